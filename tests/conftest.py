import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def live_line(config, msg):
    """Write a progress line to the run's output even while pytest captures
    the test's output (long tests keep the run's output moving): the capture
    is suspended for the write."""
    capman = config.pluginmanager.getplugin("capturemanager")
    if capman is None:
        print(msg, flush=True)
        return
    with capman.global_and_fixture_disabled():
        print(msg, flush=True)
