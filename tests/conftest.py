import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def live_line(config, msg):
    """Write a progress line to the terminal even while pytest captures the
    test's output (long tests keep the run's output moving)."""
    tr = config.pluginmanager.get_plugin("terminalreporter")
    if tr is None:
        print(msg, flush=True)
        return
    tr.write_line(str(msg))
    tw = getattr(tr, "_tw", None)
    if tw is not None and hasattr(tw, "flush"):
        tw.flush()
