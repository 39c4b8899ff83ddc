"""Host-side checks of the C-ABI library (no GPU needed, no kernel launched)."""
import ctypes as C
import os
import re

import pytest

from paper_2310_17214_amd import lbfd, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lbfd.h")).read()
    return sorted(set(re.findall(r"^\s*(?:lbfd_status|const char\*)\s+(lbfd_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    L = lbfd.lib()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(lbfd.EXPORTED)


def test_no_oracle_in_product_path():
    """The product library links nothing from the oracle and the binding
    never imports it."""
    pkg = os.path.join(ROOT, "paper_2310_17214_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".inc", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"(from|import)\s+oracle|lbfd_oracle|orc_", txt), f
    so = open(lbfd.LIB_PATH, "rb").read()
    assert b"orc_step" not in so


def _grid(**kw):
    s = W.cylinder_channel().setup
    g = lbfd.make_grid(s)
    for k, v in kw.items():
        setattr(g, k, v)
    return g


def test_workspace_bytes_and_validation():
    L = lbfd.lib()
    n = C.c_size_t()
    assert L.lbfd_workspace_bytes(C.byref(_grid()), C.byref(n)) == 0
    # D2Q9 FP64, in-place (AA) populations: 9 planes + 2 T + divu + phi, plus
    # workgroup partials and a 5-plane FP64 read scratch
    N = 128 * 64
    assert N * 8 * (9 + 4 + 5) <= n.value < N * 8 * (9 + 4 + 5) + 2 ** 20
    for bad in (dict(dim=4), dict(nx=1), dict(nz=3), dict(precision=7), dict(n_species=17)):
        assert L.lbfd_workspace_bytes(C.byref(_grid(**bad)), C.byref(n)) == lbfd.LBFD_E_INVAL
    g = _grid()
    g.lb_bc[2] = 0  # periodic LB face with a non-periodic FD face
    assert L.lbfd_workspace_bytes(C.byref(g), C.byref(n)) == lbfd.LBFD_E_INVAL
    g = _grid()
    g.lb_bc[1] = 2  # inlet on the +x face
    assert L.lbfd_workspace_bytes(C.byref(g), C.byref(n)) == lbfd.LBFD_E_UNSUPPORTED


def test_create_rejects_bad_workspace_before_touching_the_device():
    L = lbfd.lib()
    g = _grid()
    n = C.c_size_t()
    L.lbfd_workspace_bytes(C.byref(g), C.byref(n))
    h = C.c_void_p()
    assert L.lbfd_create(C.byref(g), None, n.value, None, C.byref(h)) == lbfd.LBFD_E_INVAL
    assert L.lbfd_create(C.byref(g), C.c_void_p(256), n.value - 1, None,
                         C.byref(h)) == lbfd.LBFD_E_NOMEM
    assert L.lbfd_create(C.byref(g), C.c_void_p(257), n.value, None,
                         C.byref(h)) == lbfd.LBFD_E_INVAL
    assert L.lbfd_last_error(None) == b"null context"


def test_bytes_per_cell_formula():
    """Algorithmic bytes per cell and step of the fused kernel:
    s * (2Q + 2 + 2 ns + 2 + 1) -- populations and T, Y, divu read and written
    once, phi read once."""
    assert 4 * (2 * 19 + 2 + 2 * 4 + 2 + 1) == 204


def test_largest_grids():
    """The 1024x256x256 elongated bed (D3Q19, FP32, 9 species) fits the
    indexing limits and its workspace is what the layout says (about 209 B
    per cell); a grid with more than 2^31 population slots is rejected."""
    L = lbfd.lib()
    n = C.c_size_t()
    big = dict(dim=3, nx=1024, ny=256, nz=256, precision=lbfd.FP32, n_species=9)
    g = _grid(**big)
    for f in range(6):
        g.lb_bc[f] = g.fd_bc[f] = 0
    assert L.lbfd_workspace_bytes(C.byref(g), C.byref(n)) == 0
    cells = 1024 * 256 * 256
    assert 200 * cells < n.value < 220 * cells
    g.nx, g.ny, g.nz = 1024, 1024, 128  # 19 x 134 M slots > 2^31
    assert L.lbfd_workspace_bytes(C.byref(g), C.byref(n)) == lbfd.LBFD_E_INVAL
