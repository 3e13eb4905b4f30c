"""The C-ABI library loads and exports every symbol its header declares
(no compute call: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if not h.endswith(".h"):
            continue
        txt = open(os.path.join(ROOT, "include", h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names += re.findall(r"\b(cns_[a-z0-9_]+)\s*\(", txt)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("cns_plan_create", "cns_rhs", "cns_rk4", "cns_diagnostics", "cns_init_state"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2211_16718_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libcns.so not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding's table covers the header
    assert set(declared_functions()) <= set(_lib.SIGNATURES)


def test_plan_validation_without_gpu():
    """Argument checks happen on the host before any device call."""
    from paper_2211_16718_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libcns.so not built")
    lib = _lib.load()
    h = ctypes.c_void_p()
    g = _lib.Grid(4, 16, 16, 1.0, 1.0, 1.0)
    ph = _lib.Physics(1.4, 0.72, 0.01, 1e-6, 1e-6)
    assert lib.cns_plan_create(ctypes.byref(h), ctypes.byref(g), ctypes.byref(ph), 0, None) == -1
    assert b"at least 8" in lib.cns_last_error()
    g = _lib.Grid(16, 16, 16, 1.0, 1.0, 1.0)
    bad = _lib.Physics(1.0, 0.72, 0.01, 1e-6, 1e-6)
    assert lib.cns_plan_create(ctypes.byref(h), ctypes.byref(g), ctypes.byref(bad), 0, None) == -1
    assert lib.cns_plan_create(ctypes.byref(h), ctypes.byref(g), ctypes.byref(ph), 7, None) == -1
    assert lib.cns_plan_create(ctypes.byref(h), ctypes.byref(g), ctypes.byref(ph), 0, None) == 0
    nbytes = lib.cns_workspace_bytes(h)
    assert nbytes >= (9 + 5 + 5 + 5 + 5) * 8 * 16 ** 3  # G, rhs, A, B, acc
    # no workspace bound -> compute calls refuse before touching the device
    assert lib.cns_rhs(h, ctypes.c_void_p(256), ctypes.c_void_p(512)) == -5
    assert lib.cns_set_workspace(h, ctypes.c_void_p(257), nbytes) == -1
    assert lib.cns_set_tiles(h, 4, 0, 0, 100) == -1
    assert lib.cns_plan_destroy(h) == 0


@pytest.mark.parametrize("grid,phys,msg", [
    ((1024, 1024, 512), None, b"too large"),           # 8 n3 = 2^32: past the 32-bit offsets
    ((812, 812, 812), None, None),                      # the largest cube that fits (8 n3 < 2^32)
    (None, dict(gamma=1.0), b"gamma"),
    (None, dict(mu_eff=-1e-3), b"mu_eff"),
    (None, dict(weno_eps=0.0), b"weno_eps"),
    (None, dict(weno_eps=1e31), b"weno_eps"),
    (None, dict(harten_delta=-1.0), b"harten_delta"),
    (None, dict(mu_eff=0.01, prandtl=0.0), b"prandtl"),
])
def test_plan_limits_without_gpu(grid, phys, msg):
    """Grid size and physics limits are checked on the host; a plan within them is created
    without touching the device (its workspace is the caller's)."""
    from paper_2211_16718_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libcns.so not built")
    lib = _lib.load()
    nx, ny, nz = grid or (16, 16, 16)
    g = _lib.Grid(nx, ny, nz, 1.0, 1.0, 1.0)
    p = dict(gamma=1.4, prandtl=0.72, mu_eff=0.01, weno_eps=1e-6, harten_delta=1e-6)
    p.update(phys or {})
    ph = _lib.Physics(p["gamma"], p["prandtl"], p["mu_eff"], p["weno_eps"], p["harten_delta"])
    h = ctypes.c_void_p()
    rc = lib.cns_plan_create(ctypes.byref(h), ctypes.byref(g), ctypes.byref(ph), 0, None)
    if msg is None:
        assert rc == 0
        assert lib.cns_workspace_bytes(h) > 29 * 8 * nx * ny * nz
        assert lib.cns_plan_destroy(h) == 0
    else:
        assert rc == -1 and msg in lib.cns_last_error()
