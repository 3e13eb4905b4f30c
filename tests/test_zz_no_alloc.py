"""The allocation-free diagnostics entry point (cns_diagnostics_static: scratch in a
static device array) against the plan-based cns_diagnostics, through the C-ABI: two
calls in a row, the second on a smaller box, FP64 and the mixed form, and the argument
errors it reports before any launch."""
import ctypes as C
import math

import numpy as np
import pytest

from paper_2211_16718_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2211_16718_amd import _lib  # noqa: E402
from paper_2211_16718_amd.api import Plan  # noqa: E402


def case(msg):
    print(f"[case] {msg}", flush=True)


def static_diag(lib, shape, u, precision, stream):
    nz, ny, nx = shape
    g = _lib.Grid(nx, ny, nz, 2 * math.pi, 2 * math.pi, 2 * math.pi)
    ph = _lib.Physics(1.4, 0.72, 0.01, 1e-6, 1e-6, 0)
    out = torch.full((9,), float("nan"), dtype=torch.float64, device=u.device)
    prec = _lib.CNS_FP64 if precision == "fp64" else _lib.CNS_MIXED
    rc = lib.cns_diagnostics_static(C.byref(g), C.byref(ph), prec, u.data_ptr(), out.data_ptr(),
                                    C.c_void_p(stream.cuda_stream))
    stream.synchronize()
    return rc, out


def test_static_diagnostics_equal_plan_diagnostics():
    lib = _lib.load()
    stream = torch.cuda.Stream()
    for precision in ("fp64", "mixed"):
        for shape in ((32, 32, 32), (20, 12, 36)):  # the second call on a smaller box
            case(f"static diagnostics {shape} {precision}")
            rho, vel, p, _ = I.smooth_primitives(shape, seed=5, amp=0.3, mean_vel=(0.2, 0.1, -0.1))
            plan = Plan(shape, mu_eff=0.01, precision=precision, stream=stream)
            with torch.cuda.stream(stream):
                u = plan.init_state(rho, vel, p)
                ref = plan.diagnostics(u)
            stream.synchronize()
            rc, out = static_diag(lib, shape, u, precision, stream)
            assert rc == 0, lib.cns_last_error()
            print(f"  static {out.cpu().numpy()}")
            assert torch.equal(out, ref)
            assert np.isfinite(out.cpu().numpy()).all()


def test_static_diagnostics_argument_errors():
    case("static diagnostics argument errors")
    lib = _lib.load()
    stream = torch.cuda.Stream()
    u = torch.zeros((5, 8, 8, 8), dtype=torch.float64, device="cuda")
    rc, _ = static_diag(lib, (8, 8, 4), u, "fp64", stream)  # nx < 8
    assert rc == -1
    out = torch.empty(9, dtype=torch.float64, device="cuda")
    g = _lib.Grid(8, 8, 8, 1.0, 1.0, 1.0)
    ph = _lib.Physics(1.4, 0.72, 0.01, 1e-6, 1e-6, 0)
    assert lib.cns_diagnostics_static(C.byref(g), C.byref(ph), 7, u.data_ptr(), out.data_ptr(), None) == -1
    assert lib.cns_diagnostics_static(C.byref(g), C.byref(ph), 0, None, out.data_ptr(), None) == -1
    assert lib.cns_diagnostics_static(C.byref(g), C.byref(ph), 0, u.data_ptr(), None, None) == -1
