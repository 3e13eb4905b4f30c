"""Mixed precision (FP32 state and WENO/flux arithmetic; FP64 smoothness-indicator
sums and RK4 accumulation) against the FP64 oracle and the FP64 GPU path.

The mixed form is not bitwise comparable with anything; its error is bounded by
FP32 round-off amplified by the flux difference: the interface fluxes carry a
relative error ~ a few * 2^-24 of |F|, and the difference divides by dx, so the
RHS error relative to max|RHS| is ~ 1e-7 * (N / 2 pi) * max|F| / max|RHS|.  The
tolerances below allow a factor ~10 over the values measured on the workloads.
"""
import numpy as np
import pytest

from conftest import rel_max
from paper_2211_16718_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2211_16718_amd.api import Plan  # noqa: E402


def case(msg):
    print(f"[case] {msg}", flush=True)


def test_mixed_rhs_against_oracle(orc):
    case("mixed rhs 32^3")
    n = 32
    rho, vel, p = I.hit_primitives(n, 0, 0.3)
    ph = orc.make_phys(mu_eff=0.01)
    ref = orc.rhs(orc.init_state(rho, vel, p), ph)
    plan = Plan((n, n, n), mu_eff=0.01, precision="mixed")
    got = plan.rhs(plan.init_state(rho, vel, p)).double().cpu().numpy()
    err = rel_max(got, ref)
    per_var = [rel_max(got[v], ref[v]) for v in range(5)]
    print(f"mixed rhs joint rel err {err:.3e}; per variable {per_var}")
    assert err <= 2e-5


def test_mixed_rk4_against_oracle(orc):
    case("mixed rk4 32^3 x10")
    n = 32
    rho, vel, p = I.hit_primitives(n, 0, 0.3)
    ph = orc.make_phys(mu_eff=0.01)
    u_ref = orc.init_state(rho, vel, p)
    dt = I.dt_from_speed(orc.diag(u_ref, ph)[7], n)
    uf_ref, dref = orc.rk4(u_ref, dt, 10, ph)
    plan = Plan((n, n, n), mu_eff=0.01, precision="mixed")
    u = plan.init_state(rho, vel, p)
    d = plan.rk4(u, dt, 10).cpu().numpy()
    err = rel_max(u.double().cpu().numpy(), uf_ref)
    ke_err = abs(d[-1, 0] - dref[-1, 0]) / dref[-1, 0]
    print(f"mixed rk4 state rel err {err:.3e}, KE rel err {ke_err:.3e}")
    assert err <= 2e-6
    assert ke_err <= 1e-6
    assert np.all(d[:, 8] == 0)


def test_mixed_against_fp64_gpu_128():
    case("mixed vs fp64 GPU 128^3 x5")
    n = 128
    rho, vel, p = I.hit_primitives(n, 0, 0.3)
    p64 = Plan((n, n, n), mu_eff=1 / 400)
    p32 = Plan((n, n, n), mu_eff=1 / 400, precision="mixed")
    u64 = p64.init_state(rho, vel, p)
    u32 = p32.init_state(rho, vel, p)
    dt = I.dt_from_speed(p64.diagnostics_host(u64)[7], n)
    d64 = p64.rk4(u64, dt, 5).cpu().numpy()
    d32 = p32.rk4(u32, dt, 5).cpu().numpy()
    a, b = u32.double(), u64
    per_var = [float((a[v] - b[v]).abs().max() / b[v].abs().max()) for v in range(5)]
    ke = abs(d32[-1, 0] - d64[-1, 0]) / d64[-1, 0]
    print(f"mixed vs fp64 per-variable max-norm rel err {per_var}, KE rel err {ke:.3e}")
    assert max(per_var) <= 1e-5 and ke <= 1e-6
