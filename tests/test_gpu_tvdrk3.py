"""TVD-RK3 (Shu-Osher) on the GPU against the oracle's TVD-RK3.

FP64: 1e-10 joint relative max-norm after 10 steps, as for RK4.  Mixed: the FP32
state against the FP64 oracle to the mixed form's bar.  The ensemble and graph
paths run the same fused stage kernels, so they must agree bitwise with a
single-box eager run."""
import numpy as np
import pytest

from conftest import rel_max
from paper_2211_16718_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2211_16718_amd.api import Ensemble, Plan  # noqa: E402


def case(msg):
    print(f"[case] {msg}", flush=True)


@pytest.mark.parametrize("shape,mu,steps", [((32, 32, 32), 0.01, 10), ((20, 12, 36), 0.05, 4), ((9, 17, 8), 0.0, 3)])
def test_tvdrk3_matches_oracle(orc, shape, mu, steps):
    case(f"tvdrk3 {shape} mu={mu} x{steps}")
    nz, ny, nx = shape
    n = max(shape)
    rho, vel, p = I.hit_primitives(n, 1, 0.3)
    rho, vel, p = (np.ascontiguousarray(a) for a in (rho[:nz, :ny, :nx], vel[:, :nz, :ny, :nx], p[:nz, :ny, :nx]))
    ph = orc.make_phys(mu_eff=mu)
    u_ref = orc.init_state(rho, vel, p)
    dt = I.dt_from_speed(orc.diag(u_ref, ph)[7], n)
    plan = Plan(shape, mu_eff=mu)
    u = plan.init_state(rho, vel, p)
    diag = plan.tvdrk3(u, dt, steps).cpu().numpy()
    uf_ref, diag_ref = orc.tvdrk3(u_ref, dt, steps, ph)
    err = rel_max(u.cpu().numpy(), uf_ref)
    print(f"tvdrk3 state rel err {err:.3e}")
    assert err <= 1e-10
    np.testing.assert_allclose(diag[:, :8], diag_ref[:, :8], rtol=1e-11, atol=1e-14)
    assert np.all(diag[:, 8] == 0)
    # the integrators differ at O(dt^4) per step: a wrong stage weight would show here
    u4, _ = orc.rk4(u_ref, dt, steps, ph, with_diag=False)
    assert rel_max(u.cpu().numpy(), u4) > 10 * err


def test_tvdrk3_mixed_precision(orc):
    case("tvdrk3 mixed 32^3 x5")
    rho, vel, p = I.hit_primitives(32, 2, 0.3)
    ph = orc.make_phys(mu_eff=0.01)
    u_ref = orc.init_state(rho, vel, p)
    dt = I.dt_from_speed(orc.diag(u_ref, ph)[7], 32)
    plan = Plan((32, 32, 32), mu_eff=0.01, precision="mixed")
    u = plan.init_state(rho, vel, p)
    diag = plan.tvdrk3(u, dt, 5).cpu().numpy()
    assert u.dtype == torch.float32
    uf_ref, diag_ref = orc.tvdrk3(u_ref, dt, 5, ph)
    err = rel_max(u.double().cpu().numpy(), uf_ref)
    print(f"mixed tvdrk3 rel err {err:.3e}, K rel {abs(diag[-1, 0] / diag_ref[-1, 0] - 1):.3e}")
    assert err <= 2e-6
    assert abs(diag[-1, 0] / diag_ref[-1, 0] - 1) <= 1e-6


def test_tvdrk3_ensemble_and_graph_bitwise():
    import oracle

    case("tvdrk3 ensemble + graph vs single eager")
    stream = torch.cuda.Stream()
    specs = [(24, 0.3, 200.0, 3), (16, 0.2, 500.0, 4), (20, 0.45, 120.0, 5)]
    boxes = []
    for n, mt, re, seed in specs:
        rho, vel, p = I.hit_primitives(n, seed, mt)
        smax = oracle.diag(oracle.init_state(rho, vel, p), oracle.make_phys(mu_eff=1 / re))[7]
        boxes.append(dict(shape=(n, n, n), mu_eff=1 / re, dt=I.dt_from_speed(smax, n), prim=(rho, vel, p)))
    ens = Ensemble([{k: v for k, v in b.items() if k != "prim"} for b in boxes], stream=stream)
    for i, b in enumerate(boxes):
        plan = Plan(b["shape"], mu_eff=b["mu_eff"], stream=stream)
        with torch.cuda.stream(stream):
            plan.init_state(*b["prim"], out=ens.state(i))
    ens.set_integrator("tvdrk3")
    with torch.cuda.stream(stream):
        diag = ens.run(3, graph=True)
    stream.synchronize()
    for i, b in enumerate(boxes):
        plan = Plan(b["shape"], mu_eff=b["mu_eff"], stream=stream)
        with torch.cuda.stream(stream):
            u = plan.init_state(*b["prim"])
            d = plan.tvdrk3(u, b["dt"], 3)
        stream.synchronize()
        assert torch.equal(ens.state(i), u), f"box {i}"
        assert torch.equal(diag[i], d), f"diag box {i}"
    # graph replays of a single plan equal eager steps, replay after replay
    b = boxes[0]
    pe = Plan(b["shape"], mu_eff=b["mu_eff"], stream=stream)
    pg = Plan(b["shape"], mu_eff=b["mu_eff"], stream=stream)
    pg.set_graph(True)
    with torch.cuda.stream(stream):
        ue = pe.init_state(*b["prim"])
        ug = pg.init_state(*b["prim"])
    for rep in range(3):
        with torch.cuda.stream(stream):
            pe.tvdrk3(ue, b["dt"], 2)
            pg.tvdrk3(ug, b["dt"], 2)
            pg.rk4(ug, b["dt"], 1)  # switching integrators must not replay the wrong graph
            pe.rk4(ue, b["dt"], 1)
        stream.synchronize()
        assert torch.equal(ue, ug), f"replay {rep}"
    assert ens.lib.cns_ensemble_set_integrator(ens.h, 7) == -1  # CNS_EINVAL
