"""Pins of the PyTorch restatement used for reference gradients (oracle/torch_ref.py):
its forward values equal the C oracle's, and its reverse-mode gradients equal
central differences of the C oracle."""
import math

import numpy as np
import pytest

from paper_2211_16718_amd import inputs as I

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def tr():
    from oracle import torch_ref

    return torch_ref


def setup(orc, n=12, seed=4, mu=0.02):
    rho, vel, p = I.hit_primitives(n, seed, 0.3)
    u = orc.init_state(rho, vel, p)
    return rho, vel, p, u, orc.make_phys(mu_eff=mu), mu


def test_forward_matches_c_oracle(orc, tr):
    rho, vel, p, u, ph, mu = setup(orc)
    ut = torch.from_numpy(u)
    tph = tr.make_phys(mu=mu)
    for d in range(3):
        np.testing.assert_allclose(tr.rhs_hyp_dir(ut, d, tph).numpy(), orc.rhs_hyp_dir(u, d, ph),
                                   rtol=0, atol=1e-13 * np.abs(orc.rhs_hyp_dir(u, d, ph)).max())
    v = orc.viscous(u, ph)
    np.testing.assert_allclose(tr.viscous(ut, tph).numpy(), v, rtol=0, atol=1e-13 * np.abs(v).max())
    r = orc.rhs(u, ph)
    np.testing.assert_allclose(tr.rhs(ut, tph).numpy(), r, rtol=0, atol=1e-13 * np.abs(r).max())
    # initial state map and kinetic energy
    np.testing.assert_allclose(tr.ic_state(torch.from_numpy(rho), torch.from_numpy(vel), torch.from_numpy(p),
                                           1.4).numpy(), u, rtol=1e-15, atol=1e-15)
    assert float(tr.kinetic_energy(ut)) == pytest.approx(orc.diag(u, ph)[0], rel=1e-14)


def test_forward_rk4_matches_c_oracle(orc, tr):
    rho, vel, p, u, ph, mu = setup(orc, n=10)
    dt = I.dt_from_speed(orc.diag(u, ph)[7], 10)
    uf, _ = orc.rk4(u, dt, 2, ph, with_diag=False)
    x = torch.from_numpy(u)
    for _ in range(2):
        x = tr.rk4_step(x, dt, tr.make_phys(mu=mu))
    np.testing.assert_allclose(x.numpy(), uf, rtol=0, atol=1e-13 * np.abs(uf).max())


def test_rhs_vjp_matches_central_differences_of_the_c_oracle(orc, tr):
    # <VJP(rbar), d> must equal <rbar, (R(u + h d) - R(u - h d)) / 2h> for random d
    rho, vel, p, u, ph, mu = setup(orc, n=10, seed=6)
    rng = np.random.default_rng(0)
    rbar = rng.standard_normal(u.shape)
    g = tr.rhs_vjp(torch.from_numpy(u), torch.from_numpy(rbar), tr.make_phys(mu=mu)).numpy()
    for k in range(3):
        # white-noise directions excite the WENO weights' curvature: small h (the
        # central difference converges quadratically: 3.6e-3, 4.8e-5, 4.8e-7, 6e-9
        # relative for h = 1e-4 .. 1e-7 on this state)
        d = rng.standard_normal(u.shape) * np.abs(u).mean(axis=(1, 2, 3), keepdims=True)
        h = 1e-7
        fd = (orc.rhs(u + h * d, ph) - orc.rhs(u - h * d, ph)) / (2 * h)
        lhs = float(np.sum(g * d))
        rhs = float(np.sum(rbar * fd))
        assert lhs == pytest.approx(rhs, rel=1e-7), (k, lhs, rhs)


def test_final_ke_gradient_matches_central_differences(orc, tr):
    # gradient of the final kinetic energy w.r.t. the initial velocity
    n, steps = 8, 3
    rho, vel, p = I.hit_primitives(n, 2, 0.3)
    mu = 0.02
    ph = orc.make_phys(mu_eff=mu)
    u0 = orc.init_state(rho, vel, p)
    dt = I.dt_from_speed(orc.diag(u0, ph)[7], n)
    J, gv = tr.final_ke_and_grad(torch.from_numpy(rho), torch.from_numpy(vel), torch.from_numpy(p), dt, steps,
                                 tr.make_phys(mu=mu))

    def Jc(v):
        uf, _ = orc.rk4(orc.init_state(rho, v, p), dt, steps, ph, with_diag=False)
        return orc.diag(uf, ph)[0]

    assert J == pytest.approx(Jc(vel), rel=1e-13)
    rng = np.random.default_rng(1)
    for k in range(2):
        d = I.hit_velocity(n, seed=100 + k)
        h = 1e-6
        fd = (Jc(vel + h * d) - Jc(vel - h * d)) / (2 * h)
        assert float(np.sum(gv.numpy() * d)) == pytest.approx(fd, rel=1e-6)


def test_forward_tvdrk3_matches_c_oracle(orc, tr):
    rho, vel, p, u, ph, mu = setup(orc, n=10)
    dt = I.dt_from_speed(orc.diag(u, ph)[7], 10)
    uf, _ = orc.tvdrk3(u, dt, 2, ph, with_diag=False)
    x = torch.from_numpy(u)
    for _ in range(2):
        x = tr.tvdrk3_step(x, dt, tr.make_phys(mu=mu))
    np.testing.assert_allclose(x.numpy(), uf, rtol=0, atol=1e-13 * np.abs(uf).max())


def test_final_ke_gradient_tvdrk3_matches_central_differences(orc, tr):
    n, steps = 8, 3
    rho, vel, p = I.hit_primitives(n, 2, 0.3)
    mu = 0.02
    ph = orc.make_phys(mu_eff=mu)
    u0 = orc.init_state(rho, vel, p)
    dt = I.dt_from_speed(orc.diag(u0, ph)[7], n)
    J, gv = tr.final_ke_and_grad(torch.from_numpy(rho), torch.from_numpy(vel), torch.from_numpy(p), dt, steps,
                                 tr.make_phys(mu=mu), step=tr.tvdrk3_step)

    def Jc(v):
        uf, _ = orc.tvdrk3(orc.init_state(rho, v, p), dt, steps, ph, with_diag=False)
        return orc.diag(uf, ph)[0]

    assert J == pytest.approx(Jc(vel), rel=1e-13)
    for k in range(2):
        d = I.hit_velocity(n, seed=200 + k)
        h = 1e-6
        fd = (Jc(vel + h * d) - Jc(vel - h * d)) / (2 * h)
        assert float(np.sum(gv.numpy() * d)) == pytest.approx(fd, rel=1e-6)


@pytest.mark.parametrize("weights", ["z", "m"])
def test_forward_improved_weights_match_c_oracle(orc, tr, weights):
    rho, vel, p, u, ph, mu = setup(orc, seed=7)
    code = {"z": orc.WENO_Z, "m": orc.WENO_M}[weights]
    phw = orc.make_phys(mu_eff=mu, weno_weights=code)
    ut = torch.from_numpy(u)
    tph = tr.make_phys(mu=mu, weights=weights)
    for d in range(3):
        ref = orc.rhs_hyp_dir(u, d, phw)
        np.testing.assert_allclose(tr.rhs_hyp_dir(ut, d, tph).numpy(), ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    # and the weights differ from the Jiang-Shu ones on this state
    assert np.abs(orc.rhs_hyp_dir(u, 0, phw) - orc.rhs_hyp_dir(u, 0, ph)).max() > 1e-6


@pytest.mark.parametrize("weights", ["z", "m"])
def test_rhs_vjp_improved_weights_match_central_differences(orc, tr, weights):
    rho, vel, p, u, ph, mu = setup(orc, n=10, seed=8)
    phw = orc.make_phys(mu_eff=mu, weno_weights={"z": orc.WENO_Z, "m": orc.WENO_M}[weights])
    rng = np.random.default_rng(3)
    rbar = rng.standard_normal(u.shape)
    g = tr.rhs_vjp(torch.from_numpy(u), torch.from_numpy(rbar), tr.make_phys(mu=mu, weights=weights)).numpy()
    for k in range(2):
        d = rng.standard_normal(u.shape) * np.abs(u).mean(axis=(1, 2, 3), keepdims=True)
        h = 1e-7
        fd = (orc.rhs(u + h * d, phw) - orc.rhs(u - h * d, phw)) / (2 * h)
        assert float(np.sum(g * d)) == pytest.approx(float(np.sum(rbar * fd)), rel=1e-7), k
