"""Pins of the oracle's RK4 time integration (paper Sec. 2.2: the ODE from the
spatial discretisation advanced by classical fourth-order Runge-Kutta), its
diagnostics, and the time-accurate solver as a whole (isentropic vortex)."""
import math

import numpy as np
import pytest

from paper_2211_16718_amd import inputs as I

GAMMA = 1.4


def kstar(k, h):
    return (8 * math.sin(k * h) - math.sin(2 * k * h)) / (6 * h)


def test_rk4_amplification_on_the_linear_shear_wave(orc):
    # rho u = A sin y with tiny A: d(rho u)/dt = -mu k*^2 (rho u) + O(A^3), so after
    # n steps rho u = R(z)^n A sin y with R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24,
    # z = -mu k*^2 dt.  Any wrong stage weight changes R at O(z^2) or above.
    n, mu, A = 8, 0.5, 1e-5
    h = 2 * math.pi / n
    y = I.grid_coords(n)[None, :, None] * np.ones((n, n, n))
    vel = np.zeros((3, n, n, n))
    vel[0] = A * np.sin(y)
    u = orc.init_state(np.ones((n, n, n)), vel, np.full((n, n, n), 1.0))
    dt, steps = 0.5, 6  # z ~ -0.24: large enough to see every term of R
    z = -mu * kstar(1, h) ** 2 * dt
    R = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    uf, _ = orc.rk4(u, dt, steps, orc.make_phys(mu_eff=mu), with_diag=False)
    expect = R ** steps * A * np.sin(y)
    assert np.abs(uf[1] - expect).max() <= 1e-8 * A
    # the tolerance resolves the truncation of exp(z): R^n differs from e^{nz}
    assert abs(R ** steps - math.exp(steps * z)) > 100 * 1e-8


def test_tvdrk3_amplification_on_the_linear_shear_wave(orc):
    # Shu-Osher TVD-RK3 on d(rho u)/dt = z/dt (rho u): R3(z) = 1 + z + z^2/2 + z^3/6
    n, mu, A = 8, 0.5, 1e-5
    h = 2 * math.pi / n
    y = I.grid_coords(n)[None, :, None] * np.ones((n, n, n))
    vel = np.zeros((3, n, n, n))
    vel[0] = A * np.sin(y)
    u = orc.init_state(np.ones((n, n, n)), vel, np.full((n, n, n), 1.0))
    dt, steps = 0.5, 6
    z = -mu * kstar(1, h) ** 2 * dt
    R3 = 1 + z + z * z / 2 + z ** 3 / 6
    uf, _ = orc.tvdrk3(u, dt, steps, orc.make_phys(mu_eff=mu), with_diag=False)
    assert np.abs(uf[1] - R3 ** steps * A * np.sin(y)).max() <= 1e-8 * A
    R4 = R3 + z ** 4 / 24
    assert abs(R3 ** steps - R4 ** steps) > 100 * 1e-8  # distinguishable from RK4


def test_tvdrk3_conserves_and_matches_rk4_to_third_order(orc):
    rho, vel, p = I.hit_primitives(12, 3, 0.3)
    u = orc.init_state(rho, vel, p)
    ph = orc.make_phys(mu_eff=0.01)
    d0 = orc.diag(u, ph)
    errs = []
    for dt in (0.004, 0.002):
        steps = int(round(0.008 / dt))
        u3, dg = orc.tvdrk3(u, dt, steps, ph)
        u4, _ = orc.rk4(u, dt, steps, ph, with_diag=False)
        errs.append(np.abs(u3 - u4).max())
        assert abs(dg[-1][2] - d0[2]) <= 1e-14 and abs(dg[-1][6] - d0[6]) <= 1e-14 * d0[6]
    # global error of a third-order scheme: halving dt divides the difference by ~8
    assert 6.0 < errs[0] / errs[1] < 10.0, errs


def test_rk4_keeps_a_free_stream_bitwise(orc):
    rho, vel, p = I.uniform_primitives(0, rho=0.9, vel=(0.5, 0.1, -0.3), p=1.7, shape=(8, 9, 10))
    u = orc.init_state(rho, vel, p)
    uf, _ = orc.rk4(u, 0.01, 3, orc.make_phys(mu_eff=0.01), with_diag=False)
    np.testing.assert_array_equal(uf, u)


def test_rk4_conserves_mass_momentum_energy(orc):
    rho, vel, p = I.hit_primitives(16, 1, 0.3)
    u = orc.init_state(rho, vel, p)
    ph = orc.make_phys(mu_eff=0.01)
    d0 = orc.diag(u, ph)
    dt = I.dt_from_speed(d0[7], 16)
    uf, dg = orc.rk4(u, dt, 3, ph)
    for k, scale in [(2, 1.0), (3, 1.0), (4, 1.0), (5, 1.0), (6, d0[6])]:
        assert abs(dg[-1][k] - d0[k]) <= 1e-14 * scale
    assert dg[-1][0] < d0[0]  # kinetic energy decays


def test_kinetic_energy_and_enstrophy_closed_forms(orc):
    n, A = 16, 0.4
    h = 2 * math.pi / n
    y = I.grid_coords(n)[None, :, None] * np.ones((n, n, n))
    vel = np.zeros((3, n, n, n))
    vel[0] = A * np.sin(y)
    rho = np.full((n, n, n), 1.3)
    u = orc.init_state(rho, vel, np.full((n, n, n), 1.0))
    d = orc.diag(u, orc.make_phys())
    assert d[0] == pytest.approx(0.5 * 1.3 * A * A * 0.5, rel=1e-13)  # <sin^2> = 1/2
    # omega_z = -D_y u = -A k* cos y ; Omega = 1/2 <omega^2> = A^2 k*^2 / 4
    assert d[1] == pytest.approx(A * A * kstar(1, h) ** 2 / 4, rel=1e-13)
    assert d[2] == pytest.approx(1.3, rel=1e-15)
    c = math.sqrt(GAMMA * 1.0 / 1.3)
    assert d[7] == pytest.approx(A + c, rel=1e-12)
    assert d[8] == 0


def test_diagnostics_flag_bad_points(orc):
    rho, vel, p = I.hit_primitives(8, 0, 0.3)
    u = orc.init_state(rho, vel, p)
    u[0, 1, 1, 1] = -0.5
    u[2, 3, 3, 3] = np.inf
    d = orc.diag(u, orc.make_phys())
    assert d[8] == 2


def test_isentropic_vortex_converges_to_the_exact_solution(orc):
    # Euler equations; the vortex advected by (1,1,0) is an exact solution.  A thin
    # periodic slab (nz = 8) suffices since the flow is z-independent.
    ph = orc.make_phys(mu_eff=0.0)
    errs = []
    for n in (32, 64):
        rho, vel, p = I.vortex_primitives(n, nz=8)
        u = orc.init_state(rho, vel, p)
        dtc = I.dt_from_speed(orc.diag(u, ph)[7], n)
        T = 1.0
        steps = math.ceil(T / dtc)
        uf, _ = orc.rk4(u, T / steps, steps, ph, with_diag=False)
        re, ve, pe = I.vortex_primitives(n, t=T, nz=8)
        ue = orc.init_state(re, ve, pe)
        errs.append(max(np.abs(uf[v] - ue[v]).max() for v in range(5)))
        np.testing.assert_array_equal(uf[3], 0.0)  # no z momentum ever appears
    order = math.log2(errs[0] / errs[1])
    assert order > 3.0 and errs[1] < 1e-2, errs
