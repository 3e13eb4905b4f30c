"""Pins of the oracle's full right-hand side (paper Sec. 2.1 equation (NS),
Sec. 2.2 conservative finite differences): invariants that hold exactly for
the discrete operator, and convergence to the continuous equations."""
import math

import numpy as np
import pytest

from paper_2211_16718_amd import inputs as I

GAMMA, PR = 1.4, 0.72


def hit_state(orc, n, seed=0, mt=0.3):
    rho, vel, p = I.hit_primitives(n, seed, mt)
    return orc.init_state(rho, vel, p)


def test_free_stream_is_preserved_exactly(orc):
    for shape in [(8, 8, 8), (9, 12, 10)]:
        rho, vel, p = I.uniform_primitives(0, rho=1.3, vel=(0.7, -0.4, 0.2), p=2.1, shape=shape)
        u = orc.init_state(rho, vel, p)
        r = orc.rhs(u, orc.make_phys(mu_eff=0.01))
        np.testing.assert_array_equal(r, 0.0)


@pytest.mark.parametrize("mu", [0.0, 0.01])
def test_domain_sums_of_the_rhs_vanish(orc, mu):
    # conservative differences telescope on a periodic grid
    u = hit_state(orc, 16)
    r = orc.rhs(u, orc.make_phys(mu_eff=mu))
    for v in range(5):
        assert abs(r[v].sum()) <= 1e-13 * np.abs(r[v]).sum() + 1e-300


def test_shift_equivariance_is_bitwise(orc):
    u = hit_state(orc, 16, seed=3)
    ph = orc.make_phys(mu_eff=0.01)
    r = orc.rhs(u, ph)
    for axis, s in [(1, 3), (2, -5), (3, 7)]:
        r2 = orc.rhs(np.roll(u, s, axis=axis), ph)
        np.testing.assert_array_equal(r2, np.roll(r, s, axis=axis))


def test_axis_permutation_symmetry(orc):
    # swap x and y: arrays transpose their last two axes, momentum slots 1,2 swap
    u = hit_state(orc, 12, seed=4)
    ph = orc.make_phys(mu_eff=0.02)
    r = orc.rhs(u, ph)
    up = np.ascontiguousarray(np.swapaxes(u, 2, 3)[[0, 2, 1, 3, 4]])
    rp = orc.rhs(up, ph)
    expect = np.swapaxes(r, 2, 3)[[0, 2, 1, 3, 4]]
    np.testing.assert_allclose(rp, expect, rtol=0, atol=1e-14 * np.abs(r).max())


def test_mirror_symmetry(orc):
    # x -> -x: point i maps to (-i) mod n, x-momentum changes sign.  This
    # exercises the right-biased (mirrored) WENO reconstruction.
    u = hit_state(orc, 12, seed=6)
    ph = orc.make_phys(mu_eff=0.01)
    r = orc.rhs(u, ph)
    idx = (-np.arange(12)) % 12
    sign = np.array([1, -1, 1, 1, 1])[:, None, None, None]
    um = np.ascontiguousarray(u[..., idx] * sign)
    rm = orc.rhs(um, ph)
    np.testing.assert_allclose(rm, r[..., idx] * sign, rtol=0, atol=1e-13 * np.abs(r).max())


# ---- convergence to the continuous equations ---------------------------------
def spectral_d(f, axis, length=2 * math.pi):
    n = f.shape[axis]
    k = np.fft.fftfreq(n, d=length / n) * 2 * math.pi
    shape = [1] * f.ndim
    shape[axis] = n
    return np.fft.ifft(np.fft.fft(f, axis=axis) * (1j * k).reshape(shape), axis=axis).real


def continuous_rhs(rho, vel, p, mu, gamma=GAMMA, pr=PR):
    """du/dt of the compressible NS equations with exact (spectral) derivatives
    of the grid values; accurate to round-off for the smooth fields used."""
    ax = {0: 2, 1: 1, 2: 0}
    e = p / (gamma - 1) + 0.5 * rho * (vel ** 2).sum(0)
    m = rho * vel
    out = np.zeros((5,) + rho.shape)
    for d in range(3):
        vn = vel[d]
        F = [rho * vn, m[0] * vn, m[1] * vn, m[2] * vn, (e + p) * vn]
        F[1 + d] = F[1 + d] + p
        for v in range(5):
            out[v] -= spectral_d(F[v], ax[d])
    if mu > 0:
        T = gamma * p / rho
        g = [[spectral_d(vel[a], ax[b]) for b in range(3)] for a in range(3)]
        div = g[0][0] + g[1][1] + g[2][2]
        for d in range(3):
            tau_d = [mu * (g[a][d] + g[d][a] - (2 / 3 * div if a == d else 0)) for a in range(3)]
            qd = -mu / ((gamma - 1) * pr) * spectral_d(T, ax[d])
            G = [tau_d[0], tau_d[1], tau_d[2], vel[0] * tau_d[0] + vel[1] * tau_d[1] + vel[2] * tau_d[2] - qd]
            for v in range(4):
                out[1 + v] += spectral_d(G[v], ax[d])
    return out


@pytest.mark.parametrize("mu", [0.0, 0.05])
def test_rhs_converges_to_the_continuous_equations(orc, mu):
    # smooth band-limited fields; the discrete RHS must approach the exact one at
    # the scheme's order (5 for the Euler part, 4 for the viscous part).
    errs = []
    ns = [16, 32, 64]
    spec = None
    for n in ns:
        shape = (n, n, n)
        if spec is None:
            rho, vel, p, spec = I.smooth_primitives(shape, seed=7, amp=0.4, kmax=1, mean_vel=(0.3, -0.2, 0.1))
        else:
            rho, vel, p = I.smooth_eval(shape, spec)
        u = orc.init_state(rho, vel, p)
        r = orc.rhs(u, orc.make_phys(mu_eff=mu))
        ex = continuous_rhs(rho, vel, p, mu)
        errs.append(np.abs(r - ex).max() / np.abs(ex).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert orders[-1] > (4.5 if mu == 0 else 3.7), (errs, orders)
    assert errs[-1] < 1e-5


def test_rhs_point_matches_full_grid(orc):
    u = hit_state(orc, 16, seed=8)
    ph = orc.make_phys(mu_eff=0.01)
    r = orc.rhs(u, ph)
    rng = np.random.default_rng(0)
    for _ in range(20):
        i, j, k = rng.integers(0, 16, size=3)
        np.testing.assert_array_equal(orc.rhs_point(u, i, j, k, ph), r[:, k, j, i])


def test_errors_are_reported(orc):
    u = hit_state(orc, 8)
    u[0, 1, 2, 3] = -1.0
    with pytest.raises(orc.OracleError) as e:
        orc.rhs(u, orc.make_phys())
    assert e.value.code == -4
    u = hit_state(orc, 8)
    u[4, 0, 0, 0] = np.nan
    with pytest.raises(orc.OracleError) as e:
        orc.rhs(u, orc.make_phys())
    assert e.value.code in (-3, -4)


@pytest.mark.parametrize("weights", ["z", "m"])
def test_improved_weights_rhs_invariants_and_convergence(orc, weights):
    # the WENO-Z and mapped-weight operators keep the exact invariants of the scheme
    # and converge to the continuous equations at fifth order
    phz = orc.make_phys(mu_eff=0.0, weno_weights={"z": orc.WENO_Z, "m": orc.WENO_M}[weights])
    rho, vel, p = I.uniform_primitives(0, rho=1.3, vel=(0.7, -0.4, 0.2), p=2.1, shape=(9, 12, 10))
    np.testing.assert_array_equal(orc.rhs(orc.init_state(rho, vel, p), phz), 0.0)
    u = hit_state(orc, 16)
    r = orc.rhs(u, phz)
    for v in range(5):
        assert abs(r[v].sum()) <= 1e-13 * np.abs(r[v]).sum()
    assert np.abs(r - orc.rhs(u, orc.make_phys(mu_eff=0.0))).max() > 1e-3 * np.abs(r).max()
    errs, spec = [], None
    for n in (16, 32, 64):
        if spec is None:
            rho, vel, p, spec = I.smooth_primitives((n, n, n), seed=7, amp=0.4, kmax=1, mean_vel=(0.3, -0.2, 0.1))
        else:
            rho, vel, p = I.smooth_eval((n, n, n), spec)
        r = orc.rhs(orc.init_state(rho, vel, p), phz)
        ex = continuous_rhs(rho, vel, p, 0.0)
        errs.append(np.abs(r - ex).max() / np.abs(ex).max())
    assert math.log2(errs[-2] / errs[-1]) > 4.5, errs


def test_unknown_weno_weights_are_rejected(orc):
    u = hit_state(orc, 8)
    with pytest.raises(orc.OracleError):
        orc.rhs(u, orc.make_phys(weno_weights=5))
