"""Pins of the oracle's Euler fluxes, Roe eigensystem and Harten fix
(paper Sec. 2.1 flux vectors and equation of state; Sec. 2.2 Roe flux,
|A| = X |Lambda| X^-1)."""
import numpy as np
import pytest

GAMMA = 1.4


def random_state(rng, rho=(0.5, 2.0), vel=3.0, p=(0.5, 5.0)):
    r = rng.uniform(*rho)
    v = rng.uniform(-vel, vel, size=3)
    pr = rng.uniform(*p)
    e = pr / (GAMMA - 1) + 0.5 * r * (v @ v)
    return np.array([r, r * v[0], r * v[1], r * v[2], e]), r, v, pr


def test_flux_at_rest_is_pressure_only(orc):
    rng = np.random.default_rng(0)
    for d in range(3):
        u, r, v, p = random_state(rng, vel=0.0)
        f = orc.flux(u, d, GAMMA)
        expect = np.zeros(5)
        expect[1 + d] = p
        np.testing.assert_allclose(f, expect, atol=1e-14)


def test_flux_matches_primitive_form_and_rotates_between_axes(orc):
    rng = np.random.default_rng(1)
    for _ in range(10):
        u, r, v, p = random_state(rng)
        e = u[4]
        fx = orc.flux(u, 0, GAMMA)
        np.testing.assert_allclose(fx, [r * v[0], r * v[0] ** 2 + p, r * v[0] * v[1], r * v[0] * v[2],
                                        (e + p) * v[0]], rtol=1e-13)
        # g(u) = P f(P u) with P swapping the x and y momentum slots
        perm = [0, 2, 1, 3, 4]
        gy = orc.flux(u, 1, GAMMA)
        fx_perm = orc.flux(u[perm], 0, GAMMA)
        np.testing.assert_allclose(gy, fx_perm[perm], rtol=1e-14, atol=1e-14)


def numeric_jacobian(orc, u, d, h=1e-6):
    J = np.zeros((5, 5))
    for c in range(5):
        e = np.zeros(5)
        step = h * max(1.0, abs(u[c]))
        e[c] = step
        # 4th-order central difference
        J[:, c] = (-orc.flux(u + 2 * e, d) + 8 * orc.flux(u + e, d) - 8 * orc.flux(u - e, d)
                   + orc.flux(u - 2 * e, d)) / (12 * step)
    return J


def test_eigenvectors_are_inverse_and_diagonalise_the_flux_jacobian(orc):
    rng = np.random.default_rng(2)
    for _ in range(8):
        u, *_ = random_state(rng)
        for d in range(3):
            X, Xi, lam = orc.roe_eigensystem(u, u, d, GAMMA)
            np.testing.assert_allclose(Xi @ X, np.eye(5), atol=1e-12)
            A = X @ np.diag(lam) @ Xi
            J = numeric_jacobian(orc, u, d)
            np.testing.assert_allclose(A, J, rtol=1e-7, atol=1e-7 * np.abs(J).max())


def test_roe_average_satisfies_property_U(orc):
    # Roe's defining property: f(uR) - f(uL) = A_hat (uR - uL) for any pair.
    rng = np.random.default_rng(3)
    for _ in range(20):
        uL, *_ = random_state(rng)
        uR, *_ = random_state(rng)
        for d in range(3):
            X, Xi, lam = orc.roe_eigensystem(uL, uR, d, GAMMA)
            A = X @ np.diag(lam) @ Xi
            lhs = orc.flux(uR, d, GAMMA) - orc.flux(uL, d, GAMMA)
            np.testing.assert_allclose(A @ (uR - uL), lhs, rtol=1e-11, atol=1e-11 * np.abs(lhs).max())


def test_harten_fix_is_continuous_and_bounded(orc):
    for delta in (1e-6, 0.1, 0.5):
        assert orc.harten(delta, delta) == pytest.approx(delta, rel=1e-15)
        assert orc.harten(-delta, delta) == pytest.approx(delta, rel=1e-15)
        assert orc.harten(delta * (1 - 1e-9), delta) == pytest.approx(delta, rel=1e-8)
        assert orc.harten(0.0, delta) == pytest.approx(delta / 2, rel=1e-15)
        for lam in np.linspace(-2 * delta, 2 * delta, 41):
            v = orc.harten(lam, delta)
            assert v >= abs(lam) - 1e-16 and v >= delta / 2 - 1e-16
    assert orc.harten(-0.3, 0.0) == 0.3
    assert orc.harten(0.0, 0.0) == 0.0


def test_interface_flux_of_a_uniform_stencil_is_the_physical_flux(orc):
    rng = np.random.default_rng(4)
    ph = orc.make_phys(mu_eff=0.0)
    for _ in range(10):
        u, *_ = random_state(rng)
        for d in range(3):
            F = orc.interface_flux(np.tile(u, (6, 1)), d, ph)
            np.testing.assert_allclose(F, orc.flux(u, d, GAMMA), rtol=1e-14, atol=1e-14)
