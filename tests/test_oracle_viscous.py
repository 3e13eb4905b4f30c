"""Pins of the oracle's viscous and heat-flux terms (paper Sec. 2.1 stress
tensor, heat flux, T = gamma p / rho; 4th-order central derivatives of Sec. 2.2).

The 5-point central derivative is a circulant operator with Fourier symbol
i k*, k* dx = (8 sin(k dx) - sin(2 k dx)) / 6, so for single Fourier modes the
discrete viscous terms have closed forms; for general periodic grid
functions the operator is applied through its symbol with an FFT, which is
independent of the oracle's stencil code."""
import math

import numpy as np
import pytest

from paper_2211_16718_amd import inputs as I

GAMMA, PR = 1.4, 0.72


def kstar(k, h):
    return (8 * math.sin(k * h) - math.sin(2 * k * h)) / (6 * h)


def D_spectral(f, axis, h):
    """The circulant 4th-order central derivative through its Fourier symbol."""
    n = f.shape[axis]
    k = np.fft.fftfreq(n) * n
    sym = 1j * (8 * np.sin(k * h) - np.sin(2 * k * h)) / (6 * h)
    shape = [1] * f.ndim
    shape[axis] = n
    return np.fft.ifft(np.fft.fft(f, axis=axis) * sym.reshape(shape), axis=axis).real


def state(rho, vel, p):
    import oracle

    return oracle.init_state(rho, vel, p, GAMMA)


@pytest.mark.parametrize("n", [16, 24])
def test_shear_wave_closed_form(orc, n):
    mu, A = 0.05, 0.3
    h = 2 * math.pi / n
    y = I.grid_coords(n)[None, :, None] * np.ones((n, n, n))
    rho = np.ones((n, n, n))
    p = np.full((n, n, n), 2.0)
    vel = np.zeros((3, n, n, n))
    vel[0] = A * np.sin(y)
    u = state(rho, vel, p)
    ph = orc.make_phys(mu_eff=mu, harten_delta=0.0)
    r = orc.viscous(u, ph)
    ks = kstar(1, h)
    ks2 = kstar(2, h)
    np.testing.assert_array_equal(r[0], 0.0)
    np.testing.assert_allclose(r[1], -mu * ks * ks * A * np.sin(y), atol=1e-14)
    np.testing.assert_allclose(r[2], 0.0, atol=1e-14)
    np.testing.assert_allclose(r[3], 0.0, atol=1e-14)
    # energy: mu D_y(u D_y u) = mu A^2 k* D_y(sin y cos y) = mu A^2 k* k2*/2 cos 2y
    np.testing.assert_allclose(r[4], mu * A * A * ks * 0.5 * ks2 * np.cos(2 * y), atol=1e-14)


def test_compression_wave_pins_the_stress_sign(orc):
    # v = (A sin x, 0, 0): tau_xx = mu (2 du/dx - 2/3 du/dx) = 4/3 mu du/dx with the
    # symmetric stress; the printed antisymmetric form would give -2/3.
    n, mu, A = 16, 0.07, 0.2
    h = 2 * math.pi / n
    x = I.grid_coords(n)[None, None, :] * np.ones((n, n, n))
    vel = np.zeros((3, n, n, n))
    vel[0] = A * np.sin(x)
    u = state(np.ones((n, n, n)), vel, np.full((n, n, n), 1.5))
    r = orc.viscous(u, orc.make_phys(mu_eff=mu))
    np.testing.assert_allclose(r[1], -(4.0 / 3.0) * mu * kstar(1, h) ** 2 * A * np.sin(x), atol=1e-14)


def test_cross_derivative_terms(orc):
    # v = (A sin(x + y), 0, 0): rhs_{rho v} = D_x tau_yx + D_y tau_yy
    #   = mu (D_x D_y u - 2/3 D_y D_x u) = mu/3 D_x D_y u = -mu/3 k*^2 A sin(x+y)
    n, mu, A = 16, 0.03, 0.25
    h = 2 * math.pi / n
    g = I.grid_coords(n)
    x = g[None, None, :] * np.ones((n, n, n))
    y = g[None, :, None] * np.ones((n, n, n))
    vel = np.zeros((3, n, n, n))
    vel[0] = A * np.sin(x + y)
    u = state(np.ones((n, n, n)), vel, np.full((n, n, n), 1.5))
    r = orc.viscous(u, orc.make_phys(mu_eff=mu))
    ks2 = kstar(1, h) ** 2
    np.testing.assert_allclose(r[2], -(mu / 3.0) * ks2 * A * np.sin(x + y), atol=1e-14)
    np.testing.assert_allclose(r[1], -mu * (4.0 / 3.0 + 1.0) * ks2 * A * np.sin(x + y), atol=1e-14)


def test_heat_wave_against_spectral_form_of_the_stencil(orc):
    # rho = 1 + A sin x, p const, v = 0: only the heat flux acts,
    # rhs_e = mu/((gamma-1) Pr) D_x D_x T with T = gamma p / rho.
    n, mu, A, p0 = 16, 0.04, 0.3, 1.2
    h = 2 * math.pi / n
    x = I.grid_coords(n)[None, None, :] * np.ones((n, n, n))
    rho = 1 + A * np.sin(x)
    u = state(rho, np.zeros((3, n, n, n)), np.full((n, n, n), p0))
    ph = orc.make_phys(mu_eff=mu)
    r = orc.viscous(u, ph)
    T = GAMMA * p0 / rho
    expect = mu / ((GAMMA - 1) * PR) * D_spectral(D_spectral(T, 2, h), 2, h)
    np.testing.assert_allclose(r[4], expect, atol=1e-13 * np.abs(expect).max())
    np.testing.assert_array_equal(r[0], 0.0)
    np.testing.assert_allclose(r[1:4], 0.0, atol=1e-14)


def test_viscous_operator_on_general_field_against_spectral_symbol(orc):
    # Build the viscous RHS of a smooth random field with the stencil's Fourier
    # symbol (FFT) for every derivative, and compare with the oracle.
    n = 12
    shape = (n, n, n)
    h = 2 * math.pi / n
    rho, vel, p, _ = I.smooth_primitives(shape, seed=5, amp=0.3)
    mu = 0.02
    u = state(rho, vel, p)
    r = orc.viscous(u, orc.make_phys(mu_eff=mu))
    T = GAMMA * p / rho
    axis = {0: 2, 1: 1, 2: 0}  # direction -> array axis
    grad = [[D_spectral(vel[a], axis[b], h) for b in range(3)] for a in range(3)]
    gT = [D_spectral(T, axis[b], h) for b in range(3)]
    div = grad[0][0] + grad[1][1] + grad[2][2]
    tau = [[mu * ((grad[a][b] + grad[b][a]) - (2 / 3 * div if a == b else 0)) for b in range(3)] for a in range(3)]
    kc = mu / ((GAMMA - 1) * PR)
    out = np.zeros((5,) + shape)
    for d in range(3):
        G = [np.zeros(shape), tau[0][d], tau[1][d], tau[2][d],
             vel[0] * tau[0][d] + vel[1] * tau[1][d] + vel[2] * tau[2][d] + kc * gT[d]]
        for v in range(5):
            out[v] += D_spectral(G[v], axis[d], h)
    np.testing.assert_allclose(r, out, atol=1e-13 * np.abs(out).max())
