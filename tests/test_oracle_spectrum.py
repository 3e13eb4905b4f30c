"""Pins of the oracle's energy spectrum and Taylor microscale: closed forms for
trigonometric fields, Parseval's identity, and the isotropic spectrum that the
initial-condition recipe is built on."""
import math

import numpy as np
import pytest

from oracle import spectrum as S
from paper_2211_16718_amd import inputs as I


def grid(n):
    x = I.grid_coords(n)
    return np.meshgrid(x, x, x, indexing="ij")  # z, y, x


def test_single_cosine_modes_land_in_their_shells():
    # v = sum_m A_m cos(k_m . x + phi_m) e_c: each mode gives A_m^2/4 at shell
    # round(|k_m|) and |k_m|^2 A_m^2 / 4 to the second moment, exactly.
    n = 16
    z, y, x = grid(n)
    modes = [((1, 0, 0), 0.7, 0.3, 0), ((2, 3, 1), 0.4, 1.1, 1), ((0, -5, 2), 1.3, -0.6, 2), ((4, 4, 4), 0.2, 0.0, 0)]
    vel = np.zeros((3, n, n, n))
    E_ex = np.zeros(S.nshell((n, n, n)))
    m2 = 0.0
    for (kx, ky, kz), A, ph, c in modes:
        vel[c] += A * np.cos(kx * x + ky * y + kz * z + ph)
        k = math.sqrt(kx * kx + ky * ky + kz * kz)
        E_ex[int(math.floor(k + 0.5))] += A * A / 4
        m2 += k * k * A * A / 4
    E, tot, M2 = S.spectrum_of_velocity(vel)
    np.testing.assert_allclose(E, E_ex, rtol=0, atol=1e-15)
    assert tot == pytest.approx(sum(A * A / 4 for _, A, _, _ in modes), rel=1e-14)
    assert M2 == pytest.approx(m2, rel=1e-14)
    # one shell only: lambda = sqrt(5) / |k|
    v1 = np.zeros((3, n, n, n))
    v1[1] = 0.5 * np.sin(3 * x + 4 * z)
    _, t1, m1 = S.spectrum_of_velocity(v1)
    assert S.taylor_microscale(t1, m1) == pytest.approx(math.sqrt(5) / 5.0, rel=1e-14)


def test_parseval_and_state_form():
    rng = np.random.default_rng(5)
    vel = rng.normal(size=(3, 12, 10, 14))
    length = (2.0, 3.0, 4.0)
    E, tot, _ = S.spectrum_of_velocity(vel, length)
    assert E.sum() == pytest.approx(tot, rel=1e-14)
    assert tot == pytest.approx(0.5 * (vel ** 2).sum(0).mean(), rel=1e-13)
    rho = 1.0 + 0.3 * rng.random((12, 10, 14))
    u = np.concatenate([rho[None], rho[None] * vel, np.ones((1, 12, 10, 14))])
    E2, _, _ = S.spectrum(u, length)
    np.testing.assert_allclose(E2, E, rtol=1e-12, atol=1e-16)


def test_initial_condition_follows_the_model_spectrum():
    # The recipe draws every mode with amplitude |k| exp(-(|k|/k0)^2), i.e. the
    # spectrum E ~ k^4 exp(-2 (k/k0)^2).  Its moments give lambda = 2/k0 (0.5 for
    # k0 = 4) up to sampling noise, and E peaks near k0.
    n = 64
    vel = I.hit_velocity(n, seed=0)
    E, tot, m2 = S.spectrum_of_velocity(vel)
    assert tot == pytest.approx(1.5, rel=1e-12)  # per-component rms 1
    lam = S.taylor_microscale(tot, m2)
    assert lam == pytest.approx(0.5, rel=0.05), lam
    assert 3 <= int(np.argmax(E)) <= 5
    assert E[0] <= 1e-30  # zero mean velocity
