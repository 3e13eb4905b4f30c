"""The synthetic initial conditions (paper Sec. 2.3 HIT spectrum; the
isentropic vortex) and workload draws."""
import math

import numpy as np

from paper_2211_16718_amd import inputs as I


def test_hit_velocity_energy_divergence_and_mean():
    n = 32
    v = I.hit_velocity(n, seed=0)
    # per-component rms 1 -> mean kinetic energy per unit mass 1.5 (closed form
    # of the spectrum's integral: int E dk = 3/2 u0^2)
    assert 0.5 * np.mean((v ** 2).sum(0)) == np.float64(1.5) or abs(0.5 * np.mean((v ** 2).sum(0)) - 1.5) < 1e-13
    assert np.abs(v.mean(axis=(1, 2, 3))).max() < 1e-14
    k = np.fft.fftfreq(n) * n
    vh = [np.fft.fftn(v[c]) for c in range(3)]
    div = k[None, None, :] * vh[0] + k[None, :, None] * vh[1] + k[:, None, None] * vh[2]
    assert np.abs(div).max() < 1e-10 * np.abs(vh[0]).max()


def test_hit_velocity_is_deterministic_per_seed():
    a = I.hit_velocity(16, seed=5)
    b = I.hit_velocity(16, seed=5)
    c = I.hit_velocity(16, seed=6)
    np.testing.assert_array_equal(a, b)
    assert np.abs(a - c).max() > 0.1


def test_hit_spectrum_shape():
    # shell-summed energy follows k^4 exp(-2 (k/k0)^2) up to sampling noise:
    # its peak sits at k0 = 4
    n = 32
    v = I.hit_velocity(n, seed=1)
    k = np.fft.fftfreq(n) * n
    kk = np.sqrt(k[None, None, :] ** 2 + k[None, :, None] ** 2 + k[:, None, None] ** 2)
    e = sum(np.abs(np.fft.fftn(v[c])) ** 2 for c in range(3))
    shells = np.bincount(np.rint(kk).astype(int).ravel(), weights=e.ravel())
    assert 3 <= int(np.argmax(shells[:12])) <= 5


def test_vortex_is_periodic_in_time_and_positive():
    rho0, vel0, p0 = I.vortex_primitives(32, nz=8)
    rho1, vel1, p1 = I.vortex_primitives(32, t=2 * math.pi, nz=8)
    np.testing.assert_allclose(rho1, rho0, atol=1e-12)
    np.testing.assert_allclose(vel1, vel0, atol=1e-12)
    assert rho0.min() > 0.4 and p0.min() > 0.3
    # isentropic: p = rho^gamma
    np.testing.assert_allclose(p0, rho0 ** 1.4, rtol=1e-14)


def test_ensemble_draws():
    sizes = [I.ensemble_box_params(i)[0].n for i in range(64)]
    assert set(sizes) <= {32, 48, 64, 96}
    b, _ = I.ensemble_box_params(3)
    b2, _ = I.ensemble_box_params(3)
    assert b == b2 and 0.1 <= b.mt <= 0.5 and 100 <= b.re <= 800


def test_shock_inputs_have_three_jumps_per_line():
    # density and pressure are piecewise constant along the axis (times a smooth
    # background): the jumps sit at s = pi/2, at s = 3 pi/2 (density only) and at the wrap
    shape = (24, 20, 28)
    for axis in range(3):
        rho, vel, p = I.shock_primitives(shape, axis, seed=0)
        n = shape[2 - axis]
        s = I.grid_coords(n)
        line_r = np.moveaxis(rho, 2 - axis, 0).reshape(n, -1)
        line_p = np.moveaxis(p, 2 - axis, 0).reshape(n, -1)
        jr = np.abs(np.diff(np.log(line_r), axis=0, append=np.log(line_r[:1]))).max(axis=1)
        jp = np.abs(np.diff(np.log(line_p), axis=0, append=np.log(line_p[:1]))).max(axis=1)
        big_r = set(np.nonzero(jr > 0.3)[0])
        big_p = set(np.nonzero(jp > 0.3)[0])
        i1 = int(np.searchsorted(s, 0.5 * math.pi)) - 1  # last point before pi/2
        i2 = int(np.searchsorted(s, 1.5 * math.pi)) - 1
        assert big_r == {i1, i2, n - 1}, (axis, big_r)
        assert big_p == {i1, n - 1}, (axis, big_p)  # the contact keeps the pressure
        assert rho.min() > 0.1 and p.min() > 0.09 and vel.shape == (3,) + shape
    rho, vel, p = I.shock_primitives(shape, 1, strength="strong")
    assert p.max() > 9e4 and p.min() < 1.1
