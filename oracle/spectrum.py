"""Kinetic-energy spectrum E(k) and the Taylor microscale (test infrastructure only).

The paper characterises its decaying-turbulence runs by the energy spectrum
E(k) (Sec. 2.3: the model initial spectrum and the spectrum at t/tau = 3;
Sec. 5: spectra per grid size and in time) and by the Taylor microscale lambda
that sets Re_lambda and tau = lambda/u0.  Written
from those definitions with numpy's FFT as the transform:

  v_hat(k) = (1/N) sum_x v(x) exp(-i k.x)      (N = nx ny nz points)
  E(k_s)   = sum over modes with round(|k|) = k_s of |v_hat|^2 / 2
  M2       = sum over all modes of |k|^2 |v_hat|^2 / 2
  lambda   = sqrt(5 sum_s E(k_s) / M2)           (isotropic relation)

with v = m/rho the velocity, |k| the physical wavenumber 2 pi n_d / L_d and
shells of unit width.  Shares no code with the HIP library.
"""
from __future__ import annotations

import math

import numpy as np


def wavenumbers(shape, length=(2 * math.pi,) * 3):
    """Physical wavenumber components (kz, ky, kx) broadcastable over [nz][ny][nx]."""
    nz, ny, nx = shape
    lx, ly, lz = length
    kx = np.fft.fftfreq(nx, d=1.0 / nx) * (2 * math.pi / lx)
    ky = np.fft.fftfreq(ny, d=1.0 / ny) * (2 * math.pi / ly)
    kz = np.fft.fftfreq(nz, d=1.0 / nz) * (2 * math.pi / lz)
    return kz[:, None, None], ky[None, :, None], kx[None, None, :]


def nshell(shape, length=(2 * math.pi,) * 3):
    """Number of unit-width shells: round(|k|_max) + 1 over the grid's modes."""
    kz, ky, kx = wavenumbers(shape, length)
    kmax = math.sqrt(np.max(kx ** 2) + np.max(ky ** 2) + np.max(kz ** 2))
    return int(math.floor(kmax + 0.5)) + 1


def spectrum_of_velocity(vel, length=(2 * math.pi,) * 3):
    """vel [3][nz][ny][nx] -> (E[nshell], sum E, M2)."""
    vel = np.asarray(vel, dtype=np.float64)
    shape = vel.shape[1:]
    npts = vel[0].size
    power = np.zeros(shape)
    for c in range(3):
        vh = np.fft.fftn(vel[c]) / npts
        power += 0.5 * (vh.real ** 2 + vh.imag ** 2)
    kz, ky, kx = wavenumbers(shape, length)
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    shell = np.floor(np.sqrt(k2) + 0.5).astype(np.int64)
    ns = nshell(shape, length)
    E = np.zeros(ns)
    for s in range(ns):  # plain per-shell sums
        E[s] = power[shell == s].sum()
    M2 = float((k2 * power).sum())
    return E, float(power.sum()), M2


def spectrum(u, length=(2 * math.pi,) * 3):
    """Spectrum of the velocity m/rho of a conserved state u[5][nz][ny][nx]."""
    u = np.asarray(u, dtype=np.float64)
    vel = u[1:4] / u[0]
    return spectrum_of_velocity(vel, length)


def taylor_microscale(total, m2):
    """lambda = sqrt(5 sum E / M2), i.e. u'^2 / <(du1/dx1)^2> for isotropic fields."""
    return math.sqrt(5.0 * total / m2)
