"""Seeded synthetic inputs shared by the GPU path's callers and by the tests.

This module only *draws* inputs: primitive fields (density, velocity,
pressure) on a triply periodic grid, plus the workload parameter sets.  It
contains none of the discretisation's arithmetic (no fluxes, no WENO, no
equation of state, no time stepping), so the HIP library and the CPU oracle
both receive identical primitive arrays and each converts them on its own.

Array layout: every scalar field is a C-ordered ``[nz][ny][nx]`` array (x is
fastest); a vector field is ``[3][nz][ny][nx]`` with components (u, v, w).
Grid points are ``x_i = i * L / N`` for ``i = 0 .. N-1`` on ``[0, 2*pi)``.

Decaying-turbulence initial condition (paper Sec. 2.3, the HIT decay example):
a random solenoidal velocity whose shell spectrum follows
``E(k) ~ k^4 exp(-2 (k/k0)^2)`` with ``k0 = 4``, constant density and pressure.
The paper gives no algorithm for the random field; the recipe used here is:

1. ``rng = numpy.random.default_rng(seed)``; integer wavevectors from fftfreq.
2. A complex Gaussian vector per Fourier mode; the component along ``k`` is
   projected out (divergence-free); the mean mode and every mode touching the
   Nyquist plane are zeroed.
3. Each mode is scaled by ``|k| exp(-(|k|/k0)^2)``, the square root of
   ``E(k) / (4 pi k^2)`` up to a constant.
4. ``v = Re(ifft(...))``, rescaled so the per-component rms is ``urms``
   (so the mean kinetic energy per unit mass is ``1.5 urms^2``).
5. ``rho = 1``, ``p = 1 / (gamma Mt^2)``: with ``urms = 1`` the sound speed is
   ``1/Mt``, i.e. ``Mt`` is the per-component rms velocity over sound speed,
   which matches the paper's ``u0 = 0.3``, ``c = 1`` setting after scaling
   velocity by ``1/u0``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TWO_PI = 2.0 * math.pi


def grid_coords(n: int, length: float = TWO_PI) -> np.ndarray:
    """Point coordinates ``x_i = i * length / n`` (cell centres of a periodic grid)."""
    return np.arange(n, dtype=np.float64) * (length / n)


def _fft_ifftn(a: np.ndarray) -> np.ndarray:
    try:
        import scipy.fft as sfft

        return sfft.ifftn(a, workers=-1)
    except Exception:  # pragma: no cover - scipy is present in this image
        return np.fft.ifftn(a)


def hit_velocity(n: int, seed: int | None = None, k0: float = 4.0, urms: float = 1.0,
                 rng: np.random.Generator | None = None) -> np.ndarray:
    """Random solenoidal velocity ``[3][n][n][n]`` with the HIT spectrum shape.

    ``rng`` may be passed to continue an existing stream (ensemble boxes draw
    their size and physics first, then the velocity from the same stream).
    """
    if rng is None:
        rng = np.random.default_rng(seed)
    kk = np.fft.fftfreq(n) * n  # integer wavenumbers
    kz = kk[:, None, None]
    ky = kk[None, :, None]
    kx = kk[None, None, :]
    k2 = kx * kx + ky * ky + kz * kz
    nyq = (np.abs(kx) == n // 2) | (np.abs(ky) == n // 2) | (np.abs(kz) == n // 2)
    keep = (k2 > 0) & ~nyq
    amp = np.where(keep, np.sqrt(k2) * np.exp(-k2 / (k0 * k0)), 0.0)
    inv_k2 = np.where(k2 > 0, 1.0 / np.where(k2 > 0, k2, 1.0), 0.0)

    comps = []
    for _ in range(3):
        re = rng.standard_normal((n, n, n))
        im = rng.standard_normal((n, n, n))
        comps.append(re + 1j * im)
    # divergence-free projection: v <- v - k (k.v)/|k|^2
    kdotv = kx * comps[0] + ky * comps[1] + kz * comps[2]
    proj = kdotv * inv_k2
    del kdotv
    out = np.empty((3, n, n, n), dtype=np.float64)
    for c, kc in enumerate((kx, ky, kz)):
        vh = (comps[c] - kc * proj) * amp
        comps[c] = None
        out[c] = _fft_ifftn(vh).real
        del vh
    del proj
    ms = float(np.einsum("cijk,cijk->", out, out)) / (3.0 * n ** 3)
    out *= urms / math.sqrt(ms)
    return out


def hit_primitives(n: int, seed: int, mt: float, gamma: float = 1.4, urms: float = 1.0,
                   rng: np.random.Generator | None = None):
    """``(rho [n,n,n], vel [3,n,n,n], p [n,n,n])`` for the decaying-turbulence IC."""
    vel = hit_velocity(n, seed, urms=urms, rng=rng)
    rho = np.ones((n, n, n))
    p = np.full((n, n, n), 1.0 / (gamma * mt * mt))
    return rho, vel, p


def vortex_primitives(n: int, t: float = 0.0, strength: float = 5.0, gamma: float = 1.4,
                      adv=None, radius: float = TWO_PI / 10.0,
                      nz: int | None = None, plane: str = "xy"):
    """Isentropic vortex (Euler) advected uniformly, evaluated at time ``t``.

    ``plane`` names the two axes the vortex lies in: ``"xy"`` (the default:
    invariant along z, advection ``adv = (1, 1, 0)``, arrays ``[nz][n][n]``) or
    ``"yz"`` (invariant along x, advection ``(0, 1, 1)``, arrays ``[n][n][nz]``
    with ``nz`` points along x), the same flow with the roles of the axes
    exchanged (a = x, b = y, or a = y, b = z below).
    Free stream ``rho = p = 1``, velocity ``adv``; centre ``(pi, pi)`` in the
    plane at ``t = 0``, core radius ``radius``.  With ``xt = (a - ac)/R``,
    ``r^2 = xt^2 + yt^2``::

        du = -(b / 2pi) yt exp((1 - r^2)/2),   dv = (b / 2pi) xt exp((1 - r^2)/2)
        p/rho = 1 - (gamma - 1) b^2 / (8 gamma pi^2) exp(1 - r^2)
        rho = (p/rho)^(1/(gamma-1)),  p = rho^gamma

    The centre moves with ``adv``; distances use the nearest periodic image.
    This is the exact solution of the Euler equations on the whole plane; the
    periodic box truncates it at ``r = pi/R`` core radii.
    """
    nz = n if nz is None else nz
    if plane not in ("xy", "yz"):
        raise ValueError(f"plane must be 'xy' or 'yz' (got {plane!r})")
    ia, ib, ic = (0, 1, 2) if plane == "xy" else (1, 2, 0)
    if adv is None:
        adv = (1.0, 1.0, 0.0) if plane == "xy" else (0.0, 1.0, 1.0)
    x = grid_coords(n)
    xc = math.pi + adv[ia] * t
    yc = math.pi + adv[ib] * t

    def periodic_delta(a, c):
        d = np.mod(a - c + math.pi, TWO_PI) - math.pi
        return d

    dx = periodic_delta(x, xc)[None, :] / radius  # [y][x]
    dy = periodic_delta(x, yc)[:, None] / radius
    r2 = dx * dx + dy * dy
    b = strength
    g = np.exp(0.5 * (1.0 - r2))
    du = -(b / TWO_PI) * dy * g
    dv = (b / TWO_PI) * dx * g
    temp = 1.0 - (gamma - 1.0) * b * b / (8.0 * gamma * math.pi ** 2) * np.exp(1.0 - r2)
    rho2 = temp ** (1.0 / (gamma - 1.0))
    p2 = rho2 ** gamma
    if plane == "xy":
        shape = (nz, n, n)
        place = lambda f: np.broadcast_to(f, shape).copy()  # noqa: E731  [b][a] -> [z][y][x]
    else:
        shape = (n, n, nz)
        place = lambda f: np.broadcast_to(f[:, :, None], shape).copy()  # noqa: E731  [b][a] -> [z][y][.]
    rho = place(rho2)
    p = place(p2)
    vel = np.empty((3,) + shape)
    vel[ia] = place(adv[ia] + du)
    vel[ib] = place(adv[ib] + dv)
    vel[ic] = adv[ic]
    return rho, vel, p


def shock_primitives(shape, axis: int, seed: int = 0, strength: str = "sod"):
    """Discontinuous data along ``axis`` (0 = x, 1 = y, 2 = z) on a smooth background.

    Along the line coordinate ``s`` in ``[0, 2 pi)`` the density and pressure are
    piecewise constant with three jumps per period: at ``s = pi/2`` a shock-tube
    (Sod-type) jump of density and pressure, at ``s = 3 pi/2`` a contact (density
    only, pressure continuous), and at the periodic wrap a jump of both.  Levels:
    ``"sod"``: (rho, p) = (0.125, 0.1) | (1, 1) | (0.5, 1); ``"strong"``: the same
    densities with pressures 1 | 1e5 | 1e5 (energy jumps of about 2.5e5, where
    products of four (eps + beta) factors leave the FP32 range).  Every field is
    multiplied (density, pressure) or offset (velocity) by a band-limited smooth
    random field of ``smooth_primitives``, so the transverse directions are not
    trivial.  Returns ``(rho, vel, p)``.
    """
    nz, ny, nx = (int(v) for v in shape)
    levels = {"sod": ((0.125, 0.1), (1.0, 1.0), (0.5, 1.0)),
              "strong": ((0.125, 1.0), (1.0, 1e5), (0.5, 1e5))}[strength]
    rho_s, vel_s, p_s, _ = smooth_primitives((nz, ny, nx), seed=seed, amp=0.05, mean_vel=(0.2, -0.1, 0.15))
    nline = (nx, ny, nz)[axis]
    s = grid_coords(nline)
    region = np.where(s < 0.5 * math.pi, 0, np.where(s < 1.5 * math.pi, 1, 2))
    r_line = np.array([levels[q][0] for q in region])
    p_line = np.array([levels[q][1] for q in region])
    bshape = [1, 1, 1]
    bshape[2 - axis] = nline  # arrays are [z][y][x]
    rho = rho_s * r_line.reshape(bshape)
    p = p_s * p_line.reshape(bshape)
    return rho, vel_s, p


def uniform_primitives(n: int, rho: float = 1.0, vel=(0.3, -0.2, 0.1), p: float = 1.0,
                       shape=None):
    """A free stream: constant state everywhere."""
    shape = (n, n, n) if shape is None else tuple(shape)
    r = np.full(shape, rho)
    v = np.empty((3,) + shape)
    for c in range(3):
        v[c] = vel[c]
    return r, v, np.full(shape, p)


def smooth_primitives(shape, seed: int, amp: float = 0.1, kmax: int = 2, mean_vel=(0.0, 0.0, 0.0),
                      rho0: float = 1.0, p0: float = 1.0):
    """Band-limited smooth random fields (a few Fourier modes per field).

    Used for invariant and convergence tests: every field is a sum of
    ``sin``/``cos`` modes with integer wavenumbers ``<= kmax`` and random
    amplitudes, so it is exactly periodic at every resolution.
    Returns ``(rho, vel, p, modes)``; ``modes`` lets a test re-evaluate the
    same fields on another grid (``smooth_eval``).
    """
    rng = np.random.default_rng(seed)
    modes = []
    for _f in range(5):
        terms = []
        for _t in range(4):
            k = rng.integers(-kmax, kmax + 1, size=3)
            if not k.any():
                k[0] = 1
            a = rng.uniform(-1.0, 1.0)
            ph = rng.uniform(0.0, TWO_PI)
            terms.append((k, a, ph))
        modes.append(terms)
    spec = dict(modes=modes, amp=amp, mean_vel=tuple(mean_vel), rho0=rho0, p0=p0)
    rho, vel, p = smooth_eval(shape, spec)
    return rho, vel, p, spec


def smooth_eval(shape, spec):
    nz, ny, nx = shape
    z = grid_coords(nz)[:, None, None]
    y = grid_coords(ny)[None, :, None]
    x = grid_coords(nx)[None, None, :]
    fields = []
    for terms in spec["modes"]:
        f = np.zeros(shape)
        for k, a, ph in terms:
            f = f + a * np.sin(k[0] * x + k[1] * y + k[2] * z + ph)
        fields.append(f / len(terms))
    amp = spec["amp"]
    rho = spec["rho0"] * (1.0 + 0.5 * amp * fields[0])
    p = spec["p0"] * (1.0 + 0.5 * amp * fields[4])
    vel = np.empty((3,) + tuple(shape))
    for c in range(3):
        vel[c] = spec["mean_vel"][c] + amp * fields[1 + c]
    return rho, vel, p


def dt_from_speed(max_speed: float, n_min: int, cfl: float = 0.5, length: float = TWO_PI) -> float:
    """Time step ``cfl * dx / max_speed`` with ``max_speed = max over points and
    directions of |v_d| + c`` (a per-direction CFL, not summed over directions)."""
    return cfl * (length / n_min) / max_speed


# --------------------------------------------------------------------------------------
# Workload parameter sets (synthetic stand-ins for the paper's HIT-decay runs)
# --------------------------------------------------------------------------------------
GAMMA = 1.4
PRANDTL = 0.72
WENO_EPS = 1e-6
HARTEN_DELTA = 1e-6
CFL = 0.5


@dataclass
class Workload:
    name: str
    n: int
    steps: int
    mt: float = 0.3
    re: float = 100.0  # mu_eff = 1/re ; re = inf -> Euler
    seed: int = 0
    precision: str = "fp64"
    extra: dict = field(default_factory=dict)

    @property
    def mu_eff(self) -> float:
        return 0.0 if math.isinf(self.re) else 1.0 / self.re


WORKLOADS = {
    "hit32": Workload("hit32_re100_rk4x10", 32, 10, mt=0.3, re=100.0),
    "hit128": Workload("hit128_re400_rk4x100", 128, 100, mt=0.3, re=400.0),
    "hit512": Workload("hit512_re1600_rk4x20", 512, 20, mt=0.3, re=1600.0),
    "adjoint128": Workload("hit128_re400_rk4x200_adjoint", 128, 200, mt=0.3, re=400.0,
                           extra=dict(ckpt_every=20)),
}


@dataclass
class EnsembleBox:
    index: int
    n: int
    mt: float
    re: float


def ensemble_box_params(i: int):
    """Box ``i`` of the uneven ensemble: draws N, Mt, Re, then the velocity,
    all from ``default_rng(i)``.  Returns ``(EnsembleBox, rng)`` with the rng
    positioned for the velocity draw."""
    rng = np.random.default_rng(i)
    n = int(rng.choice([32, 48, 64, 96]))
    mt = float(rng.uniform(0.1, 0.5))
    re = float(rng.uniform(100.0, 800.0))
    return EnsembleBox(i, n, mt, re), rng


def ensemble_box_primitives(i: int, gamma: float = GAMMA):
    box, rng = ensemble_box_params(i)
    rho, vel, p = hit_primitives(box.n, None, box.mt, gamma=gamma, rng=rng)
    return box, rho, vel, p
