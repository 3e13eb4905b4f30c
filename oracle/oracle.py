"""ctypes wrapper of the C oracle (test infrastructure only).

Arrays are numpy float64, C-contiguous: a conserved state is ``[5][nz][ny][nx]``.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

from . import build_oracle

_LIB = None
NDIAG = 9
DIAG_NAMES = ("K", "Omega", "rho_mean", "mx_mean", "my_mean", "mz_mean", "e_mean", "max_speed", "bad")

ERRORS = {0: "ok", -1: "EINVAL", -3: "ENONFINITE", -4: "ENONPHYSICAL"}


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed: {ERRORS.get(code, code)}")
        self.code = code


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double)]


class Phys(C.Structure):
    _fields_ = [("gamma", C.c_double), ("prandtl", C.c_double), ("mu_eff", C.c_double),
                ("weno_eps", C.c_double), ("harten_delta", C.c_double), ("weno_weights", C.c_int)]


_dp = C.POINTER(C.c_double)


def lib():
    """The oracle library: ``CNS_ORACLE_LIBRARY`` may name another build of the same
    source (the benchmark's ``-march=native`` build); else the in-tree build."""
    global _LIB
    if _LIB is None:
        path = os.environ.get("CNS_ORACLE_LIBRARY") or build_oracle.LIB
        if path == build_oracle.LIB and not os.path.exists(path):
            build_oracle.build()
        L = C.CDLL(path)
        L.oracle_weno5.restype = C.c_double
        L.oracle_weno5.argtypes = [C.c_double] * 6 + [_dp]
        L.oracle_weno5z.restype = C.c_double
        L.oracle_weno5z.argtypes = [C.c_double] * 6 + [_dp]
        L.oracle_weno5m.restype = C.c_double
        L.oracle_weno5m.argtypes = [C.c_double] * 6 + [_dp]
        L.oracle_weno_map.restype = C.c_double
        L.oracle_weno_map.argtypes = [C.c_double, C.c_double]
        L.oracle_flux.restype = None
        L.oracle_flux.argtypes = [_dp, C.c_int, C.c_double, _dp]
        L.oracle_roe_eigensystem.argtypes = [_dp, _dp, C.c_int, C.c_double, _dp, _dp, _dp]
        L.oracle_harten.restype = C.c_double
        L.oracle_harten.argtypes = [C.c_double, C.c_double]
        L.oracle_interface_flux.argtypes = [_dp, C.c_int, C.POINTER(Phys), _dp]
        for name in ("oracle_rhs", "oracle_viscous", "oracle_diag"):
            getattr(L, name).argtypes = [C.POINTER(Grid), C.POINTER(Phys), _dp, _dp]
        L.oracle_rhs_hyp_dir.argtypes = [C.POINTER(Grid), C.POINTER(Phys), _dp, C.c_int, _dp]
        L.oracle_rhs_point.argtypes = [C.POINTER(Grid), C.POINTER(Phys), _dp, C.c_int, C.c_int, C.c_int, _dp]
        L.oracle_rk4.argtypes = [C.POINTER(Grid), C.POINTER(Phys), _dp, C.c_double, C.c_int, _dp]
        L.oracle_tvdrk3.argtypes = [C.POINTER(Grid), C.POINTER(Phys), _dp, C.c_double, C.c_int, _dp]
        L.oracle_init_state.argtypes = [C.POINTER(Grid), C.c_double, _dp, _dp, _dp, _dp]
        L.oracle_num_threads.restype = C.c_int
        L.oracle_cs_rhs_jvp.argtypes = [C.POINTER(Grid), C.POINTER(Phys), _dp, _dp, C.c_double, _dp, _dp]
        L.oracle_cs_step_jvp.argtypes = [C.POINTER(Grid), C.POINTER(Phys), C.c_int, _dp, _dp, C.c_double, C.c_int,
                                         C.c_double, _dp, _dp, _dp]
        L.oracle_adjoint_rk4.argtypes = [C.POINTER(Grid), C.POINTER(Phys), C.c_int, _dp, C.c_double, C.c_int,
                                         C.c_double, _dp, _dp]
        _LIB = L
    return _LIB


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], "need C-contiguous float64"
    return a.ctypes.data_as(_dp)


def _chk(rc, what):
    if rc != 0:
        raise OracleError(rc, what)


def make_grid(shape, length=(2 * math.pi,) * 3) -> Grid:
    """``shape`` is (nz, ny, nx); ``length`` is (lx, ly, lz)."""
    nz, ny, nx = shape
    return Grid(nx, ny, nz, length[0], length[1], length[2])


WENO_JS, WENO_Z, WENO_M = 0, 1, 2


def make_phys(gamma=1.4, prandtl=0.72, mu_eff=0.01, weno_eps=1e-6, harten_delta=1e-6, weno_weights=WENO_JS) -> Phys:
    return Phys(gamma, prandtl, mu_eff, weno_eps, harten_delta, weno_weights)


def weno5(a, b, c, d, e, eps=1e-6, parts=False, weights=WENO_JS):
    buf = (C.c_double * 9)()
    fn = {WENO_JS: lib().oracle_weno5, WENO_Z: lib().oracle_weno5z, WENO_M: lib().oracle_weno5m}[weights]
    r = fn(a, b, c, d, e, eps, buf)
    if parts:
        return r, np.array(buf[:])
    return r


def weno_map(w, d):
    """The weight mapping of the mapped WENO weights (Henrick et al. 2005)."""
    return lib().oracle_weno_map(w, d)


def flux(u, direction, gamma=1.4):
    u = np.ascontiguousarray(u, dtype=np.float64)
    f = np.zeros(5)
    lib().oracle_flux(_ptr(u), direction, gamma, _ptr(f))
    return f


def roe_eigensystem(uL, uR, direction, gamma=1.4):
    uL = np.ascontiguousarray(uL, dtype=np.float64)
    uR = np.ascontiguousarray(uR, dtype=np.float64)
    X = np.zeros(25)
    Xi = np.zeros(25)
    lam = np.zeros(5)
    _chk(lib().oracle_roe_eigensystem(_ptr(uL), _ptr(uR), direction, gamma, _ptr(X), _ptr(Xi), _ptr(lam)),
         "roe_eigensystem")
    return X.reshape(5, 5), Xi.reshape(5, 5), lam


def harten(lam, delta):
    return lib().oracle_harten(lam, delta)


def interface_flux(stencil, direction, phys: Phys):
    s = np.ascontiguousarray(stencil, dtype=np.float64).reshape(30)
    F = np.zeros(5)
    _chk(lib().oracle_interface_flux(_ptr(s), direction, C.byref(phys), _ptr(F)), "interface_flux")
    return F


def init_state(rho, vel, p, gamma=1.4, length=(2 * math.pi,) * 3):
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    vel = np.ascontiguousarray(vel, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    g = make_grid(rho.shape, length)
    u = np.zeros((5,) + rho.shape)
    _chk(lib().oracle_init_state(C.byref(g), gamma, _ptr(rho), _ptr(vel), _ptr(p), _ptr(u)), "init_state")
    return u


def _grid_of(u, length):
    return make_grid(u.shape[1:], length)


def rhs(u, phys: Phys, length=(2 * math.pi,) * 3):
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty_like(u)
    g = _grid_of(u, length)
    _chk(lib().oracle_rhs(C.byref(g), C.byref(phys), _ptr(u), _ptr(out)), "rhs")
    return out


def rhs_hyp_dir(u, direction, phys: Phys, length=(2 * math.pi,) * 3):
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty_like(u)
    g = _grid_of(u, length)
    _chk(lib().oracle_rhs_hyp_dir(C.byref(g), C.byref(phys), _ptr(u), direction, _ptr(out)), "rhs_hyp_dir")
    return out


def viscous(u, phys: Phys, length=(2 * math.pi,) * 3):
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty_like(u)
    g = _grid_of(u, length)
    _chk(lib().oracle_viscous(C.byref(g), C.byref(phys), _ptr(u), _ptr(out)), "viscous")
    return out


def rhs_point(u, i, j, k, phys: Phys, length=(2 * math.pi,) * 3):
    """RHS at point (x=i, y=j, z=k)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(5)
    g = _grid_of(u, length)
    _chk(lib().oracle_rhs_point(C.byref(g), C.byref(phys), _ptr(u), int(i), int(j), int(k), _ptr(out)),
         "rhs_point")
    return out


def rk4(u, dt, nsteps, phys: Phys, length=(2 * math.pi,) * 3, with_diag=True):
    """Returns ``(u_final, diag[nsteps][9])`` (the input array is not modified)."""
    u = np.array(u, dtype=np.float64, order="C", copy=True)
    g = _grid_of(u, length)
    diag = np.zeros((max(nsteps, 1), NDIAG))
    rc = lib().oracle_rk4(C.byref(g), C.byref(phys), _ptr(u), float(dt), int(nsteps),
                          _ptr(diag) if with_diag else None)
    _chk(rc, "rk4")
    return u, diag[:nsteps]


def tvdrk3(u, dt, nsteps, phys: Phys, length=(2 * math.pi,) * 3, with_diag=True):
    """Third-order TVD Runge-Kutta; returns ``(u_final, diag[nsteps][9])``."""
    u = np.array(u, dtype=np.float64, order="C", copy=True)
    g = _grid_of(u, length)
    diag = np.zeros((max(nsteps, 1), NDIAG))
    rc = lib().oracle_tvdrk3(C.byref(g), C.byref(phys), _ptr(u), float(dt), int(nsteps),
                             _ptr(diag) if with_diag else None)
    _chk(rc, "tvdrk3")
    return u, diag[:nsteps]


def diag(u, phys: Phys, length=(2 * math.pi,) * 3):
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(NDIAG)
    g = _grid_of(u, length)
    _chk(lib().oracle_diag(C.byref(g), C.byref(phys), _ptr(u), _ptr(out)), "diag")
    return out


def num_threads():
    return lib().oracle_num_threads()


# ---- complex-step derivatives (cns_oracle_cs.c): the oracle's own arithmetic in
# complex numbers, Im F(u + i h d) / h = F'(u) d to rounding ----
CS_STEP = 1e-20


def rhs_jvp_cs(u, d, phys: Phys, length=(2 * math.pi,) * 3, h=CS_STEP):
    """``(R'(u) d, Re R(u + i h d))``: the derivative of the right-hand side along d."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    assert d.shape == u.shape
    jvp = np.zeros_like(u)
    val = np.zeros_like(u)
    g = _grid_of(u, length)
    _chk(lib().oracle_cs_rhs_jvp(C.byref(g), C.byref(phys), _ptr(u), _ptr(d), float(h), _ptr(jvp), _ptr(val)),
         "cs_rhs_jvp")
    return jvp, val


def step_jvp_cs(u0, d, dt, nsteps, phys: Phys, scheme="rk4", length=(2 * math.pi,) * 3, h=CS_STEP):
    """Derivatives along d of ``nsteps`` steps of ``scheme`` ("rk4" or "tvdrk3") from u0:
    returns ``(du_N, dK, K)``, the final state's derivative, the derivative of the final
    mean kinetic energy and that energy."""
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    assert d.shape == u0.shape
    du = np.zeros_like(u0)
    dK = C.c_double(0.0)
    K = C.c_double(0.0)
    g = _grid_of(u0, length)
    sch = {"rk4": 0, "tvdrk3": 1}[scheme]
    _chk(lib().oracle_cs_step_jvp(C.byref(g), C.byref(phys), sch, _ptr(u0), _ptr(d), float(dt), int(nsteps), float(h),
                                  _ptr(du), C.pointer(dK), C.pointer(K)), "cs_step_jvp")
    return du, dK.value, K.value


def adjoint_cs(u0, dt, nsteps, phys: Phys, scheme="rk4", length=(2 * math.pi,) * 3, h=CS_STEP):
    """``(dK/du0, K)``: the gradient of the final mean kinetic energy after ``nsteps``
    steps of ``scheme`` with respect to every component of u0, each entry its own
    complex-step derivative (5 N^3 runs: small grids only)."""
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    grad = np.zeros_like(u0)
    K = C.c_double(0.0)
    g = _grid_of(u0, length)
    sch = {"rk4": 0, "tvdrk3": 1}[scheme]
    _chk(lib().oracle_adjoint_rk4(C.byref(g), C.byref(phys), sch, _ptr(u0), float(dt), int(nsteps), float(h),
                                  _ptr(grad), C.pointer(K)), "adjoint_rk4")
    return grad, K.value
