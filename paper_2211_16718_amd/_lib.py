"""ctypes loader of the in-tree HIP library ``libcns.so`` (C-ABI in include/cns.h).

Argument marshalling only.  There is no CPU fallback: if the library is
missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# CNS_LIBRARY may name another build of the same library (same C-ABI)
LIB_PATH = os.environ.get("CNS_LIBRARY") or os.path.join(HERE, "libcns.so")

CNS_OK = 0
CNS_NDIAG = 9
CNS_FP64 = 0
CNS_MIXED = 1
CNS_RK4 = 0
CNS_WENO_JS = 0
CNS_WENO_Z = 1
CNS_WENO_M = 2
CNS_TVDRK3 = 1
CNS_NKERNEL = 6
KERNEL_NAMES = ("visc_prim", "visc_flux", "sweep_x", "sweep_y", "sweep_z_rk4", "diagnostics")
ERRORS = {0: "CNS_OK", -1: "CNS_EINVAL", -2: "CNS_EHIP", -3: "CNS_ENONFINITE", -4: "CNS_ENONPHYSICAL",
          -5: "CNS_EWORKSPACE", -6: "CNS_EUNSUPPORTED"}


class CnsError(RuntimeError):
    def __init__(self, code: int, what: str, msg: str):
        super().__init__(f"{what}: {ERRORS.get(code, code)}: {msg}")
        self.code = code


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double)]


class Physics(C.Structure):
    _fields_ = [("gamma", C.c_double), ("prandtl", C.c_double), ("mu_eff", C.c_double),
                ("weno_eps", C.c_double), ("harten_delta", C.c_double), ("weno_weights", C.c_int32)]


_vp = C.c_void_p
_dp = C.POINTER(C.c_double)
# name -> (restype, argtypes); mirrors include/cns.h
SIGNATURES = {
    "cns_plan_create": (C.c_int, [C.POINTER(_vp), C.POINTER(Grid), C.POINTER(Physics), C.c_int32, _vp]),
    "cns_plan_destroy": (C.c_int, [_vp]),
    "cns_workspace_bytes": (C.c_size_t, [_vp]),
    "cns_set_workspace": (C.c_int, [_vp, _vp, C.c_size_t]),
    "cns_set_tiles": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "cns_set_x_kernel": (C.c_int, [_vp, C.c_int32]),
    "cns_init_state": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "cns_rhs": (C.c_int, [_vp, _vp, _vp]),
    "cns_rhs_dir": (C.c_int, [_vp, _vp, C.c_int32, _vp]),
    "cns_viscous": (C.c_int, [_vp, _vp, _vp]),
    "cns_rk4": (C.c_int, [_vp, _vp, C.c_double, C.c_int32, _vp]),
    "cns_tvdrk3": (C.c_int, [_vp, _vp, C.c_double, C.c_int32, _vp]),
    "cns_diagnostics": (C.c_int, [_vp, _vp, _vp]),
    "cns_spectrum_shells": (C.c_int, [_vp]),
    "cns_spectrum": (C.c_int, [_vp, _vp, _vp, C.c_int32, _vp]),
    "cns_diagnostics_host": (C.c_int, [_vp, _vp, _dp]),
    "cns_max_wave_speed": (C.c_int, [_vp, _vp, _vp]),
    "cns_diagnostics_static": (C.c_int, [C.POINTER(Grid), C.POINTER(Physics), C.c_int32, _vp, _vp, _vp]),
    "cns_plan_graph_captures": (C.c_int64, [_vp]),
    "cns_ensemble_graph_captures": (C.c_int64, [_vp]),
    "cns_profile_enable": (C.c_int, [_vp, C.c_int32]),
    "cns_profile_read": (C.c_int, [_vp, _dp, C.POINTER(C.c_int64)]),
    "cns_set_graph": (C.c_int, [_vp, C.c_int32]),
    "cns_ensemble_create": (C.c_int, [C.POINTER(_vp), C.c_int32, C.POINTER(Grid), C.POINTER(Physics), _dp,
                                      C.c_int32, _vp, C.POINTER(C.c_int64), _vp]),
    "cns_ensemble_destroy": (C.c_int, [_vp]),
    "cns_ensemble_workspace_bytes": (C.c_size_t, [_vp]),
    "cns_ensemble_set_workspace": (C.c_int, [_vp, _vp, C.c_size_t]),
    "cns_ensemble_set_tiles": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "cns_ensemble_get_tiles": (C.c_int, [_vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "cns_ensemble_autotune": (C.c_int, [_vp, C.c_char_p]),
    "cns_ensemble_get_launch": (C.c_int, [_vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                          C.POINTER(C.c_int64)]),
    "cns_ensemble_set_launch": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int64, C.c_int64]),
    "cns_ensemble_run": (C.c_int, [_vp, C.c_int32, _vp, C.c_int32]),
    "cns_ensemble_set_integrator": (C.c_int, [_vp, C.c_int32]),
    "cns_ensemble_profile_enable": (C.c_int, [_vp, C.c_int32]),
    "cns_ensemble_profile_read": (C.c_int, [_vp, _dp, C.POINTER(C.c_int64)]),
    "cns_adjoint_workspace_bytes": (C.c_size_t, [_vp, C.c_int32, C.c_int32]),
    "cns_rhs_vjp": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.c_size_t]),
    "cns_adjoint_rk4": (C.c_int, [_vp, _vp, C.c_double, C.c_int32, C.c_int32, _vp, C.c_size_t, _vp, _vp]),
    "cns_adjoint_tvdrk3": (C.c_int, [_vp, _vp, C.c_double, C.c_int32, C.c_int32, _vp, C.c_size_t, _vp, _vp]),
    "cns_adjoint_forward": (C.c_int, [_vp, C.c_int32, _vp, C.c_double, C.c_int32, C.c_int32, _vp, C.c_size_t, _vp]),
    "cns_adjoint_reverse": (C.c_int, [_vp, C.c_int32, C.c_double, C.c_int32, C.c_int32, _vp, C.c_size_t, _vp]),
    "cns_ic_vjp": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "cns_stream_copy": (C.c_int, [_vp, _vp, C.c_size_t, _vp]),
    "cns_last_error": (C.c_char_p, []),
}

_LIB = None


def load():
    """Load libcns.so (built by ``paper_2211_16718_amd.build``); raise if absent."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def check(rc: int, what: str):
    if rc != CNS_OK:
        msg = load().cns_last_error().decode(errors="replace")
        raise CnsError(rc, what, msg)
