"""Python binding of the HIP library (argument marshalling only).

PyTorch supplies device memory and the stream; every step of the computation
runs in the library's kernels.  A state is a contiguous tensor of shape
``(5, nz, ny, nx)`` (float64 for ``precision="fp64"``, float32 for
``precision="mixed"``) on the plan's device.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from . import _lib
from ._lib import CNS_NDIAG, CNS_RK4, CNS_TVDRK3, check

TWO_PI = 2.0 * math.pi


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


def _scheme(name):
    return {"rk4": CNS_RK4, "tvdrk3": CNS_TVDRK3}[name]


def _weno_code(weno):
    """``"js"``: Jiang-Shu weights (the paper's); ``"z"``: WENO-Z weights (Borges et al.
    2008); ``"m"``: mapped weights (Henrick et al. 2005)."""
    return {"js": _lib.CNS_WENO_JS, "z": _lib.CNS_WENO_Z, "m": _lib.CNS_WENO_M}[weno]


class Plan:
    """One periodic box: grid, physics, precision, stream and workspace."""

    def __init__(self, shape, length=(TWO_PI, TWO_PI, TWO_PI), gamma=1.4, prandtl=0.72, mu_eff=0.01,
                 weno_eps=1e-6, harten_delta=1e-6, precision="fp64", device="cuda:0", stream=None, weno="js"):
        self.lib = _lib.load()
        nz, ny, nx = (int(s) for s in shape)
        self.shape = (nz, ny, nx)
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the HIP library needs a GPU device")
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        prec = _lib.CNS_FP64 if precision == "fp64" else _lib.CNS_MIXED
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.grid = _lib.Grid(nx, ny, nz, *length)
        self.phys = _lib.Physics(gamma, prandtl, mu_eff, weno_eps, harten_delta, _weno_code(weno))
        h = C.c_void_p()
        check(self.lib.cns_plan_create(C.byref(h), C.byref(self.grid), C.byref(self.phys), prec,
                                       C.c_void_p(self.stream.cuda_stream)), "cns_plan_create")
        self.h = h
        nbytes = int(self.lib.cns_workspace_bytes(h))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        check(self.lib.cns_set_workspace(h, _ptr(self.workspace), nbytes), "cns_set_workspace")

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.cns_plan_destroy(h)
            self.h = None

    # ---- helpers -------------------------------------------------------
    def _state(self, u: torch.Tensor, name="u"):
        if u.dtype != self.dtype or u.device != self.device or not u.is_contiguous() \
                or tuple(u.shape) != (5,) + self.shape:
            raise ValueError(f"{name} must be a contiguous {self.dtype} tensor of shape {(5,) + self.shape} "
                             f"on {self.device}")
        return u

    def empty_state(self):
        return torch.empty((5,) + self.shape, dtype=self.dtype, device=self.device)

    def set_tiles(self, seg=(0, 0, 0), block=0):
        check(self.lib.cns_set_tiles(self.h, int(seg[0]), int(seg[1]), int(seg[2]), int(block)), "cns_set_tiles")

    def set_x_kernel(self, kind: str = "rows"):
        """``"rows"`` (whole rows in LDS, default) or ``"march"`` for the x sweep."""
        check(self.lib.cns_set_x_kernel(self.h, 0 if kind == "rows" else 1), "cns_set_x_kernel")

    # ---- calls ---------------------------------------------------------
    def set_graph(self, enable=True):
        """Replay cns_rk4 from a captured hipGraph (needs a non-default stream)."""
        check(self.lib.cns_set_graph(self.h, 1 if enable else 0), "cns_set_graph")

    def init_state(self, rho, vel, p, out=None) -> torch.Tensor:
        """Conserved state from primitive arrays (numpy or tensors, float64)."""
        def dev(a):
            t = torch.as_tensor(np.ascontiguousarray(a) if isinstance(a, np.ndarray) else a,
                                dtype=torch.float64, device=self.device)
            return t.contiguous()
        with torch.cuda.stream(self.stream):
            r, v, pp = dev(rho), dev(vel), dev(p)
            for name, t, want in (("rho", r, self.shape), ("vel", v, (3,) + self.shape), ("p", pp, self.shape)):
                if tuple(t.shape) != want:
                    raise ValueError(f"{name} must have shape {want} (got {tuple(t.shape)})")
            u = self.empty_state() if out is None else self._state(out, "out")
            check(self.lib.cns_init_state(self.h, _ptr(r), _ptr(v), _ptr(pp), _ptr(u)), "cns_init_state")
        self._keep = (r, v, pp)  # alive until the stream has consumed them
        return u

    def rhs(self, u, out=None):
        self._state(u)
        out = self.empty_state() if out is None else self._state(out, "out")
        check(self.lib.cns_rhs(self.h, _ptr(u), _ptr(out)), "cns_rhs")
        return out

    def rhs_dir(self, u, direction, out=None):
        self._state(u)
        out = self.empty_state() if out is None else self._state(out, "out")
        check(self.lib.cns_rhs_dir(self.h, _ptr(u), int(direction), _ptr(out)), "cns_rhs_dir")
        return out

    def viscous(self, u, out=None):
        self._state(u)
        out = self.empty_state() if out is None else self._state(out, "out")
        check(self.lib.cns_viscous(self.h, _ptr(u), _ptr(out)), "cns_viscous")
        return out

    def rk4(self, u, dt, nsteps, diag=True):
        """Advance ``u`` in place by classical RK4; returns the per-step diagnostics
        tensor ``[nsteps][9]`` (float64, device) or None."""
        return self._steps("cns_rk4", u, dt, nsteps, diag)

    def tvdrk3(self, u, dt, nsteps, diag=True):
        """Advance ``u`` in place by third-order TVD Runge-Kutta (Shu-Osher); returns
        the per-step diagnostics as :meth:`rk4`."""
        return self._steps("cns_tvdrk3", u, dt, nsteps, diag)

    def _steps(self, fn, u, dt, nsteps, diag):
        self._state(u)
        d = torch.empty((max(int(nsteps), 1), CNS_NDIAG), dtype=torch.float64, device=self.device) if diag else None
        check(getattr(self.lib, fn)(self.h, _ptr(u), float(dt), int(nsteps), _ptr(d) if d is not None else None), fn)
        return d[:nsteps] if d is not None else None

    def spectrum(self, u):
        """Kinetic-energy spectrum of the velocity m/rho: ``(E, moments)``, device float64
        tensors ``[nshell]`` and ``[3]`` = (sum E, sum |k|^2 |v_hat|^2 / 2, Taylor
        microscale), all computed by the library."""
        self._state(u)
        ns = int(self.lib.cns_spectrum_shells(self.h))
        if ns < 1:
            check(ns, "cns_spectrum_shells")
        E = torch.empty(ns, dtype=torch.float64, device=self.device)
        mom = torch.empty(3, dtype=torch.float64, device=self.device)
        check(self.lib.cns_spectrum(self.h, _ptr(u), _ptr(E), ns, _ptr(mom)), "cns_spectrum")
        return E, mom

    @staticmethod
    def taylor_microscale(moments):
        """The Taylor microscale that :meth:`spectrum` returned in ``moments[2]``."""
        return float(moments[2])

    def max_wave_speed(self, u, out=None):
        """max over points and directions of |v_d| + c (device float64 tensor ``[1]``)."""
        self._state(u)
        out = torch.empty(1, dtype=torch.float64, device=self.device) if out is None else out
        check(self.lib.cns_max_wave_speed(self.h, _ptr(u), _ptr(out)), "cns_max_wave_speed")
        return out

    def graph_captures(self):
        """Graph captures made so far (replays of an unchanged run reuse one capture)."""
        n = int(self.lib.cns_plan_graph_captures(self.h))
        if n < 0:
            check(n, "cns_plan_graph_captures")
        return n

    def diagnostics(self, u, out=None):
        self._state(u)
        out = torch.empty(CNS_NDIAG, dtype=torch.float64, device=self.device) if out is None else out
        check(self.lib.cns_diagnostics(self.h, _ptr(u), _ptr(out)), "cns_diagnostics")
        return out

    def diagnostics_host(self, u, raise_bad=True):
        self._state(u)
        out = np.zeros(CNS_NDIAG)
        rc = self.lib.cns_diagnostics_host(self.h, _ptr(u), out.ctypes.data_as(C.POINTER(C.c_double)))
        if rc != 0 and (raise_bad or rc not in (-3, -4)):
            check(rc, "cns_diagnostics_host")
        return out

    # ---- adjoint (FP64) -----------------------------------------------------
    def _adj_ws(self, nsteps, ckpt_every):
        n = int(self.lib.cns_adjoint_workspace_bytes(self.h, int(nsteps), int(ckpt_every)))
        ws = getattr(self, "_adj_buf", None)
        if ws is None or ws.numel() < n:
            ws = torch.empty(n, dtype=torch.uint8, device=self.device)
            self._adj_buf = ws
        return ws, n

    def rhs_vjp(self, u, rbar, out=None):
        """``(dR/du)^T rbar`` at ``u``."""
        self._state(u)
        self._state(rbar, "rbar")
        out = self.empty_state() if out is None else self._state(out, "out")
        check(self.lib.cns_rhs_vjp(self.h, _ptr(u), _ptr(rbar), _ptr(out), None, 0), "cns_rhs_vjp")
        return out

    def adjoint_rk4(self, u0, dt, nsteps, ckpt_every):
        """``(J, dJ/du0)`` for J = mean kinetic energy after ``nsteps`` RK4 steps."""
        return self._adjoint("cns_adjoint_rk4", u0, dt, nsteps, ckpt_every)

    def adjoint_tvdrk3(self, u0, dt, nsteps, ckpt_every):
        """``(J, dJ/du0)`` for J = mean kinetic energy after ``nsteps`` TVD-RK3 steps."""
        return self._adjoint("cns_adjoint_tvdrk3", u0, dt, nsteps, ckpt_every)

    def _adjoint(self, fn, u0, dt, nsteps, ckpt_every):
        self._state(u0)
        ws, n = self._adj_ws(nsteps, ckpt_every)
        J = torch.empty(1, dtype=torch.float64, device=self.device)
        g = self.empty_state()
        check(getattr(self.lib, fn)(self.h, _ptr(u0), float(dt), int(nsteps), int(ckpt_every), _ptr(ws), n,
                                    _ptr(J), _ptr(g)), fn)
        return J, g

    def adjoint_workspace(self, nsteps, ckpt_every):
        """A device buffer for :meth:`adjoint_forward` / :meth:`adjoint_reverse` (the
        caller keeps it between the two calls)."""
        n = int(self.lib.cns_adjoint_workspace_bytes(self.h, int(nsteps), int(ckpt_every)))
        return torch.empty(n, dtype=torch.uint8, device=self.device)

    def adjoint_forward(self, u0, dt, nsteps, ckpt_every, ws, scheme="rk4"):
        """J = mean kinetic energy after ``nsteps`` steps of ``scheme`` from ``u0``; keeps
        the checkpoints in ``ws`` for :meth:`adjoint_reverse`."""
        self._state(u0)
        J = torch.empty(1, dtype=torch.float64, device=self.device)
        check(self.lib.cns_adjoint_forward(self.h, _scheme(scheme), _ptr(u0), float(dt), int(nsteps),
                                           int(ckpt_every), _ptr(ws), ws.numel(), _ptr(J)), "cns_adjoint_forward")
        return J

    def adjoint_reverse(self, dt, nsteps, ckpt_every, ws, scheme="rk4"):
        """dJ/du0 from the workspace :meth:`adjoint_forward` filled."""
        g = self.empty_state()
        check(self.lib.cns_adjoint_reverse(self.h, _scheme(scheme), float(dt), int(nsteps), int(ckpt_every),
                                           _ptr(ws), ws.numel(), _ptr(g)), "cns_adjoint_reverse")
        return g

    def ic_vjp(self, rho, vel, ubar):
        """Transpose of the initial-state map at fixed density and pressure."""
        out = torch.empty((3,) + self.shape, dtype=torch.float64, device=self.device)
        check(self.lib.cns_ic_vjp(self.h, _ptr(rho), _ptr(vel), _ptr(ubar), _ptr(out)), "cns_ic_vjp")
        return out

    # ---- per-kernel timing -------------------------------------------------
    def profile(self, enable=True):
        check(self.lib.cns_profile_enable(self.h, 1 if enable else 0), "cns_profile_enable")

    def profile_read(self):
        """``{kernel: (total_ms, launches)}`` since the last ``profile(True)``."""
        ms = np.zeros(_lib.CNS_NKERNEL)
        cnt = np.zeros(_lib.CNS_NKERNEL, dtype=np.int64)
        check(self.lib.cns_profile_read(self.h, ms.ctypes.data_as(C.POINTER(C.c_double)),
                                        cnt.ctypes.data_as(C.POINTER(C.c_int64))), "cns_profile_read")
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(_lib.KERNEL_NAMES)}


def _align_elems(dtype):
    return 256 // torch.tensor([], dtype=dtype).element_size()


class Ensemble:
    """Independent periodic boxes of uneven sizes advanced together.

    ``boxes``: list of dicts with ``shape`` (nz, ny, nx), ``mu_eff``, ``dt`` and
    optionally ``length``, ``gamma``, ``prandtl``, ``weno_eps``, ``harten_delta``, ``weno``
    (``"js"`` or ``"z"``, the same for every box).
    The states live in one packed device buffer; ``state(i)`` is box i's view.
    """

    def __init__(self, boxes, precision="fp64", device="cuda:0", stream=None):
        self.lib = _lib.load()
        self.device = torch.device(device)
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        prec = _lib.CNS_FP64 if precision == "fp64" else _lib.CNS_MIXED
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nb = len(boxes)
        self.shapes = [tuple(int(x) for x in b["shape"]) for b in boxes]
        al = _align_elems(self.dtype)
        offs, o = [], 0
        for sh in self.shapes:
            offs.append(o)
            n = 5 * sh[0] * sh[1] * sh[2]
            o += (n + al - 1) // al * al
        self.offsets = offs
        self.u = torch.zeros(max(o, al), dtype=self.dtype, device=self.device)
        grids = (_lib.Grid * nb)()
        phys = (_lib.Physics * nb)()
        dts = (C.c_double * nb)()
        for i, b in enumerate(boxes):
            nz, ny, nx = self.shapes[i]
            L = b.get("length", (TWO_PI, TWO_PI, TWO_PI))
            grids[i] = _lib.Grid(nx, ny, nz, *L)
            phys[i] = _lib.Physics(b.get("gamma", 1.4), b.get("prandtl", 0.72), b["mu_eff"],
                                   b.get("weno_eps", 1e-6), b.get("harten_delta", 1e-6),
                                   _weno_code(b.get("weno", "js")))
            dts[i] = float(b["dt"])
        coffs = (C.c_int64 * nb)(*offs)
        h = C.c_void_p()
        check(self.lib.cns_ensemble_create(C.byref(h), nb, grids, phys, dts, prec, _ptr(self.u), coffs,
                                           C.c_void_p(self.stream.cuda_stream)), "cns_ensemble_create")
        self.h = h
        self.nbox = nb
        nbytes = int(self.lib.cns_ensemble_workspace_bytes(h))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)  # the zero fill of the packed states is complete
        check(self.lib.cns_ensemble_set_workspace(h, _ptr(self.workspace), nbytes), "cns_ensemble_set_workspace")

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.cns_ensemble_destroy(h)
            self.h = None

    def state(self, i) -> torch.Tensor:
        nz, ny, nx = self.shapes[i]
        n = 5 * nz * ny * nx
        return self.u[self.offsets[i]:self.offsets[i] + n].view(5, nz, ny, nx)

    def set_tiles(self, box=-1, seg=(0, 0, 0), block=0):
        check(self.lib.cns_ensemble_set_tiles(self.h, int(box), int(seg[0]), int(seg[1]), int(seg[2]), int(block)),
              "cns_ensemble_set_tiles")

    def get_tiles(self, box):
        seg = (C.c_int32 * 3)()
        blk = C.c_int32()
        check(self.lib.cns_ensemble_get_tiles(self.h, int(box), seg, C.byref(blk)), "cns_ensemble_get_tiles")
        return tuple(seg), blk.value

    def get_launch(self, box):
        """``(rows, sweep_grid, tile_grid)``: rows per block of box's x rows kernel and the
        launched blocks of the sweeps and tiled kernels (0: one per virtual block)."""
        r, gs, gt = C.c_int32(), C.c_int64(), C.c_int64()
        check(self.lib.cns_ensemble_get_launch(self.h, int(box), C.byref(r), C.byref(gs), C.byref(gt)),
              "cns_ensemble_get_launch")
        return r.value, gs.value, gt.value

    def set_launch(self, box=-1, rows=0, sweep_grid=0, tile_grid=0):
        """Launch shapes by hand (see :meth:`get_launch`); results do not change."""
        check(self.lib.cns_ensemble_set_launch(self.h, int(box), int(rows), int(sweep_grid), int(tile_grid)),
              "cns_ensemble_set_launch")

    def autotune(self, cache_path=None):
        check(self.lib.cns_ensemble_autotune(self.h, cache_path.encode() if cache_path else None),
              "cns_ensemble_autotune")

    def set_integrator(self, scheme):
        """``"rk4"`` (default) or ``"tvdrk3"`` for :meth:`run`."""
        code = {"rk4": CNS_RK4, "tvdrk3": CNS_TVDRK3}[scheme]
        check(self.lib.cns_ensemble_set_integrator(self.h, code), "cns_ensemble_set_integrator")

    def run(self, nsteps, diag=True, graph=True):
        """nsteps steps of every box; returns diagnostics ``[nbox][nsteps][9]`` or None."""
        d = torch.empty((self.nbox, max(int(nsteps), 1), CNS_NDIAG), dtype=torch.float64,
                        device=self.device) if diag else None
        check(self.lib.cns_ensemble_run(self.h, int(nsteps), _ptr(d) if d is not None else None,
                                        1 if graph else 0), "cns_ensemble_run")
        return d[:, :nsteps] if d is not None else None

    def graph_captures(self):
        """Graph captures made so far (replays of an unchanged run reuse one capture)."""
        n = int(self.lib.cns_ensemble_graph_captures(self.h))
        if n < 0:
            check(n, "cns_ensemble_graph_captures")
        return n

    def profile(self, enable=True):
        check(self.lib.cns_ensemble_profile_enable(self.h, 1 if enable else 0), "cns_ensemble_profile_enable")

    def profile_read(self):
        ms = np.zeros(_lib.CNS_NKERNEL)
        cnt = np.zeros(_lib.CNS_NKERNEL, dtype=np.int64)
        check(self.lib.cns_ensemble_profile_read(self.h, ms.ctypes.data_as(C.POINTER(C.c_double)),
                                                 cnt.ctypes.data_as(C.POINTER(C.c_int64))),
              "cns_ensemble_profile_read")
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(_lib.KERNEL_NAMES)}
