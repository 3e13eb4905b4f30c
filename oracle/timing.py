"""Timing of the oracle for the benchmark's CPU baseline (test infrastructure only).

``python -m oracle.timing --prims FILE.npz --mu MU [--native] [--length L]`` builds the
state from the primitives ``rho [nz,ny,nx]``, ``vel [3,nz,ny,nx]``, ``p [nz,ny,nx]`` in
the file, times one evaluation of the oracle's right-hand side on it and prints one
JSON line: the seconds, the points, the OpenMP threads the oracle used, and which
build ran.  ``--native`` first compiles the oracle with ``-march=native`` for this host
(into a temporary directory) and checks on a small state that it returns bitwise what
the in-tree build returns.  The thread count follows ``OMP_NUM_THREADS``.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _rhs_with(path, u, mu):
    """RHS of u by the oracle library at `path` (loaded on its own handle)."""
    from oracle import oracle as O

    L = C.CDLL(path)
    L.oracle_rhs.argtypes = [C.POINTER(O.Grid), C.POINTER(O.Phys), O._dp, O._dp]
    out = np.zeros_like(u)
    g = O.make_grid(u.shape[1:])
    ph = O.make_phys(mu_eff=mu)
    rc = L.oracle_rhs(C.byref(g), C.byref(ph), O._ptr(u), O._ptr(out))
    if rc != 0:
        raise RuntimeError(f"oracle_rhs returned {rc}")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--prims", required=True)
    ap.add_argument("--mu", type=float, required=True)
    ap.add_argument("--native", action="store_true")
    args = ap.parse_args(argv)
    from oracle import build_oracle

    build = "in-tree (-O2 -ffp-contract=off)"
    same = None
    if args.native:
        tmp = tempfile.mkdtemp(prefix="cns_oracle_native_")
        path = build_oracle.build(native=True, out=os.path.join(tmp, "libcns_oracle_native.so"))
        # the native build against the in-tree one on a small smooth state
        from paper_2211_16718_amd import inputs as I
        import oracle

        r, v, p, _ = I.smooth_primitives((12, 10, 14), seed=3, amp=0.3)
        us = oracle.init_state(r, v, p)
        same = bool(np.array_equal(_rhs_with(path, us, args.mu), _rhs_with(build_oracle.LIB, us, args.mu)))
        os.environ["CNS_ORACLE_LIBRARY"] = path
        build = "-O2 -march=native -ffp-contract=off"
    import oracle

    d = np.load(args.prims, mmap_mode="r")
    u = oracle.init_state(np.asarray(d["rho"]), np.asarray(d["vel"]), np.asarray(d["p"]))
    ph = oracle.make_phys(mu_eff=args.mu)
    oracle.rhs(np.ascontiguousarray(u[:, :8, :8, :8]), ph)  # load the library, start the threads
    t0 = time.perf_counter()
    oracle.rhs(u, ph)
    sec = time.perf_counter() - t0
    print(json.dumps({"seconds": sec, "points": int(np.prod(u.shape[1:])), "threads": oracle.num_threads(),
                      "build": build, "native_bitwise_equal_to_in_tree": same}), flush=True)


if __name__ == "__main__":
    main()
