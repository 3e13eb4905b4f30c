#!/usr/bin/env python3
"""Throughput of the FP64 WENO5-Roe / central-viscous RK4 path on one MI355X.

Workload (default): 512^3 triply periodic decaying turbulence (seeded synthetic IC
with the HIT spectrum, Mt = 0.3, Re = 1600, gamma = 1.4, Pr = 0.72), classical RK4
at CFL 0.5 with the diagnostics (kinetic energy, enstrophy, means, wave speed) reduced
after every step.  One "step" is one RK4 step = 4 right-hand-side evaluations of the
whole grid.  ``--workload hit128`` runs the 128^3, Re = 400 case instead.

Metric: grid-point RHS evaluations per second (4 * N^3 per step), with the state
resident in HBM before the timed region starts.

Prints one JSON line.  ``roofline`` describes the kernel with the largest share of the
step, timed with HIP events on the plan's stream; ``step_hbm`` relates the bytes a step
must move to the step time; ``cpu_baseline`` times the CPU oracle (built for the host)
on one RHS evaluation of the same state on all host threads, with a one-thread sample.

``--summarize DIR`` instead reads rocprofv3 CSV output (a kernel trace and the
FETCH_SIZE / WRITE_SIZE counter runs, each taken with ``--calibrate-copy-gib``) and
writes ``profiles/traffic.json`` and a Markdown table of bytes and rates per kernel.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP64 operations per grid point of one launch (add, sub, mul, div and
# sqrt count one each; an FMA counts two), from the kernels' formulation:
#   point flux 18, WENO5 L+R pair 122 x 10 scalars, Roe dissipation 116,
#   interface flux 20, viscous interface flux 24, difference 10, plus the output
#   update (write 0 / accumulate 5 / fused RK4 stage ~30).
FLOPS_PER_POINT = {
    "sweep_x": 18 + 1220 + 5 + 116 + 20 + 24 + 10,
    "sweep_y": 18 + 1220 + 5 + 116 + 20 + 24 + 10 + 5,
    "sweep_z_rk4": 18 + 1220 + 5 + 116 + 20 + 24 + 10 + 30,
    "visc_flux": 13 + 12 * 5 + 40,  # primitives of the point, 12 derivatives, tau/q/G
    "diagnostics": 120,
}
# Algorithmic HBM bytes per grid point of one launch (FP64): each array element
# read or written once; the fused RK4 stage is averaged over the four stages
# (u^n read in stages 2-4, the accumulator written in stage 2 and read in stage 4).
BYTES_PER_POINT = {
    "sweep_x": 8 * (5 + 4 + 5),            # u, 4 viscous fluxes -> rhs
    "sweep_y": 8 * (5 + 4 + 5 + 5),        # + rhs read-modify-write
    "sweep_z_rk4": 8 * (5 + 4 + 5 + 5) + 8 * (15 + 5 + 5) // 4,  # u, G, rhs -> next stage; + u^n, acc
    "visc_flux": 8 * (5 + 9),              # u -> 9 viscous-flux fields
    "diagnostics": 8 * 5,
}
# The mixed form (FP32 state, G and rhs; FP64 accumulator, updated in every stage): u^n
# read in stages 2-3, the accumulator written in stage 1, updated in stages 2-3 and read
# in stage 4.
BYTES_PER_POINT_MIXED = {
    "sweep_x": 4 * (5 + 4 + 5),
    "sweep_y": 4 * (5 + 4 + 5 + 5),
    "sweep_z_rk4": 4 * (5 + 4 + 5 + 5) + (40 + 100 + 100 + 40) // 4,
    "visc_flux": 4 * (5 + 9),
    "diagnostics": 4 * 5,
}
# compulsory bytes of a fused RK4 step (three state arrays: u^n, the stage state and the
# FP64 accumulator), per point-RHS
COMPULSORY_BYTES_PER_POINT_RHS = 160
PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector (256 CU x 64 lanes x 2 x 2.4 GHz)
PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector (published; its 2x over FP64 needs packed FP32)
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E
PEAK_VALU_LANE_INSTR = 256 * 4 * 16 * 2.4e9  # VALU lane-instructions per second (3.93e13)
# rocprofv3 kernel names -> the library's kernel kinds
KERNEL_KIND_OF = (("k_sweep_x_rows", "sweep_x"), ("k_sweep_x_chunks", "sweep_x"), ("k_visc_flux", "visc_flux"), ("k_diag_partial", "diagnostics"),
                  ("k_diag_final", "diagnostics_final"), ("k_stream_copy", "stream_copy"),
                  ("k_init_state", "init_state"), ("k_speed_", "max_wave_speed"))


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_digest():
    """SHA-256 of the sources the step's kernels are built from (counters taken on other
    sources are stale)."""
    import hashlib

    h = hashlib.sha256()
    for f in ("cns_kernels.hip", "cns_device.h", "cns_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2211_16718_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="hit512", choices=["hit512", "hit128"],
                    help="hit512: 512^3, Re 1600 (the default); hit128: 128^3, Re 400")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="fp64 (the named workload) or the mixed form, for profiling it alone")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the mixed-precision, ensemble, adjoint and option measurements")
    ap.add_argument("--extras", default="mixed_512,ensemble_64,adjoint_128,options_128",
                    help="comma-separated subset of the extra measurements to run")
    ap.add_argument("--copy-gib", type=float, default=4.0,
                    help="size of the streaming-copy bandwidth reference (GiB)")
    ap.add_argument("--calibrate-copy-gib", type=float, default=0.0,
                    help="before the workload, run the streaming copy once on a buffer of this many GiB "
                         "(a known-size dispatch for hardware byte counters)")
    ap.add_argument("--summarize", metavar="DIR", default=None,
                    help="summarize rocprofv3 CSV output under DIR (kt/, fetch/, write/) instead of running")
    ap.add_argument("--summary-title", default="")
    return ap.parse_args()


def stream_copy(lib, src, dst, nbytes, stream):
    from paper_2211_16718_amd._lib import check

    check(lib.cns_stream_copy(src.data_ptr(), dst.data_ptr(), int(nbytes), stream.cuda_stream), "cns_stream_copy")


def copy_reference(gib, stream):
    """Read + write bandwidth of the library's streaming copy (median of 5 copies of `gib` GiB)."""
    import torch

    from paper_2211_16718_amd import _lib

    lib = _lib.load()
    nb = int(gib * (1 << 30)) // 16 * 16
    src = torch.ones(nb // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    stream_copy(lib, src, dst, nb, stream)  # warm
    times = []
    for _ in range(5):
        sec, _ = _timed(stream, lambda: stream_copy(lib, src, dst, nb, stream))
        times.append(sec)
    assert torch.equal(src[:1024], dst[:1024]) and torch.equal(src[-1024:], dst[-1024:])
    times.sort()
    del src, dst
    return {"bytes_moved": 2 * nb, "GBs": 2 * nb / times[2] / 1e9, "kernel": "cns_stream_copy (16-byte "
            "non-temporal loads and stores, 2048 x 256 threads)"}


def main():
    args = parse()
    if args.summarize:
        return summarize(args.summarize, args.summary_title)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "domain decomposition is not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2211_16718_amd import _lib
    from paper_2211_16718_amd import inputs as I
    from paper_2211_16718_amd.api import Plan

    wl = I.WORKLOADS[args.workload]
    n, mu = wl.n, 1.0 / wl.re
    fp64 = args.precision == "fp64"
    if args.calibrate_copy_gib > 0:
        nb = int(args.calibrate_copy_gib * (1 << 30)) // 16 * 16
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        stream_copy(_lib.load(), src, dst, nb, torch.cuda.current_stream())
        torch.cuda.synchronize()
        del src, dst
    t0 = time.perf_counter()
    rho, vel, p = I.hit_primitives(n, wl.seed, wl.mt)
    log(f"initial condition {n}^3 in {time.perf_counter() - t0:.1f} s")
    plan = Plan((n, n, n), mu_eff=mu, precision=args.precision, device="cuda:0")
    u = plan.init_state(rho, vel, p)
    smax = float(plan.max_wave_speed(u).item())
    dt = I.dt_from_speed(smax, n, cfl=I.CFL)
    stream = plan.stream

    # untimed warmup
    if args.warmup > 0:
        plan.rk4(u, dt, args.warmup)
    torch.cuda.synchronize()
    u_start = u.clone()

    # timed region: exactly K steps, state resident in HBM
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    diag = plan.rk4(u, dt, args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    diag_h = diag.cpu().numpy()
    if np.any(diag_h[:, 8] > 0):
        print("bench: non-finite or non-physical state during the timed run", file=sys.stderr)
        sys.exit(3)
    log(f"timed {args.steps} steps: {gpu_ms / args.steps:.3f} ms/step")

    seconds = gpu_ms / 1e3
    point_rhs = 4.0 * n ** 3 * args.steps
    value = point_rhs / seconds

    # per-kernel timing of the same K steps (events around every launch)
    u.copy_(u_start)
    plan.profile(True)
    plan.rk4(u, dt, args.steps)
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile(False)
    kernels = {}
    for name, (ms, cnt) in prof.items():
        if cnt:
            kernels[name] = {"avg_ms": ms / cnt, "launches": cnt, "share": None, "total_ms": ms}
    tot = sum(k["total_ms"] for k in kernels.values())
    for k in kernels.values():
        k["share"] = k["total_ms"] / tot
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    avg_s = kernels[dom]["avg_ms"] / 1e3
    flops = FLOPS_PER_POINT[dom] * n ** 3
    achieved = flops / avg_s / 1e12
    del u_start
    copy = copy_reference(args.copy_gib, stream)
    log(f"streaming copy reference {copy['GBs']:.0f} GB/s")

    traffic, traffic_note = None, "no counters for these kernel sources at this size"
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tfile):
        try:
            t = json.load(open(tfile))
            if t.get("kernel_source_sha256") == kernel_source_digest() and dom in t.get("kernels", {}) \
                    and t.get("n") == n and t.get("precision", "fp64") == args.precision:
                traffic = t["kernels"][dom]["bytes_per_launch"]
                traffic_note = (f"FETCH_SIZE x {t['fetch_scale']:.3f} + WRITE_SIZE x {t['write_scale']:.3f} per "
                                "dispatch (scales from a streaming copy of known size)")
        except Exception:
            traffic = None
    # VALU instructions per point of the dominant kernel (SQ_INSTS_VALU counters taken on
    # the same kernel sources), as a fraction of the issue peak: one wave64 VALU
    # instruction per SIMD every 4 cycles = 256 x 4 x 16 lanes x 2.4 GHz lane-instructions/s
    valu = None
    vfile = os.path.join(ROOT, "profiles", "valu.json")
    if os.path.exists(vfile):
        try:
            v = json.load(open(vfile))
            if fp64 and v.get("kernel_source_sha256") == kernel_source_digest() and dom in v.get("kernels", {}):
                per = v["kernels"][dom]["valu_per_point"]
                valu = {"valu_instructions_per_point": round(per, 1),
                        "valu_issue_frac": round(per * n ** 3 / avg_s / PEAK_VALU_LANE_INSTR, 4)}
        except Exception:
            valu = None
    peak = PEAK_FP64_TFLOPS if fp64 else PEAK_FP32_TFLOPS
    bpp_tab = BYTES_PER_POINT if fp64 else BYTES_PER_POINT_MIXED
    bpp = bpp_tab[dom]
    roofline = {
        "bound": "alu",
        "kernel": dom,
        "achieved": round(achieved, 3),
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": round(achieved / peak, 4),
        "traffic": traffic,
        "traffic_source": traffic_note,
        "algorithmic_bytes_per_launch": bpp * n ** 3,
        "hbm_frac_algorithmic": round(bpp * n ** 3 / avg_s / 1e9 / PEAK_HBM_GBS, 4),
        "flops_per_point": FLOPS_PER_POINT[dom],
        "avg_launch_ms": round(kernels[dom]["avg_ms"], 5),
    }
    if traffic:
        roofline["hbm_GBs_measured_bytes"] = round(traffic / avg_s / 1e9, 1)
        roofline["hbm_frac_measured_bytes"] = round(traffic / avg_s / 1e9 / PEAK_HBM_GBS, 4)
    if valu:
        roofline.update(valu)

    # the whole step against HBM: the bytes the step's launches must move (each array
    # element read or written once per launch), and the compulsory bytes of a fused step
    step_s = gpu_ms / 1e3 / args.steps
    design = sum(bpp_tab[k] * n ** 3 * kernels[k]["launches"] / args.steps for k in kernels if k in bpp_tab)
    compulsory = COMPULSORY_BYTES_PER_POINT_RHS * 4 * n ** 3 * (1 if fp64 else 110 / 160)
    step_hbm = {
        "design_bytes_per_step": int(design),
        "design_GBs": round(design / step_s / 1e9, 1),
        "design_frac_of_peak": round(design / step_s / 1e9 / PEAK_HBM_GBS, 4),
        "design_frac_of_copy": round(design / step_s / 1e9 / copy["GBs"], 4),
        "compulsory_bytes_per_point_rhs": COMPULSORY_BYTES_PER_POINT_RHS if fp64 else 110,
        "compulsory_frac_of_peak": round(compulsory / step_s / 1e9 / PEAK_HBM_GBS, 4),
        "copy_reference_GBs": round(copy["GBs"], 1),
        "copy_reference_frac_of_peak": round(copy["GBs"] / PEAK_HBM_GBS, 4),
    }
    del plan, u
    torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline and fp64:
        cpu = cpu_baseline(n, mu, wl, rho, vel, p, value)

    extras = {}
    if not args.no_extras:
        wanted = set(args.extras.split(","))
        prims512 = (rho, vel, p) if n == 512 else None
        for name, fn in (("mixed_512", lambda: bench_mixed(prims512)), ("ensemble_64", bench_ensemble),
                         ("adjoint_128", bench_adjoint), ("options_128", lambda: bench_options(prims512))):
            if name not in wanted:
                continue
            t0 = time.perf_counter()
            try:
                extras[name] = fn()
            except Exception as e:  # report, keep the main line
                extras[name] = {"error": f"{type(e).__name__}: {e}"}
            log(f"extra {name} in {time.perf_counter() - t0:.1f} s")
            torch.cuda.empty_cache()

    out = {
        "metric": "grid-point RHS evaluations per second (FP64 WENO5-Roe + central viscous, RK4)" if fp64 else
                  "grid-point RHS evaluations per second (mixed FP32/FP64 WENO5-Roe + central viscous, RK4)",
        "value": value,
        "unit": "point-RHS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": gpu_ms / args.steps,
        "wall_ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if fp64 else "f32+f64",
        "data": "synthetic (seeded HIT-spectrum initial condition)",
        "config": {"workload": f"hit{n}_re{int(wl.re)}_rk4_diag_every_step" + ("" if fp64 else "_mixed"),
                   "grid": [n, n, n], "re": wl.re, "mt": wl.mt, "cfl": I.CFL, "dt": dt, "precision": args.precision,
                   "launches": "eager (18 per step)"},
        "roofline": roofline,
        "step_hbm": step_hbm,
        "kernels": {k: {"avg_ms": round(v["avg_ms"], 5), "launches": v["launches"], "share": round(v["share"], 4)}
                    for k, v in kernels.items()},
        "cpu_baseline": cpu,
    }
    out.update(extras)
    print(json.dumps(out), flush=True)


def _child_json(argv, env=None, timeout=600):
    r = subprocess.run(argv, env=env, capture_output=True, text=True, timeout=timeout, cwd=ROOT)
    if r.returncode != 0:
        raise RuntimeError(f"{' '.join(argv[:4])}... exited {r.returncode}: {r.stderr[-400:]}")
    return json.loads(r.stdout.strip().splitlines()[-1])


def cpu_baseline(n, mu, wl, rho, vel, p, gpu_value):
    """The oracle, built for this host (-O2 -march=native -ffp-contract=off), timed on one
    RHS evaluation of the benchmark's own state on every host thread; a one-thread sample
    on one RHS of the 128^3 state of the same physics; the oracle beside the GPU on the
    other configurations (in-tree build)."""
    import numpy as np

    from paper_2211_16718_amd import inputs as I

    t0 = time.perf_counter()
    tmp = tempfile.mkdtemp(prefix="cns_bench_")
    out = {"kind": "oracle", "unit": "point-RHS/s"}
    try:
        f = os.path.join(tmp, "prims.npz")
        np.savez(f, rho=rho, vel=vel, p=p)
        d = _child_json([sys.executable, "-m", "oracle.timing", "--prims", f, "--mu", repr(mu), "--native"])
        os.remove(f)
        out.update({"value": d["points"] / d["seconds"], "cores": d["threads"],
                    "sample": f"one RHS evaluation of the same {n}^3 state ({d['points']} point-RHS) in "
                              f"{d['seconds']:.1f} s on {d['threads']} OpenMP threads; oracle built "
                              f"{d['build']}, bitwise equal to the in-tree build: {d['native_bitwise_equal_to_in_tree']}",
                    "gpu_over_oracle": gpu_value * d["seconds"] / d["points"]})
        m = 128
        r1, v1, p1 = I.hit_primitives(m, wl.seed, wl.mt)
        f1 = os.path.join(tmp, "prims128.npz")
        np.savez(f1, rho=r1, vel=v1, p=p1)
        d1 = _child_json([sys.executable, "-m", "oracle.timing", "--prims", f1, "--mu", repr(mu), "--native"],
                         env=dict(os.environ, OMP_NUM_THREADS="1"))
        out["one_core"] = {"value": d1["points"] / d1["seconds"], "unit": "point-RHS/s", "cores": d1["threads"],
                           "kind": "oracle", "sample": f"one RHS evaluation of the {m}^3 state of the same physics "
                                                       f"in {d1['seconds']:.1f} s ({d1['build']})",
                           "gpu_over_one_core": gpu_value * d1["seconds"] / d1["points"]}
    except Exception as e:
        out["error"] = f"{type(e).__name__}: {e}"
    finally:
        import shutil

        shutil.rmtree(tmp, ignore_errors=True)
    out["host"] = _host_cpu()
    out["configs"] = _oracle_configs()
    log(f"cpu baseline in {time.perf_counter() - t0:.1f} s")
    return out


def _timed(stream, fn):
    import torch

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    r = fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3, r


def _oracle_configs():
    """The oracle beside the GPU path on the other configurations, all host threads: the
    32^3 workload in full (10 RK4 steps), the first 32^3 and 96^3 boxes of the uneven
    ensemble (2 RK4 steps each), and the gradient of the final kinetic energy at 16^3 (2
    RK4 steps; the restatement runs op by op, several seconds per step) from
    the PyTorch CPU restatement.  Each with the GPU time of the same work."""
    import torch

    import oracle
    from oracle import torch_ref
    from paper_2211_16718_amd import inputs as I
    from paper_2211_16718_amd.adjoint import FinalKineticEnergy
    from paper_2211_16718_amd.api import Plan

    def both(n, rho, vel, p, mu, steps):
        ph = oracle.make_phys(mu_eff=mu)
        uh = oracle.init_state(rho, vel, p)
        plan = Plan((n, n, n), mu_eff=mu)
        u = plan.init_state(rho, vel, p)
        dt = I.dt_from_speed(plan.diagnostics_host(u)[7], n)
        plan.rk4(plan.empty_state().copy_(u), dt, 1)  # warm
        gsec, _ = _timed(plan.stream, lambda: plan.rk4(u, dt, steps))
        t0 = time.perf_counter()
        oracle.rk4(uh, dt, steps, ph)
        csec = time.perf_counter() - t0
        work = 4.0 * n ** 3 * steps
        return {"grid": n, "steps": steps, "oracle_point_rhs_per_s": work / csec, "oracle_s": csec,
                "gpu_point_rhs_per_s": work / gsec, "gpu_s": gsec, "gpu_over_oracle": csec / gsec}

    out = {"cores": oracle.num_threads()}
    wl = I.WORKLOADS["hit32"]
    out["hit32_rk4x10"] = both(32, *I.hit_primitives(32, wl.seed, wl.mt), 1.0 / wl.re, 10)
    for want in (32, 96):
        i = next(i for i in range(64) if I.ensemble_box_params(i)[0].n == want)
        box, rho, vel, p = I.ensemble_box_primitives(i)
        out[f"ensemble_box{i}_n{want}_rk4x2"] = both(want, rho, vel, p, 1.0 / box.re, 2)
    n, steps, mu = 16, 2, 1.0 / 400
    rho, vel, p = I.hit_primitives(n, 0, 0.3)
    plan = Plan((n, n, n), mu_eff=mu)
    dt = I.dt_from_speed(plan.diagnostics_host(plan.init_state(rho, vel, p))[7], n)
    r, v, q = (torch.from_numpy(a).cuda() for a in (rho, vel, p))

    def grad():
        v0 = v.clone().requires_grad_(True)
        FinalKineticEnergy.apply(v0, r, q, plan, dt, steps, 1).backward()
        return v0.grad

    grad()  # warm
    gsec, _ = _timed(plan.stream, grad)
    t0 = time.perf_counter()
    torch_ref.final_ke_and_grad(rho, vel, p, dt, steps, torch_ref.make_phys(mu=mu))
    csec = time.perf_counter() - t0
    out[f"adjoint16_rk4x{steps}"] = {"grid": n, "steps": steps, "torch_cpu_s": csec, "torch_cpu_threads": torch.get_num_threads(),
                               "gpu_s": gsec, "gpu_over_cpu": csec / gsec}
    return out


def _host_cpu():
    """The host CPU the oracle ran on: model name, logical CPUs, sockets, physical cores,
    the CPUs this process may use and OMP_NUM_THREADS."""
    model, sockets, cores = None, set(), set()
    phys = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name" and model is None:
                    model = v
                elif k == "physical id":
                    phys = v
                    sockets.add(v)
                elif k == "core id":
                    cores.add((phys, v))
    except OSError:
        pass
    info = {"model": model, "logical_cpus": os.cpu_count(), "sockets": len(sockets) or None,
            "physical_cores": len(cores) or None,
            "usable_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}
    try:
        r = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20)
        keep = ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)", "NUMA node(s)")
        info["lscpu"] = {k.strip(): v.strip() for k, _, v in (ln.partition(":") for ln in r.stdout.splitlines())
                         if k.strip() in keep}
    except Exception:
        pass
    return info


def bench_mixed(prims=None, n=512, steps=20):
    """512^3, Re = 1600: mixed precision against the FP64 path at the same size."""
    import numpy as np  # noqa: F401
    import torch  # noqa: F401

    from paper_2211_16718_amd import inputs as I
    from paper_2211_16718_amd.api import Plan

    wl = I.WORKLOADS["hit512"]
    rho, vel, p = prims if prims is not None else I.hit_primitives(n, wl.seed, wl.mt)
    out = {"config": {"workload": f"hit{n}_re1600_rk4x{steps}", "grid": [n, n, n], "steps": steps}}
    res = {}
    for prec in ("fp64", "mixed"):
        plan = Plan((n, n, n), mu_eff=1.0 / wl.re, precision=prec)
        u = plan.init_state(rho, vel, p)
        if prec == "fp64":
            dt = I.dt_from_speed(float(plan.max_wave_speed(u).item()), n)
        plan.rk4(plan.empty_state().copy_(u), dt, 1, diag=False)  # warm
        sec, diag = _timed(plan.stream, lambda: plan.rk4(u, dt, steps))
        res[prec] = (u, diag.cpu().numpy(), sec)
        out[prec] = {"value": 4.0 * n ** 3 * steps / sec, "unit": "point-RHS/s", "ms_per_step": sec * 1e3 / steps,
                     "bytes_per_state": int(u.numel() * u.element_size())}
        del plan
    u64, d64, _ = res["fp64"]
    u32, d32, _ = res["mixed"]
    per_var = [float((u32[v].double() - u64[v]).abs().max() / u64[v].abs().max()) for v in range(5)]
    out["mixed_vs_fp64"] = {"max_norm_rel_err_per_variable": per_var,
                            "ke_rel_err_final": float(abs(d32[-1, 0] - d64[-1, 0]) / d64[-1, 0]),
                            "enstrophy_rel_err_final": float(abs(d32[-1, 1] - d64[-1, 1]) / d64[-1, 1])}
    out["speedup_mixed_over_fp64"] = out["mixed"]["value"] / out["fp64"]["value"]
    return out


def bench_ensemble(nbox=64, steps=50):
    """64 boxes of sizes drawn from {32,48,64,96}, 50 RK4 steps, one captured graph."""
    import torch

    from paper_2211_16718_amd import inputs as I
    from paper_2211_16718_amd.api import Ensemble, Plan

    stream = torch.cuda.Stream()
    boxes, prims = [], []
    for i in range(nbox):
        box, rho, vel, p = I.ensemble_box_primitives(i)
        boxes.append(dict(shape=(box.n,) * 3, mu_eff=1.0 / box.re, dt=1.0))
        prims.append((rho, vel, p))
    # dt per box from the GPU diagnostics of its initial state
    for b, pr in zip(boxes, prims):
        pl = Plan(b["shape"], mu_eff=b["mu_eff"], stream=stream)
        with torch.cuda.stream(stream):
            smax = pl.diagnostics_host(pl.init_state(*pr))[7]
        b["dt"] = I.dt_from_speed(smax, b["shape"][0])
    ens = Ensemble(boxes, stream=stream)
    for i, (b, pr) in enumerate(zip(boxes, prims)):
        pl = Plan(b["shape"], mu_eff=b["mu_eff"], stream=stream)
        with torch.cuda.stream(stream):
            pl.init_state(*pr, out=ens.state(i))
    stream.synchronize()
    t0 = time.perf_counter()
    ens.autotune(None)
    tune_s = time.perf_counter() - t0
    u_start = ens.u.clone()
    with torch.cuda.stream(stream):
        ens.run(steps, graph=True)  # capture + warm: the timed call replays this capture
    stream.synchronize()
    ens.u.copy_(u_start)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        sec, diag = _timed(stream, lambda: ens.run(steps, graph=True))
    assert ens.graph_captures() == 1
    pts = sum(b["shape"][0] ** 3 for b in boxes)
    shapes = {}
    for i, b in enumerate(boxes):
        n = b["shape"][0]
        if n not in shapes:
            seg, blk = ens.get_tiles(i)
            rows, gs, gt = ens.get_launch(i)
            shapes[n] = {"seg_yz": seg[1:], "block": blk, "rows": rows, "sweep_grid": gs, "tile_grid": gt}
    return {"config": {"workload": f"ensemble{nbox}_rk4x{steps}", "boxes": nbox, "points": pts,
                       "sizes": sorted({b["shape"][0] for b in boxes})}, "launch_shapes": shapes,
            "value": 4.0 * pts * steps / sec, "unit": "point-RHS/s", "ms_per_step": sec * 1e3 / steps,
            "autotune_s": tune_s, "graph": True,
            "bad_points": int((diag[..., 8] > 0).sum().item())}


def bench_adjoint(n=128, steps=200, ckpt=20):
    """128^3, Re = 400: J = final kinetic energy after 200 steps and dJ/dv0."""
    import torch

    from paper_2211_16718_amd import inputs as I
    from paper_2211_16718_amd.adjoint import FinalKineticEnergy
    from paper_2211_16718_amd.api import Plan

    rho, vel, p = (torch.from_numpy(a).cuda() for a in I.hit_primitives(n, 0, 0.3))
    plan = Plan((n, n, n), mu_eff=1.0 / 400)
    u0 = plan.init_state(rho, vel, p)
    dt = I.dt_from_speed(plan.diagnostics_host(u0)[7], n)
    fsec, _ = _timed(plan.stream, lambda: plan.rk4(u0, dt, steps, diag=False))

    def grad():
        v0 = vel.clone().requires_grad_(True)
        J = FinalKineticEnergy.apply(v0, rho, p, plan, dt, steps, ckpt)
        J.backward()
        return J, v0.grad

    grad()  # warm: the workspace allocation and the first launches stay out of the timing
    gsec, (J, g) = _timed(plan.stream, grad)
    # J alone: the autograd forward (the steps with checkpoints), no reverse sweep
    v0 = vel.clone().requires_grad_(True)
    jsec, _ = _timed(plan.stream, lambda: FinalKineticEnergy.apply(v0, rho, p, plan, dt, steps, ckpt))
    out = {"config": {"workload": f"hit{n}_re400_rk4x{steps}_adjoint", "ckpt_every": ckpt},
           "forward_s": fsec, "gradient_s": gsec, "gradient_over_forward": gsec / fsec,
           "autograd_forward_s": jsec, "reverse_over_forward": (gsec - jsec) / fsec,
           "value": 4.0 * n ** 3 * steps / gsec, "unit": "point-RHS/s (forward-step equivalents of the gradient)",
           "J": float(J.detach()), "grad_norm": float(g.norm())}
    # one vector-Jacobian product against one right-hand side at the same state
    rbar = torch.randn(u0.shape, dtype=torch.float64, device=u0.device)
    ub = plan.rhs_vjp(u0, rbar)
    r = plan.rhs(u0)
    psec, _ = _timed(plan.stream, lambda: [plan.rhs_vjp(u0, rbar, out=ub) for _ in range(20)])
    rsec, _ = _timed(plan.stream, lambda: [plan.rhs(u0, out=r) for _ in range(20)])
    out["product_ms"], out["rhs_ms"] = psec / 20 * 1e3, rsec / 20 * 1e3
    out["product_over_rhs"] = psec / rsec
    # the same gradient through the TVD-RK3 integrator (checkpoints every ckpt steps)
    plan.tvdrk3(plan.init_state(rho, vel, p), dt, 1, diag=False)
    u3 = plan.init_state(rho, vel, p)
    f3, _ = _timed(plan.stream, lambda: plan.tvdrk3(u3, dt, steps, diag=False))

    def grad3():
        v0 = vel.clone().requires_grad_(True)
        J = FinalKineticEnergy.apply(v0, rho, p, plan, dt, steps, ckpt, "tvdrk3")
        J.backward()
        return J, v0.grad

    grad3()
    g3, (J3, _) = _timed(plan.stream, grad3)
    out["tvdrk3"] = {"forward_s": f3, "gradient_s": g3, "gradient_over_forward": g3 / f3, "J": float(J3.detach())}
    # one segment (checkpoint interval = all steps): the forward pass keeps the start and
    # stage states of every step in HBM (4 states per step) and nothing is recomputed
    need = int(plan.lib.cns_adjoint_workspace_bytes(plan.h, steps, steps))
    if need < 0.8 * torch.cuda.mem_get_info()[0]:
        g20 = g.clone()
        ckpt_all = steps

        def grad1():
            v0 = vel.clone().requires_grad_(True)
            J = FinalKineticEnergy.apply(v0, rho, p, plan, dt, steps, ckpt_all)
            J.backward()
            return J, v0.grad

        grad1()
        gsec1, (J1, g1) = _timed(plan.stream, grad1)
        out["one_segment"] = {"ckpt_every": steps, "workspace_GB": need / 1e9, "gradient_s": gsec1,
                              "gradient_over_forward": gsec1 / fsec,
                              "max_abs_diff_vs_ckpt": float((g1 - g20).abs().max())}
        plan._adj_buf = None
        torch.cuda.empty_cache()
    return out


def bench_options(prims512=None, n=128, steps=20):
    """The same 128^3 workload with the TVD-RK3 integrator, with WENO-Z and with mapped
    weights, the RHS alone, and the time of one energy spectrum (128^3 and 512^3)."""
    import torch

    from paper_2211_16718_amd import inputs as I
    from paper_2211_16718_amd.api import Plan

    wl = I.WORKLOADS["hit128"]
    rho, vel, p = I.hit_primitives(n, wl.seed, wl.mt)
    out = {"config": {"workload": f"hit{n}_re400", "grid": [n, n, n], "steps": steps}}
    plan = Plan((n, n, n), mu_eff=1.0 / wl.re)
    u = plan.init_state(rho, vel, p)
    dt = I.dt_from_speed(plan.diagnostics_host(u)[7], n)
    plan.tvdrk3(plan.empty_state().copy_(u), dt, 1, diag=False)  # warm
    sec, _ = _timed(plan.stream, lambda: plan.tvdrk3(u, dt, steps))
    out["tvdrk3"] = {"value": 3.0 * n ** 3 * steps / sec, "unit": "point-RHS/s", "ms_per_step": sec * 1e3 / steps}
    pz = Plan((n, n, n), mu_eff=1.0 / wl.re, weno="z")
    uz = pz.init_state(rho, vel, p)
    pz.rk4(pz.empty_state().copy_(uz), dt, 1, diag=False)
    sec, _ = _timed(pz.stream, lambda: pz.rk4(uz, dt, steps))
    out["rk4_wenoz"] = {"value": 4.0 * n ** 3 * steps / sec, "unit": "point-RHS/s", "ms_per_step": sec * 1e3 / steps}
    pm = Plan((n, n, n), mu_eff=1.0 / wl.re, weno="m")
    um = pm.init_state(rho, vel, p)
    pm.rk4(pm.empty_state().copy_(um), dt, 1, diag=False)
    sec, _ = _timed(pm.stream, lambda: pm.rk4(um, dt, steps))
    out["rk4_wenom"] = {"value": 4.0 * n ** 3 * steps / sec, "unit": "point-RHS/s", "ms_per_step": sec * 1e3 / steps}
    del pm, um
    # the RHS alone (cns_rhs: viscous fluxes and the three sweeps, no stage update)
    r = plan.empty_state()
    plan.rhs(u, r)
    reps = 20
    sec, _ = _timed(plan.stream, lambda: [plan.rhs(u, r) for _ in range(reps)])
    out["rhs_only"] = {"value": n ** 3 * reps / sec, "unit": "point-RHS/s", "ms": sec * 1e3 / reps}
    plan.spectrum(u)  # warm
    reps = 5
    sec, (E, mom) = _timed(plan.stream, lambda: [plan.spectrum(u) for _ in range(reps)][-1])
    out["spectrum_128"] = {"ms": sec * 1e3 / reps, "taylor_microscale": Plan.taylor_microscale(mom),
                           "k_peak": int(torch.argmax(E).item())}
    del plan, pz, u, uz
    torch.cuda.empty_cache()
    m = 512
    r5, v5, p5 = prims512 if prims512 is not None else I.hit_primitives(m, 0, 0.3)
    p512 = Plan((m, m, m), mu_eff=1.0 / 1600)
    u5 = p512.init_state(r5, v5, p5)
    p512.spectrum(u5)
    sec, (E, mom) = _timed(p512.stream, lambda: p512.spectrum(u5))
    out["spectrum_512"] = {"ms": sec * 1e3, "taylor_microscale": Plan.taylor_microscale(mom)}
    return out


# ---------------------------------------------------------------------------------------
# rocprofv3 summaries
# ---------------------------------------------------------------------------------------
def _csv_rows(d, suffix):
    import csv

    rows = []
    for root, _, files in os.walk(d):
        for f in sorted(files):
            if f.endswith(suffix):
                with open(os.path.join(root, f), newline="") as fh:
                    rows += list(csv.DictReader(fh))
    return rows


def kernel_kind(name):
    """The library's kernel kind of a rocprofv3 kernel name (template arguments decide
    the direction and the output mode of a marching sweep)."""
    if "k_sweep<" in name and "k_sweep_x_rows" not in name:
        args = [a.strip() for a in name.split("k_sweep<", 1)[1].split(">", 1)[0].split(",")]
        d, mode = int(args[2]), int(args[3])
        return ("sweep_x", "sweep_y", "sweep_z_rk4" if mode == 2 else "sweep_z")[d]
    for key, kind in KERNEL_KIND_OF:
        if key in name:
            return kind
    return name.split("(")[0].replace("void ", "").replace("cns::", "")


def summarize(d, title):
    """Per-kernel bytes and rates from rocprofv3 CSV output under d: kt/ (kernel trace),
    fetch/ (FETCH_SIZE) and write/ (WRITE_SIZE).  d/meta.json gives the grid size, the
    precision, the bytes of one calibration copy and the commands that made the runs.
    Writes profiles/traffic.json and prints a Markdown table."""
    meta = json.load(open(os.path.join(d, "meta.json")))
    n, prec = meta["n"], meta.get("precision", "fp64")
    copy_bytes = meta["copy_bytes"]
    trace = _csv_rows(os.path.join(d, "kt"), "kernel_trace.csv")
    dur = {}
    for r in trace:
        dur.setdefault(r["Kernel_Name"], []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))

    def counter(sub, cname):
        vals = {}
        for r in _csv_rows(os.path.join(d, sub), "counter_collection.csv"):
            if r.get("Counter_Name") == cname:
                vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * 1024.0)
        return vals

    fetch, write = counter("fetch", "FETCH_SIZE"), counter("write", "WRITE_SIZE")
    copy_name = next(k for k in fetch if "k_stream_copy" in k)
    fetch_scale = copy_bytes / (sorted(fetch[copy_name])[len(fetch[copy_name]) // 2])
    write_scale = copy_bytes / (sorted(write[copy_name])[len(write[copy_name]) // 2])
    copy_ns = sorted(dur.get(copy_name, [0]))[len(dur.get(copy_name, [0])) // 2]
    copy_GBs = 2 * copy_bytes / copy_ns if copy_ns else None
    bpp = BYTES_PER_POINT if prec == "fp64" else BYTES_PER_POINT_MIXED
    kinds, rows = {}, []
    for name in sorted(set(fetch) & set(write), key=lambda k: -sum(dur.get(k, [0]))):
        kind = kernel_kind(name)
        fb = sum(fetch[name]) / len(fetch[name]) * fetch_scale
        wb = sum(write[name]) / len(write[name]) * write_scale
        ns = sum(dur[name]) / len(dur[name]) if name in dur else None
        alg = bpp.get(kind, 0) * n ** 3 if kind in bpp else None
        rows.append((name, kind, ns, fb, wb, alg))
        if kind not in kinds or (ns or 0) > (kinds[kind]["avg_launch_ns"] or 0):
            kinds[kind] = {"bytes_per_launch": int(fb + wb), "fetch_bytes": int(fb), "write_bytes": int(wb),
                           "avg_launch_ns": ns, "dispatches": len(fetch[name])}
    out = {"n": n, "precision": prec, "kernel_source_sha256": kernel_source_digest(), "fetch_scale": fetch_scale,
           "write_scale": write_scale, "copy_reference_GBs": copy_GBs, "kernels": kinds}
    # the benchmark line reads the counters of its own workload (512^3 FP64) only
    headline = n == 512 and prec == "fp64"
    if headline:
        with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as f:
            json.dump(out, f, indent=1)
    sq = summarize_sq(d, n, dur)
    lines = [f"# {title}", "", "Commands (each in its own run, from /tmp, `TMPDIR=/tmp`):", "", "```"]
    lines += meta.get("commands", []) + ["```", ""]
    lines.append(f"Calibration: each run first copies {copy_bytes / 1e9:.2f} GB with the library's streaming copy "
                 f"(`k_stream_copy`); FETCH_SIZE reads {1 / fetch_scale:.3f} and WRITE_SIZE {1 / write_scale:.3f} "
                 f"of the copied bytes, so the table scales them by {fetch_scale:.3f} and {write_scale:.3f}. "
                 + (f"The copy ran at {copy_GBs:.0f} GB/s (read + write) in the kernel trace." if copy_GBs else ""))
    lines += ["", "| kernel | avg ms | fetch GB | write GB | achieved TB/s | of 8 TB/s peak | of streaming copy | "
                  "algorithmic GB | algorithmic / measured bytes |", "|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for name, kind, ns, fb, wb, alg in rows:
        if ns is None:
            continue
        tbs = (fb + wb) / ns / 1e3
        short = name.split("(")[0].replace("void ", "").replace("cns::", "")
        lines.append(f"| `{short}` | {ns / 1e6:.3f} | {fb / 1e9:.2f} | {wb / 1e9:.2f} | {tbs:.2f} | "
                     f"{tbs * 1e3 / PEAK_HBM_GBS:.2f} | " + (f"{tbs * 1e3 / copy_GBs:.2f}" if copy_GBs else "-") +
                     " | " + (f"{alg / 1e9:.2f} | {alg / (fb + wb):.2f} |" if alg else "- | - |"))
    traced_only = sorted(set(dur) - set(fetch), key=lambda k: -sum(dur[k]))
    if traced_only:
        # launched by the multi-step kernel trace only (the counter runs take one step)
        lines += ["", "In the kernel trace only (the counter runs take one step): " + "; ".join(
            f"`{k.split('(')[0].replace('void ', '').replace('cns::', '')}` {len(dur[k])} launches, "
            f"{sum(dur[k]) / len(dur[k]) / 1e6:.3f} ms average" for k in traced_only) + "."]
    lines += ["", "Algorithmic bytes: every array element a kernel must read or write, once (the z sweep with "
                  "the fused update averaged over the four RK4 stages).  Kernel times: the kernel trace of the first "
                  "command."]
    if sq:
        lines += ["", "Shader counters (rocprofv3 `--pmc`, one pass per line of the commands above that names SQ_ "
                      "counters; per dispatch, averaged over the dispatches of the kernel): VALU instructions per "
                      "grid point (SQ_INSTS_VALU x 64 lanes / points), the VALU issue fraction (those lane-"
                      "instructions over the kernel time at 256 CU x 4 SIMD x 16 lanes x 2.4 GHz), and the share of "
                      "wave cycles spent waiting (SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES) and issuing VALU work "
                      "(SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES).", "",
                  "| kernel | VALU instr / point | VALU issue frac | wait / wave cycles | VALU active / wave cycles | "
                  "LDS bank conflicts / LDS instr | other counters |", "|---|---:|---:|---:|---:|---:|---|"]
        for kind, c in sq.items():
            def g(k):
                return c.get(k)
            valu_pt = g("SQ_INSTS_VALU") * 64 / n ** 3 if g("SQ_INSTS_VALU") else None
            ns = c.get("_avg_ns")
            issue = valu_pt * n ** 3 / (ns * 1e-9) / PEAK_VALU_LANE_INSTR if valu_pt and ns else None
            wait = g("SQ_WAIT_INST_ANY") / g("SQ_WAVE_CYCLES") if g("SQ_WAIT_INST_ANY") and g("SQ_WAVE_CYCLES") else None
            act = g("SQ_ACTIVE_INST_VALU") / g("SQ_WAVE_CYCLES") if g("SQ_ACTIVE_INST_VALU") and g("SQ_WAVE_CYCLES") \
                else None
            bank = g("SQ_LDS_BANK_CONFLICT") / g("SQ_INSTS_LDS") if g("SQ_LDS_BANK_CONFLICT") is not None and \
                g("SQ_INSTS_LDS") else None
            other = ", ".join(f"{k} {v:.3g}" for k, v in sorted(c.items()) if not k.startswith("_") and k not in
                              ("SQ_INSTS_VALU", "SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES", "SQ_ACTIVE_INST_VALU",
                               "SQ_LDS_BANK_CONFLICT", "SQ_INSTS_LDS"))

            def fmt(x, f):
                return f.format(x) if x is not None else "-"
            lines.append(f"| {kind} | {fmt(valu_pt, '{:.0f}')} | {fmt(issue, '{:.2f}')} | {fmt(wait, '{:.2f}')} | "
                         f"{fmt(act, '{:.2f}')} | {fmt(bank, '{:.3f}')} | {other} |")
        if headline:
            with open(os.path.join(ROOT, "profiles", "valu.json"), "w") as f:
                json.dump({"n": n, "precision": prec, "kernel_source_sha256": kernel_source_digest(),
                           "kernels": {k: {"valu_per_point": c["SQ_INSTS_VALU"] * 64 / n ** 3} for k, c in sq.items()
                                       if c.get("SQ_INSTS_VALU")}}, f, indent=1)
    print("\n".join(lines))


def summarize_sq(d, n, dur):
    """Mean per-dispatch shader counters per kernel kind from every d/sq*/ counter run."""
    sums, cnt = {}, {}
    for sub in sorted(os.listdir(d)):
        if not sub.startswith("sq"):
            continue
        for r in _csv_rows(os.path.join(d, sub), "counter_collection.csv"):
            kind = kernel_kind(r["Kernel_Name"])
            key = (kind, r["Counter_Name"])
            sums[key] = sums.get(key, 0.0) + float(r["Counter_Value"])
            cnt[key] = cnt.get(key, 0) + 1
    out = {}
    for (kind, cname), v in sums.items():
        out.setdefault(kind, {})[cname] = v / cnt[(kind, cname)]
    for name, ds in dur.items():
        kind = kernel_kind(name)
        if kind in out:
            out[kind]["_avg_ns"] = sum(ds) / len(ds)
    return out


if __name__ == "__main__":
    main()
