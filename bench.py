#!/usr/bin/env python3
"""Throughput of the FP64 WENO5-Roe / central-viscous RK4 path on one MI355X.

Workload: 128^3 triply periodic decaying turbulence (seeded synthetic IC with the
HIT spectrum, Mt = 0.3, Re = 400, gamma = 1.4, Pr = 0.72), classical RK4 at
CFL 0.5 with kinetic energy and enstrophy reduced after every step.  One "step"
is one RK4 step = 4 right-hand-side evaluations of the whole grid.

Metric: grid-point RHS evaluations per second (4 * N^3 per step), with the
state resident in HBM before the timed region starts.

Prints one JSON line.  The roofline object describes the kernel with the
largest share of the step, timed with HIP events on the plan's stream; the
cpu_baseline object times the CPU oracle on a bounded sample of the same
workload on the host's cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
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
PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector (256 CU x 64 lanes x 2 x 2.4 GHz)
PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector (published; its 2x over FP64 needs packed FP32)
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E
PEAK_VALU_LANE_INSTR = 256 * 4 * 16 * 2.4e9  # VALU lane-instructions per second (3.93e13)


def kernel_source_digest():
    """SHA-256 of the sources the sweep kernels are built from (counters taken on other
    sources are stale)."""
    import hashlib

    h = hashlib.sha256()
    for f in ("cns_kernels.hip", "cns_device.h"):
        h.update(open(os.path.join(ROOT, "paper_2211_16718_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=128, help="grid points per direction (128 = the named workload)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="fp64 (the named workload) or the mixed form, for profiling it alone")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=2, help="RK4 steps of the oracle sample")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the mixed-precision 512^3, ensemble and adjoint measurements")
    ap.add_argument("--extras", default="mixed_512,ensemble_64,adjoint_128,options_128",
                    help="comma-separated subset of the extra measurements to run")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="before the workload, copy a buffer of this many MiB device-to-device once "
                         "(a known-size reference for hardware byte counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "domain decomposition is not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2211_16718_amd import inputs as I
    from paper_2211_16718_amd.api import Plan

    if args.calibrate_copy_mib > 0:
        nb = args.calibrate_copy_mib << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    n = args.n
    wl = I.WORKLOADS["hit128"]
    mu = 1.0 / wl.re
    rho, vel, p = I.hit_primitives(n, wl.seed, wl.mt)
    fp64 = args.precision == "fp64"
    plan = Plan((n, n, n), mu_eff=mu, precision=args.precision, device="cuda:0")
    u = plan.init_state(rho, vel, p)
    smax = plan.diagnostics_host(u)[7]
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
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tfile):
        try:
            t = json.load(open(tfile))
            if fp64 and t.get("kernel_source_sha256") == kernel_source_digest() and dom in t.get("kernels", {}) \
                    and t.get("n") == n:
                traffic = t["kernels"][dom]["bytes_per_launch"]
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
    bpp = (BYTES_PER_POINT if fp64 else BYTES_PER_POINT_MIXED)[dom]
    roofline = {
        "bound": "alu",
        "kernel": dom,
        "achieved": round(achieved, 3),
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": round(achieved / peak, 4),
        "traffic": traffic,
        "algorithmic_bytes_per_launch": bpp * n ** 3,
        "hbm_frac_algorithmic": round(bpp * n ** 3 / avg_s / 1e9 / PEAK_HBM_GBS, 4),
        "flops_per_point": FLOPS_PER_POINT[dom],
        "avg_launch_ms": round(kernels[dom]["avg_ms"], 5),
    }
    if valu:
        roofline.update(valu)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        ph = oracle.make_phys(mu_eff=mu)
        uh = oracle.init_state(rho, vel, p)
        oracle.rhs(np.ascontiguousarray(uh[:, :8, :8, :8]), ph)  # load the library
        t0 = time.perf_counter()
        oracle.rk4(uh, dt, args.cpu_steps, ph)
        ct = time.perf_counter() - t0
        cpu = {"value": 4.0 * n ** 3 * args.cpu_steps / ct, "unit": "point-RHS/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"{args.cpu_steps} RK4 steps (with diagnostics) of the same {n}^3 workload, "
                         f"{ct:.1f} s, OpenMP over grid points"}
        cpu["host"] = _host_cpu()
        cpu["configs"] = _oracle_configs()
        cpu1 = _oracle_one_core(n, mu)
        if cpu1:
            cpu["one_core"] = cpu1
            cpu["one_core"]["gpu_over_one_core"] = value / cpu1["value"]

    extras = {}
    if not args.no_extras:
        del plan
        torch.cuda.empty_cache()
        wanted = set(args.extras.split(","))
        for name, fn in (("mixed_512", bench_mixed), ("ensemble_64", bench_ensemble), ("adjoint_128", bench_adjoint),
                         ("options_128", bench_options)):
            if name not in wanted:
                continue
            try:
                extras[name] = fn()
            except Exception as e:  # report, keep the main line
                extras[name] = {"error": f"{type(e).__name__}: {e}"}
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
        "config": {"workload": f"hit{n}_re400_rk4_diag_every_step" + ("" if fp64 else "_mixed"), "grid": [n, n, n],
                   "re": wl.re, "mt": wl.mt, "cfl": I.CFL, "dt": dt, "precision": args.precision},
        "roofline": roofline,
        "kernels": {k: {"avg_ms": round(v["avg_ms"], 5), "launches": v["launches"], "share": round(v["share"], 4)}
                    for k, v in kernels.items()},
        "cpu_baseline": cpu,
    }
    out.update(extras)
    print(json.dumps(out), flush=True)


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
    """The host CPU the oracle ran on: model name, logical CPUs, sockets, OMP_NUM_THREADS."""
    model, sockets = None, set()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k = k.strip()
                if k == "model name" and model is None:
                    model = v.strip()
                elif k == "physical id":
                    sockets.add(v.strip())
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count(), "sockets": len(sockets) or None,
            "usable_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def _oracle_one_core(n, mu):
    """The oracle's RHS on one host thread (the paper's GPU-vs-one-core comparison), in a
    child process started with OMP_NUM_THREADS=1: one RHS evaluation of the same input."""
    import subprocess

    code = (
        "import json, sys, time\n"
        f"sys.path.insert(0, {ROOT!r})\n"
        "import numpy as np\n"
        "import oracle\n"
        "from paper_2211_16718_amd import inputs as I\n"
        f"n, mu = {n}, {mu!r}\n"
        "wl = I.WORKLOADS['hit128']\n"
        "rho, vel, p = I.hit_primitives(n, wl.seed, wl.mt)\n"
        "ph = oracle.make_phys(mu_eff=mu)\n"
        "uh = oracle.init_state(rho, vel, p)\n"
        "oracle.rhs(np.ascontiguousarray(uh[:, :8, :8, :8]), ph)\n"
        "t0 = time.perf_counter()\n"
        "oracle.rhs(uh, ph)\n"
        "ct = time.perf_counter() - t0\n"
        "print(json.dumps({'value': n ** 3 / ct, 'seconds': ct, 'cores': oracle.num_threads()}))\n"
    )
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
        d = json.loads(r.stdout.strip().splitlines()[-1])
    except Exception:
        return None
    return {"value": d["value"], "unit": "point-RHS/s", "cores": d["cores"], "kind": "oracle",
            "sample": f"one RHS evaluation of the same {n}^3 state, {d['seconds']:.1f} s"}


def bench_mixed(n=512, steps=20):
    """512^3, Re = 1600: mixed precision against the FP64 path at the same size."""
    import numpy as np
    import torch

    from paper_2211_16718_amd import inputs as I
    from paper_2211_16718_amd.api import Plan

    wl = I.WORKLOADS["hit512"]
    rho, vel, p = I.hit_primitives(n, wl.seed, wl.mt)
    out = {"config": {"workload": f"hit{n}_re1600_rk4x{steps}", "grid": [n, n, n], "steps": steps}}
    res = {}
    for prec in ("fp64", "mixed"):
        plan = Plan((n, n, n), mu_eff=1.0 / wl.re, precision=prec)
        u = plan.init_state(rho, vel, p)
        if prec == "fp64":
            dt = I.dt_from_speed(plan.diagnostics_host(u)[7], n)
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
    return {"config": {"workload": f"ensemble{nbox}_rk4x{steps}", "boxes": nbox, "points": pts,
                       "sizes": sorted({b["shape"][0] for b in boxes})},
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

    gsec, (J, g) = _timed(plan.stream, grad)
    out = {"config": {"workload": f"hit{n}_re400_rk4x{steps}_adjoint", "ckpt_every": ckpt},
           "forward_s": fsec, "gradient_s": gsec, "gradient_over_forward": gsec / fsec,
           "value": 4.0 * n ** 3 * steps / gsec, "unit": "point-RHS/s (forward-step equivalents of the gradient)",
           "J": float(J.detach()), "grad_norm": float(g.norm())}
    # the same gradient through the TVD-RK3 integrator (checkpoints every ckpt steps)
    plan.tvdrk3(plan.init_state(rho, vel, p), dt, 1, diag=False)
    u3 = plan.init_state(rho, vel, p)
    f3, _ = _timed(plan.stream, lambda: plan.tvdrk3(u3, dt, steps, diag=False))

    def grad3():
        v0 = vel.clone().requires_grad_(True)
        J = FinalKineticEnergy.apply(v0, rho, p, plan, dt, steps, ckpt, "tvdrk3")
        J.backward()
        return J, v0.grad

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

        gsec1, (J1, g1) = _timed(plan.stream, grad1)
        out["one_segment"] = {"ckpt_every": steps, "workspace_GB": need / 1e9, "gradient_s": gsec1,
                              "gradient_over_forward": gsec1 / fsec,
                              "max_abs_diff_vs_ckpt": float((g1 - g20).abs().max())}
        plan._adj_buf = None
        torch.cuda.empty_cache()
    return out


def bench_options(n=128, steps=20):
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
    r5, v5, p5 = I.hit_primitives(m, 0, 0.3)
    p512 = Plan((m, m, m), mu_eff=1.0 / 1600)
    u5 = p512.init_state(r5, v5, p5)
    p512.spectrum(u5)
    sec, (E, mom) = _timed(p512.stream, lambda: p512.spectrum(u5))
    out["spectrum_512"] = {"ms": sec * 1e3, "taylor_microscale": Plan.taylor_microscale(mom)}
    return out


if __name__ == "__main__":
    main()
