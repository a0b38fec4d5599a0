#!/usr/bin/env python3
"""Throughput of the SPV hot path on one MI355X: cell-steps/s.

A step is one full pass of the hot path through the C-ABI (forces and
update, geometry and empty-circumcircle test, device repair of failed rings)
on the synthetic spv_n100k workload: N = 100000 cells uniform-random in a
periodic box of side sqrt(N), p0 = 3.9, v0 = 0.1, Dr = 1, mu = 1, dt = 0.01,
FP64.  `value` = N * steps / wall seconds of the timed steps, inputs resident
in HBM.  The JSON line also carries the roofline of the dominant kernel
(algorithmic bytes per launch / average launch time from HIP events on the
library's stream) and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6  # MI355X dense FP64 vector

# Algorithmic HBM bytes per cell per launch (FP64, mean ring length 6;
# neighbour gathers served by cache).
BYTES_PER_CELL = {
    # force+update: read x,y,theta (24), deg (1), ring (24), opp (24), own a,b (16), tag (4);
    # write x,y,theta (24)
    "force_update": 24 + 1 + 24 + 24 + 16 + 4 + 24,
    # geometry+test: read x,y (16), deg (1), ring (24), opp (24), A0,P0 (16);
    # write A,P,a,b (32)
    "geometry_test": 16 + 1 + 24 + 24 + 16 + 32,
}


# HBM bytes per launch of the force kernel, per workload and kernel layout
# (force_mode 1: lanes per cell, 2: per item), from the rocprofv3
# FETCH_SIZE / WRITE_SIZE runs (calibrated against a plain copy; the
# summaries are in profiles/), valid only for the force kernels' source as it
# was then: the digest covers the shared device header and the kernel file up
# to the geometry section (constants, helpers, the force kernels).
MEASURED_TRAFFIC = {
    ("spv_n100k", "force_update", 1): {"bytes": 20.69e6,
                                    "source_sha256": "420f9cb40282218c4c831cc4fd68e0cb6d7ccdbda9839b03ae7e4caf14a73af1"},
    ("spv_n1m", "force_update", 2): {"bytes": 200.52e6,
                                  "source_sha256": "420f9cb40282218c4c831cc4fd68e0cb6d7ccdbda9839b03ae7e4caf14a73af1"},
}

# FP64 FLOPs per launch of the force kernel, per workload and kernel layout,
# from the rocprofv3 SQ_INSTS_VALU_{FMA,ADD,MUL}_F64 counters
# ((2 FMA + ADD + MUL) x 64 lanes; profiles/), valid for the same source
# digest as the traffic.
MEASURED_FP64_FLOPS = {
    ("spv_n100k", "force_update", 1): {"flops": 221.9e6,
                                    "source_sha256": "420f9cb40282218c4c831cc4fd68e0cb6d7ccdbda9839b03ae7e4caf14a73af1"},
    ("spv_n1m", "force_update", 2): {"flops": 2061.8e6,
                                  "source_sha256": "420f9cb40282218c4c831cc4fd68e0cb6d7ccdbda9839b03ae7e4caf14a73af1"},
}


def force_source_digest():
    import hashlib
    csrc = os.path.join(ROOT, "paper_1702_02939_amd", "csrc")
    h = hashlib.sha256()
    h.update(open(os.path.join(csrc, "spv_common.hpp"), "rb").read())
    k = open(os.path.join(csrc, "spv_kernels.hpp"), "rb").read()
    h.update(k[:k.index(b"// ---------------------------------------------------------------- geometry + validity test")])
    return h.hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--workload", default="spv_n100k")
    ap.add_argument("--cpu-sample-steps", type=int, default=80)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--headline-only", action="store_true", help="skip the mixed / batched / 1e6 runs")
    ap.add_argument("--no-timing", action="store_true", help="skip the kernel-timing pass")
    ap.add_argument("--timing-steps", type=int, default=2000)
    ap.add_argument("--no-autotune", action="store_true",
                    help="run with the default scheduling knobs instead of the library's tuned ones")
    ap.add_argument("--batch-steps", type=int, default=5000)
    ap.add_argument("--big-steps", type=int, default=2000)
    ap.add_argument("--sweep-steps", type=int, default=2000)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MiB",
                    help="first run one device-to-device copy of this many MiB (HBM counter calibration)")
    return ap.parse_args()


def cpu_baseline(w, nsteps):
    """The oracle (serial C: full Bowyer-Watson each step, dual-number forces)
    on the same workload, a bounded number of steps from the same start."""
    import numpy as np

    import oracle
    from paper_1702_02939_amd import inputs
    n, L = w["N"], w["L"]
    x, y = inputs.uniform_positions(n, L, L, w["seed"])
    xq, yq, Lx, Ly, q = oracle.prepare(x, y, L, L)
    th = oracle.theta0(w["seed"], n)
    t0 = time.perf_counter()
    oracle.run(xq, yq, th, Lx, Ly, q, 1.0, w["p0"], mu=w["mu"], v0=w["v0"], Dr=w["Dr"], dt=w["dt"],
               seed=w["seed"], nsteps=nsteps)
    dt = time.perf_counter() - t0
    # run() also triangulates the final state once: nsteps + 1 triangulations
    return {"value": n * nsteps / dt, "unit": "cell-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{w['N']} cells, {nsteps} steps from the random start (serial, 1 thread), {dt:.1f} s"}


def timed_run(spv, make, steps, warmup, timing=True):
    """Create via make() (outside the timed region: this includes the
    autotuner's trials when it has no cached choice), warm up, time `steps`
    steps; returns a dict."""
    import torch
    sysm, ncells = make()
    tuning = sysm.tuning()
    sysm.step(warmup)
    _, _, _, c0 = sysm.observables()
    if timing:
        spv.spv_set_timing(sysm.h, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    half = steps // 2
    sysm.step(steps - half)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sysm.step(half)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    second = time.perf_counter() - t1
    E, qbar, sumA, c1 = sysm.observables()
    kt = {name: spv.spv_kernel_time(sysm.h, k) for name, k in
          (("force_update", spv.K_FORCE), ("geometry_test", spv.K_GEOM), ("repair", spv.K_REPAIR))}
    sysm.close()
    return {"value": ncells * steps / wall, "ms_per_step": wall * 1e3 / steps, "cells": ncells, "steps": steps,
            "steady_value": ncells * half / second if half else None,
            "kernels": kt, "repairs_per_step": float(c1[1] - c0[1]) / steps,
            "rounds_per_step": float(c1[2] - c0[2]) / steps, "E": E, "qbar": qbar, "sumA": sumA,
            "path": {"graph_periods": int(c1[8] - c0[8]), "dense_steps": int(c1[9] - c0[9]),
                     "host_rounds": int(c1[10] - c0[10]), "host_recovered_steps": int(c1[11] - c0[11]),
                     "resorts": int(c1[5] - c0[5])},
            "tuning": tuning}


AUTOTUNE = 1


def single(spv, inputs, name, precision, p0=None, **knobs):
    w = inputs.WORKLOADS[name]

    def make():
        x, y = inputs.uniform_positions(w["N"], w["L"], w["L"], w["seed"])
        prm = spv.Params(mu=w["mu"], v0=w["v0"], Dr=w["Dr"], dt=w["dt"], seed=w["seed"], precision=precision,
                         autotune=0 if knobs else AUTOTUNE, **knobs)
        return spv.System(x, y, w["L"], w["L"], p0=w["p0"] if p0 is None else p0, params=prm), w["N"]
    return make


def sweeps(spv, inputs, steps, warmup):
    """The paper's solid-to-fluid sweep (target shape index 3.8 / 3.9 / 4.0
    at v0 = 0.1, N = 1e5, FP64) and the re-sort interval ablation (Hilbert
    order; 10 / 32 / 100 / 1000 steps between re-sorts, and row-major bins at
    32) on spv_n100k."""
    out = {"p0_sweep": {}, "resort_ablation": {}}
    for p0 in (3.8, 3.9, 4.0):
        r = timed_run(spv, single(spv, inputs, "spv_n100k", spv.SPV_FP64, p0=p0), steps, warmup, timing=False)
        out["p0_sweep"][str(p0)] = {"value": r["value"], "ms_per_step": r["ms_per_step"],
                                    "repairs_per_step": r["repairs_per_step"]}
    for every in (10, 32, 100, 1000):
        r = timed_run(spv, single(spv, inputs, "spv_n100k", spv.SPV_FP64, resort_every=every), steps, warmup,
                      timing=False)
        out["resort_ablation"][str(every)] = {"value": r["value"], "ms_per_step": r["ms_per_step"]}
    r = timed_run(spv, single(spv, inputs, "spv_n100k", spv.SPV_FP64, resort_every=32, bin_order=1), steps,
                  warmup, timing=False)
    out["resort_ablation"]["32_row_major_bins"] = {"value": r["value"], "ms_per_step": r["ms_per_step"]}
    return out


def batched(spv, inputs, precision):
    def make():
        systems = inputs.batch_systems()
        N_s = [s_["N"] for s_ in systems]
        L_s = [s_["L"] for s_ in systems]
        x = __import__("numpy").concatenate([s_["x"] for s_ in systems])
        y = __import__("numpy").concatenate([s_["y"] for s_ in systems])
        prm = spv.Params(mu=1.0, Dr=1.0, dt=0.01, precision=precision, autotune=AUTOTUNE)
        sysm = spv.System.batch(N_s, L_s, x, y, [s_["p0"] for s_ in systems], v0_s=[s_["v0"] for s_ in systems],
                                seed_s=[s_["seed"] for s_ in systems], params=prm)
        return sysm, sum(N_s)
    return make


def adjoint_cost(spv, inputs):
    """spv_n4096_adjoint workload: gradient of the time-averaged mean shape
    index over T steps (checkpoint every k) w.r.t. per-cell p0; cost of
    forward+backward relative to the plain FP64 forward of the same T steps."""
    import numpy as np
    import torch
    w = inputs.WORKLOADS["spv_n4096_adjoint"]
    n, L, T, k = w["N"], w["L"], w["steps"], w["ckpt"]
    x, y = inputs.uniform_positions(n, L, L, w["seed"])
    p0 = inputs.per_cell_p0(n, w["p0"], w["p0_sigma"], w["seed"])
    prm = spv.Params(mu=w["mu"], v0=w["v0"], Dr=w["Dr"], dt=w["dt"], seed=w["seed"])

    def fresh():
        s = spv.System(x, y, L, L, P0=p0, params=prm)
        s.step(200)  # leave the random-start transient
        return s
    s = fresh()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(T)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    s.close()
    s = fresh()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Q = s.traj_forward(T, k)
    t1 = time.perf_counter()
    g = s.traj_backward(1.0)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    s.close()
    return {"cells": n, "steps": T, "ckpt_every": k, "Q": Q, "grad_norm": float(np.linalg.norm(g)),
            "plain_forward_ms": t_plain * 1e3, "traj_forward_ms": (t1 - t0) * 1e3,
            "traj_backward_ms": (t2 - t1) * 1e3, "adjoint_over_forward": (t2 - t0) / t_plain}


def alu_roofline(workload, dom, mode, avg_s):
    """The same kernel against the FP64 vector peak, from its counted FP64
    operations (None when there are no counters for this workload or they
    predate the kernel's source)."""
    mf = MEASURED_FP64_FLOPS.get((workload, dom, mode))
    if not mf or mf["source_sha256"] != force_source_digest() or avg_s <= 0:
        return None
    tf = mf["flops"] / avg_s / 1e12
    return {"achieved": tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tf / FP64_PEAK_TFLOPS,
            "flops_per_launch": mf["flops"]}


def roofline_of(kt, ncells):
    dom = max(("force_update", "geometry_test"), key=lambda k: kt[k][0])
    ms, launches = kt[dom]
    avg_s = ms / 1e3 / max(launches, 1)
    bytes_per_launch = BYTES_PER_CELL[dom] * ncells
    achieved = bytes_per_launch / avg_s / 1e9 if avg_s > 0 else 0.0
    return dom, avg_s, bytes_per_launch, achieved


def main():
    global AUTOTUNE
    args = parse()
    AUTOTUNE = 0 if args.no_autotune else 1
    if args.gpus != 1:
        print(json.dumps({"error": "the SPV step runs on one GPU; sharding across GPUs is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    from paper_1702_02939_amd import inputs, spv

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        nel = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = inputs.WORKLOADS[args.workload]
    # timed region 1: throughput (steps replayed as captured graphs, no events)
    head = timed_run(spv, single(spv, inputs, args.workload, spv.SPV_FP64), args.steps, args.warmup, timing=False)
    n = head["cells"]
    # timed region 2: kernel durations from HIP events around every launch
    # (timing mode launches each step's kernels one by one on the same stream)
    kt = {k: (0.0, 0) for k in ("force_update", "geometry_test", "repair")}
    if not args.no_timing:
        kt = timed_run(spv, single(spv, inputs, args.workload, spv.SPV_FP64), args.timing_steps, args.warmup,
                       timing=True)["kernels"]
    dom, avg_s, bytes_per_launch, achieved = roofline_of(kt, n)
    mode = head["tuning"].get("force_mode")
    mt = MEASURED_TRAFFIC.get((args.workload, dom, mode))
    traffic = mt["bytes"] if mt and mt["source_sha256"] == force_source_digest() else None
    out = {
        "metric": "cell-steps/s",
        "value": head["value"],
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "N": n, "L": w["L"], "p0": w["p0"], "v0": w["v0"], "Dr": w["Dr"],
                   "mu": w["mu"], "dt": w["dt"], "precision": "fp64", "tuning": head["tuning"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": dom,
                     "bytes_per_launch": bytes_per_launch, "avg_launch_us": avg_s * 1e6},
        "roofline_fp64_alu": alu_roofline(args.workload, dom, mode, avg_s),
        "kernels_ms_total": {k: v[0] for k, v in kt.items()},
        "kernel_launches": {k: v[1] for k, v in kt.items()},
        "steady_state_value": head["steady_value"],
        "repairs_per_step": head["repairs_per_step"],
        "repair_rounds_per_step": head["rounds_per_step"],
        "path": head["path"],
        "observables": {"E": head["E"], "qbar": head["qbar"], "sumA": head["sumA"]},
    }
    if not args.headline_only:
        extra = {}
        runs = [
            ("spv_n100k_mixed", single(spv, inputs, "spv_n100k", spv.SPV_MIXED), args.steps, args.warmup),
            ("batched_sweep_256_mixed", batched(spv, inputs, spv.SPV_MIXED), args.batch_steps, 200),
            ("batched_sweep_256_fp64", batched(spv, inputs, spv.SPV_FP64), args.batch_steps, 200),
            ("spv_n1m_fp64", single(spv, inputs, "spv_n1m", spv.SPV_FP64), args.big_steps, 100),
            ("spv_n1m_mixed", single(spv, inputs, "spv_n1m", spv.SPV_MIXED), args.big_steps, 100),
        ]
        for name, make, steps, warm in runs:
            r = timed_run(spv, make, steps, warm, timing=False)
            r["kernels"] = timed_run(spv, make, max(steps // 10, 50), warm, timing=True)["kernels"]
            d, a_s, bpl, ach = roofline_of(r["kernels"], r["cells"])
            extra[name] = {"value": r["value"], "unit": "cell-steps/s", "ms_per_step": r["ms_per_step"],
                           "cells": r["cells"], "steps": steps, "warmup": warm,
                           "repairs_per_step": r["repairs_per_step"], "tuning": r["tuning"], "path": r["path"],
                           "kernel_avg_us": {k: (v[0] * 1e3 / max(v[1], 1)) for k, v in r["kernels"].items()},
                           "roofline_frac_hbm": ach / HBM_PEAK_GBS, "dominant_kernel": d}
            print(f"[bench] {name}: {r['value']:.3e} cell-steps/s", file=sys.stderr, flush=True)
        extra["mixed_vs_fp64_speedup_n100k"] = extra["spv_n100k_mixed"]["value"] / head["value"]
        extra["adjoint_n4096"] = adjoint_cost(spv, inputs)
        extra.update(sweeps(spv, inputs, args.sweep_steps, args.warmup))
        print(f"[bench] adjoint/forward: {extra['adjoint_n4096']['adjoint_over_forward']:.2f}", file=sys.stderr,
              flush=True)
        out["extra"] = extra
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_sample_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
