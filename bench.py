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

# Algorithmic HBM bytes (FP64, mean ring length 6; neighbour gathers served
# by cache) per kernel class over a timed window, from the cell count, the
# steps and launches, and the repair counters of the window:
#   force_update   per cell and launch: read x,y,theta (24), deg (1), ring (24),
#                  opp (24), own a,b (16), tag (4); write x,y,theta (24) = 117
#   geometry_test  per cell and launch: read x,y (16), deg (1), ring (24),
#                  opp (24), A0,P0 (16); write A,P,a,b (32) = 113
#   repair         per candidate gathered: its x,y (16) and index (4) = 20;
#                  per repaired cell: old ring row (64), new ring (24), deg (1) = 89
#   cell_list      the scan of the step's bin counts: per bin the count read,
#                  the start written, the count cleared = 12 (the per-cell
#                  part -- bin, slot and count update in the force kernel's
#                  update, the placement in the all-cells pass -- is in those
#                  kernels' time)
#   resort         per cell: every per-cell array read and written once
#                  (x,y,theta 24, tag,sys 8, A0,P0 16, A,P,a,b 32, deg 1,
#                  ring,opp 48, each way) plus ring and opp renumbering reads
#                  (48), key, permutation and inverse (16) = 322
# The other classes (re-tests, tail, flag compaction, host rounds) are timed
# but carry no byte model.
FORCE_B, GEOM_B = 117, 113
CAND_B, REPAIRED_B = 20, 89
LIST_CELL_B, LIST_BIN_B = 0, 12
RESORT_B = 322
STEP_B = 244  # algorithmic bytes of a whole step per cell (three streaming passes)
LIST_LAUNCHES, RESORT_LAUNCHES = 2, 9  # launches of one cell list (its scan) / one re-sort


def class_bytes(cls, r):
    """Algorithmic bytes of kernel class cls over the timed window of run r
    (None without a model)."""
    n, steps, launches = r["cells"], r["steps"], r["kernels"][cls][1]
    if cls == "force_update":
        return FORCE_B * n * launches
    if cls == "geometry_test":
        return GEOM_B * n * launches
    if cls == "repair":
        return CAND_B * r["candidates"] + REPAIRED_B * r["repaired"]
    if cls == "cell_list":
        return (LIST_CELL_B * n + LIST_BIN_B * r["bins"]) * (launches // LIST_LAUNCHES)
    if cls == "resort":
        return RESORT_B * n * (launches // RESORT_LAUNCHES)
    return None


# Measured HBM bytes per launch (rocprofv3 FETCH_SIZE and WRITE_SIZE,
# calibrated against a plain device copy; the summaries are in profiles/) per
# (workload, kernel class, force-kernel layout), valid only for the kernel
# source they were taken on (digest of the device headers): any later change
# of the kernels nulls roofline.traffic.
MEASURED_TRAFFIC = {
    ("spv_n100k", "repair", 1): {"bytes_per_launch": 18.297e6, "source_sha256":
                                 "a382cd4b05eb0d17b4c7e5b523e9e01f630b53fbc037442ef4dd1831fbe7495a"},
    ("spv_n100k", "force_update", 1): {"bytes_per_launch": 17.324e6, "source_sha256":
                                       "a382cd4b05eb0d17b4c7e5b523e9e01f630b53fbc037442ef4dd1831fbe7495a"},
    ("spv_n100k", "geometry_test", 1): {"bytes_per_launch": 15.310e6, "source_sha256":
                                        "a382cd4b05eb0d17b4c7e5b523e9e01f630b53fbc037442ef4dd1831fbe7495a"},
}


def source_digest():
    import hashlib
    csrc = os.path.join(ROOT, "paper_1702_02939_amd", "csrc")
    h = hashlib.sha256()
    for f in ("spv_common.hpp", "spv_exact.hpp", "spv_kernels.hpp"):
        h.update(open(os.path.join(csrc, f), "rb").read())
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
    ap.add_argument("--no-autotune", action="store_true",
                    help="run with the default scheduling knobs instead of the library's tuned ones")
    ap.add_argument("--batch-steps", type=int, default=5000)
    ap.add_argument("--big-steps", type=int, default=2000)
    ap.add_argument("--sweep-steps", type=int, default=2000)
    ap.add_argument("--hybrid-steps", type=int, default=200)
    ap.add_argument("--ablation-steps", type=int, default=1000)
    ap.add_argument("--avm-steps", type=int, default=2000)
    ap.add_argument("--avm-cpu-steps", type=int, default=20)
    ap.add_argument("--avm-only", action="store_true", help="run only the active vertex model runs (profiling)")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64",
                    help="arithmetic of the headline runs (mixed: for profiling the FP32 geometry and forces)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MiB",
                    help="first run one device-to-device copy of this many MiB (HBM counter calibration)")
    return ap.parse_args()


def _oracle_sample(w, nsteps):
    """nsteps of the oracle on workload w from its random start; returns the
    seconds the steps took (setup excluded)."""
    import oracle
    from paper_1702_02939_amd import inputs
    n, L = w["N"], w["L"]
    x, y = inputs.uniform_positions(n, L, L, w["seed"])
    xq, yq, Lx, Ly, q = oracle.prepare(x, y, L, L)
    th = oracle.theta0(w["seed"], n)
    t0 = time.perf_counter()
    oracle.run(xq, yq, th, Lx, Ly, q, 1.0, w["p0"], mu=w["mu"], v0=w["v0"], Dr=w["Dr"], dt=w["dt"],
               seed=w["seed"], nsteps=nsteps)
    return time.perf_counter() - t0


def _oracle_copies(w, nsteps, procs):
    """The same oracle sample in `procs` independent processes at once (fresh
    interpreters that load only the oracle): the host's aggregate rate on
    independent systems.  Returns (cell-steps/s over the slowest copy, its
    seconds)."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    with ctx.Pool(procs) as pool:
        times = pool.starmap(_oracle_sample, [(w, nsteps)] * procs)
    slow = max(times)
    return procs * w["N"] * nsteps / slow, slow


def cpu_baseline(w, nsteps, copies_steps=None):
    """The oracle (serial C: full Bowyer-Watson each step, dual-number forces)
    on the same workload, a bounded number of steps from the same start; and
    the same sample run as independent copies, one per available core (up to
    16), for the host's aggregate rate."""
    n = w["N"]
    copies_steps = nsteps if copies_steps is None else copies_steps
    dt = _oracle_sample(w, nsteps)
    # run() also triangulates the final state once: nsteps + 1 triangulations
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    affinity = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    out = {"value": n * nsteps / dt, "unit": "cell-steps/s", "cores": 1, "kind": "oracle",
           "sample": f"{w['N']} cells, {nsteps} steps from the random start (serial, 1 thread), {dt:.1f} s",
           "host_cpu": cpu, "host_nproc": os.cpu_count(), "host_affinity": affinity}
    procs = max(1, min(16, affinity or 1))
    if copies_steps > 0 and procs > 1:
        v, slow = _oracle_copies(w, copies_steps, procs)
        out["independent_copies"] = {
            "value": v, "unit": "cell-steps/s", "processes": procs,
            "sample": f"{procs} copies of {w['N']} cells x {copies_steps} steps, one process each, "
                      f"slowest {slow:.1f} s"}
    return out


def count_bins(sysm, bin_factor):
    """Cell-list bins of a handle (the library's rule: per system,
    floor(L / (bin_factor * mean spacing)) per side)."""
    S, _ = sysm.size()
    nb = 0
    for k in range(S):
        Lx, Ly, _ = sysm.system_box(k)
        _, n = sysm.system_range(k)
        h = bin_factor * math.sqrt(Lx * Ly / n)
        nb += max(1, math.floor(Lx / h)) * max(1, math.floor(Ly / h))
    return nb


def timed_run(spv, make, steps, warmup, timing=True):
    """Create via make() (outside the timed region: this includes the
    autotuner's trials when it has no cached choice), warm up, time `steps`
    steps; returns a dict.  With timing, every kernel launch of the timed
    steps carries HIP events on the library's stream (the steps run as
    without timing, except that no captured graph replays)."""
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
    kt = {name: spv.spv_kernel_time(sysm.h, k) for name, k in spv.KERNEL_CLASSES.items()} if timing else None
    bins = count_bins(sysm, tuning["bin_factor"])
    sysm.close()
    return {"value": ncells * steps / wall, "ms_per_step": wall * 1e3 / steps, "cells": ncells, "steps": steps,
            "steady_value": ncells * half / second if half else None,
            "kernels": kt, "repairs_per_step": float(c1[1] - c0[1]) / steps,
            "repaired": int(c1[1] - c0[1]), "candidates": int(c1[12] - c0[12]), "bins": bins,
            "rounds_per_step": float(c1[2] - c0[2]) / steps, "E": E, "qbar": qbar, "sumA": sumA,
            "path": {"graph_periods": int(c1[8] - c0[8]), "dense_steps": int(c1[9] - c0[9]),
                     "host_rounds": int(c1[10] - c0[10]), "host_recovered_steps": int(c1[11] - c0[11]),
                     "resorts": int(c1[5] - c0[5])},
            "tuning": tuning}


def kernel_table(r):
    """Per kernel class over the timed window: total ms, launches, ms per
    step, and (with a byte model) algorithmic GB/s and its HBM fraction."""
    out = {}
    for cls, (ms, launches) in r["kernels"].items():
        if launches == 0:
            continue
        e = {"ms": ms, "launches": launches, "ms_per_step": ms / r["steps"], "avg_launch_us": ms * 1e3 / launches}
        b = class_bytes(cls, r)
        if b is not None and ms > 0:
            e["bytes"] = b
            e["GBs"] = b / (ms * 1e-3) / 1e9
            e["hbm_frac"] = e["GBs"] / HBM_PEAK_GBS
        out[cls] = e
    return out


def roofline(r, workload, mode):
    """The roofline object for the dominant kernel class (largest total time
    in the timed window): achieved = algorithmic bytes / kernel time."""
    table = kernel_table(r)
    dom = max(table, key=lambda k: table[k]["ms"])
    e = table[dom]
    achieved = e.get("GBs")
    mt = MEASURED_TRAFFIC.get((workload, dom, mode))
    traffic = None
    if mt and mt["source_sha256"] == source_digest():
        traffic = mt["bytes_per_launch"]
    # the counter-measured bytes over the same live launch time (wasted
    # re-reads included), beside the algorithmic figure
    measured = traffic / (e["avg_launch_us"] * 1e-6) / 1e9 if traffic else None
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved is not None else None, "traffic": traffic,
            "measured_achieved": measured, "measured_frac": measured / HBM_PEAK_GBS if measured else None,
            "kernel": dom, "avg_launch_us": e["avg_launch_us"], "launches": e["launches"],
            "share_of_kernel_time": e["ms"] / sum(v["ms"] for v in table.values()),
            "bytes_per_launch": e["bytes"] / e["launches"] if "bytes" in e else None}, table


AUTOTUNE = 1


def single(spv, inputs, name, precision, p0=None, **knobs):
    w = inputs.WORKLOADS[name]

    def make():
        x, y = inputs.uniform_positions(w["N"], w["L"], w["L"], w["seed"])
        prm = spv.Params(mu=w["mu"], v0=w["v0"], Dr=w["Dr"], dt=w["dt"], seed=w["seed"], precision=precision,
                         autotune=0 if knobs else AUTOTUNE, **knobs)
        return spv.System(x, y, w["L"], w["L"], p0=w["p0"] if p0 is None else p0, params=prm), w["N"]
    return make


def sweeps(spv, inputs, steps, warmup, hybrid_steps, ablation_steps):
    """The paper's solid-to-fluid sweep (target shape index 3.8 / 3.9 / 4.0
    at v0 = 0.1, N = 1e5, FP64), the hybrid comparison mode at the same
    points, and the spatial-sort ablation at N = 1e6 (state beyond the 256 MB
    Infinity Cache)."""
    out = {"p0_sweep": {}, "hybrid": {}, "resort_ablation_n1m": {}}
    w = inputs.WORKLOADS["spv_n100k"]
    for p0 in (3.8, 3.9, 4.0):
        r = timed_run(spv, single(spv, inputs, "spv_n100k", spv.SPV_FP64, p0=p0), steps, warmup, timing=False)
        out["p0_sweep"][str(p0)] = {"value": r["value"], "ms_per_step": r["ms_per_step"],
                                    "repairs_per_step": r["repairs_per_step"], "path": r["path"]}
        # hybrid comparison mode (device test, host repair with the worklist
        # and positions copied to the host every step with failures) against
        # the device repair over the same steps: both from the state after
        # the warm-up (saved from a device handle, loaded into each)
        dev = single(spv, inputs, "spv_n100k", spv.SPV_FP64, p0=p0)()[0]
        dev.step(warmup)
        state = dev.save_state()
        dev.close()
        res = {}
        for mode in (0, 1):
            def make(p0=p0, state=state, mode=mode):
                x, y = inputs.uniform_positions(w["N"], w["L"], w["L"], w["seed"])
                prm = spv.Params(mu=w["mu"], v0=w["v0"], Dr=w["Dr"], dt=w["dt"], seed=w["seed"], repair_mode=mode)
                h = spv.System(x, y, w["L"], w["L"], p0=p0, params=prm)
                h.load_state(state)
                return h, w["N"]
            res[mode] = timed_run(spv, make, hybrid_steps, 0, timing=False)
        out["hybrid"][str(p0)] = {"steps": hybrid_steps, "after_warmup": warmup,
                                  "hybrid_value": res[1]["value"], "hybrid_ms_per_step": res[1]["ms_per_step"],
                                  "device_value": res[0]["value"], "device_ms_per_step": res[0]["ms_per_step"],
                                  "repairs_per_step": res[1]["repairs_per_step"],
                                  "device_over_hybrid": res[0]["value"] / res[1]["value"]}
        print(f"[bench] p0={p0}: device {res[0]['value']:.3e}, hybrid {res[1]['value']:.3e} cell-steps/s",
              file=sys.stderr, flush=True)
    # spatial-sort ablation (Sec. II.B): re-sort every 10 / 100 / 1000 steps
    # (periods are shortened while the drift bound would pass a bin side) and
    # never (-1: the memory order of creation, repairs on a per-step cell
    # list), with Hilbert-ordered or row-major bins
    for every in (10, 100, 1000, -1):
        for order, name in ((0, "hilbert"), (1, "row_major")):
            r = timed_run(spv, single(spv, inputs, "spv_n1m", spv.SPV_FP64, resort_every=every, bin_order=order),
                          ablation_steps, 100, timing=False)
            out["resort_ablation_n1m"][f"{every}_{name}"] = {
                "value": r["value"], "ms_per_step": r["ms_per_step"], "steady_state_value": r["steady_value"],
                "resorts": r["path"]["resorts"], "steps": ablation_steps, "warmup": 100}
            print(f"[bench] re-sort {every} {name}: {r['value']:.3e} cell-steps/s", file=sys.stderr, flush=True)
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


# Active vertex model, algorithmic bytes per cell-step (two vertices per
# cell): geometry 113 (degree, the first eight list entries, two vertex
# positions, A0 and P0 in; A, P, a, b out), force and move 136 (per vertex
# position, neighbour and cell rows, a third of three cells' a, b, theta,
# the new position out), first T1 marking pass with the director rotation
# 80, the other passes about 8 (flag bytes).
AVM_STEP_B = 337


def avm_runs(spv, inputs, steps):
    """The active vertex model from the Voronoi network of uniform-random
    points: cell-steps/s with the memory order kept along a Hilbert curve
    (every 1000 or 100 steps), by rows of bins, or never sorted (the
    caller's order, spatially random)."""
    import torch
    out = {}
    for name in ("avm_n100k", "avm_n1m"):
        w = inputs.WORKLOADS[name]
        n, L = w["N"], w["L"]
        nsteps = steps if name == "avm_n100k" else max(steps // 5, 100)
        x, y = inputs.uniform_positions(n, L, L, w["seed"])
        s = spv.System(x, y, L, L)
        vx, vy, off, cv = spv.spv_voronoi_network(s.h, s.N)
        s.close()
        res = {}
        for label, re, bo in (("hilbert_every_1000", 0, 0), ("row_major_every_1000", 0, 1),
                              ("hilbert_every_100", 100, 0), ("never_sorted", -1, 0)):
            prm = spv.AvmParams(mu=w["mu"], v0=w["v0"], Dr=w["Dr"], dt=w["dt"], seed=w["seed"],
                                t1_length=w["t1"], t1_new_length=w["t1_new"], resort_every=re, bin_order=bo)
            a = spv.AVM(vx, vy, off, cv, L, L, p0=w["p0"], params=prm)
            a.step(104)  # past the first T1 burst of a Voronoi start
            torch.cuda.synchronize()
            c0 = a.observables()[2]
            t0 = time.perf_counter()
            a.step(nsteps)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            c1 = a.observables()[2]
            a.close()
            d = c1 - c0
            v = n * nsteps / dt
            res[label] = {"value": v, "unit": "cell-steps/s", "ms_per_step": dt / nsteps * 1e3, "steps": nsteps,
                          "t1_per_step": float(d[1]) / nsteps, "t1_rounds_per_step": float(d[2]) / nsteps,
                          "host_rounds": int(d[3]), "graph_batches": int(d[4]), "resorts": int(d[5]),
                          "roofline_step": {"bytes_per_cell_step": AVM_STEP_B, "achieved": AVM_STEP_B * v / 1e9,
                                            "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                            "frac": AVM_STEP_B * v / 1e9 / HBM_PEAK_GBS}}
            print(f"[bench] {name} {label}: {v:.3e} cell-steps/s", file=sys.stderr, flush=True)
        res["hilbert_over_never"] = res["hilbert_every_1000"]["value"] / res["never_sorted"]["value"]
        out[name] = res
    return out


def avm_cpu_baseline(inputs, nsteps):
    """The oracle's active vertex model on the host (one thread): nsteps
    steps of the avm_n100k workload from its Voronoi network, a bounded
    sample that includes the first burst of T1 transitions (which the device
    figures skip)."""
    import oracle
    w = inputs.WORKLOADS["avm_n100k"]
    n, L = w["N"], w["L"]
    x, y = inputs.uniform_positions(n, L, L, w["seed"])
    xq, yq, Lx, Ly, q = oracle.prepare(x, y, L, L)
    vx, vy, off, cv = oracle.voronoi_network(xq, yq, Lx, Ly, q)
    th = oracle.theta0(w["seed"], n)
    t0 = time.perf_counter()
    oracle.avm_run(vx, vy, th, Lx, Ly, q, off, cv, 1.0, w["p0"], KA=1.0, KP=1.0, mu=w["mu"], v0=w["v0"], Dr=w["Dr"],
                   dt=w["dt"], seed=w["seed"], l_t1=w["t1"], l_new=w["t1_new"], nsteps=nsteps)
    dt = time.perf_counter() - t0
    return {"value": n * nsteps / dt, "unit": "cell-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"avm_n100k, {nsteps} steps from the Voronoi network (includes the first T1 burst)"}


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
    if args.avm_only:
        print(json.dumps({"avm": avm_runs(spv, inputs, args.avm_steps)}))
        return
    w = inputs.WORKLOADS[args.workload]
    prec = spv.SPV_MIXED if args.precision == "mixed" else spv.SPV_FP64
    # timed region 1: throughput (no events) -> value
    head = timed_run(spv, single(spv, inputs, args.workload, prec), args.steps, args.warmup, timing=False)
    n = head["cells"]
    mode = head["tuning"].get("force_mode")
    # timed region 2: the same window of the same trajectory (a fresh handle,
    # the same warm-up and steps) with HIP events on every kernel launch ->
    # the time of each kernel class and the roofline of the dominant one
    rl, table = None, None
    if not args.no_timing:
        tr = timed_run(spv, single(spv, inputs, args.workload, prec), args.steps, args.warmup, timing=True)
        rl, table = roofline(tr, args.workload, mode)
        rl["timed_ms_per_step"] = tr["ms_per_step"]
        if prec != spv.SPV_FP64:  # the counter-measured traffic is that of the FP64 kernels
            rl["traffic"] = rl["measured_achieved"] = rl["measured_frac"] = None
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
        "dtype": "f64" if prec == spv.SPV_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "N": n, "L": w["L"], "p0": w["p0"], "v0": w["v0"], "Dr": w["Dr"],
                   "mu": w["mu"], "dt": w["dt"], "precision": args.precision, "tuning": head["tuning"]},
        "roofline": rl,
        # the whole step's algorithmic bytes (three streaming passes) at the
        # measured rate, against HBM peak
        "roofline_step": {"bytes_per_cell_step": STEP_B, "achieved": STEP_B * head["value"] / 1e9,
                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": STEP_B * head["value"] / 1e9 / HBM_PEAK_GBS},
        "kernels": table,
        "steady_state_value": head["steady_value"],
        "repairs_per_step": head["repairs_per_step"],
        "candidates_per_repair": head["candidates"] / max(head["repaired"], 1),
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
            # kernel classes over the first tenth of the same window (events
            # keep the steps eager)
            tr = timed_run(spv, make, max(steps // 10, 50), warm, timing=True)
            rr, tab = roofline(tr, name, r["tuning"].get("force_mode"))
            extra[name] = {"value": r["value"], "unit": "cell-steps/s", "ms_per_step": r["ms_per_step"],
                           "steady_state_value": r["steady_value"],
                           "cells": r["cells"], "steps": steps, "warmup": warm,
                           "repairs_per_step": r["repairs_per_step"], "tuning": r["tuning"], "path": r["path"],
                           "kernels_timed_steps": tr["steps"],
                           "kernels": {k: {"avg_launch_us": v["avg_launch_us"], "ms_per_step": v["ms_per_step"],
                                           "hbm_frac": v.get("hbm_frac")} for k, v in tab.items()},
                           "dominant_kernel": rr["kernel"], "roofline_frac_hbm": rr["frac"]}
            print(f"[bench] {name}: {r['value']:.3e} cell-steps/s", file=sys.stderr, flush=True)
        extra["mixed_vs_fp64_speedup_n100k"] = extra["spv_n100k_mixed"]["value"] / head["value"]
        extra["adjoint_n4096"] = adjoint_cost(spv, inputs)
        extra.update(sweeps(spv, inputs, args.sweep_steps, args.warmup, args.hybrid_steps, args.ablation_steps))
        extra["avm"] = avm_runs(spv, inputs, args.avm_steps)
        if not args.no_cpu_baseline:
            extra["avm"]["cpu_baseline"] = avm_cpu_baseline(inputs, args.avm_cpu_steps)
        print(f"[bench] adjoint/forward: {extra['adjoint_n4096']['adjoint_over_forward']:.2f}", file=sys.stderr,
              flush=True)
        out["extra"] = extra
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_sample_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
