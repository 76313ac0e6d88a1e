"""Benchmark of the MRS filament hot path on one MI355X.

One step = one forward-Euler time step of a resident ensemble: rod forces
with the half-angle mid frames (packed straight into source records), the
all-pairs MRS sum of U and Omega, and the fixed-order FP64 reduction fused
with the position/frame update.  The headline workload is 100 filaments x
128 points (12,800 points); its value is pair interactions per second of the
FP32-compensated path, with the FP64 path measured the same way beside it.

Prints ONE JSON line.  --gpus N > 1 is not supported (one GPU per run).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MRS pair interactions/s (FP32-comp vs FP64) at 1 GPU; p50/p99 solve latency"
PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector, published
PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector, published
FLOPS_PER_PAIR = 92       # algorithmic flops of one (target, source) evaluation, FMA = 2


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    import synth

    if name == "config2":
        return synth.config2(), "100 filaments x 128 points (12,800 points) in [0,10]^3, eps = 1.5/128"
    if name == "config5":
        return synth.config5(), "1,000 filaments x 256 points (256,000 points) in [0,50]^3, eps = 1.5/256"
    raise SystemExit(f"unknown workload {name}")


def measure(mrs, ctx, e, prec, steps, warmup, dt):
    """Timed eager steps with per-kernel HIP events on the launch stream."""
    import torch

    rod = mrs.rod_params(*(getattr(e.rod(), k) for k in ("a", "b", "omega0", "ds")))
    ens = mrs.mrs_ensemble_create(ctx, e.offsets, e.X, e.D, e.f, e.n, e.eps, e.mu, rod)
    try:
        mrs.mrs_ensemble_step(ctx, ens, mrs.MRS_EULER, dt, warmup, prec, True)
        # latency of single synchronous steps
        lat = []
        for _ in range(max(steps, 20)):
            t0 = time.perf_counter()
            mrs.mrs_ensemble_step(ctx, ens, mrs.MRS_EULER, dt, 1, prec, True)
            lat.append((time.perf_counter() - t0) * 1e3)
        # throughput: K steps queued back to back, kernel events on
        mrs.mrs_profile_reset(ctx)
        mrs.mrs_profile_enable(ctx, True)
        torch.cuda.synchronize()
        mrs.mrs_context_synchronize(ctx)
        t0 = time.perf_counter()
        mrs.mrs_ensemble_step(ctx, ens, mrs.MRS_EULER, dt, steps, prec, True)
        mrs.mrs_context_synchronize(ctx)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        mrs.mrs_profile_enable(ctx, False)
        kname = "pairs_tile_f32c" if prec == mrs.MRS_FP32C else "pairs_tile_f64"
        n_k, ms_k = mrs.mrs_profile_query(ctx, kname)
        kernels = {}
        for k in ("rod_forces", "pairs_tile", "pairs_split", "reduce_euler"):
            n, ms = mrs.mrs_profile_query(ctx, k)
            if n:
                kernels[k] = {"launches": n, "avg_us": 1e3 * ms / n}
        mrs.mrs_profile_reset(ctx)
        # graph-replayed steps (one HIP graph launch per 50 steps)
        mrs.mrs_batch_step(ctx, [ens], mrs.MRS_EULER, dt, steps, prec, True, use_graph=True)
        t0 = time.perf_counter()
        mrs.mrs_batch_step(ctx, [ens], mrs.MRS_EULER, dt, steps, prec, True, use_graph=True)
        wall_graph = time.perf_counter() - t0
        Xg, Dg, _, _ = mrs.mrs_ensemble_get(ctx, ens)
        return {
            "wall_s": wall,
            "wall_graph_s": wall_graph,
            "lat_ms": lat,
            "kernel": kname,
            "kernel_launches": n_k,
            "kernel_avg_s": (ms_k / n_k) * 1e-3 if n_k else float("nan"),
            "kernels": kernels,
            "finite": bool(np.all(np.isfinite(Xg)) and np.all(np.isfinite(Dg))),
        }
    finally:
        mrs.mrs_ensemble_destroy(ens)


def cpu_baseline(mrs, ctx, e, prec_list):
    """The FP64 oracle as it stands, on this host's cores, on a bounded sample:
    the rod forces of the whole ensemble plus the MRS sum for a subset of
    targets; also the GPU's max relative error on that subset."""
    import oracle

    n_t = min(e.N, 1024)
    idx = np.sort(np.random.default_rng(7).choice(e.N, n_t, replace=False))
    t0 = time.perf_counter()
    reps = 0
    while True:
        g, m = oracle.rod_forces(e.offsets, e.X, e.D, e.rod(), e.f, e.n)
        Uo, Wo = oracle.mrs_field(e.X[idx], e.X, g, m, e.eps, e.mu)
        reps += 1
        if time.perf_counter() - t0 > 10.0 or reps >= 50:
            break
    dt = time.perf_counter() - t0
    pairs = reps * n_t * e.N
    errs = {}
    rod = mrs.rod_params(*(getattr(e.rod(), k) for k in ("a", "b", "omega0", "ds")))
    ens = mrs.mrs_ensemble_create(ctx, e.offsets, e.X, e.D, e.f, e.n, e.eps, e.mu, rod)
    try:
        for prec in prec_list:
            mrs.mrs_ensemble_eval(ctx, ens, prec, True)
            _, _, U, W = mrs.mrs_ensemble_get(ctx, ens)
            errs["fp32c" if prec == mrs.MRS_FP32C else "fp64"] = {
                "U": oracle.rel_err(U[idx], Uo), "Omega": oracle.rel_err(W[idx], Wo)}
    finally:
        mrs.mrs_ensemble_destroy(ens)
    return {
        "value": pairs / dt,
        "unit": "pairs/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"rod forces of all {e.N} points + MRS sum for {n_t} seeded targets x {e.N} sources, "
                  f"repeated {reps}x ({dt:.1f} s)",
    }, errs


def roofline(pairs_per_launch, avg_s, peak_tflops, traffic=None):
    ach = FLOPS_PER_PAIR * pairs_per_launch / avg_s / 1e12
    return {"bound": "alu", "achieved": round(ach, 3), "peak": peak_tflops, "unit": "TFLOP/s",
            "frac": round(ach / peak_tflops, 4), "traffic": traffic}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="config2", choices=["config2", "config5"])
    ap.add_argument("--dt", type=float, default=1e-6)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the library is single-GPU; see the sharding notes)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2604_12083_amd as mrs

    assert torch.cuda.is_available(), "needs a GPU"
    e, desc = workload(args.workload)
    ctx = mrs.mrs_context_create(0)
    try:
        pairs_step = e.N * e.N
        res = {}
        for prec, tag in ((mrs.MRS_FP32C, "fp32c"), (mrs.MRS_FP64, "fp64")):
            log(f"measure {tag} N={e.N} steps={args.steps}")
            res[tag] = measure(mrs, ctx, e, prec, args.steps, args.warmup, args.dt)
        cpu, errs = (None, None)
        if not args.no_cpu:
            log("cpu baseline (oracle)")
            cpu, errs = cpu_baseline(mrs, ctx, e, [mrs.MRS_FP32C, mrs.MRS_FP64])
    finally:
        mrs.mrs_context_destroy(ctx)

    def summary(r, peak):
        lat = np.array(r["lat_ms"])
        return {
            "value": args.steps * pairs_step / r["wall_s"],
            "ms_per_step": 1e3 * r["wall_s"] / args.steps,
            "ms_per_step_graph": 1e3 * r["wall_graph_s"] / args.steps,
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
            "roofline": roofline(pairs_step, r["kernel_avg_s"], peak),
            "kernels_avg_us": {k: round(v["avg_us"], 2) for k, v in r["kernels"].items()},
        }

    s32 = summary(res["fp32c"], PEAK_FP32_TFLOPS)
    s64 = summary(res["fp64"], PEAK_FP64_TFLOPS)
    line = {
        "metric": METRIC,
        "value": s32["value"],
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": s32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32c",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}; one forward-Euler step (rod forces + MRS U/Omega "
                               f"+ frame update), dt={args.dt}",
                   "n_points": e.N, "pairs_per_step": pairs_step, "precision": "fp32c"},
        "latency_ms": s32["latency_ms"],
        "ms_per_step_graph": s32["ms_per_step_graph"],
        "kernels_avg_us": s32["kernels_avg_us"],
        "roofline": s32["roofline"],
        "fp64": s64,
        "cpu_baseline": cpu,
        "max_rel_err_vs_oracle": errs,
        "finite": res["fp32c"]["finite"] and res["fp64"]["finite"],
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
