"""Benchmark of the MRS filament hot path on one MI355X.

One step = one forward-Euler time step of a resident ensemble: rod forces
with the half-angle mid frames (packed straight into source records), the
all-pairs MRS sum of U and Omega, and the fixed-order FP64 reduction fused
with the position/frame update.  The headline workload is 100 filaments x
128 points (12,800 points); its value is pair interactions per second of the
FP32-compensated path, with the FP64 path measured the same way beside it.
The default run adds two legs to the same line: one-shot evaluations of the
1,000-filament, 256,000-point ensemble in both precisions (pair-kernel
roofline from its own events; max relative error on its 2,048-target check
subset from the CPU leg) and 16 fine-propagator slices of 3,200 points
advanced by RK4 steps as one batched graph launch against one launch per
kernel per slice.

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

# HBM bytes per pair-kernel launch from hardware counters (FETCH_SIZE x 2.0 +
# WRITE_SIZE x 1.0, the factors a 256 MiB device copy reads), valid only for
# the pair-kernel source (sha256 of the kernel file and its device header,
# concatenated), the exact work list (sha256 of the blocks `mrs_plan_items`
# gives for the workload) and the schedule (0 grid, 1 persistent) they were
# taken on: any other kernel, decomposition or schedule reports null.
KERNEL_SRCS = [os.path.join(ROOT, "paper_2604_12083_amd", "csrc", f) for f in ("mrs_pairs.hip", "mrs_device_pairs.h")]
KERNEL_SHA = "40f34d49df4e05869d604daebf4eddf5ac4a3fb0ed492161478c62626b0aa46b"
MEASURED_TRAFFIC = {
    ("ens12800", "fp32c", "678ec7c5e5d82ecf", 0): (3544.88 * 2.0 + 37200.0) * 1024,
    ("ens12800", "fp64", "adb3c89bda2d142d", 0): (4134.13 * 2.0 + 30000.0) * 1024,
    ("ens256000", "fp32c", "4a2b01f9e8a27aa9", 1): (321384.91 * 2.0 + 264767.56) * 1024,
    ("ens256000", "fp64", "571ba5e594123b76", 1): (467335.21 * 2.0 + 396579.69) * 1024,
    ("swim", "fp32c", "72ec18efbf0e53ad", 1): (41684.76 * 2.0 + 177658.77) * 1024,
    ("swim", "fp64", "df10004c75444124", 1): (74857.08 * 2.0 + 148478.23) * 1024,
}


def measured_traffic(mrs, workload_name, tag, n, prec, n_cu, sched=0):
    import hashlib

    h = hashlib.sha256()
    try:
        for src in KERNEL_SRCS:
            with open(src, "rb") as fh:
                h.update(fh.read())
    except OSError:
        return None
    if h.hexdigest() != KERNEL_SHA:
        return None
    _, items = mrs.mrs_plan_items(n, prec, n_cu)
    v = MEASURED_TRAFFIC.get((workload_name, tag, hashlib.sha256(items.tobytes()).hexdigest()[:16], int(sched)))
    return None if v is None else round(v)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    """(ensemble, description, swimming parameters or None)."""
    import synth

    if name == "rod64":
        return synth.rod64(), "1 filament x 64 points, eps = 1.5/64", None
    if name == "ens12800":
        return synth.ens12800(), "100 filaments x 128 points (12,800 points) in [0,10]^3, eps = 1.5/128", None
    if name == "ens256000":
        return synth.ens256000(), "1,000 filaments x 256 points (256,000 points) in [0,50]^3, eps = 1.5/256", None
    if name == "swim":
        e = synth.swimmers(1000, box=40.0, seed=12)
        p = synth.swim_params(e)
        return e, ("1,000 straight swimmers x 51 points (51,000 points), length 1, eps = 4 ds, in [0,40]^2 at "
                   f"z = 1 +- 0.1; waveform A={p.wave[0]}, k=2 pi, f={p.wave[2]:.4g}; Lennard-Jones sigma = 3 eps, "
                   f"energy {p.lj[1]}"), p
    if name == "swim25":
        # the largest configuration of the paper's timing table: 25 swimmers of 51 points
        e = synth.swimmers(25, box=4.0, seed=25)
        p = synth.swim_params(e)
        return e, ("25 straight swimmers x 51 points (1,275 points), length 1, eps = 4 ds, in [0,4]^2 at "
                   f"z = 1 +- 0.1; waveform A={p.wave[0]}, k=2 pi, f={p.wave[2]:.4g}; Lennard-Jones sigma = 3 eps, "
                   f"energy {p.lj[1]}"), p
    raise SystemExit(f"unknown workload {name}")


SETTLE_S = 0.5  # untimed steps before the warm-up, so that the shader clock has settled


def measure(mrs, ctx, e, prec, steps, warmup, dt, integ=None, swim=None):
    """Timed eager steps; HIP events on the launch stream bracket the
    dominant pair kernel inside the timed region.  Before the warm-up, untimed
    steps run for SETTLE_S seconds (the clock of a fresh process ramps up
    over the first launches)."""
    import torch

    integ = mrs.MRS_EULER if integ is None else integ
    rp = swim.rod if swim is not None else e.rod()
    rod = mrs.rod_params(*(getattr(rp, k) for k in ("a", "b", "omega0", "ds")))
    ens = mrs.mrs_ensemble_create(ctx, e.offsets, e.X, e.D, e.f, e.n, e.eps, e.mu, rod)
    if swim is not None:
        mrs.mrs_ensemble_set_swimming(ctx, ens, swim.wave, swim.lj)
    try:
        t_settle = time.perf_counter()
        settle_steps = 0
        while time.perf_counter() - t_settle < SETTLE_S:
            mrs.mrs_ensemble_step(ctx, ens, integ, dt, 5, prec, True)
            settle_steps += 5
        settle_s = time.perf_counter() - t_settle
        mrs.mrs_ensemble_set_state(ctx, ens, e.X, e.D)
        mrs.mrs_ensemble_set_time(ctx, ens, 0.0)
        mrs.mrs_ensemble_step(ctx, ens, integ, dt, warmup, prec, True)
        # latency of single synchronous steps
        lat = []
        for _ in range(max(steps, 20)):
            t0 = time.perf_counter()
            mrs.mrs_ensemble_step(ctx, ens, integ, dt, 1, prec, True)
            lat.append((time.perf_counter() - t0) * 1e3)
        # throughput: K steps queued back to back; HIP events bracket the
        # dominant pair kernel only, on the stream it is launched on
        split = mrs.mrs_tune_get(ctx, e.N, prec)["mode"] == 1
        kname = ("pairs_split_f32c" if prec == mrs.MRS_FP32C else "pairs_split_f64") if split else \
            ("pairs_tile_f32c" if prec == mrs.MRS_FP32C else "pairs_tile_f64")
        mrs.mrs_profile_reset(ctx)
        mrs.mrs_profile_select(ctx, kname)
        mrs.mrs_profile_enable(ctx, True)
        clock_before = mrs.mrs_profile_clock(ctx)
        torch.cuda.synchronize()
        mrs.mrs_context_synchronize(ctx)
        t0 = time.perf_counter()
        mrs.mrs_ensemble_step(ctx, ens, integ, dt, steps, prec, True)
        mrs.mrs_context_synchronize(ctx)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        clock_after = mrs.mrs_profile_clock(ctx)
        mrs.mrs_profile_enable(ctx, False)
        n_k, ms_k = mrs.mrs_profile_query(ctx, kname)
        # every kernel of the step, from a short untimed pass
        mrs.mrs_profile_reset(ctx)
        mrs.mrs_profile_select(ctx, "")
        mrs.mrs_profile_enable(ctx, True)
        mrs.mrs_ensemble_step(ctx, ens, integ, dt, min(steps, 20), prec, True)
        mrs.mrs_profile_enable(ctx, False)
        kernels = {}
        for k in ("lj_forces", "rod_forces", "pairs_tile", "pairs_split", "reduce_euler", "reduce_rk_stage",
                  "reduce_rk_final"):
            n, ms = mrs.mrs_profile_query(ctx, k)
            if n:
                kernels[k] = {"launches": n, "avg_us": 1e3 * ms / n}
        mrs.mrs_profile_reset(ctx)
        # graph-replayed steps (one HIP graph launch per 50 steps)
        mrs.mrs_batch_step(ctx, [ens], integ, dt, steps, prec, True, use_graph=True)
        t0 = time.perf_counter()
        mrs.mrs_batch_step(ctx, [ens], integ, dt, steps, prec, True, use_graph=True)
        wall_graph = time.perf_counter() - t0
        Xg, Dg, _, _ = mrs.mrs_ensemble_get(ctx, ens)
        return {
            "settle_s": settle_s,
            "settle_steps": settle_steps,
            "clock_mhz": {"before": round(clock_before, 1), "after": round(clock_after, 1)},
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


def cpu_baseline(mrs, ctx, e, prec_list, swim=None, workload_name=""):
    """The FP64 oracle as it stands, on this host's cores, on a bounded sample:
    the rod forces of the whole ensemble plus the MRS sum for a subset of
    targets (the 2,048-target check subset at 256,000 points, else 1,024
    seeded targets); also the same on one core, and the GPU's max relative
    error on that subset."""
    import oracle
    import synth

    if workload_name == "ens256000":
        idx = synth.ens256000_subset(e.N)
    else:
        idx = np.sort(np.random.default_rng(7).choice(e.N, min(e.N, 1024), replace=False))
    n_t = len(idx)
    rp = swim.rod if swim is not None else e.rod()
    kw = {} if swim is None else {"wave": swim.wave, "t": 0.0, "lj": swim.lj}

    def timed_reps(limit_s):
        t0 = time.perf_counter()
        reps = 0
        while True:
            g, m = oracle.rod_forces(e.offsets, e.X, e.D, rp, e.f, e.n, **kw)
            Uo, Wo = oracle.mrs_field(e.X[idx], e.X, g, m, e.eps, e.mu)
            reps += 1
            if time.perf_counter() - t0 > limit_s or reps >= 5000:
                return reps, time.perf_counter() - t0, Uo, Wo

    cores = oracle.num_threads()
    reps, dt, Uo, Wo = timed_reps(10.0)
    oracle.set_num_threads(1)
    try:
        reps1, dt1, _, _ = timed_reps(3.0)
    finally:
        oracle.set_num_threads(cores)
    pairs = reps * n_t * e.N
    errs = {}
    rod = mrs.rod_params(*(getattr(rp, k) for k in ("a", "b", "omega0", "ds")))
    ens = mrs.mrs_ensemble_create(ctx, e.offsets, e.X, e.D, e.f, e.n, e.eps, e.mu, rod)
    if swim is not None:
        mrs.mrs_ensemble_set_swimming(ctx, ens, swim.wave, swim.lj)
    try:
        for prec in prec_list:
            mrs.mrs_ensemble_eval(ctx, ens, prec, True)
            _, _, U, W = mrs.mrs_ensemble_get(ctx, ens)
            errs["fp32c" if prec == mrs.MRS_FP32C else "fp64"] = {
                "U": oracle.rel_err(U[idx], Uo), "Omega": oracle.rel_err(W[idx], Wo)}
    finally:
        mrs.mrs_ensemble_destroy(ens)
    out = {
        "value": pairs / dt,
        "unit": "pairs/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"rod forces of all {e.N} points + MRS sum for {n_t} seeded targets x {e.N} sources, "
                  f"repeated {reps}x ({dt:.1f} s)",
        "value_1core": reps1 * n_t * e.N / dt1,
        "cpu": cpu_model(),
    }
    if n_t < e.N:
        # time of one full N^2 evaluation at the measured rate (not measured)
        out["extrapolated_full_eval_s"] = e.N * e.N / out["value"]
    return out, errs


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


# Algorithmic bytes per point of the frame update: the rod stage reads X, D
# (96 B) and writes the point's source record (48 B); with FP32C it also
# writes the source-block descriptors, reading X again (24 B) and writing the
# anchored position (16 B) and 1/64 of a 64-B block descriptor.  The Euler
# update reads X, D, U, Omega (144 B) and writes X, D (96 B).
ROD_BYTES_PER_POINT = {"fp64": 144, "fp32c": 144 + 24 + 16 + 1}
EULER_BYTES_PER_POINT = 240


def frame_update_gbps(n_points, kernels, prec="fp64"):
    out = {}
    for name, nbytes in (("rod_forces", ROD_BYTES_PER_POINT[prec]), ("reduce_euler", EULER_BYTES_PER_POINT)):
        if name in kernels and kernels[name]["avg_us"] > 0:
            out[name] = round(nbytes * n_points / (kernels[name]["avg_us"] * 1e-6) / 1e9, 1)
    return out


def roofline(pairs_per_launch, avg_s, peak_tflops, traffic=None):
    ach = FLOPS_PER_PAIR * pairs_per_launch / avg_s / 1e12
    return {"bound": "alu", "achieved": round(ach, 3), "peak": peak_tflops, "unit": "TFLOP/s",
            "frac": round(ach / peak_tflops, 4), "traffic": traffic}


def bench_large(mrs, ctx, n_cu, reps32=3, reps64=2):
    """One-shot U, Omega evaluations (rod forces + MRS sum + reduction) of the
    256,000-point ensemble, FP32C then FP64, with HIP events around the pair
    kernel; returns the leg's summary and the GPU results on the seeded
    2,048-target check subset (compared with the oracle in the CPU leg)."""
    import synth

    e = synth.ens256000()
    idx = synth.ens256000_subset(e.N)
    rod = mrs.rod_params(*(getattr(e.rod(), k) for k in ("a", "b", "omega0", "ds")))
    ens = mrs.mrs_ensemble_create(ctx, e.offsets, e.X, e.D, e.f, e.n, e.eps, e.mu, rod)
    out, subset = {"n_points": e.N, "pairs_per_eval": e.N * e.N}, {}
    try:
        for prec, tag, reps, peak in ((mrs.MRS_FP32C, "fp32c", reps32, PEAK_FP32_TFLOPS),
                                      (mrs.MRS_FP64, "fp64", reps64, PEAK_FP64_TFLOPS)):
            log(f"large ensemble {tag}: {reps} evaluations of {e.N} points")
            mrs.mrs_ensemble_eval(ctx, ens, prec, True)  # plan and warm-up
            kname = "pairs_tile_f32c" if prec == mrs.MRS_FP32C else "pairs_tile_f64"
            mrs.mrs_profile_reset(ctx)
            mrs.mrs_profile_select(ctx, kname)
            mrs.mrs_profile_enable(ctx, True)
            t0 = time.perf_counter()
            for _ in range(reps):
                mrs.mrs_ensemble_eval(ctx, ens, prec, True)
            wall = (time.perf_counter() - t0) / reps
            mrs.mrs_profile_enable(ctx, False)
            n_k, ms_k = mrs.mrs_profile_query(ctx, kname)
            mrs.mrs_profile_reset(ctx)
            _, _, U, W = mrs.mrs_ensemble_get(ctx, ens)
            subset[tag] = (U[idx], W[idx])
            out[tag] = {"evals": reps, "ms_per_eval": 1e3 * wall, "pairs_per_s": e.N * e.N / wall,
                        "pair_kernel_us": 1e3 * ms_k / n_k,
                        "roofline": roofline(e.N * e.N, 1e-3 * ms_k / n_k, peak,
                                             measured_traffic(mrs, "ens256000", tag, e.N, prec, n_cu,
                                                              mrs.mrs_tune_get(ctx, e.N, prec)["schedule"]))}
    finally:
        mrs.mrs_ensemble_destroy(ens)
    return out, subset


def oracle_large_subset(subset):
    """The oracle on the 256,000-point ensemble's 2,048-target check subset
    (rod forces of every point, then the MRS sum for the subset): its time and
    the GPU's max relative error there."""
    import oracle
    import synth

    e = synth.ens256000()
    idx = synth.ens256000_subset(e.N)
    t0 = time.perf_counter()
    g, m = oracle.rod_forces(e.offsets, e.X, e.D, e.rod(), e.f, e.n)
    Uo, Wo = oracle.mrs_field(e.X[idx], e.X, g, m, e.eps, e.mu)
    dt = time.perf_counter() - t0
    errs = {tag: {"U": oracle.rel_err(U, Uo), "Omega": oracle.rel_err(W, Wo)} for tag, (U, W) in subset.items()}
    return {"value": len(idx) * e.N / dt, "unit": "pairs/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"rod forces of all {e.N} points + MRS sum for the {len(idx)}-target check subset, once "
                      f"({dt:.1f} s)"}, errs


def bench_tune(mrs, sizes, reps=7, tune_reps=5):
    """The tuner against the automatic configuration: for each size (sinusoidal
    128-point filaments at the density of 100 in a box of side 10; the tuner
    itself times straight ones) and precision, mrs_autotune in a fresh
    context, then `reps` interleaved evaluations (mrs_eval_device, device time
    of all its kernels) with the automatic entry and with the tuned one."""
    import torch

    import synth

    rows = []
    for n in sizes:
        F = n // 128
        e = synth.filaments(F, 128, 10.0 * (F / 100.0) ** (1.0 / 3.0), 4000 + F)
        dX, df, dn = (torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0") for a in (e.X, e.f, e.n))
        dU, dW = torch.empty_like(dX), torch.empty_like(dX)
        s = torch.cuda.current_stream()
        for prec, tag in ((mrs.MRS_FP32C, "fp32c"), (mrs.MRS_FP64, "fp64")):
            ctx = mrs.mrs_context_create(0)
            try:
                auto = mrs.mrs_tune_get(ctx, e.N, prec)
                auto_entry = (auto["mode"], auto["targets_per_lane"], 1 if auto["mode"] == 1 else 0, 0)
                log(f"tune N={e.N} {tag}: automatic {auto}")
                t0 = time.perf_counter()
                best, best_ms = mrs.mrs_autotune(ctx, e.N, prec, tune_reps)
                tune_s = time.perf_counter() - t0
                tuned = mrs.mrs_tune_get(ctx, e.N, prec)
                entry = (best["mode"], best["targets_per_lane"], best["chunks"], best["schedule"])
                times = {"automatic": [], "tuned": []}
                for r in range(reps + 1):
                    for name, cfg in (("automatic", auto_entry), ("tuned", entry)):
                        mrs.mrs_tune_set(ctx, e.N, prec, *cfg)
                        mrs.mrs_profile_reset(ctx)
                        mrs.mrs_profile_select(ctx, "")
                        mrs.mrs_profile_enable(ctx, True)
                        mrs.mrs_eval_device(ctx, e.N, dX, df, dn, e.eps, e.mu, prec, dU, dW, s)
                        mrs.mrs_profile_enable(ctx, False)
                        _, ms = mrs.mrs_profile_query(ctx)
                        if r > 0:
                            times[name].append(ms)
                mrs.mrs_profile_reset(ctx)
                a, t = float(np.median(times["automatic"])), float(np.median(times["tuned"]))
                rows.append({"n_points": e.N, "prec": tag, "automatic": auto, "tuned": tuned,
                             "automatic_us": 1e3 * a, "tuned_us": 1e3 * t, "ratio": t / a,
                             "tuner_best_us": 1e3 * best_ms, "tune_s": tune_s})
                log(f"  tuned {tuned} in {tune_s:.1f} s: automatic {1e3 * a:.1f} us, tuned {1e3 * t:.1f} us")
            finally:
                mrs.mrs_context_destroy(ctx)
    return rows


def bench_slices(mrs, ctx, steps, args):
    """16 Parareal fine slices (32 x 100 points each), RK4 at dt = 1e-5, FP32C:
    one batched launch sequence replayed from HIP graphs vs one launch per
    kernel per slice per stage."""
    import synth

    base, slices = synth.slices()
    rod = mrs.rod_params(*(getattr(base.rod(), k) for k in ("a", "b", "omega0", "ds")))

    def make():
        return [mrs.mrs_ensemble_create(ctx, e.offsets, e.X, e.D, e.f, e.n, e.eps, e.mu, rod) for e in slices]

    hb, hp = make(), make()
    try:
        warm = max(1, min(10, steps // 10))
        mrs.mrs_batch_step(ctx, hb, mrs.MRS_RK4, 1e-5, warm, mrs.MRS_FP32C, True, use_graph=True)
        for h in hp:
            mrs.mrs_ensemble_step(ctx, h, mrs.MRS_RK4, 1e-5, warm, mrs.MRS_FP32C, True)
        t0 = time.perf_counter()
        mrs.mrs_batch_step(ctx, hb, mrs.MRS_RK4, 1e-5, steps, mrs.MRS_FP32C, True, use_graph=True)
        tb = time.perf_counter() - t0
        t0 = time.perf_counter()
        for h in hp:
            mrs.mrs_ensemble_step(ctx, h, mrs.MRS_RK4, 1e-5, steps, mrs.MRS_FP32C, True)
        tp = time.perf_counter() - t0
        same = all(np.array_equal(mrs.mrs_ensemble_get(ctx, a)[0], mrs.mrs_ensemble_get(ctx, b)[0])
                   for a, b in zip(hb, hp))
    finally:
        for h in hb + hp:
            mrs.mrs_ensemble_destroy(h)
    pairs = len(slices) * slices[0].N ** 2 * 4 * steps
    return {"slices": len(slices), "points_per_slice": slices[0].N, "rk4_steps": steps,
            "batched_graph_s": tb, "plain_s": tp, "batched_pairs_per_s": pairs / tb,
            "plain_pairs_per_s": pairs / tp, "speedup": tp / tb, "identical_results": bool(same)}


def bench_copies(mrs, ctx, e, dt, copies=(4, 8), reps=10):
    """The FP32C pair kernel over one launch of n copies of the ensemble
    (`reps` batched forward-Euler steps queued back to back, as the
    headline's steps are) for the two copy counts, interleaved, HIP events
    around the pair launches: the marginal cost of one copy in a longer grid
    (difference of the two, which cancels the fixed cost of a launch and is
    taken under the same sustained load), with its roofline, and the fixed
    cost that remains of the smaller launch."""
    rod = mrs.rod_params(*(getattr(e.rod(), k) for k in ("a", "b", "omega0", "ds")))
    lo, hi = copies
    hs = [mrs.mrs_ensemble_create(ctx, e.offsets, e.X, e.D, e.f, e.n, e.eps, e.mu, rod) for _ in range(hi)]
    try:
        times = {lo: [], hi: []}
        for n in times:  # plans and warm-up
            mrs.mrs_batch_step(ctx, hs[:n], mrs.MRS_EULER, dt, 2, mrs.MRS_FP32C, True, use_graph=False)
        for _ in range(3):
            for n in times:
                mrs.mrs_profile_reset(ctx)
                mrs.mrs_profile_select(ctx, "pairs_tile")
                mrs.mrs_profile_enable(ctx, True)
                mrs.mrs_batch_step(ctx, hs[:n], mrs.MRS_EULER, dt, reps, mrs.MRS_FP32C, True, use_graph=False)
                mrs.mrs_profile_enable(ctx, False)
                k, ms = mrs.mrs_profile_query(ctx, "pairs_tile")
                times[n].append(1e3 * ms / k)
        mrs.mrs_profile_reset(ctx)
    finally:
        for h in hs:
            mrs.mrs_ensemble_destroy(h)
    tl, th = float(np.median(times[lo])), float(np.median(times[hi]))
    marginal = (th - tl) / (hi - lo)
    return {"copies": list(copies), "pair_launch_us": {str(lo): tl, str(hi): th},
            "fixed_us": tl - lo * marginal, "marginal_us_per_copy": marginal,
            "marginal_roofline": roofline(e.N * e.N, 1e-6 * marginal, PEAK_FP32_TFLOPS)}


def bench_parareal(mrs, ctx, prec, tol, coarse_steps):
    """Parareal on one GPU for the 3,200-point slice base ensemble (external torques
    scaled by 1e-2): 16 slices of 200 RK4 steps at dt = 1e-5 (fine), forward
    Euler with `coarse_steps` steps per slice (coarse), against the serial
    fine solve of the same 3,200 steps."""
    import synth

    base, _ = synth.slices(n_slices=1)
    rod = mrs.rod_params(*(getattr(base.rod(), k) for k in ("a", "b", "omega0", "ds")))
    # external torques scaled by 1e-2: with N(0,1) torques the frames spin at
    # ~3e4 rad/s and no explicit-Euler coarse step of the slice is meaningful
    tq = 1e-2 * base.n
    mk = lambda: mrs.mrs_ensemble_create(ctx, base.offsets, base.X, base.D, base.f, tq, base.eps, base.mu, rod)

    def reset(h):
        mrs.mrs_ensemble_set_state(ctx, h, base.X, base.D)
        mrs.mrs_ensemble_set_time(ctx, h, 0.0)

    a, b = mk(), mk()
    try:
        # warm-up calls: the slice workers and the plans and graphs of every
        # iteration's batch (slices k..16) stay with the ensemble
        mrs.mrs_parareal(ctx, a, 16, mrs.MRS_RK4, 1e-5, 200, coarse_steps, 16, tol, prec, True)
        mrs.mrs_ensemble_step(ctx, b, mrs.MRS_RK4, 1e-5, 10, prec, True)
        reset(a)
        reset(b)
        t0 = time.perf_counter()
        it, hist = mrs.mrs_parareal(ctx, a, 16, mrs.MRS_RK4, 1e-5, 200, coarse_steps, 16, tol, prec, True)
        tpar = time.perf_counter() - t0
        c = mk()
        try:
            mrs.mrs_parareal_pipelined(ctx, c, 16, mrs.MRS_RK4, 1e-5, 200, coarse_steps, 16, tol, prec, True)
            reset(c)
            t0 = time.perf_counter()
            itp, histp = mrs.mrs_parareal_pipelined(ctx, c, 16, mrs.MRS_RK4, 1e-5, 200, coarse_steps, 16, tol, prec,
                                                    True)
            tpipe = time.perf_counter() - t0
            same = itp == it and np.array_equal(histp, hist) and np.array_equal(
                mrs.mrs_ensemble_get(ctx, c)[0], mrs.mrs_ensemble_get(ctx, a)[0])
        finally:
            mrs.mrs_ensemble_destroy(c)
        t0 = time.perf_counter()
        mrs.mrs_ensemble_step(ctx, b, mrs.MRS_RK4, 1e-5, 16 * 200, prec, True)
        tser = time.perf_counter() - t0
        Xa = mrs.mrs_ensemble_get(ctx, a)[0]
        Xb = mrs.mrs_ensemble_get(ctx, b)[0]
        disp = np.linalg.norm(Xb - base.X, axis=1)
        eta = float(np.max(np.linalg.norm(Xa - Xb, axis=1) / np.linalg.norm(Xb, axis=1)))
        eta_disp = float(np.max(np.linalg.norm(Xa - Xb, axis=1) / disp))
    finally:
        mrs.mrs_ensemble_destroy(a)
        mrs.mrs_ensemble_destroy(b)
    return {"slices": 16, "fine": "RK4 x 200 at dt=1e-5 per slice", "coarse": f"Euler x {coarse_steps} per slice",
            "iterations": it, "increments": [float(x) for x in hist], "tol": tol, "parareal_s": tpar,
            "pipelined_s": tpipe, "pipelined_identical": bool(same),
            "serial_fine_s": tser, "speedup_vs_serial": tser / tpar,
            "eta_vs_serial_fine": eta, "error_relative_to_displacement": eta_disp}


def bench_schedules(mrs, ctx, prec, integ="RK4", iters=4, fine_steps=(5, 20, 50, 200), coarse_steps=10):
    """Regular against pipelined Parareal (Sec. II.D) on one GPU for several
    fine/coarse cost ratios r: 16 slices of the 3,200-point slice ensemble,
    fine `integ` x fine_steps, coarse Euler x coarse_steps, a fixed number of
    iterations (tol = 0), so both schedules do the same work.  Each schedule
    runs twice on one ensemble from the same start state: the first call
    builds the slice workers, plans and graphs (`*_first_s`), the second
    reuses them (`*_s`)."""
    import synth

    base, _ = synth.slices(n_slices=1)
    rod = mrs.rod_params(*(getattr(base.rod(), k) for k in ("a", "b", "omega0", "ds")))
    tq = 1e-2 * base.n
    mk = lambda: mrs.mrs_ensemble_create(ctx, base.offsets, base.X, base.D, base.f, tq, base.eps, base.mu, rod)
    out = []
    for fs in fine_steps:
        stages = {"RK2": 2, "RK4": 4}[integ]
        row = {"fine": integ, "fine_steps": fs, "coarse_steps": coarse_steps, "r_evals": stages * fs / coarse_steps}
        for name, fn, kw in (("regular", mrs.mrs_parareal, {}), ("pipelined", mrs.mrs_parareal_pipelined, {}),
                             ("pipelined_g1", mrs.mrs_parareal_pipelined, {"group": 1})):
            log(f"parareal schedules: {name} {integ} fine_steps={fs}")
            h = mk()
            try:
                for key in ("_first_s", "_s"):
                    mrs.mrs_ensemble_set_state(ctx, h, base.X, base.D)
                    mrs.mrs_ensemble_set_time(ctx, h, 0.0)
                    t0 = time.perf_counter()
                    fn(ctx, h, 16, getattr(mrs, "MRS_" + integ), 1e-5, fs, coarse_steps, iters, 0.0, prec, True,
                       **kw)
                    row[name + key] = time.perf_counter() - t0
            finally:
                mrs.mrs_ensemble_destroy(h)
        out.append(row)
    return out


def bench_serving(mrs, ctx, n_req, rates, slots, budget, tick_pairs=0, admission=0, max_wait=0.0):
    """Serving: the fixed request sequence at Poisson arrival rates; continuous
    batching (many slots, admission order `admission`) vs one request at a
    time (one slot, arrival order)."""
    import synth

    reqs = synth.serving_requests()[:n_req]
    ens = [synth.filaments(r.n_fil, r.M, 10.0, r.seed) for r in reqs]
    out = {"requests": n_req, "points": [e.N for e in ens], "kinds": [r.kind for r in reqs]}
    rods = [mrs.rod_params(*(getattr(e.rod(), k) for k in ("a", "b", "omega0", "ds"))) for e in ens]

    def run(rate, nslots):
        log(f"serving {n_req} requests at {rate} req/s with {nslots} slots")
        arr = synth.poisson_arrivals(n_req, rate)
        srv = mrs.mrs_server_start(ctx, mrs.MRS_FP32C, budget, nslots)
        mrs.mrs_server_set_tick_pairs(srv, int(tick_pairs) if nslots > 1 else 0)
        if nslots > 1:
            mrs.mrs_server_set_admission(srv, admission, max_wait)
        tickets = []
        try:
            t0 = time.monotonic()
            for i, (r, e) in enumerate(zip(reqs, ens)):
                delay = t0 + arr[i] - time.monotonic()
                if delay > 0:
                    time.sleep(delay)
                tickets.append(mrs.mrs_server_submit(srv, r.kind, e.offsets, e.X, e.D, e.f, e.n, e.eps, e.mu,
                                                     rods[i], dt=1e-5, nsteps=50, integ=mrs.MRS_RK4))
            lat, kinds = [], []
            for i, t in enumerate(tickets):
                st, info, _ = mrs.mrs_server_wait(srv, t, ens[i].N, timeout_s=600)
                assert st == mrs.MRS_OK, st
                lat.append(info.t_done - info.t_submit)
                kinds.append(reqs[i].kind)
            wall = time.monotonic() - t0
            stats = mrs.mrs_server_stats_get(srv)
        finally:
            mrs.mrs_server_stop(srv)
        lat = np.array(lat) * 1e3
        kinds = np.array(kinds)
        res = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
               "pairs_per_s": stats["pairs"] / wall, "wall_s": wall, "ticks": stats["ticks"],
               "offered_req_per_s": rate, "device_busy_s": stats["busy_s"],
               "device_busy_frac": stats["busy_s"] / wall}
        for k, name in ((0, "eval"), (1, "rk4x50")):
            if np.any(kinds == k):
                res[f"p50_ms_{name}"] = float(np.percentile(lat[kinds == k], 50))
                res[f"p99_ms_{name}"] = float(np.percentile(lat[kinds == k], 99))
        # small requests: fewer points than the median request of the sequence
        pts = np.array([e.N for e in ens])
        small = pts < np.median(pts)
        if np.any(small):
            res["p50_ms_small"] = float(np.percentile(lat[small], 50))
            res["p99_ms_small"] = float(np.percentile(lat[small], 99))
            res["small_max_points"] = int(pts[small].max())
        return res

    out["admission"] = {"order": ["arrival", "least-work"][admission], "max_wait_s": max_wait,
                        "tick_pairs": tick_pairs, "slots": slots}
    out["batched"] = {str(r): run(r, slots) for r in rates}
    out["one_at_a_time"] = {str(rates[-1]): run(rates[-1], 1)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="ens12800",
                    choices=["rod64", "ens12800", "ens256000", "swim", "swim25", "slices", "serving", "parareal",
                             "copy", "tune"])
    ap.add_argument("--requests", type=int, default=32, help="serving: prefix of the request sequence")
    ap.add_argument("--rates", default="10,100,1000", help="serving: Poisson arrival rates (req/s)")
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--tick-pairs", type=float, default=5e9, help="serving: pair budget of one serving tick")
    ap.add_argument("--admission", default="least-work", choices=["arrival", "least-work"],
                    help="serving: admission order of queued requests")
    ap.add_argument("--max-wait", type=float, default=10.0,
                    help="serving, least-work order: age (s) after which a request is admitted in arrival order")
    ap.add_argument("--dt", type=float, default=None, help="time step (default 1e-4 for rod64, else 1e-6)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="default workload only: skip the 256,000-point and the 16-slice legs")
    args = ap.parse_args()
    if args.dt is None:
        args.dt = 1e-4 if args.workload == "rod64" else 1e-6
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the library is single-GPU; see the sharding notes)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2604_12083_amd as mrs

    assert torch.cuda.is_available(), "needs a GPU"
    if args.workload == "copy":
        # counter calibration: a plain device copy of 256 MiB (read 256 MiB, write 256 MiB) per launch
        nbytes = 256 << 20
        a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(args.warmup):
            b.copy_(a)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        print(json.dumps({"metric": "device copy GB/s (counter calibration)", "value": 2 * nbytes / dt / 1e9,
                          "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
                          "vs_baseline": None, "dtype": "f64", "data": "synthetic",
                          "config": {"workload": "copy of 256 MiB float64", "bytes_read": nbytes,
                                     "bytes_written": nbytes}}), flush=True)
        return
    if args.workload == "tune":
        sizes = (1536, 3200, 6400, 12800, 25600, 51200, 102400, 256000)
        rows = bench_tune(mrs, sizes)
        worst = max(r["ratio"] for r in rows)
        print(json.dumps({"metric": "pair-kernel tuner: tuned / automatic evaluation time, worst size",
                          "value": worst, "unit": "ratio", "n_gpus": 1, "steps": 7, "warmup": 1,
                          "ms_per_step": None, "higher_is_better": False, "scaling": "strong",
                          "vs_baseline": None, "dtype": "f32c+f64", "data": "synthetic",
                          "config": {"workload": "tuner: sinusoidal 128-point filaments, 1,536 to 256,000 points"},
                          "tune": rows}), flush=True)
        return
    if args.workload in ("slices", "serving", "parareal"):
        ctx = mrs.mrs_context_create(0)
        try:
            if args.workload == "parareal":
                r = {tag: bench_parareal(mrs, ctx, p, tol, 10) for tag, p, tol in
                     (("fp64", mrs.MRS_FP64, 1e-12), ("fp32c", mrs.MRS_FP32C, 1e-6))}
                r["schedules_fp32c"] = bench_schedules(mrs, ctx, mrs.MRS_FP32C)
                r["schedules_fp32c_rk2"] = bench_schedules(mrs, ctx, mrs.MRS_FP32C, integ="RK2")
                line = {"metric": "Parareal wall time on one GPU vs serial fine (32 filaments x 100 points, 16 slices)",
                        "value": r["fp32c"]["speedup_vs_serial"], "unit": "x", "n_gpus": 1, "steps": 3200,
                        "warmup": 1, "ms_per_step": 1e3 * r["fp32c"]["parareal_s"] / 3200,
                        "higher_is_better": True, "scaling": "strong", "vs_baseline": None, "dtype": "f32c",
                        "data": "synthetic",
                        "config": {"workload": "parareal: 32 filaments x 100 points (torques x 1e-2), 16 slices"},
                        "parareal": r}
            elif args.workload == "slices":
                r = bench_slices(mrs, ctx, args.steps, args)
                line = {"metric": METRIC, "value": r["batched_pairs_per_s"], "unit": "pairs/s", "n_gpus": 1,
                        "steps": args.steps, "warmup": args.warmup,
                        "ms_per_step": 1e3 * r["batched_graph_s"] / args.steps, "higher_is_better": True,
                        "scaling": "weak", "vs_baseline": None, "dtype": "f32c", "data": "synthetic",
                        "config": {"workload": "slices: 16 Parareal fine slices x (32 filaments x 100 points), "
                                               "RK4 dt=1e-5, batched + HIP graph vs plain per-slice launches"},
                        "slices": r}
            else:
                rates = [float(x) for x in args.rates.split(",")]
                r = bench_serving(mrs, ctx, args.requests, rates, args.slots, int(args.budget_gb * (1 << 30)),
                                  args.tick_pairs, ["arrival", "least-work"].index(args.admission), args.max_wait)
                best = r["batched"][str(rates[-1])]
                line = {"metric": METRIC, "value": best["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1,
                        "steps": args.requests, "warmup": 0, "ms_per_step": best["p50_ms"],
                        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32c",
                        "data": "synthetic",
                        "config": {"workload": f"serving: first {args.requests} requests of the serving sequence, "
                                               "Poisson arrivals, continuous batching"},
                        "serving": r}
        finally:
            mrs.mrs_context_destroy(ctx)
        print(json.dumps(line), flush=True)
        return
    e, desc, swim = workload(args.workload)
    # the swimming workload steps with the paper's fine propagator (RK2, 2 stages)
    integ, stages, step_name = ((mrs.MRS_RK2, 2, "midpoint RK2") if swim is not None else
                                (mrs.MRS_EULER, 1, "forward-Euler"))
    import torch

    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    ctx = mrs.mrs_context_create(0)
    try:
        pairs_step = stages * e.N * e.N
        res = {}
        for prec, tag in ((mrs.MRS_FP32C, "fp32c"), (mrs.MRS_FP64, "fp64")):
            log(f"measure {tag} N={e.N} steps={args.steps}")
            res[tag] = measure(mrs, ctx, e, prec, args.steps, args.warmup, args.dt, integ, swim)
            res[tag]["chunks"] = mrs.mrs_tune_get(ctx, e.N, prec)["chunks"]
            res[tag]["traffic"] = measured_traffic(mrs, args.workload, tag, e.N, prec, n_cu,
                                                   mrs.mrs_tune_get(ctx, e.N, prec)["schedule"])
        extra = args.workload == "ens12800" and not args.no_extra
        large = slices_leg = large_subset = copies_leg = None
        if extra:
            large, large_subset = bench_large(mrs, ctx, n_cu)
            log(f"16 slices x 3,200 points, {args.steps} RK4 steps: batched graph vs plain")
            slices_leg = bench_slices(mrs, ctx, args.steps, args)
            log("12,800-point pair kernel: 4 and 8 copies in one launch")
            copies_leg = bench_copies(mrs, ctx, e, args.dt)
        cpu, errs = (None, None)
        if not args.no_cpu:
            log("cpu baseline (oracle)")
            cpu, errs = cpu_baseline(mrs, ctx, e, [mrs.MRS_FP32C, mrs.MRS_FP64], swim, args.workload)
            if large_subset is not None:
                log("oracle on the 256,000-point check subset")
                cpu["large_subset"], large["max_rel_err_vs_oracle"] = oracle_large_subset(large_subset)
    finally:
        mrs.mrs_context_destroy(ctx)

    def summary(r, peak, tag):
        lat = np.array(r["lat_ms"])
        return {
            "value": args.steps * pairs_step / r["wall_s"],
            "ms_per_step": 1e3 * r["wall_s"] / args.steps,
            "ms_per_step_graph": 1e3 * r["wall_graph_s"] / args.steps,
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
            "roofline": roofline(e.N * e.N, r["kernel_avg_s"], peak, r["traffic"]),
            "source_chunks": r["chunks"],
            "settle_s": round(r["settle_s"], 3),
            "clock_mhz": r["clock_mhz"],
            "kernels_avg_us": {k: round(v["avg_us"], 2) for k, v in r["kernels"].items()},
            "frame_update_GBps": frame_update_gbps(e.N, r["kernels"], tag),
        }

    s32 = summary(res["fp32c"], PEAK_FP32_TFLOPS, "fp32c")
    s64 = summary(res["fp64"], PEAK_FP64_TFLOPS, "fp64")
    if cpu:
        cpu["gpu_over_oracle"] = {"fp32c": s32["value"] / cpu["value"], "fp64": s64["value"] / cpu["value"]}
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
        "config": {"workload": f"{args.workload}: {desc}; one {step_name} step ({stages} x (rod forces + MRS "
                               f"U/Omega) + frame update), dt={args.dt}",
                   "n_points": e.N, "pairs_per_step": pairs_step, "precision": "fp32c"},
        "latency_ms": s32["latency_ms"],
        "ms_per_step_graph": s32["ms_per_step_graph"],
        "kernels_avg_us": s32["kernels_avg_us"],
        "frame_update_GBps": s32["frame_update_GBps"],
        "roofline": s32["roofline"],
        "fp64": s64,
        "cpu_baseline": cpu,
        "max_rel_err_vs_oracle": errs,
        "finite": res["fp32c"]["finite"] and res["fp64"]["finite"],
        "settle_s": s32["settle_s"],
        "clock_mhz": s32["clock_mhz"],
    }
    if large is not None:
        line["large_256000"] = large
    if slices_leg is not None:
        line["slices_16x3200"] = slices_leg
        line["pairs_copies_12800"] = copies_leg
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
