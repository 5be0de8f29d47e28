"""Benchmark of the transient F-statistic map on one MI355X.

Default workload (the headline `value`): exponential window, 1 frequency
bin, 5000 slots of T_sft = 1800 s (about 104 days, 15% gaps), 1000 t0 values
at T_sft spacing by 1000 tau values from 2 T_sft to 30 days, FP32 data sums
with FP64 antenna sums (the plain method).  One step computes the full 2F
map (written to device memory) and the per-bin max 2F, argmax and logB, with
the atoms already resident on the device.

Metric: cells*SFTs/s, where a cell's count is the number of SFTs present in
its window, truncated at the data end (the paper's N_sums of appendix A,
eq. Nsums-exp, counted over present SFTs).

The same JSON line also carries, unless --no-extras:
  exp_256_bins   256 bins sharing one set of antenna atoms, split hi + lo
                 half-precision (f16x3) and bf16 (bf16x3) parts on matrix
                 cores against the plain FP32 form, each with its 2F error
                 against the oracle on sampled cells;
  uneven_batch   64 uneven candidates as one batch (one captured graph, one
                 persistent fused launch, the matrix-core launch) in FP32,
                 F16X3 and BF16X3, against one map per call;
  serving        a Poisson request stream (F16X3 requests) with continuous
                 batching, p50/p99, a load ramp and the sequential plain FP32
                 baseline;
  cpu_baseline   the FP64 oracle on the host cores (all threads and one).

Prints ONE JSON line.  Options:
  --gpus N       only 1 is supported (the path runs on one GPU)
  --steps K      timed steps (default 20)
  --warmup W     untimed steps (default 3; continued until 0.3 s of untimed
                 work has run, so that the timed steps see settled clocks)
  --workload     exp1bin (default) | exp256 | rect | rect256 | batch
  --prec         fp32 (default) | fp64 | f16x3 | bf16x3 | recur64
  --no-extras, --no-cpu-baseline, --serve-seconds S (0 skips serving)
"""
from __future__ import annotations

import argparse
import contextlib
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import tfsynth  # noqa: E402

T = tfsynth.T_SFT
PEAK_ALU_TFLOPS = 78.6    # non-packed FP32 and FP64 vector FMA, 256 CU x 64 lanes x 2 x 2.4 GHz
PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0  # dense bf16 and fp16 matrix cores
MATRIX_PRECS = ("f16x3", "bf16x3")
DTYPES = {"fp32": "f32+f64", "fp64": "f64", "bf16x3": "bf16x3(f32 acc)+f64", "f16x3": "f16x3(f32 acc)+f64",
          "recur64": "f64"}


def mfma_taus(atoms, win, prec="bf16x3", taus_per_block: int = 8, min_band: int = 64, min_bins: int = 2):
    """Boolean mask of the taus whose sums run on the matrix cores in
    F16X3 or BF16X3 -- the library's planning rule restated: exponential
    windows of at least 2 bins with a block of 8 consecutive taus whose
    shortest band (the slots of [t0, t0 + 3 tau) over the row with the
    largest offset from the slot grid, capped at the data end) is at least
    64 slots; the matrix cores take the blocks whose shortest band is at
    least 64 slots (BF16X3) or 24 slots (F16X3)."""
    keep = np.zeros(win.n_tau, dtype=bool)
    if win.kind != "exp" or atoms.n_bins < min_bins:
        return keep
    T_ = atoms.t_sft
    T0 = int(atoms.timestamps[0])
    k0 = -(-(win.t0 - T0) // T_)
    delta = T0 + k0 * T_ - win.t0
    cap = max(0, atoms.n_slots - int(min(k0.min(), atoms.n_slots)))
    span = 3 * win.tau
    dmax = int(delta.max())
    lcol = np.where(span > dmax, -(-(span - dmax) // T_), 0)
    lcol = np.minimum(lcol, cap)
    long_block = False
    for b0 in range(0, win.n_tau, taus_per_block):
        if lcol[b0:b0 + taus_per_block].min() >= min_band:
            long_block = True
    if not long_block:
        return keep
    band = 24 if prec == "f16x3" else min_band
    for b0 in range(0, win.n_tau, taus_per_block):
        if lcol[b0:b0 + taus_per_block].min() >= band:
            keep[b0:b0 + taus_per_block] = True
    return keep


def mfma_cells(atoms, win, prec="bf16x3"):
    """cells*present SFTs*bins of the tau blocks that run on the matrix
    cores (the others run on the VALU)."""
    keep = mfma_taus(atoms, win, prec)
    if not keep.any():
        return 0
    sub = tfsynth.Window(win.kind, win.t0, win.tau[keep])
    return work_counts(atoms, sub)[0]


def split_form(atoms, win, prec):
    """Whether the library plans this exponential map in the split form (A/B/C
    pass, then F_a, F_b only): FP32, at least 8 bins, and a median slot span
    of its 64-row tiles within the band stage (448 slots) -- the library's
    default rule, restated to count the fused kernel's own flops."""
    if prec != "fp32" or atoms.n_bins < 8:
        return False
    T0 = int(atoms.timestamps[0])
    k0 = np.minimum(-(-(win.t0 - T0) // atoms.t_sft), atoms.n_slots)
    spans = [int(k0[min(s + 63, len(k0) - 1)] - k0[s]) for s in range(0, len(k0), 64)]
    return sorted(spans)[len(spans) // 2] <= 448


def work_counts(atoms, win):
    """(cells*present SFTs, cells*slots) summed over bins: each cell counts
    the SFT start times in [t0, t0 + span) with span = tau (rect) or 3 tau
    (exp), truncated at the end of the data."""
    ts = atoms.timestamps
    T0 = int(ts[0])
    t_end = T0 + atoms.t_data
    span = win.tau if win.kind == "rect" else 3 * win.tau
    present = 0
    slots = 0
    for t0 in win.t0.tolist():
        ends = t0 + span
        present += int((np.searchsorted(ts, ends, "left") - np.searchsorted(ts, t0, "left")).sum())
        s_lo = min(max(0, -(-(t0 - T0) // atoms.t_sft)), atoms.n_slots)
        s_hi = np.minimum(-(-(np.minimum(ends, t_end) - T0) // atoms.t_sft), atoms.n_slots)
        slots += int(np.maximum(s_hi - s_lo, 0).sum())
    return present * atoms.n_bins, slots * atoms.n_bins


WORKLOADS = {
    "exp1bin": ("exp window, 1 bin, 5000 slots (15% gaps), 1000 t0 x 1000 tau "
                "(2 T_sft .. 30 d), T_sft = 1800 s", tfsynth.workload_exp_1bin),
    "exp256": ("exp window, 256 bins sharing a,b, 2000 slots (10% gaps), 500 t0 x 500 tau "
               "(2 .. 501 T_sft)", tfsynth.workload_exp_bins),
    "rect": ("rect window, 1 bin, 200 slots (10% gaps), 100 t0 x 199 tau", tfsynth.workload_rect_small),
}


def make_workload(name):
    if name == "rect256":
        atoms, _ = tfsynth.workload_exp_bins()
        win = tfsynth.regular_window("rect", 0, T, 500, 2 * T, T, 500)
        return "rect window, 256 bins, 2000 slots (10% gaps), 500 t0 x 500 tau", atoms, win
    desc, fn = WORKLOADS[name]
    atoms, win = fn()
    return desc, atoms, win


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(atoms, win, threads: int, budget_s: float):
    """cells*present SFTs/s of the FP64 oracle with `threads` threads over an
    evenly spaced sample of t0 rows sized to about budget_s of CPU time."""
    import oracle
    probe_rows = max(1, min(win.n_t0, max(8, threads)))
    sub = tfsynth.Window(win.kind, win.t0[:probe_rows], win.tau)
    t = time.perf_counter()
    oracle.fmap_atoms(atoms, sub, threads)
    dt = max(time.perf_counter() - t, 1e-6)
    rows = int(min(win.n_t0, max(probe_rows, probe_rows * budget_s / threads / dt)))
    rows = max(threads, rows - rows % threads) if rows >= threads else rows
    rows = min(rows, win.n_t0)
    idx = np.linspace(0, win.n_t0 - 1, rows).round().astype(int)
    sample = tfsynth.Window(win.kind, win.t0[np.unique(idx)], win.tau)
    present, _ = work_counts(atoms, sample)
    t = time.perf_counter()
    oracle.fmap_atoms(atoms, sample, threads)
    dt = time.perf_counter() - t
    return present / dt, sample.n_t0, dt


def cpu_baseline(atoms, win, budget_s: float = 20.0):
    """The FP64 oracle on the host cores over a bounded sample of t0 rows:
    all threads (the reported value) and one thread."""
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    rate, rows, dt = _oracle_rate(atoms, win, threads, budget_s)
    rate1, rows1, dt1 = _oracle_rate(atoms, win, 1, min(budget_s, 8.0))
    return {"value": rate, "unit": "cells*SFTs/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": "%d of %d t0 rows (evenly spaced) x all %d tau, all %d bins; %.1f s wall"
                      % (rows, win.n_t0, win.n_tau, atoms.n_bins, dt),
            "single_thread": {"value": rate1, "unit": "cells*SFTs/s", "cores": 1,
                              "sample": "%d t0 rows x all %d tau; %.1f s wall" % (rows1, win.n_tau, dt1)}}


def traffic_from_profile(workload: str, kernel_file: str, variant=None):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, each scaled by a
    plain copy's reading), or None when the counters are missing, the
    kernel source changed since they were taken, or they were taken on
    another build variant of the kernel."""
    import hashlib
    meta = os.path.join(ROOT, "profiles", kernel_file + "_" + workload + ".json")
    if not os.path.exists(meta):
        return None
    m = json.load(open(meta))
    src = os.path.join(ROOT, "paper_1805_05652_amd", "csrc", m.get("source", "kernels.hip"))
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != m["kernels_source_sha256"]:
        return None
    if variant is not None and m.get("variant") != variant:
        return None
    return m["traffic_bytes_per_launch"]


def _percentiles(lat_ms):
    return float(np.percentile(lat_ms, 50)), float(np.percentile(lat_ms, 99))


def serving(ctx, seed: int = 4000, rate_hz: float = 200.0, duration_s: float = 15.0,
            precision: str = "f16x3", pool: int = 400, ramp=(300.0, 500.0, 700.0, 900.0, 1100.0, 1300.0),
            ramp_s: float = 4.0):
    """Served maps: a Poisson stream of map requests over resident atoms.

    Requests (slots log-uniform [200, 10000], grids U{100..2000}^2, 1..64
    bins, window type random, linspace grids) arrive at `rate_hz` for
    `duration_s`.  Their atoms come from a pool of `pool` resident candidates
    (request i uses candidate i mod pool, drawn from the same distribution),
    each request with its own grid and window type.  Requests are submitted
    at their arrival times and polled; latency is arrival to observed
    completion.  Streams: the offered rate with continuous batching (up to
    16 requests per launch); the first requests with one request per slot; a
    ramp of offered rates (each `ramp_s` long) up to the highest sustained
    one; every request of the first 1000 at t = 0 (the loop's capacity).  The
    baseline runs the same requests one after another through tfstat_fmap in
    plain FP32 and derives FIFO latencies from the measured service times and
    the same arrivals."""
    reqs = tfsynth.request_stream(seed, rate_hz, duration_s)
    pool_atoms = []
    for r in reqs[:pool]:
        atoms = tfsynth.make_atoms(r["seed"], r["n_slots"], 0.10, r["n_bins"])
        pool_atoms.append((ctx.upload_atoms(atoms), atoms.n_bins, atoms))
    jobs = []
    for i, r in enumerate(reqs):
        aid, nb, atoms = pool_atoms[i % len(pool_atoms)]
        jobs.append((r["arrival"], aid, tfsynth.request_window(atoms, r), nb))
    pool_atoms = [(aid, nb) for aid, nb, _ in pool_atoms]
    ctx.fmap(jobs[0][1], jobs[0][2], precision)   # warm the kernels

    def run_stream(sel, max_batch, stretch=1.0):
        ctx.serve_config(max_batch)
        t_start = time.perf_counter() + 0.05
        pending = {}
        lat = []
        i = 0
        while i < len(sel) or pending:
            now = time.perf_counter() - t_start
            while i < len(sel) and stretch * sel[i][0] <= now:
                arr, aid, win, nb = sel[i]
                pending[ctx.submit(aid, win, precision)] = (arr, nb)
                i += 1
            for t, (arr, nb) in list(pending.items()):
                if ctx.poll(t, nb) is not None:
                    lat.append(time.perf_counter() - t_start - stretch * arr)
                    del pending[t]
            if not pending and i < len(sel):
                time.sleep(max(0.0, min(0.0005, stretch * sel[i][0] - (time.perf_counter() - t_start))))
        return time.perf_counter() - t_start, np.array(lat) * 1e3

    wall, lat = run_stream(jobs, 16)
    first = [j for j in jobs if j[0] < 5.0]
    wall1, lat1 = run_stream(first, 1)
    ramp_out = []
    for r in ramp:
        sel = [j for j in jobs if j[0] * rate_hz / r < ramp_s]
        w, l = run_stream(sel, 16, stretch=rate_hz / r)
        served = len(sel) / w
        p50, p99 = _percentiles(l)
        ramp_out.append({"offered_rate_hz": r, "requests": len(sel), "maps_per_s": served,
                         "p50_ms": p50, "p99_ms": p99})
        if served < 0.9 * r:
            break
    sustained = [x["offered_rate_hz"] for x in ramp_out if x["maps_per_s"] >= 0.95 * x["offered_rate_hz"]]
    cap = jobs[:1000]
    wall_c, _ = run_stream(cap, 16, stretch=0.0)
    # sequential plain FP32 baseline on the same requests
    svc = []
    for arr, aid, win, nb in jobs:
        t0 = time.perf_counter()
        ctx.fmap(aid, win, "fp32")
        svc.append(time.perf_counter() - t0)
    free_at = 0.0
    seq_lat = []
    for (arr, _, _, _), sv in zip(jobs, svc):
        start = max(arr, free_at)
        free_at = start + sv
        seq_lat.append(free_at - arr)
    for aid, _ in pool_atoms:
        ctx.free(aid)
    seq_lat = np.array(seq_lat) * 1e3
    p50, p99 = _percentiles(lat)
    p50_1, p99_1 = _percentiles(lat1)
    sp50, sp99 = _percentiles(seq_lat)
    return {
        "requests": len(jobs), "offered_rate_hz": rate_hz, "duration_s": duration_s,
        "precision": precision, "admission": "continuous batching, up to 16 requests per fused launch",
        "maps_per_s": len(jobs) / wall,
        "bin_maps_per_s": sum(j[3] for j in jobs) / wall,
        "p50_ms": p50, "p99_ms": p99, "tail_samples_above_p99": int((lat > p99).sum()),
        "ramp": ramp_out,
        "max_sustained_offered_hz": max([rate_hz] + sustained) if len(jobs) / wall >= 0.95 * rate_hz
        else None,
        "all_at_once": {"requests": len(cap), "maps_per_s": len(cap) / wall_c,
                        "bin_maps_per_s": sum(j[3] for j in cap) / wall_c},
        "one_request_per_slot": {"requests": len(first), "maps_per_s": len(first) / wall1,
                                 "p50_ms": p50_1, "p99_ms": p99_1},
        "sequential_fp32": {"maps_per_s": len(jobs) / sum(svc),
                            "service_s_by_window": {
                                k: float(sum(sv for (_, _, w, _), sv in zip(jobs, svc) if w.kind == k))
                                for k in ("rect", "exp")},
                            "p50_ms": sp50, "p99_ms": sp99},
        "workload": "Poisson %.0f/s for %.0f s (%d requests) over %d resident candidates; slots "
                    "log-uniform [200, 10000], grids U{100..2000}, bins U{1..64}, rect or exp at "
                    "random, linspace grids" % (rate_hz, duration_s, len(jobs), len(pool_atoms)),
    }


def sampled_error(twoF, res, atoms, win, n_cells: int, seed: int):
    """Largest relative 2F error, |2F_gpu - 2F_oracle| / max(2F_oracle, 1), of a
    device map over n_cells random cells plus every bin's argmax cell,
    against the FP64 oracle at those cells."""
    import oracle
    import torch
    rng = np.random.default_rng(seed)
    mi = np.concatenate([rng.integers(0, win.n_t0, n_cells), [r["m"] for r in res]]).astype(np.int32)
    ni = np.concatenate([rng.integers(0, win.n_tau, n_cells), [r["n"] for r in res]]).astype(np.int32)
    ref = oracle.cells_atoms(atoms, win, mi, ni)
    got = twoF[:, torch.from_numpy(mi.astype(np.int64)).to(twoF.device),
               torch.from_numpy(ni.astype(np.int64)).to(twoF.device)].cpu().numpy().astype(np.float64)
    return float((np.abs(got - ref) / np.maximum(np.abs(ref), 1.0)).max()), int(mi.shape[0])


def roofline_for(atoms, win, prec, prof, workload):
    """Roofline of the dominant kernel of one map computation from the
    per-kernel HIP-event times of the timed steps."""
    mfma = win.kind == "exp" and prec in MATRIX_PRECS and prof["mfma"][0] > 0
    recur = win.kind == "exp" and prec == "recur64" and prof["recur"][0] > 0
    dom = "mfma" if mfma else ("recur" if recur else ("exp" if win.kind == "exp" else "rect"))
    n_launch, k_ms = prof[dom]
    avg_ms = k_ms / max(n_launch, 1)
    present, _ = work_counts(atoms, win)
    if recur:
        # FP64 flops of the recurrence: the boundary window per tau (w^2 and
        # one FMA per antenna and data channel per slot), two passes per row
        # of (scale + head FMA + tail FMA) per channel, and the finalize
        # (about 30 flops per cell and bin)
        ch = 3 + 4 * atoms.n_bins
        band = np.minimum(-(-3 * win.tau // atoms.t_sft), atoms.n_slots)
        flops = float((band * (1 + 2 * ch)).sum()) + win.n_tau * win.n_t0 * (2 * 5 * ch + 30 * atoms.n_bins)
        roof = {"bound": "alu", "achieved": flops / (avg_ms * 1e-3) / 1e12, "peak": PEAK_ALU_TFLOPS,
                "unit": "TFLOP/s"}
    elif mfma:
        # 4 complex-by-real MACs = 8 flops per cell*SFT*bin, issued as three
        # half-precision or bf16 products (hi*hi + hi*lo + lo*hi): 24
        # matrix-core flops, counted over the tau blocks the matrix-core
        # kernel runs
        long_cells = mfma_cells(atoms, win, prec)
        flops = 24.0 * long_cells
        roof = {"bound": "mfma", "achieved": flops / (avg_ms * 1e-3) / 1e12, "peak": PEAK_BF16_TFLOPS,
                "unit": "TFLOP/s", "cells_sfts_bins": long_cells}
    elif win.kind == "exp":
        # 4 FMA (F_a, F_b) per cell*SFT*bin + 3 FP64 FMA (A, B, C) per cell*SFT
        # per group of bins sharing a lane; in the split form the A/B/C pass
        # is its own kernel and the dominant one sums F_a, F_b only
        bg = 1 if (prec == "fp64" or atoms.n_bins == 1) else (4 if atoms.n_bins >= 4 else 2)
        cells = present // atoms.n_bins
        split = prof["abc"][0] > 0
        flops = 8.0 * present + (0.0 if split else 6.0 * cells * ((atoms.n_bins + bg - 1) // bg))
        roof = {"bound": "alu", "achieved": flops / (avg_ms * 1e-3) / 1e12, "peak": PEAK_ALU_TFLOPS,
                "unit": "TFLOP/s"}
    else:
        # the map write: 4 bytes per cell*bin
        byts = 4.0 * atoms.n_bins * win.n_t0 * win.n_tau
        roof = {"bound": "hbm", "achieved": byts / (avg_ms * 1e-3) / 1e9, "peak": PEAK_HBM_GBS,
                "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = traffic_from_profile(workload, {"exp": "exp_valu", "rect": "rect",
                                                      "mfma": "exp_mfma", "recur": "exp_recur"}[dom],
                                           prec if mfma else None)
    roof["kernel"] = dom
    roof["kernel_avg_ms"] = avg_ms
    return roof


@contextlib.contextmanager
def no_gc():
    """Python's cyclic collector paused over a timed region (collected
    first), so that a collection pass does not land inside one step."""
    gc.collect()
    gc.disable()
    try:
        yield
    finally:
        gc.enable()


SETTLE_S = 0.3   # untimed work before the timed steps, so that the clocks have ramped


def settle(step, warmup):
    """The `warmup` untimed steps, continued until SETTLE_S seconds have
    passed: a cold GPU runs its first milliseconds of work at lower clocks."""
    import torch
    t = time.perf_counter()
    n = 0
    while n < warmup or (time.perf_counter() - t < SETTLE_S and n < 100000):
        step()
        n += 1
        if n % 16 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()


def time_map(ctx, aid, atoms, win, prec, twoF, steps, warmup, workload):
    """Times `steps` calls of tfstat_fmap (map written to twoF when given)
    after `warmup` untimed ones (at least SETTLE_S seconds of them);
    per-kernel device times from HIP events."""
    import torch
    res = None
    ctx.profile(True)
    # the collector's pass happens before the warmup, so that no idle gap
    # (clocks fall back within tens of milliseconds) separates the warmup
    # from the timed steps
    with no_gc():
        settle(lambda: ctx.fmap(aid, win, prec, out=twoF), warmup)
        ctx.profile_reset()
        t0 = time.perf_counter()
        for _ in range(steps):
            res, _ = ctx.fmap(aid, win, prec, out=twoF)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    ctx.profile(False)
    prof = ctx.profile_read()
    ms = (t1 - t0) * 1e3 / steps
    present, _ = work_counts(atoms, win)
    return {"ms_per_step": ms, "value": present / (ms * 1e-3), "res": res,
            "roofline": roofline_for(atoms, win, prec, prof, workload),
            "kernels_ms": {k: (v[1] / v[0] if v[0] else None) for k, v in prof.items()}}


def bench_exp256(args, tf, torch):
    """256 frequency bins sharing one set of antenna atoms (2000 slots, 10%
    gaps, 500 x 500 grid, map written): the batched mixed-precision forms
    (split hi + lo half-precision or bf16 parts on matrix cores, FP32
    accumulation, A/B/C/D in FP64) against the plain FP32 VALU form, each
    with its largest 2F error against the FP64 oracle on sampled cells."""
    atoms, win = tfsynth.workload_exp_bins()
    present, slots = work_counts(atoms, win)
    ctx = tf.Context(0, arena_bytes=2 << 30)
    aid = ctx.upload_atoms(atoms)
    twoF = torch.empty((atoms.n_bins, win.n_t0, win.n_tau), dtype=torch.float32, device="cuda:0")
    out = {"workload": "exp window, 256 bins sharing a,b, 2000 slots (10% gaps), 500 t0 x 500 tau "
                       "(2 .. 501 T_sft), map written",
           "cells_sfts_bins": present, "cells_slots_bins": slots, "unit": "cells*SFTs*bins/s"}
    for prec in ("f16x3", "bf16x3", "fp32"):
        r = time_map(ctx, aid, atoms, win, prec, twoF, args.steps, args.warmup, "exp256")
        err, n = sampled_error(twoF, r["res"], atoms, win, 2000, 2561)
        out[prec] = {"ms_per_step": r["ms_per_step"], "value": r["value"], "roofline": r["roofline"],
                     "kernels_ms": r["kernels_ms"],
                     "max_rel_err_2F_vs_oracle": err,
                     "oracle_cells_compared": "%d cells x 256 bins (random + each bin's argmax)" % n}
    for prec in MATRIX_PRECS:
        out["speedup_%s_vs_fp32" % prec] = out["fp32"]["ms_per_step"] / out[prec]["ms_per_step"]
    ctx.free(aid)
    ctx.close()
    return out


def bench_batch(args, tf, torch, prec):
    """The uneven batch: 64 follow-up candidates (slots log-uniform in
    [500, 8000], gaps U[0, 0.3], grids U{100..1500}^2, 1..16 bins, rect and
    exp alternating) as one planned batch -- one captured graph with one
    persistent fused launch per step (and, in F16X3 / BF16X3, one matrix-core
    launch for the exponential maps of 2 or more bins) -- against the same
    maps computed one map per call.  Returns the record of the step."""
    cands = [tfsynth.candidate(i) for i in range(64)]
    exp_present = exp_slots = rect_cells = 0
    abc_cells_sfts = 0   # A/B/C inside the fused kernel (not split-form or matrix-core maps)
    valu_present = 0     # exp cells*SFTs*bins summed on the VALU
    mfma_present = 0     # exp cells*SFTs*bins on the matrix cores
    for a, w in cands:
        if w.kind == "exp":
            p, sl = work_counts(a, w)
            exp_present += p
            exp_slots += sl
            mc = mfma_cells(a, w, prec) if prec in MATRIX_PRECS else 0
            mfma_present += mc
            valu_present += p - mc
            if not split_form(a, w, "fp32" if prec in MATRIX_PRECS else prec) and mc == 0:
                abc_cells_sfts += p // a.n_bins
        else:
            rect_cells += w.n_t0 * w.n_tau * a.n_bins
    ctx = tf.Context(0, arena_bytes=24 << 30)
    ids = [ctx.upload_atoms(a) for a, _ in cands]
    items = list(zip(ids, [w for _, w in cands]))
    t = time.perf_counter()
    batch = ctx.batch(items, prec, tune=not args.no_tune)
    plan_s = time.perf_counter() - t
    step_ms, step_graph_ms = [], []
    with no_gc():
        settle(batch.run, args.warmup)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ts = time.perf_counter()
            res = batch.run()
            step_ms.append((time.perf_counter() - ts) * 1e3)
            step_graph_ms.append(batch.stats()["last_ms"])
        t1 = time.perf_counter()
    st = batch.stats()
    ms = (t1 - t0) * 1e3 / args.steps
    # the fused kernel and the matrix-core launch alone, timed with HIP
    # events on their stream (direct launches)
    fused, mm = [], []
    for _ in range(3):
        timed = batch.run(timed=True)
        fused.append(batch.stats()["last_fused_ms"])
        mm.append(batch.stats()["last_mfma_ms"])
    # one map per call: the same maps, sequentially, plain launches
    for aid, w in items[:4]:
        ctx.fmap(aid, w, prec)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    seq = [ctx.fmap(aid, w, prec)[0] for aid, w in items]
    torch.cuda.synchronize()
    seq_ms = (time.perf_counter() - ts) * 1e3
    same = all(r1 == r2 for a, b in zip(res, seq) for r1, r2 in zip(a, b))
    same = same and timed == res
    # every map's 2F against the oracle on sampled cells (the maps of the
    # single-map path, whose results the batch reproduces bit for bit)
    err = 0.0
    n_cmp = 0
    for i, ((a, w), aid) in enumerate(zip(cands, ids)):
        r, twoF = ctx.fmap(aid, w, prec, want_map=True)
        e, n = sampled_error(twoF, r, a, w, 64, 3100 + i)
        err = max(err, e)
        n_cmp += n * a.n_bins
        del twoF
    fused_ms = float(np.mean(fused))
    mfma_ms = float(np.mean(mm))
    # algorithmic flops of the fused kernel: 4 FMA per exp cell*SFT*bin summed
    # there, 3 FP64 FMA (A, B, C) per exp cell*SFT of the maps whose A, B, C it
    # sums (split-form and matrix-core maps have theirs from the pre-pass
    # launch), about 30 FP64 flops per rect cell*bin
    flops = 8.0 * valu_present + 6.0 * abc_cells_sfts + 30.0 * rect_cells
    roof_f = {"bound": "alu", "achieved": flops / (fused_ms * 1e-3) / 1e12, "peak": PEAK_ALU_TFLOPS,
              "unit": "TFLOP/s", "kernel": "fused", "kernel_avg_ms": fused_ms,
              "traffic": traffic_from_profile("batch_" + prec, "fused", st["variant"])}
    roof_f["frac"] = roof_f["achieved"] / roof_f["peak"]
    roof = roof_f
    out = {
        "workload": "uneven batch: 64 candidates, 32 exp + 32 rect maps, 1-16 bins",
        "value": exp_present / (ms * 1e-3), "unit": "cells*SFTs*bins/s", "ms_per_step": ms,
        "precision": prec,
        "exp_cells_sfts_bins": exp_present, "exp_cells_slots_bins": exp_slots,
        "rect_cells_bins": rect_cells, "maps": len(cands), "bin_maps": st["n_results"],
        "variant": st["variant"], "groups": st["groups"], "tiles": st["n_tiles"],
        "tune_ms": st["tune_ms"], "plan_s": plan_s, "graph_ms": st["last_ms"],
        "step_ms": [round(x, 3) for x in step_ms],
        "step_graph_ms": [round(x, 3) for x in step_graph_ms],
        "sequential_ms": seq_ms, "speedup_vs_sequential": seq_ms / ms,
        "results_equal_sequential": bool(same),
        "max_rel_err_2F_vs_oracle": err,
        "oracle_cells_compared": "%d cell-bins (64 random cells + each bin's argmax, every map)" % n_cmp,
    }
    if prec in MATRIX_PRECS:
        # the matrix-core launch: 24 matrix-core flops per cell*SFT*bin it sums
        roof_m = {"bound": "mfma", "achieved": 24.0 * mfma_present / (mfma_ms * 1e-3) / 1e12,
                  "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s", "kernel": "mfma_batch",
                  "kernel_avg_ms": mfma_ms, "cells_sfts_bins": mfma_present,
                  "traffic": traffic_from_profile("batch_" + prec, "mfma_batch", prec)}
        roof_m["frac"] = roof_m["achieved"] / roof_m["peak"]
        out["roofline_fused"] = roof_f
        out["roofline_mfma"] = roof_m
        roof = roof_m if mfma_ms >= fused_ms else roof_f
    out["roofline"] = roof
    batch.close()
    for aid in ids:
        ctx.free(aid)
    ctx.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="exp1bin",
                    choices=["exp1bin", "exp256", "rect", "rect256", "batch"])
    ap.add_argument("--no-tune", action="store_true", help="batch: default launch width")
    ap.add_argument("--no-alternatives", action="store_true",
                    help="skip timing the recurrence form of the same map")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline only: skip the 256-bin and uneven-batch records")
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp64", "f16x3", "bf16x3", "recur64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-map", action="store_true",
                    help="do not write the 2F map (per-bin results only)")
    ap.add_argument("--serve-seconds", type=float, default=15.0,
                    help="length of the served request stream (0 skips it)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-prec", default="f16x3", choices=["fp32", "fp64", "f16x3", "bf16x3", "recur64"])
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="instead of the map, time a plain device-to-device copy of this many "
                         "bytes (calibrates HBM byte counters)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py: this path runs on one GPU; --gpus %d is not supported (use --gpus 1)"
              % args.gpus, file=sys.stderr)
        return 2

    import torch
    import paper_1805_05652_amd as tf

    if args.copy_bytes:
        n = args.copy_bytes // 4
        src = torch.rand(n, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(args.warmup):
            dst.copy_(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        print(json.dumps({"copy_bytes": 4 * n, "ms_per_copy": ms,
                          "GBps_read_plus_write": 8 * n / (ms * 1e-3) / 1e9}), flush=True)
        return 0

    metric = "F-map cells*SFTs/s (exp window) and served maps/s with p50/p99 latency"
    if args.workload == "batch":
        if args.prec not in ("fp32", "fp64", "f16x3", "bf16x3"):
            print("bench.py: the batch runs in fp32, fp64, f16x3 or bf16x3", file=sys.stderr)
            return 2
        b = bench_batch(args, tf, torch, args.prec)
        out = {"metric": metric, "value": b.pop("value"), "unit": b.pop("unit"), "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup, "settle_s": SETTLE_S,
               "ms_per_step": b.pop("ms_per_step"),
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": DTYPES[args.prec],
               "data": "synthetic",
               "roofline": b.pop("roofline"),
               "config": {"workload": b.pop("workload"), "parallelism": "single GPU"}, "batch": b}
        print(json.dumps(out), flush=True)
        return 0

    desc, atoms, win = make_workload(args.workload)
    present, slots = work_counts(atoms, win)
    ctx = tf.Context(0, arena_bytes=(24 << 30) if args.serve_seconds > 0 else (4 << 30))
    aid = ctx.upload_atoms(atoms)
    twoF = None if args.no_map else torch.empty((atoms.n_bins, win.n_t0, win.n_tau),
                                                  dtype=torch.float32, device="cuda:0")
    r = time_map(ctx, aid, atoms, win, args.prec, twoF, args.steps, args.warmup, args.workload)
    out = {
        "metric": metric,
        "value": r["value"],
        "unit": "cells*SFTs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle_s": SETTLE_S,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[args.prec],
        "data": "synthetic",
        "config": {"workload": desc, "n_slots": atoms.n_slots, "n_sft": atoms.n_sft,
                   "n_t0": win.n_t0, "n_tau": win.n_tau, "n_bins": atoms.n_bins,
                   "window": win.kind, "precision": args.prec, "cells_sfts": present,
                   "cells_slots": slots, "map_written": not args.no_map,
                   "parallelism": "single GPU"},
        "roofline": r["roofline"],
        "kernels_ms": r["kernels_ms"],
        "result_bin0": r["res"][0],
    }
    if twoF is not None and args.workload != "rect256":
        err, n = sampled_error(twoF, r["res"], atoms, win, 2000, 1001)
        out["max_rel_err_2F_vs_oracle"] = err
        out["oracle_cells_compared"] = "%d cells x %d bins (random + each bin's argmax)" % (n, atoms.n_bins)
    if win.kind == "exp" and args.prec == "fp32" and not args.no_alternatives:
        # the same map by the O(1)-per-cell recurrence (all FP64), for context
        for _ in range(2):
            ctx.fmap(aid, win, "recur64", out=twoF)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            rres, _ = ctx.fmap(aid, win, "recur64", out=twoF)
        torch.cuda.synchronize()
        rms = (time.perf_counter() - t0) * 1e3 / args.steps
        out["alternatives"] = {"recur64": {"ms_per_step": rms, "value": present / (rms * 1e-3),
                                           "max2F_bin0": rres[0]["max2F"], "logB_bin0": rres[0]["logB"]}}
    ctx.free(aid)
    if args.workload == "exp1bin" and not args.no_extras:
        ctx.close()
        out["exp_256_bins"] = bench_exp256(args, tf, torch)
        ub = {p: bench_batch(args, tf, torch, p) for p in ("fp32",) + MATRIX_PRECS}
        for p in MATRIX_PRECS:
            ub["speedup_%s_vs_fp32" % p] = ub["fp32"]["ms_per_step"] / ub[p]["ms_per_step"]
        out["uneven_batch"] = ub
        ctx = tf.Context(0, arena_bytes=24 << 30)
    if args.serve_seconds > 0:
        out["serving"] = serving(ctx, rate_hz=args.serve_rate, duration_s=args.serve_seconds,
                                 precision=args.serve_prec)
    ctx.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(atoms, win)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
