"""Benchmark of the transient F-statistic map on one MI355X.

Default workload: exponential window, 1 frequency bin, 5000 slots of
T_sft = 1800 s (about 104 days, 15% gaps), 1000 t0 values at T_sft spacing by
1000 tau values from 2 T_sft to 30 days, FP32 data sums with FP64 antenna
sums (the plain method).  One step computes the full 2F map (written to
device memory) and the per-bin max 2F, argmax and logB, with the atoms
already resident on the device.

Metric: cells*SFTs/s, where a cell's count is the number of SFTs present in
its window, truncated at the data end (the paper's N_sums of appendix A,
eq. Nsums-exp, counted over present SFTs).

Prints ONE JSON line.  Options:
  --gpus N       only 1 is supported (the path runs on one GPU)
  --steps K      timed steps (default 20)
  --warmup W     untimed steps (default 3)
  --workload     exp1bin (default) | exp256 | rect | rect256
  --prec         fp32 (default) | fp64
  --no-cpu-baseline   skip timing the CPU oracle
"""
from __future__ import annotations

import argparse
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
PEAK_BF16_TFLOPS = 2500.0  # dense bf16 matrix cores


def mfma_cells(atoms, win, taus_per_block: int = 8, min_band: int = 64):
    """cells*present SFTs*bins of the tau blocks long enough for the matrix
    cores (blocks of 8 consecutive taus whose longest band, in slots, is at
    least 64; shorter ones run on the VALU).  Rows must start on slots."""
    T_ = atoms.t_sft
    span = 3 * win.tau
    lcol = -(-span // T_)
    keep = np.zeros(win.n_tau, dtype=bool)
    for b0 in range(0, win.n_tau, taus_per_block):
        if lcol[b0:b0 + taus_per_block].max() >= min_band:
            keep[b0:b0 + taus_per_block] = True
    sub = tfsynth.Window(win.kind, win.t0, win.tau[keep])
    return work_counts(atoms, sub)[0]


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


def cpu_baseline(atoms, win, budget_s: float = 20.0):
    """The FP64 oracle on the host cores over a bounded sample of t0 rows."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    # size the sample from a short probe
    probe_rows = max(1, min(win.n_t0, 8))
    sub = tfsynth.Window(win.kind, win.t0[:probe_rows], win.tau)
    t = time.perf_counter()
    oracle.fmap_atoms(atoms, sub, threads)
    dt = max(time.perf_counter() - t, 1e-6)
    # budget_s is CPU time (wall time x threads)
    rows = int(min(win.n_t0, max(probe_rows, probe_rows * budget_s / threads / dt)))
    rows = max(threads, rows - rows % threads) if rows >= threads else rows
    rows = min(rows, win.n_t0)
    idx = np.linspace(0, win.n_t0 - 1, rows).round().astype(int)
    sample = tfsynth.Window(win.kind, win.t0[np.unique(idx)], win.tau)
    present, _ = work_counts(atoms, sample)
    t = time.perf_counter()
    oracle.fmap_atoms(atoms, sample, threads)
    dt = time.perf_counter() - t
    return {"value": present / dt, "unit": "cells*SFTs/s", "cores": threads, "kind": "oracle",
            "sample": "%d of %d t0 rows (evenly spaced) x all %d tau, all %d bins; %.1f s wall"
                      % (sample.n_t0, win.n_t0, win.n_tau, atoms.n_bins, dt)}


def traffic_from_profile(workload: str, kernel_file: str):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, each scaled by a
    plain copy's reading), or None when the counters are missing or the
    kernel source changed since they were taken."""
    import hashlib
    meta = os.path.join(ROOT, "profiles", kernel_file + "_" + workload + ".json")
    if not os.path.exists(meta):
        return None
    m = json.load(open(meta))
    src = os.path.join(ROOT, "paper_1805_05652_amd", "csrc", m.get("source", "kernels.hip"))
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != m["kernels_source_sha256"]:
        return None
    return m["traffic_bytes_per_launch"]


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="exp1bin", choices=["exp1bin", "exp256", "rect", "rect256"])
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp64", "bf16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
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

    desc, atoms, win = make_workload(args.workload)
    present, slots = work_counts(atoms, win)
    ctx = tf.Context(0, arena_bytes=4 << 30)
    aid = ctx.upload_atoms(atoms)
    twoF = torch.empty((atoms.n_bins, win.n_t0, win.n_tau), dtype=torch.float32, device="cuda:0")
    for _ in range(args.warmup):
        ctx.fmap(aid, win, args.prec, out=twoF)
    torch.cuda.synchronize()
    ctx.profile_reset()
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = None
    for _ in range(args.steps):
        res, _ = ctx.fmap(aid, win, args.prec, out=twoF)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.profile(False)
    prof = ctx.profile_read()
    ms = (t1 - t0) * 1e3 / args.steps
    value = present / (ms * 1e-3)

    mfma = win.kind == "exp" and args.prec == "bf16x3" and prof["mfma"][0] > 0
    dom = "mfma" if mfma else ("exp" if win.kind == "exp" else "rect")
    n_launch, k_ms = prof[dom]
    avg_ms = k_ms / max(n_launch, 1)
    if mfma:
        # 4 complex-by-real MACs = 8 flops per cell*SFT*bin, issued as three
        # bf16 products (hi*hi + hi*lo + lo*hi): 24 bf16 flops, counted over
        # the tau blocks the matrix-core kernel runs
        long_cells = mfma_cells(atoms, win)
        flops = 24.0 * long_cells
        roof = {"bound": "mfma", "achieved": flops / (avg_ms * 1e-3) / 1e12, "peak": PEAK_BF16_TFLOPS,
                "unit": "TFLOP/s", "cells_sfts_bins": long_cells}
    elif win.kind == "exp":
        # 4 FMA (F_a, F_b) per cell*SFT*bin + 3 FP64 FMA (A, B, C) per cell*SFT
        # per group of bins sharing a lane
        bg = 1 if (args.prec == "fp64" or atoms.n_bins == 1) else (4 if atoms.n_bins >= 4 else 2)
        cells = present // atoms.n_bins
        flops = 8.0 * present + 6.0 * cells * ((atoms.n_bins + bg - 1) // bg)
        roof = {"bound": "alu", "achieved": flops / (avg_ms * 1e-3) / 1e12, "peak": PEAK_ALU_TFLOPS,
                "unit": "TFLOP/s"}
    else:
        # the map write: 4 bytes per cell*bin
        byts = 4.0 * atoms.n_bins * win.n_t0 * win.n_tau
        roof = {"bound": "hbm", "achieved": byts / (avg_ms * 1e-3) / 1e9, "peak": PEAK_HBM_GBS,
                "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = traffic_from_profile(args.workload, "exp_valu" if dom == "exp" else "rect")
    roof["kernel"] = dom
    roof["kernel_avg_ms"] = avg_ms
    out = {
        "metric": "F-map cells*SFTs/s (exp window)",
        "value": value,
        "unit": "cells*SFTs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.prec == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "n_slots": atoms.n_slots, "n_sft": atoms.n_sft,
                   "n_t0": win.n_t0, "n_tau": win.n_tau, "n_bins": atoms.n_bins,
                   "window": win.kind, "precision": args.prec, "cells_sfts": present,
                   "cells_slots": slots, "parallelism": "single GPU"},
        "roofline": roof,
        "kernels_ms": {k: (v[1] / v[0] if v[0] else None) for k, v in prof.items()},
        "result_bin0": res[0],
    }
    ctx.free(aid)
    ctx.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(atoms, win)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
