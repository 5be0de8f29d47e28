"""Timing model of the F-statistic map and its fit on this GPU (appendix A).

The paper models the cost of one map as
    rect:  c_SFTs N_SFT + c_sums^r N_sums^r + c_F N_t0 N_tau   (eq. cost-rect-Nsums)
    exp:   c_SFTs N_SFT + c_sums^e N_sums^e + c_F N_t0 N_tau   (eq. cost-exp-Nsums)
with the effective numbers of summation steps
    N_sums^r = sum_m min(T_data - t0_m, tau_max) / T_sft          (eq. Nsums-rect)
    N_sums^e = sum_m sum_n min(T_data - t0_m, 3 tau_n) / T_sft    (eq. Nsums-exp)
(t0_m measured from the start of the data), and fits the four constants in
three steps: c_SFTs on short data sets (N_sums <= 100) alone, then
c_sums^r and c_F on rectangular maps with c_SFTs fixed, then c_sums^e on
exponential maps with c_SFTs and c_F fixed.  The PGM constants follow in
the embedded case from eq. cost-rect-convert and eq. cost-exp-convert.

A GPU call also has a fixed cost per map (launches and the host round
trip) that the CPU model has no term for; `fit_paper` follows the paper's
steps as they are, and `fit_with_offset` adds a constant c_0 fitted in the
first step beside c_SFTs (the data sets of step 1 then span many N_SFT).

Running this module times tfstat_fmap on the GPU over a grid of setups
(T_data, N_t0, N_tau, window) and prints both fits as one JSON line:
    python -m paper_1805_05652_amd.timing_model [--reps 5] [--quick]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

T_SFT = 1800


def n_sums_rect(t0_rel, tau, t_data, t_sft=T_SFT) -> float:
    """eq. Nsums-rect: t0_rel are start times from the data start (s)."""
    t0_rel = np.asarray(t0_rel, dtype=np.float64)
    tau_max = float(np.max(tau))
    return float(np.sum(np.minimum(t_data - t0_rel, tau_max)) / t_sft)


def n_sums_exp(t0_rel, tau, t_data, t_sft=T_SFT) -> float:
    """eq. Nsums-exp."""
    t0_rel = np.asarray(t0_rel, dtype=np.float64)[:, None]
    tau = np.asarray(tau, dtype=np.float64)[None, :]
    return float(np.sum(np.minimum(t_data - t0_rel, 3.0 * tau)) / t_sft)


def _lstsq(X, y, w=None):
    """Least squares with relative weights (each run's time counts with the
    same relative precision); returns coefficients and their standard errors."""
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if w is None:
        w = 1.0 / np.maximum(y, 1e-300)
    Xw = X * w[:, None]
    yw = y * w
    coef, *_ = np.linalg.lstsq(Xw, yw, rcond=None)
    res = yw - Xw @ coef
    dof = max(len(y) - X.shape[1], 1)
    s2 = float(res @ res) / dof
    try:
        cov = s2 * np.linalg.inv(Xw.T @ Xw)
        err = np.sqrt(np.maximum(np.diag(cov), 0.0))
    except np.linalg.LinAlgError:
        err = np.full(X.shape[1], np.nan)
    return coef, err


def fit_paper(runs, short_max_sums: float = 100.0):
    """The three steps of appendix A.  runs: dicts with keys kind ('rect' or
    'exp'), n_sft, n_sums, n_cells (= N_t0 N_tau) and t (seconds).  Step 1
    uses the short runs (N_sums <= short_max_sums); steps 2 and 3 use the
    others (the paper leaves open whether the short runs enter them again;
    here they serve step 1 only)."""
    short = [r for r in runs if r["n_sums"] <= short_max_sums]
    if not short:
        raise ValueError("step 1 needs runs with N_sums <= %g" % short_max_sums)
    c_sft, e_sft = _lstsq([[r["n_sft"]] for r in short], [r["t"] for r in short])
    runs = [r for r in runs if r["n_sums"] > short_max_sums]
    rect = [r for r in runs if r["kind"] == "rect"]
    y = [r["t"] - c_sft[0] * r["n_sft"] for r in rect]
    (c_rs, c_f), (e_rs, e_f) = _lstsq([[r["n_sums"], r["n_cells"]] for r in rect], y,
                                      w=1.0 / np.array([r["t"] for r in rect]))
    ex = [r for r in runs if r["kind"] == "exp"]
    y = [r["t"] - c_sft[0] * r["n_sft"] - c_f * r["n_cells"] for r in ex]
    (c_es,), (e_es,) = _lstsq([[r["n_sums"]] for r in ex], y, w=1.0 / np.array([r["t"] for r in ex]))
    return {"c_SFTs": (float(c_sft[0]), float(e_sft[0])), "c_sums_rect": (float(c_rs), float(e_rs)),
            "c_F": (float(c_f), float(e_f)), "c_sums_exp": (float(c_es), float(e_es))}


def fit_with_offset(runs, short_max_sums: float = 100.0):
    """The same three steps with a constant per-map cost c_0 fitted beside
    c_SFTs in step 1 and held fixed afterwards."""
    short = [r for r in runs if r["n_sums"] <= short_max_sums]
    (c0, c_sft), (e0, e_sft) = _lstsq([[1.0, r["n_sft"]] for r in short], [r["t"] for r in short])
    base = lambda r: c0 + c_sft * r["n_sft"]  # noqa: E731
    runs = [r for r in runs if r["n_sums"] > short_max_sums]
    rect = [r for r in runs if r["kind"] == "rect"]
    (c_rs, c_f), (e_rs, e_f) = _lstsq([[r["n_sums"], r["n_cells"]] for r in rect],
                                      [r["t"] - base(r) for r in rect],
                                      w=1.0 / np.array([r["t"] for r in rect]))
    ex = [r for r in runs if r["kind"] == "exp"]
    (c_es,), (e_es,) = _lstsq([[r["n_sums"]] for r in ex],
                              [r["t"] - base(r) - c_f * r["n_cells"] for r in ex],
                              w=1.0 / np.array([r["t"] for r in ex]))
    return {"c_0": (float(c0), float(e0)), "c_SFTs": (float(c_sft), float(e_sft)),
            "c_sums_rect": (float(c_rs), float(e_rs)), "c_F": (float(c_f), float(e_f)),
            "c_sums_exp": (float(c_es), float(e_es))}


def predict(fit, run) -> float:
    """Modelled time of one run (keys as in fit_paper) from a fit: eq.
    cost-rect-Nsums or eq. cost-exp-Nsums, plus c_0 when the fit has one."""
    c_sums = fit["c_sums_rect"][0] if run["kind"] == "rect" else fit["c_sums_exp"][0]
    return (fit.get("c_0", (0.0, 0.0))[0] + fit["c_SFTs"][0] * run["n_sft"] + c_sums * run["n_sums"]
            + fit["c_F"][0] * run["n_cells"])


def pgm_constants(fit, n_sft, n_t0, n_tau, tau_min, tau_max, dtau, t_sft=T_SFT):
    """PGM's per-step constants in the embedded case (eq. cost-rect-convert,
    eq. cost-exp-convert), with the fitted constants' central values."""
    c_sft = fit["c_SFTs"][0]
    c_f = fit["c_F"][0]
    c_rect = fit["c_sums_rect"][0] + t_sft / tau_max * (c_sft * n_sft / n_t0 + c_f * n_tau)
    c_exp = 3.0 * fit["c_sums_exp"][0] + t_sft / (tau_min + 0.5 * dtau) * (c_sft * n_sft / (n_t0 * n_tau) + c_f)
    return {"c_rect_PGM": c_rect, "c_exp_PGM": c_exp}


# ---------------------------------------------------------------------------
# Timing runs on the GPU
# ---------------------------------------------------------------------------
def setups(quick: bool = False):
    """(n_slots, n_t0, n_tau, kind) covering short and long data, small and
    large grids, embedded and truncated windows (section 4.1 grids:
    t0 over [0, T_data - 2 T_sft], tau over [2 T_sft, T_data])."""
    out = []
    slots = [8, 16, 24, 48, 96, 480, 2000, 5000] if not quick else [8, 24, 96, 2000]
    grids = ([(2, 2), (3, 3), (10, 10), (50, 20), (100, 100), (300, 300), (1000, 500)] if not quick
             else [(2, 2), (10, 10), (300, 300)])
    for k in slots:
        for n_t0, n_tau in grids:
            for kind in ("rect", "exp"):
                out.append((k, min(n_t0, k - 2), min(n_tau, k - 2), kind))
    return out


def time_runs(reps: int = 5, quick: bool = False, precision: str = "fp32", seed: int = 9000,
              on_result=None):
    """Times tfstat_fmap over `setups(quick)`: one untimed call, then the
    median of `reps` timed calls per setup.  on_result(atoms, win, results),
    when given, receives each setup's per-bin results."""
    import torch
    import paper_1805_05652_amd as tf
    import tfsynth
    runs = []
    ctx = tf.Context(0, arena_bytes=8 << 30)
    try:
        for i, (k, n_t0, n_tau, kind) in enumerate(setups(quick)):
            atoms = tfsynth.make_atoms(seed + i, k, 0.0, n_bins=1)
            win = tfsynth.linspace_grid(atoms, kind, n_t0, n_tau)
            aid = ctx.upload_atoms(atoms)
            res, _ = ctx.fmap(aid, win, precision)
            if on_result is not None:
                on_result(atoms, win, res)
            ts = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t = time.perf_counter()
                ctx.fmap(aid, win, precision)
                ts.append(time.perf_counter() - t)
            ctx.free(aid)
            t0_rel = win.t0 - atoms.timestamps[0]
            t_data = atoms.t_data
            ns = n_sums_rect(t0_rel, win.tau, t_data) if kind == "rect" else n_sums_exp(t0_rel, win.tau, t_data)
            runs.append({"kind": kind, "n_slots": k, "n_sft": atoms.n_sft, "n_t0": win.n_t0,
                         "n_tau": win.n_tau, "n_cells": win.n_t0 * win.n_tau, "n_sums": ns,
                         "t": float(np.median(ts))})
            print("run %d/%d %s K=%d %dx%d  %.3f ms" % (i + 1, len(setups(quick)), kind, k, win.n_t0,
                                                      win.n_tau, 1e3 * runs[-1]["t"]),
                  file=sys.stderr, flush=True)
    finally:
        ctx.close()
    return runs


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    args = ap.parse_args(argv)
    runs = time_runs(args.reps, args.quick, args.precision)
    paper = fit_paper(runs)
    offs = fit_with_offset(runs)
    # PGM comparison in the embedded example of the paper's footnote: one
    # year of data, tau in [0.5, 14.5] days
    day = 86400
    conv = dict(n_sft=17532, n_t0=17532, n_tau=29, tau_min=0.5 * day, tau_max=14.5 * day, dtau=0.5 * day)
    print(json.dumps({"precision": args.precision, "runs": runs, "fit_paper": paper,
                      "fit_with_offset": offs, "pgm_paper_fit": pgm_constants(paper, **conv),
                      "pgm_offset_fit": pgm_constants(offs, **conv)}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
