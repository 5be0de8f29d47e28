"""Seeded synthetic inputs for transient F-statistic maps.

This module simulates what the map computation consumes: per-SFT "atoms"
(antenna-pattern products a^2, b^2, ab and the complex matched-filter values
F_a, F_b) on a slot grid of T_sft = 1800 s with data gaps, Gaussian noise,
optional injected transient signals, and the (t0, tau) search grids of the
benchmark workloads.  It computes no part of the F-statistic map itself: no
windowed sums, no determinant, no F, no marginalisation.  Both the GPU path's
tests/benchmark and the CPU oracle's tests draw their inputs from here.

Noise model.  Each SFT j of bin b carries one complex sample
x_jb ~ CN(0, 1) (real and imaginary parts N(0, 1/2)) and the atoms are
F_a = a_j x_jb, F_b = b_j x_jb.  With this model the data vector (F_a, F_b)
summed over any window is complex Gaussian with covariance equal to the
windowed antenna matrix, which is what makes 2F chi-square with 4 degrees of
freedom in pure noise (section 2 of the paper defines F as a likelihood ratio
against Gaussian noise).  F_a and F_b are rounded to float32-representable
values, matching the single-precision atoms of the paper's implementation, so
that every consumer sees exactly the same inputs.

Signal model.  An injection adds s_j = h exp(i chi) env(t_j) (a_j - i b_j) to
x_j, where env is the transient envelope (rectangular or exponentially
decaying with a 3 tau cutoff, the two window shapes of section 2).  For a
search window that matches the envelope this raises the expected 2F by
2 h^2 (A + B).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

T_SFT = 1800
P_SIDEREAL = 86164.0


@dataclasses.dataclass
class Injection:
    bin: int
    kind: str          # "rect" or "exp"
    t0: int            # seconds
    tau: int           # seconds
    h: float
    chi: float = 0.0


@dataclasses.dataclass
class Atoms:
    timestamps: np.ndarray     # int64 [n_sft], SFT start times, on T0 + k*t_sft
    a: np.ndarray              # float64 [n_sft] signed antenna pattern a_j
    b: np.ndarray              # float64 [n_sft]
    a2: np.ndarray             # float64 [n_sft]
    b2: np.ndarray             # float64 [n_sft]
    ab: np.ndarray             # float64 [n_sft]
    fa: np.ndarray             # float64 [n_bins, n_sft, 2] (re, im), float32-exact
    fb: np.ndarray             # float64 [n_bins, n_sft, 2]
    t_sft: int = T_SFT
    phi_a: float = 0.0
    phi_b: float = 0.0
    injections: List[Injection] = dataclasses.field(default_factory=list)

    @property
    def n_sft(self) -> int:
        return int(self.timestamps.shape[0])

    @property
    def n_bins(self) -> int:
        return int(self.fa.shape[0])

    @property
    def n_slots(self) -> int:
        ts = self.timestamps
        return int((ts[-1] - ts[0]) // self.t_sft) + 1

    @property
    def t_data(self) -> int:
        return self.n_slots * self.t_sft


@dataclasses.dataclass
class Window:
    kind: str                  # "rect" or "exp"
    t0: np.ndarray             # int64 [n_t0], strictly increasing
    tau: np.ndarray            # int64 [n_tau], strictly increasing, > 0
    # Set when the grid is regular, so callers may pass (min, step, count).
    t0_regular: Optional[tuple] = None
    tau_regular: Optional[tuple] = None
    # kind "shape": samples of the window shape s(x), x = (t - t0) / tau,
    # evenly spaced over [0, num/den]; support = (num, den)
    shape: Optional[np.ndarray] = None
    support: tuple = (1, 1)

    @property
    def n_t0(self) -> int:
        return int(self.t0.shape[0])

    @property
    def n_tau(self) -> int:
        return int(self.tau.shape[0])


def regular_window(kind: str, t0_min: int, dt0: int, n_t0: int,
                   tau_min: int, dtau: int, n_tau: int) -> Window:
    t0 = t0_min + dt0 * np.arange(n_t0, dtype=np.int64)
    tau = tau_min + dtau * np.arange(n_tau, dtype=np.int64)
    return Window(kind, t0, tau, (int(t0_min), int(dt0), int(n_t0)),
                  (int(tau_min), int(dtau), int(n_tau)))


def list_window(kind: str, t0: Sequence[int], tau: Sequence[int]) -> Window:
    t0 = np.asarray(t0, dtype=np.int64)
    tau = np.asarray(tau, dtype=np.int64)
    return Window(kind, t0, tau)


def shape_window(base: Window, shape, support=(1, 1)) -> Window:
    """The grid of `base` with a general window shape: samples of s(x),
    x = (t - t0) / tau, evenly spaced over [0, num/den], support = (num, den)."""
    return Window("shape", base.t0, base.tau, base.t0_regular, base.tau_regular,
                  np.ascontiguousarray(shape, dtype=np.float64), (int(support[0]), int(support[1])))


def slot_timestamps(rng: np.random.Generator, n_slots: int, gap_frac: float,
                    t_sft: int = T_SFT, T0: int = 0) -> np.ndarray:
    """Start times of the SFTs present on a grid of n_slots slots.

    Exactly round(gap_frac * n_slots) slots are dropped, chosen by the seeded
    generator; the first and last slots are always kept so the data span is
    exactly n_slots * t_sft.
    """
    n_drop = int(round(gap_frac * n_slots))
    keep = np.ones(n_slots, dtype=bool)
    if n_drop > 0:
        if n_drop > n_slots - 2:
            raise ValueError("too many gaps for the span")
        drop = rng.choice(np.arange(1, n_slots - 1), size=n_drop, replace=False)
        keep[drop] = False
    return T0 + np.nonzero(keep)[0].astype(np.int64) * t_sft


def _envelope(kind: str, ts: np.ndarray, t0: int, tau: int) -> np.ndarray:
    """Amplitude envelope of a simulated transient signal at SFT times."""
    dt = (ts - t0).astype(np.float64)
    if kind == "rect":
        return ((ts >= t0) & (ts < t0 + tau)).astype(np.float64)
    if kind == "exp":
        on = (ts >= t0) & (ts < t0 + 3 * tau)
        return np.where(on, np.exp(-np.where(on, dt, 0.0) / tau), 0.0)
    raise ValueError(kind)


def make_atoms(seed: int, n_slots: int, gap_frac: float, n_bins: int = 1,
               injections: Sequence[Injection] = (), t_sft: int = T_SFT,
               T0: int = 0, min_abs_cos: float = 0.2,
               noise: bool = True) -> Atoms:
    """Seeded atoms with noise and injections.

    Antenna patterns: a = 0.5 cos(2 pi t / P_sid + phi_a),
    b = 0.5 sin(2 pi t / P_sid + phi_b), with phi_a, phi_b uniform.  The
    phases are redrawn (deterministically) while |cos(phi_b - phi_a)| is below
    min_abs_cos, because at cos = 0 the two patterns are collinear and every
    window is degenerate.
    """
    rng = np.random.default_rng(seed)
    ts = slot_timestamps(rng, n_slots, gap_frac, t_sft, T0)
    while True:
        phi_a, phi_b = rng.uniform(0.0, 2.0 * math.pi, size=2)
        if abs(math.cos(phi_b - phi_a)) >= min_abs_cos:
            break
    ph = 2.0 * math.pi * ts.astype(np.float64) / P_SIDEREAL
    a = 0.5 * np.cos(ph + phi_a)
    b = 0.5 * np.sin(ph + phi_b)
    n = ts.shape[0]
    if noise:
        x = (rng.standard_normal((n_bins, n)) + 1j * rng.standard_normal((n_bins, n))) * math.sqrt(0.5)
    else:
        x = np.zeros((n_bins, n), dtype=np.complex128)
    for inj in injections:
        env = _envelope(inj.kind, ts, inj.t0, inj.tau)
        x[inj.bin] += inj.h * np.exp(1j * inj.chi) * env * (a - 1j * b)
    fa_c = (a[None, :] * x).astype(np.complex64)
    fb_c = (b[None, :] * x).astype(np.complex64)
    fa = np.stack([fa_c.real, fa_c.imag], axis=-1).astype(np.float64)
    fb = np.stack([fb_c.real, fb_c.imag], axis=-1).astype(np.float64)
    return Atoms(ts, a, b, a * a, b * b, a * b, np.ascontiguousarray(fa),
                 np.ascontiguousarray(fb), t_sft, float(phi_a), float(phi_b),
                 list(injections))


# ---------------------------------------------------------------------------
# Benchmark workloads.  Seeds are (workload index) * 1000 + candidate index.
# ---------------------------------------------------------------------------

def workload_rect_small():
    """Rectangular window, 1 bin, 200 slots with 10% gaps; t0 over the first
    100 slots, tau from 2 to 200 slots in steps of one SFT (19,900 cells)."""
    inj = [Injection(0, "rect", 30 * T_SFT, 60 * T_SFT, 0.4, chi=0.3)]
    atoms = make_atoms(0, 200, 0.10, 1, inj)
    win = regular_window("rect", 0, T_SFT, 100, 2 * T_SFT, T_SFT, 199)
    return atoms, win


def exp_tau_grid_30d(n_tau: int = 1000) -> np.ndarray:
    """tau from 2 T_sft to 30 days in n_tau steps rounded to whole seconds."""
    lo, hi = 2 * T_SFT, 30 * 86400
    n = np.arange(n_tau, dtype=np.int64)
    return lo + np.round(n * (hi - lo) / (n_tau - 1)).astype(np.int64)


def workload_exp_1bin(n_slots: int = 5000, n_t0: int = 1000, n_tau: int = 1000):
    """Exponential window, 1 bin, 5000 slots (~104 days) with 15% gaps;
    t0 over the first 1000 slots, tau from 2 T_sft to 30 days."""
    inj = [Injection(0, "exp", 200 * T_SFT, 10 * 86400, 0.2, chi=1.1)]
    atoms = make_atoms(1000, n_slots, 0.15, 1, inj)
    t0 = T_SFT * np.arange(n_t0, dtype=np.int64)
    win = Window("exp", t0, exp_tau_grid_30d(n_tau), (0, T_SFT, n_t0), None)
    return atoms, win


def workload_exp_bins(n_bins: int = 256, n_slots: int = 2000, n_t0: int = 500,
                      n_tau: int = 500, seed: int = 2000):
    """Exponential window, many frequency bins sharing a, b; 2000 slots with
    10% gaps; injections in 4 seeded bins."""
    rng = np.random.default_rng(seed + 1)
    inj_bins = rng.choice(n_bins, size=min(4, n_bins), replace=False)
    inj = []
    for b in inj_bins:
        t0 = int(rng.integers(0, n_t0)) * T_SFT
        tau = int(rng.integers(2, n_tau + 2)) * T_SFT
        inj.append(Injection(int(b), "exp", t0, tau, 0.2, float(rng.uniform(0, 2 * math.pi))))
    atoms = make_atoms(seed, n_slots, 0.10, n_bins, inj)
    win = regular_window("exp", 0, T_SFT, n_t0, 2 * T_SFT, T_SFT, n_tau)
    return atoms, win


def linspace_grid(atoms: Atoms, kind: str, n_t0: int, n_tau: int) -> Window:
    """The paper's timing-test grid: t0 in [T0, T0 + T_data - 2 T_sft] and
    tau in [2 T_sft, T_data], evenly spaced and rounded to whole seconds."""
    T0 = int(atoms.timestamps[0])
    td = atoms.t_data
    t0 = T0 + np.round(np.linspace(0, td - 2 * atoms.t_sft, n_t0)).astype(np.int64)
    tau = np.round(np.linspace(2 * atoms.t_sft, td, n_tau)).astype(np.int64)
    return Window(kind, np.unique(t0), np.unique(tau))


def candidate(index: int, seed_base: int = 3000, max_slots: int = 8000,
              max_grid: int = 1500, max_bins: int = 16):
    """One follow-up candidate of the uneven batch: slots log-uniform in
    [500, max_slots], gap fraction U[0, 0.3], grid sizes U{100..max_grid},
    1..max_bins bins, rect for even and exp for odd index, injections in about
    10% of candidates."""
    rng = np.random.default_rng(seed_base + index)
    n_slots = int(round(math.exp(rng.uniform(math.log(500), math.log(max_slots)))))
    gap = float(rng.uniform(0.0, 0.3))
    n_t0 = int(rng.integers(100, max_grid + 1))
    n_tau = int(rng.integers(100, max_grid + 1))
    n_bins = int(rng.integers(1, max_bins + 1))
    kind = "rect" if index % 2 == 0 else "exp"
    inj = []
    if rng.uniform() < 0.1:
        t0 = int(rng.integers(0, n_slots // 2)) * T_SFT
        tau = int(rng.integers(2, max(3, n_slots // 4))) * T_SFT
        inj.append(Injection(int(rng.integers(0, n_bins)), kind, t0, tau, 0.2,
                             float(rng.uniform(0, 2 * math.pi))))
    atoms = make_atoms(seed_base * 10 + index, n_slots, gap, n_bins, inj)
    win = linspace_grid(atoms, kind, min(n_t0, n_slots - 1), min(n_tau, n_slots - 1))
    return atoms, win


def request_stream(seed: int, rate_hz: float, duration_s: float,
                   max_slots: int = 10000, max_grid: int = 2000,
                   max_bins: int = 64):
    """Poisson arrival times and per-request shapes of the serving workload.

    Returns a list of dicts with arrival time (s) and the request's seed and
    shape; atoms are generated per request by `request_atoms`.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        n_slots = int(round(math.exp(rng.uniform(math.log(200), math.log(max_slots)))))
        out.append(dict(
            arrival=t,
            seed=int(rng.integers(0, 2**31 - 1)),
            n_slots=n_slots,
            n_t0=int(rng.integers(100, max_grid + 1)),
            n_tau=int(rng.integers(100, max_grid + 1)),
            n_bins=int(rng.integers(1, max_bins + 1)),
            kind="rect" if rng.uniform() < 0.5 else "exp",
        ))
    return out


def request_window(atoms: Atoms, req: dict) -> Window:
    """The request's grid (window type, N_t0 x N_tau, linspace) over `atoms`;
    grid sizes are capped at the atoms' slots - 1."""
    return linspace_grid(atoms, req["kind"], min(req["n_t0"], atoms.n_slots - 1),
                         min(req["n_tau"], atoms.n_slots - 1))


def request_atoms(req: dict):
    atoms = make_atoms(req["seed"], req["n_slots"], 0.10, req["n_bins"])
    return atoms, request_window(atoms, req)
