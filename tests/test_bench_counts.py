"""The benchmark's unit of work (cells x SFTs in the window, the paper's
N_sums of appendix A counted over SFTs) against the closed forms the
appendix gives for its special cases."""
import numpy as np
import pytest

import bench
import tfsynth

T = tfsynth.T_SFT


def _gapless(n_slots, n_bins=1):
    return tfsynth.make_atoms(0, n_slots, 0.0, n_bins=n_bins)


def test_rect_embedded_case():
    """Embedded case (every window inside the data): N_sums^rect sums the
    slots of every cell; for the largest tau it is N_t0 tau_max / T_sft
    (eq. Nsums-rect reduces to PGM's N_t0 tau_max / T_sft)."""
    atoms = _gapless(400)
    win = tfsynth.regular_window("rect", 0, T, 50, 2 * T, T, 100)   # t0 + tau <= 151 T
    present, slots = bench.work_counts(atoms, win)
    assert present == slots
    # each cell (m, n) holds exactly tau_n / T slots
    assert present == win.n_t0 * int((win.tau // T).sum())
    one = tfsynth.Window("rect", win.t0, win.tau[-1:])
    assert bench.work_counts(atoms, one)[0] == win.n_t0 * int(win.tau[-1] // T)


def test_rect_timing_grid_half():
    """On the timing grid of section 4.1 (N_t0 dt0 = N_tau dtau = T_data - 2 T)
    the rectangular count for tau_max is about 0.5 N_t0 tau_max / T_sft."""
    K = 2000
    atoms = _gapless(K)
    n = K - 2
    win = tfsynth.regular_window("rect", 0, T, n, 2 * T, T, n)
    one = tfsynth.Window("rect", win.t0, np.array([K * T], dtype=np.int64))
    got = bench.work_counts(atoms, one)[0]
    assert got == pytest.approx(0.5 * n * K, rel=0.01)


def test_exp_embedded_case():
    """Embedded exponential case: N_sums^exp = 3 N_t0 sum_n tau_n / T_sft
    (eq. Nsums-exp) when 3 tau_n is a whole number of SFTs."""
    atoms = _gapless(1000)
    win = tfsynth.regular_window("exp", 0, T, 40, 2 * T, T, 60)    # 3 * 61 T + 40 T < 1000 T
    present, slots = bench.work_counts(atoms, win)
    assert present == slots == 3 * win.n_t0 * int((win.tau // T).sum())


def test_exp_truncation_and_gaps():
    """Windows past the data end are truncated; gaps reduce the SFT count but
    not the slot count."""
    atoms = tfsynth.make_atoms(3, 300, 0.2, n_bins=3)
    win = tfsynth.regular_window("exp", 250 * T, T, 10, 30 * T, T, 5)
    present, slots = bench.work_counts(atoms, win)
    per_bin_slots = sum(min(300 - (250 + m), 3 * (30 + k)) for m in range(10) for k in range(5))
    assert slots == 3 * per_bin_slots
    assert present < slots


def test_workload_counts_match_recipes():
    atoms, win = tfsynth.workload_exp_1bin()
    present, slots = bench.work_counts(atoms, win)
    assert slots == 2162207818
    assert 0.84 * slots < present < 0.86 * slots       # 15% gaps
