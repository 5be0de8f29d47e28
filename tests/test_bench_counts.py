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


def test_work_counts_brute_force():
    """Off-slot start times, gaps, windows before, inside and past the data:
    work_counts equals a per-cell count of the SFT start times and of the
    slot start times in [t0, t0 + span), cut at the data end."""
    atoms = tfsynth.make_atoms(11, 120, 0.25, n_bins=2)
    ts = atoms.timestamps
    T0 = int(ts[0])
    t_end = T0 + atoms.t_data
    t0 = np.array([-3 * T - 5, -1, 0, 7, T + 1, 40 * T + 900, 118 * T, 130 * T], dtype=np.int64)
    tau = np.array([1, T - 1, T, 2 * T + 3, 17 * T, 200 * T], dtype=np.int64)
    for kind, mult in (("rect", 1), ("exp", 3)):
        win = tfsynth.list_window(kind, t0, tau)
        present = slots = 0
        for a in t0.tolist():
            for t in tau.tolist():
                e = a + mult * t
                present += sum(1 for s in ts.tolist() if a <= s < e)
                slots += sum(1 for k in range(atoms.n_slots) if a <= T0 + k * T < min(e, t_end))
        assert bench.work_counts(atoms, win) == (present * 2, slots * 2), kind


def test_mfma_cells_blocks():
    """The matrix-core share counts exactly the tau blocks of 8 whose
    shortest band (ceil(3 tau / T_sft) slots for rows on slot starts) is at
    least 64, for maps of at least 2 bins; one-bin maps run on the VALU."""
    atoms = _gapless(600, n_bins=5)
    tau = np.concatenate([np.full(8, 30 * T), np.full(8, 21 * T), [21 * T + 1] * 7 + [10 * T],
                          np.full(3, 40 * T)]).astype(np.int64)
    win = tfsynth.list_window("exp", np.arange(20, dtype=np.int64) * T, tau)
    # blocks: all bands 90 (in), all 63 (out), seven 64 and one 30 (out), three 120 (in)
    keep = np.r_[np.ones(8, bool), np.zeros(16, bool), np.ones(3, bool)]
    want = bench.work_counts(atoms, tfsynth.list_window("exp", win.t0, tau[keep]))[0]
    assert bench.mfma_cells(atoms, win) == want
    assert 0 < want < bench.work_counts(atoms, win)[0]
    assert bench.mfma_cells(_gapless(600, n_bins=1), win) == 0
    assert bench.mfma_cells(atoms, tfsynth.list_window("rect", win.t0, tau)) == 0
    # F16X3: blocks whose bands are all at least 24 slots, in a map that has
    # a block of 64 (here every block: its shortest band is 30)
    assert bench.mfma_cells(atoms, win, "f16x3") == bench.work_counts(atoms, win)[0]
    short = tfsynth.list_window("exp", win.t0, tau[8:24])
    assert bench.mfma_cells(atoms, short, "f16x3") == 0
    # a block whose shortest band is 23 slots (3 tau = 22.67 T) stays off
    tau23 = np.concatenate([np.full(8, 30 * T), np.full(8, 7 * T + 1000)]).astype(np.int64)
    w23 = tfsynth.list_window("exp", win.t0, tau23)
    assert bench.mfma_cells(atoms, w23, "f16x3") == \
        bench.work_counts(atoms, tfsynth.list_window("exp", win.t0, tau23[:8]))[0]


def test_mfma_taus_offsets_and_data_end():
    """Rows off the slot grid shorten the band by the largest offset: with
    3 tau = 64 T - 600 s, a row on a slot start holds 64 slot starts in
    [t0, t0 + 3 tau), a row 1799 s before a slot start only 63.  Bands are
    capped at the data end seen from the earliest row."""
    atoms = _gapless(600, n_bins=4)
    tau = np.full(8, (64 * T - 600) // 3, dtype=np.int64)
    assert 3 * tau[0] == 64 * T - 600
    assert bench.mfma_taus(atoms, tfsynth.list_window("exp", np.array([0, T]), tau)).all()
    assert not bench.mfma_taus(atoms, tfsynth.list_window("exp", np.array([0, T + 1]), tau)).any()
    # rows near the data end: 600 - 540 = 60 slots left
    assert not bench.mfma_taus(atoms, tfsynth.list_window("exp", np.array([540 * T, 550 * T]),
                                                          np.full(8, 100 * T))).any()
    assert bench.mfma_taus(atoms, tfsynth.list_window("exp", np.array([530 * T, 550 * T]),
                                                      np.full(8, 100 * T))).all()
