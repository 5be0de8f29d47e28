"""The seeded generator: reproducibility, exact gap counts, float32-exact
matched-filter atoms."""
import numpy as np

import tfsynth

T = tfsynth.T_SFT


def test_reproducible_and_seed_dependent():
    a1 = tfsynth.make_atoms(5, 300, 0.2, 3)
    a2 = tfsynth.make_atoms(5, 300, 0.2, 3)
    a3 = tfsynth.make_atoms(6, 300, 0.2, 3)
    assert np.array_equal(a1.timestamps, a2.timestamps)
    assert np.array_equal(a1.fa, a2.fa) and np.array_equal(a1.fb, a2.fb)
    assert not np.array_equal(a1.fa[:, :10], a3.fa[:, :10])


def test_gap_count_and_span():
    for K, g in [(200, 0.1), (5000, 0.15), (777, 0.3), (50, 0.0)]:
        at = tfsynth.make_atoms(1, K, g)
        assert at.n_sft == K - int(round(g * K))
        assert at.timestamps[0] == 0 and at.timestamps[-1] == (K - 1) * T
        assert at.n_slots == K
        assert np.all(at.timestamps % T == 0)
        assert np.all(np.diff(at.timestamps) > 0)


def test_atoms_float32_exact_and_consistent():
    at = tfsynth.make_atoms(2, 100, 0.1, 2)
    assert np.array_equal(at.fa, at.fa.astype(np.float32).astype(np.float64))
    assert np.array_equal(at.fb, at.fb.astype(np.float32).astype(np.float64))
    assert np.array_equal(at.a2, at.a * at.a) and np.array_equal(at.ab, at.a * at.b)
    assert abs(np.cos(at.phi_b - at.phi_a)) >= 0.2


def test_workload_shapes():
    at, w = tfsynth.workload_rect_small()
    assert (at.n_slots, at.n_sft, w.n_t0, w.n_tau) == (200, 180, 100, 199)
    at, w = tfsynth.workload_exp_1bin()
    assert (at.n_slots, at.n_sft, w.n_t0, w.n_tau) == (5000, 4250, 1000, 1000)
    assert w.tau[0] == 2 * T and w.tau[-1] == 30 * 86400
    assert np.all(np.diff(w.tau) > 0)
    at, w = tfsynth.candidate(3)
    assert w.kind == "exp" and 1 <= at.n_bins <= 16
    assert np.all(np.diff(w.t0) > 0) and np.all(np.diff(w.tau) > 0)
    reqs = tfsynth.request_stream(4, 200.0, 1.0)
    assert 120 < len(reqs) < 300
