"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle on
the same seeded inputs.

Tolerances (floating point):
  * 2F: |2F_gpu - 2F_oracle| <= tol * max(2F_oracle, 1) with tol = 1e-4 for
    FP32 sums and 1e-9 for FP64 sums; the stored map is float32, so map
    comparisons also allow its rounding (2^-23 relative).
  * logB: absolute 1e-3.
  * argmax: exact, or a near-tie: 2F_oracle at the GPU's argmax is at least
    (1 - 1e-4) * max 2F_oracle.
  * degenerate cells (2F = 0 in the oracle) are exactly 0 on the GPU.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import tfsynth

pytestmark = pytest.mark.gpu

from checks import TOL, check_map, check_results

T = tfsynth.T_SFT


@pytest.fixture(scope="module")
def ctx():
    import paper_1805_05652_amd as tf
    c = tf.Context(0, arena_bytes=3 << 30)
    yield c
    c.close()


def _case(msg):
    print("case:", msg, flush=True)


DENSE_ONLY = 1 << 30   # tiling: every map on the band-staged form
RUNS_ALWAYS = 0        # tiling: every map on the runs form


class tiling:
    """Sets the exponential tiling thresholds for the maps planned inside."""

    def __init__(self, ctx, runs_min_spread, split_min_bins=-1):
        self.ctx, self.v, self.s = ctx, runs_min_spread, split_min_bins

    def __enter__(self):
        self.ctx.tiling_config(self.v, self.s)

    def __exit__(self, *exc):
        self.ctx.tiling_config(-1, -1)


def run_and_check(ctx, atoms, win, prec):
    aid = ctx.upload_atoms(atoms)
    try:
        res, twoF = ctx.fmap(aid, win, prec, want_map=True)
        ref = oracle.fmap_atoms(atoms, win)
        err = check_map(twoF.cpu().numpy(), ref, TOL[prec])
        check_results(res, ref, win, TOL[prec])
        return res, ref, err
    finally:
        ctx.free(aid)


# ---------------------------------------------------------------------------
# Small cases spanning several tiles with ragged tails
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rect_small_workload(ctx, prec):
    _case("rect small workload " + prec)
    atoms, win = tfsynth.workload_rect_small()
    run_and_check(ctx, atoms, win, prec)


@pytest.mark.parametrize("n_t0,n_tau", [(1, 1), (63, 64), (64, 65), (65, 1), (130, 129)])
def test_rect_tile_edges(ctx, n_t0, n_tau):
    """Rect tiles are 64 rows x 64 taus with one reduction per tile: grids
    one row / one tau short of, at and past a tile edge, every cell of the
    map and the per-bin results against the oracle (two bins)."""
    _case("rect tile edges %d x %d" % (n_t0, n_tau))
    atoms = tfsynth.make_atoms(260 + n_t0, 300, 0.1, n_bins=2)
    win = tfsynth.regular_window("rect", 2 * T + 5, T, n_t0, T + 3, 2 * T, n_tau)
    run_and_check(ctx, atoms, win, "fp64")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind", ["rect", "exp"])
def test_ragged_grid_with_edges(ctx, prec, kind):
    """t0 off the slot grid, before the data and after it; tau not a multiple
    of T_sft, shorter than one SFT and longer than the data; 3 bins."""
    _case("ragged edges %s %s" % (kind, prec))
    atoms = tfsynth.make_atoms(101, 300, 0.2, n_bins=3,
                               injections=[tfsynth.Injection(2, kind, 40 * T, 30 * T, 1.2)])
    rng = np.random.default_rng(5)
    t0 = np.unique(np.concatenate([
        [-5 * T - 77, -T, -1, 0, 1, T - 1],
        rng.integers(0, 300 * T, size=120),
        [299 * T, 299 * T + 1, 300 * T + 5, 400 * T]]))
    tau = np.unique(np.concatenate([
        [1, T - 1, T, T + 1, 2 * T],
        rng.integers(2 * T, 200 * T, size=37),
        [300 * T, 1000 * T]]))
    win = tfsynth.list_window(kind, t0, tau)
    run_and_check(ctx, atoms, win, prec)


@pytest.mark.parametrize("n_bins", [1, 2, 3, 5, 8])
def test_exp_bins_groups(ctx, n_bins):
    _case("exp bins %d" % n_bins)
    atoms = tfsynth.make_atoms(200 + n_bins, 180, 0.1, n_bins=n_bins)
    win = tfsynth.regular_window("exp", 0, T, 130, 2 * T, T, 77)
    run_and_check(ctx, atoms, win, "fp32")


@pytest.mark.parametrize("form", ["dense", "default"])
def test_exp_sparse_rows_read_through_cache(ctx, form):
    """Rows 10 slots apart: a 64-row tile spans more slots than one LDS stage
    (band-staged form: each lane reads its slots through the caches; by
    default: the runs form)."""
    _case("exp sparse rows " + form)
    atoms = tfsynth.make_atoms(301, 900, 0.1, n_bins=2)
    win = tfsynth.regular_window("exp", 0, 10 * T, 85, 2 * T, 7 * T + 13, 30)
    with tiling(ctx, DENSE_ONLY if form == "dense" else -1):
        run_and_check(ctx, atoms, win, "fp32")
        run_and_check(ctx, atoms, win, "fp64")


@pytest.mark.parametrize("step,n_bins", [(13, 1), (16, 1), (5, 2), (7, 5)])
@pytest.mark.parametrize("form", ["dense", "runs"])
def test_exp_row_spread_staging_limits(ctx, step, n_bins, form):
    """64-row tiles spanning 819 and 1008 slots (one bin: staged in shorter
    rounds, then read through the caches) and 315 and 441 slots (two and five
    bins: staged in shorter rounds); ragged band ends.  Both tile forms."""
    _case("exp row spread step %d bins %d %s" % (step, n_bins, form))
    atoms = tfsynth.make_atoms(311 + step, 1500, 0.1, n_bins=n_bins)
    win = tfsynth.regular_window("exp", 3 * T + 40, step * T, 100, 2 * T, 9 * T + 17, 40)
    with tiling(ctx, DENSE_ONLY if form == "dense" else RUNS_ALWAYS):
        run_and_check(ctx, atoms, win, "fp32")


@pytest.mark.parametrize("prec,n_bins,kind", [("fp32", 1, "exp"), ("fp32", 3, "exp"), ("fp32", 6, "exp"),
                                              ("fp64", 2, "exp"), ("fp32", 5, "shape")])
def test_exp_rows_far_apart(ctx, prec, n_bins, kind):
    """t0 rows 23 slots apart with an offset (a 64-row tile spans 1449 slots,
    more than an LDS stage holds), ragged row and tau counts, windows past the
    data end, bins that leave a partial bin group; also a shape window."""
    _case("exp rows far apart %s %d %s" % (prec, n_bins, kind))
    atoms = tfsynth.make_atoms(331 + n_bins, 2200, 0.15, n_bins=n_bins,
                               injections=[tfsynth.Injection(0, "exp", 500 * T, 80 * T, 1.0)])
    base = tfsynth.regular_window("exp", 7 * T + 300, 23 * T, 90, 2 * T, 11 * T + 13, 130)
    win = _bump_window(base) if kind == "shape" else base
    run_and_check(ctx, atoms, win, prec)


def test_exp_long_bands_many_chunks(ctx):
    """Bands longer than several LDS chunks and truncated at the data end."""
    _case("exp long bands")
    atoms = tfsynth.make_atoms(401, 1500, 0.15,
                               injections=[tfsynth.Injection(0, "exp", 100 * T, 200 * T, 0.6)])
    win = tfsynth.regular_window("exp", 0, T, 200, 2 * T, 61 * T, 24)
    run_and_check(ctx, atoms, win, "fp32")


def _runs_case(case):
    """Maps for the runs form, from consecutive rows (every slot shared by 64
    rows) to rows 31 slots apart; ragged tiles, edges, bin groups, shapes."""
    if case.startswith("ragged"):
        atoms = tfsynth.make_atoms(111, 300, 0.2, n_bins=3,
                                   injections=[tfsynth.Injection(2, "exp", 40 * T, 30 * T, 1.2)])
        rng = np.random.default_rng(15)
        t0 = np.unique(np.concatenate([[-5 * T - 77, -T, -1, 0, 1, T - 1],
                                       rng.integers(0, 300 * T, size=120),
                                       [299 * T, 299 * T + 1, 300 * T + 5, 400 * T]]))
        tau = np.unique(np.concatenate([[1, T - 1, T, T + 1, 2 * T], rng.integers(2 * T, 200 * T, size=37),
                                        [300 * T, 1000 * T]]))
        return atoms, tfsynth.list_window("exp", t0, tau)
    if case.startswith("bins"):
        n_bins = int(case[4:])
        atoms = tfsynth.make_atoms(220 + n_bins, 700, 0.1, n_bins=n_bins)
        return atoms, tfsynth.regular_window("exp", 5 * T + 9, 7 * T, 93, 2 * T, 5 * T + 1, 41)
    if case == "consecutive":
        atoms = tfsynth.make_atoms(231, 500, 0.1, n_bins=2)
        return atoms, tfsynth.regular_window("exp", 0, T, 130, 2 * T, T, 77)
    if case == "far31":
        atoms = tfsynth.make_atoms(232, 3100, 0.15, n_bins=1,
                                   injections=[tfsynth.Injection(0, "exp", 900 * T, 60 * T, 1.0)])
        return atoms, tfsynth.regular_window("exp", 2 * T + 500, 31 * T, 97, 2 * T, 13 * T, 36)
    if case.startswith("shape"):
        atoms = tfsynth.make_atoms(233, 900, 0.1, n_bins=5)
        base = tfsynth.regular_window("exp", 100, 9 * T, 90, 2 * T, 3 * T + 7, 45)
        return atoms, _bump_window(base)
    raise ValueError(case)


@pytest.mark.parametrize("case,prec", [("ragged", "fp32"), ("ragged", "fp64"), ("bins1", "fp32"),
                                       ("bins2", "fp32"), ("bins5", "fp32"), ("bins8", "fp32"),
                                       ("bins1", "fp64"), ("consecutive", "fp32"), ("far31", "fp32"),
                                       ("far31", "fp64"), ("shape", "fp32"), ("shape", "fp64")])
def test_exp_runs_form(ctx, case, prec):
    """The runs form on every map (tiling threshold 0): t0 off the slot grid,
    before and after the data, taus shorter than one SFT and longer than the
    data, partial bin groups, groups of four tau blocks with a ragged last
    group, shape windows."""
    _case("exp runs form %s %s" % (case, prec))
    atoms, win = _runs_case(case)
    with tiling(ctx, RUNS_ALWAYS):
        run_and_check(ctx, atoms, win, prec)


def test_exp_forms_agree(ctx):
    """The two forms of the same map agree within the FP32 tolerance, and
    each is bitwise repeatable."""
    _case("exp forms agree")
    atoms, win = _runs_case("bins5")
    aid = ctx.upload_atoms(atoms)
    try:
        out = {}
        for name, v in (("dense", DENSE_ONLY), ("runs", RUNS_ALWAYS)):
            with tiling(ctx, v):
                a, ma = ctx.fmap(aid, win, "fp32", want_map=True)
                b, mb = ctx.fmap(aid, win, "fp32", want_map=True)
            assert torch_equal(ma, mb)
            out[name] = (a, ma.cpu().numpy().astype(np.float64))
        d, r = out["dense"][1], out["runs"][1]
        assert np.all((d == 0) == (r == 0))
        assert np.max(np.abs(d - r) / np.maximum(np.abs(d), 1.0)) <= 2e-4
    finally:
        ctx.free(aid)


@pytest.mark.parametrize("case", ["bins8", "bins9", "bins12", "ragged12", "shape10", "tail"])
def test_exp_split_form(ctx, case):
    """The split form (A, B, C once per cell, then F_a, F_b four bins per
    lane) against the oracle: 8, 9 and 12 bins (a partial last group), t0
    off the slot grid and before/after the data, shape windows, and bands
    reaching past the data end; also against the form without the split."""
    _case("exp split form " + case)
    if case.startswith("bins"):
        n_bins = int(case[4:])
        atoms = tfsynth.make_atoms(240 + n_bins, 420, 0.12, n_bins=n_bins,
                                   injections=[tfsynth.Injection(3, "exp", 90 * T, 25 * T, 1.0)])
        win = tfsynth.regular_window("exp", 7 + 2 * T, T, 150, 2 * T, 3 * T + 11, 43)
    elif case == "ragged12":
        atoms = tfsynth.make_atoms(251, 300, 0.2, n_bins=12)
        rng = np.random.default_rng(25)
        t0 = np.unique(np.concatenate([[-5 * T - 77, -T, -1, 0, 1, T - 1],
                                       rng.integers(0, 300 * T, size=120), [299 * T + 1, 300 * T + 5]]))
        tau = np.unique(np.concatenate([[1, T - 1, T, 2 * T], rng.integers(2 * T, 200 * T, size=29),
                                        [300 * T, 1000 * T]]))
        win = tfsynth.list_window("exp", t0, tau)
    elif case == "shape10":
        atoms = tfsynth.make_atoms(252, 500, 0.1, n_bins=10)
        win = _bump_window(tfsynth.regular_window("exp", 100, 2 * T, 140, 2 * T, 5 * T + 7, 33))
    else:
        atoms = tfsynth.make_atoms(253, 260, 0.1, n_bins=8)
        win = tfsynth.regular_window("exp", 0, T, 200, 20 * T, 11 * T, 30)
    res, ref, err = run_and_check(ctx, atoms, win, "fp32")
    aid = ctx.upload_atoms(atoms)
    try:
        with tiling(ctx, -1, 0):
            other, m_other = ctx.fmap(aid, win, "fp32", want_map=True)
        _, m_split = ctx.fmap(aid, win, "fp32", want_map=True)
        a = m_split.cpu().numpy().astype(np.float64)
        b = m_other.cpu().numpy().astype(np.float64)
        assert np.all((a == 0) == (b == 0))
        assert np.max(np.abs(a - b) / np.maximum(np.abs(b), 1.0)) <= 2e-4
    finally:
        ctx.free(aid)


def torch_equal(a, b):
    import torch
    return bool(torch.equal(a, b))


def test_single_cell_and_single_sft(ctx):
    _case("single cell / single sft")
    atoms = tfsynth.make_atoms(5, 2, 0.0)
    for kind in ("rect", "exp"):
        win = tfsynth.regular_window(kind, 0, T, 1, 5 * T, T, 1)
        run_and_check(ctx, atoms, win, "fp32")
    one = tfsynth.Atoms(np.array([7 * T], dtype=np.int64), np.array([0.3]), np.array([0.1]),
                        np.array([0.09]), np.array([0.01]), np.array([0.03]),
                        np.array([[[0.5, -0.25]]]), np.array([[[0.125, 1.0]]]))
    for kind in ("rect", "exp"):
        win = tfsynth.regular_window(kind, 6 * T, T, 3, T, T, 3)
        res, ref, _ = run_and_check(ctx, one, win, "fp64")
        assert np.all(ref == 0.0)


def test_degenerate_windows(ctx):
    """Collinear antenna patterns make every window rank one (D = 0), and a
    pattern vanishing at some SFTs makes single-SFT windows badly scaled;
    both must give exactly 2F = 0 where the oracle does."""
    _case("degenerate windows")
    base = tfsynth.make_atoms(81, 400, 0.1, n_bins=2)
    x = base.fa[..., 0] / np.where(base.a == 0, 1, base.a)
    a = base.a.copy()
    a[::7] *= 1e-5
    for b_of_a in (lambda a: 2 * a, lambda a: base.b):
        b = b_of_a(a)
        fa = np.stack([a * x, 0 * x], -1)
        fb = np.stack([b * x, 0 * x], -1)
        atoms = tfsynth.Atoms(base.timestamps, a, b, a * a, b * b, a * b, fa, fb)
        for kind in ("rect", "exp"):
            win = tfsynth.regular_window(kind, 0, T, 390, T // 2, T, 12)
            for prec in ("fp64", "fp32"):
                run_and_check(ctx, atoms, win, prec)


def test_loud_injection_argmax(ctx):
    _case("loud injection")
    t0, tau = 40 * T, 25 * T
    for kind in ("rect", "exp"):
        atoms = tfsynth.make_atoms(91, 150, 0.1, injections=[tfsynth.Injection(0, kind, t0, tau, 4.5)])
        win = tfsynth.regular_window(kind, 0, T, 100, 2 * T, T, 140)
        res, ref, _ = run_and_check(ctx, atoms, win, "fp32")
        assert res[0]["max2F"] > (150 if kind == "rect" else 80)


# ---------------------------------------------------------------------------
# Full-size workloads, in the launch configuration the benchmark times
# ---------------------------------------------------------------------------

def test_full_exp_1bin_fp32(ctx):
    """5000 slots, 1000 x 1000 grid, tau to 30 days: every cell against the
    oracle's full map, and the per-bin results."""
    _case("full exp 1 bin fp32")
    atoms, win = tfsynth.workload_exp_1bin()
    aid = ctx.upload_atoms(atoms)
    try:
        res, twoF = ctx.fmap(aid, win, "fp32", want_map=True)
        res2, _ = ctx.fmap(aid, win, "fp32", want_map=False)
        assert res == res2, "results depend on whether the map is written"
    finally:
        ctx.free(aid)
    ref = oracle.fmap_atoms(atoms, win)
    err = check_map(twoF.cpu().numpy(), ref, 1e-4)
    check_results(res, ref, win, 1e-4)
    print("full exp 1 bin: max rel err %.3e" % err, flush=True)


@pytest.fixture(scope="module")
def exp256_oracle():
    """The 256-bin exponential workload and its full FP64 oracle map (every
    cell of every bin: 4.3e10 cells*SFTs*bins, computed once per module)."""
    atoms, win = tfsynth.workload_exp_bins()
    ref = oracle.fmap_atoms(atoms, win)
    return atoms, win, ref


@pytest.mark.parametrize("prec", ["fp32", "f16x3", "bf16x3"])
def test_full_exp_256_bins_every_cell(ctx, exp256_oracle, prec):
    """256 bins sharing antenna atoms, 2000 slots, 500 x 500 grid: every cell
    of every bin against the oracle's full map at the 2F tolerance, and the
    per-bin max 2F, argmax and logB against the oracle's reduction."""
    _case("full exp 256 bins every cell " + prec)
    atoms, win, ref = exp256_oracle
    aid = ctx.upload_atoms(atoms)
    try:
        res, twoF = ctx.fmap(aid, win, prec, want_map=True)
    finally:
        ctx.free(aid)
    err = check_map(twoF.cpu().numpy(), ref, TOL[prec])
    check_results(res, ref, win, TOL[prec])
    print("full exp 256 bins %s: max rel err %.3e over %d cells" % (prec, err, ref.size), flush=True)


@pytest.mark.parametrize("case", ["mixed_spacing", "few_taus", "many_segments"])
def test_abc_scan_rows(ctx, case):
    """The A/B/C of matrix-core maps come from a scan of the row recurrence
    (64 rows per chunk, several segments per tau).  Rows that share a first
    slot, rows one slot and far apart (windows that end before the next row
    starts), rows before the data and past its end, taus shorter than one
    SFT, grids of 64 k +- 1 rows over several chunks and segments: every
    cell's 2F and the per-bin results against the oracle (F16X3)."""
    _case("abc scan " + case)
    rng = np.random.default_rng({"mixed_spacing": 91, "few_taus": 92, "many_segments": 93}[case])
    atoms = tfsynth.make_atoms(9100 + len(case), 900, 0.15, n_bins=5,
                               injections=[tfsynth.Injection(2, "exp", 200 * T, 40 * T, 1.0)])
    T0 = int(atoms.timestamps[0])
    if case == "mixed_spacing":
        # steps of 0 (same slot), a few seconds, one slot, and far apart
        steps = rng.choice([7, 300, T, T + 11, 3 * T, 40 * T], size=192)
        t0 = T0 - 30 * T + np.cumsum(steps)
        tau = np.concatenate([[T // 3, T - 1], np.arange(2, 60, 3) * T + 17, [300 * T, 2000 * T]])
    elif case == "few_taus":
        t0 = T0 - 5 * T + np.arange(129) * (T // 2)
        tau = np.array([5 * T, 70 * T + 3, 400 * T], dtype=np.int64)
    else:
        # 700 rows x 600 taus: segments of three 64-row chunks
        t0 = T0 + 20 * T + np.arange(700) * T + 13
        tau = np.arange(1, 601) * (T // 2)
    win = tfsynth.list_window("exp", np.unique(t0.astype(np.int64)), tau.astype(np.int64))
    _, _, err = run_and_check(ctx, atoms, win, "f16x3")
    print("abc scan %s: %d rows, %d taus, max rel err %.3e" % (case, win.n_t0, win.n_tau, err), flush=True)


@pytest.mark.parametrize("prec", ["f16x3", "bf16x3"])
@pytest.mark.parametrize("case", ["offset", "tail", "sparse_rows"])
def test_matrix_ragged(ctx, case, prec):
    """Matrix-core path: 21 bins (ragged bin tile), rows off the slot grid by
    a common offset, a partial row tile, bands past the data end, rows three
    slots apart."""
    _case("%s %s" % (prec, case))
    atoms = tfsynth.make_atoms(3, 777, 0.1, n_bins=21,
                               injections=[tfsynth.Injection(4, "exp", 90 * T, 50 * T, 0.8)])
    if case == "offset":
        win = tfsynth.regular_window("exp", 5 * T + 77, T, 123, 2 * T, 3 * T + 5, 61)
    elif case == "tail":
        win = tfsynth.regular_window("exp", 700 * T, T, 77, 2 * T, 40 * T, 9)
    else:
        win = tfsynth.regular_window("exp", 0, 3 * T, 90, 2 * T, 5 * T, 30)
    _, _, err = run_and_check(ctx, atoms, win, prec)
    print("%s %s: max rel err %.3e" % (prec, case, err), flush=True)


def _kernel_launches(ctx, fn):
    ctx.profile_reset()
    ctx.profile(True)
    try:
        out = fn()
    finally:
        ctx.profile(False)
    return out, ctx.profile_read()


@pytest.mark.parametrize("prec", ["f16x3", "bf16x3"])
@pytest.mark.parametrize("case", ["linspace", "stride7", "before_after", "bins5", "bins37", "bins1_valu", "bins3",
                                  "one_row_tile", "long_and_short", "scaled", "bins70", "bins64_stride3",
                                  "bins150", "bins520", "bins2", "bins4", "bins48", "bins49"])
def test_matrix_any_grid(ctx, case, prec):
    """Matrix cores for exponential windows on any t0 grid (weights computed
    per row): linspace rows with their own offsets, rows 7 slots apart, rows
    before and after the data, ragged bin counts (partial 16-bin column
    tiles), a one-bin map (FP32 path) and a three-bin one, a single partial row
    tile, tau blocks with short bands beside long ones (FP32 F-only tiles),
    and data far outside the half-precision range with one all-zero bin
    (the half-precision path's column scaling).  Maps of 2 to 48 bins take
    the transposed work item (one bin per item; 2 and 4 bins: one bin per
    XCD, 8 or more: bins dealt over the XCDs, others in plain order), maps
    of 49 to 520 bins the work items of four column tiles with shared
    weights (49 bins: the smallest such map; 70 bins: a last group of one
    column tile and three waves without one; 70, 150 and 520 bins: 2, 3 and
    9 column groups, each with its own order of work items over the XCDs).
    Every cell and the per-bin results against the oracle."""
    _case("%s any grid %s" % (prec, case))
    n_bins = {"bins5": 5, "bins37": 37, "bins1_valu": 1, "bins3": 3, "bins70": 70, "bins64_stride3": 64,
              "bins150": 150, "bins520": 520, "bins2": 2, "bins4": 4, "bins48": 48, "bins49": 49}.get(case, 24)
    atoms = tfsynth.make_atoms(811, 1400, 0.12, n_bins=n_bins,
                               injections=[tfsynth.Injection(min(4, n_bins - 1), "exp", 300 * T, 60 * T, 1.0)])
    if case == "scaled":
        # F is unchanged when F_a, F_b scale by s and a^2, b^2, ab by s^2:
        # s = 2^20 puts the data far beyond the half-precision range; bin 7
        # holds no data at all (2F = 0 everywhere)
        fa, fb = atoms.fa * 2.0 ** 20, atoms.fb * 2.0 ** 20
        fa[7] = 0.0
        fb[7] = 0.0
        atoms = dataclasses.replace(atoms, fa=fa, fb=fb, a2=atoms.a2 * 2.0 ** 40, b2=atoms.b2 * 2.0 ** 40,
                                    ab=atoms.ab * 2.0 ** 40)
    if case in ("linspace", "bins5", "bins37", "bins1_valu", "bins3", "scaled", "bins70", "bins2", "bins4", "bins48",
                "bins49"):
        win = tfsynth.linspace_grid(atoms, "exp", 260, 110)
    elif case == "bins64_stride3":
        win = tfsynth.regular_window("exp", 50 * T + 3, 3 * T, 150, 2 * T, 4 * T + 9, 75)
    elif case in ("bins150", "bins520"):
        win = tfsynth.linspace_grid(atoms, "exp", 70, 40)
    elif case == "stride7":
        win = tfsynth.regular_window("exp", 333, 7 * T, 150, 2 * T, 5 * T + 17, 70)
    elif case == "before_after":
        win = tfsynth.regular_window("exp", -40 * T - 11, 13 * T, 140, 3 * T, 9 * T + 1, 60)
    elif case == "one_row_tile":
        win = tfsynth.regular_window("exp", 100 * T + 7, 3 * T, 37, 40 * T, 11 * T, 21)
    else:
        tau = np.concatenate([np.arange(2, 30) * T + 11, np.arange(30, 80, 2) * T + 3, [900 * T, 1500 * T]])
        win = tfsynth.list_window("exp", 5 + np.arange(0, 1300, 9) * T, tau)
    aid = ctx.upload_atoms(atoms)
    try:
        (res, twoF), prof = _kernel_launches(ctx, lambda: ctx.fmap(aid, win, prec, want_map=True))
        ref = oracle.fmap_atoms(atoms, win)
        err = check_map(twoF.cpu().numpy(), ref, TOL[prec])
        check_results(res, ref, win, TOL[prec])
        assert (prof["mfma"][0] > 0) == (case != "bins1_valu"), prof["mfma"]
        # the same map again: bitwise repeatable
        res2, _ = ctx.fmap(aid, win, prec)
        assert res2 == res
    finally:
        ctx.free(aid)
    print("%s %s: max rel err %.3e" % (prec, case, err), flush=True)


def test_f16x3_bin_scales(ctx):
    """Half-precision parts with each bin's data scaled by its own power of
    two (2^-40 .. 2^40, beyond both ends of the half-precision range) and a
    non-power-of-two scale on one bin: every cell's 2F against the oracle of
    the scaled atoms (2F grows with the square of the scale, so the logB of
    such bins is compared through max 2F and argmax only)."""
    _case("f16x3 bin scales")
    n_bins = 18
    atoms = tfsynth.make_atoms(813, 900, 0.1, n_bins=n_bins)
    k = np.linspace(-40, 40, n_bins).round().astype(int)
    scale = np.ldexp(1.0, k)
    scale[5] = 3.0e-3
    fa = (atoms.fa * scale[:, None, None]).astype(np.float32).astype(np.float64)
    fb = (atoms.fb * scale[:, None, None]).astype(np.float32).astype(np.float64)
    atoms = dataclasses.replace(atoms, fa=fa, fb=fb)
    win = tfsynth.linspace_grid(atoms, "exp", 130, 70)
    aid = ctx.upload_atoms(atoms)
    try:
        res, twoF = ctx.fmap(aid, win, "f16x3", want_map=True)
    finally:
        ctx.free(aid)
    ref = oracle.fmap_atoms(atoms, win)
    got = twoF.cpu().numpy().astype(np.float64)
    mx, am, _ = oracle.reduce(ref)
    worst = 0.0
    for b in range(n_bins):
        # relative to the bin's own largest 2F (the floor of 1 would hide
        # the tiny bins)
        e = np.abs(got[b] - ref[b]).max() / mx[b]
        worst = max(worst, e)
        assert e <= TOL["f16x3"], (b, e)
        assert abs(res[b]["max2F"] - mx[b]) <= TOL["f16x3"] * mx[b], (b, res[b]["max2F"], mx[b])
        idx = res[b]["m"] * win.n_tau + res[b]["n"]
        assert idx == am[b] or ref[b].ravel()[idx] >= (1 - 1e-4) * mx[b], (b, idx, am[b])
    print("f16x3 bin scales: max err relative to each bin's max 2F %.3e" % worst, flush=True)


@pytest.mark.parametrize("case", ["stride1", "stride3_delta", "past_end", "before_data", "bins5",
                                  "irregular"])
def test_recur64_edges(ctx, case):
    """Exponential sums by the t0 recurrence: strides, a common offset,
    rows past the end of the data and before its start, ragged bin groups,
    and an irregular grid (direct FP64 sums)."""
    _case("recur64 " + case)
    if case == "stride1":
        atoms = tfsynth.make_atoms(1, 150, 0.2, 2)
        win = tfsynth.regular_window("exp", 0, T, 100, 2 * T, 3 * T + 7, 9)
    elif case == "stride3_delta":
        atoms = tfsynth.make_atoms(2, 200, 0.1, 1)
        win = tfsynth.regular_window("exp", 77, 3 * T, 70, T // 2, 5 * T, 8)
    elif case == "past_end":
        atoms = tfsynth.make_atoms(3, 120, 0.3, 1)
        win = tfsynth.regular_window("exp", 60 * T, T, 90, 2 * T, 11 * T, 6)
    elif case == "before_data":
        atoms = tfsynth.make_atoms(4, 120, 0.1, 1)
        win = tfsynth.regular_window("exp", -20 * T - 5, 2 * T, 40, 2 * T, 13 * T, 5)
    elif case == "bins5":
        atoms = tfsynth.make_atoms(5, 700, 0.15, 5,
                                   injections=[tfsynth.Injection(3, "exp", 100 * T, 60 * T, 1.0)])
        win = tfsynth.regular_window("exp", 0, T, 300, 2 * T, 4 * T, 70)
    else:
        atoms = tfsynth.make_atoms(6, 300, 0.1, 2)
        win = tfsynth.list_window("exp", [0, 5 * T, 7 * T + 3, 40 * T, 41 * T], [2 * T, 9 * T, 70 * T])
    run_and_check(ctx, atoms, win, "recur64")


def test_full_exp_1bin_recur64(ctx):
    """The 1-bin benchmark workload by the recurrence, every cell."""
    _case("full exp 1 bin recur64")
    atoms, win = tfsynth.workload_exp_1bin()
    aid = ctx.upload_atoms(atoms)
    try:
        res, twoF = ctx.fmap(aid, win, "recur64", want_map=True)
    finally:
        ctx.free(aid)
    ref = oracle.fmap_atoms(atoms, win)
    err = check_map(twoF.cpu().numpy(), ref, 1e-8)
    check_results(res, ref, win, 1e-8)
    print("full exp 1 bin recur64: max rel err %.3e" % err, flush=True)


def test_full_rect_workload_results(ctx):
    """Rectangular window over the 256-bin atoms, 500 x 500 grid: every cell
    and the per-bin results against the oracle."""
    _case("full rect 256 bins")
    atoms, win = tfsynth.workload_exp_bins()
    win = tfsynth.regular_window("rect", 0, T, 500, 2 * T, T, 500)
    aid = ctx.upload_atoms(atoms)
    try:
        res, twoF = ctx.fmap(aid, win, "fp64", want_map=True)
    finally:
        ctx.free(aid)
    ref = oracle.fmap_atoms(atoms, win)
    check_map(twoF.cpu().numpy(), ref, TOL["fp64"])
    check_results(res, ref, win, TOL["fp64"])


# ---------------------------------------------------------------------------
# logB of stored maps, determinism
# ---------------------------------------------------------------------------

def test_logB_of_stored_map(ctx):
    import torch
    _case("logB stored map")
    rng = np.random.default_rng(23)
    maps = rng.chisquare(4, size=(3, 123, 457)).astype(np.float32)
    maps[1, 7, 9] = 1400.0      # exp(700) overflows a double without the shift
    dev = torch.from_numpy(maps).to("cuda:0")
    got = ctx.logB(dev)
    _, _, lb = oracle.reduce(maps.astype(np.float64))
    assert np.allclose(got, lb, atol=1e-9, rtol=0)


def test_deterministic_repeat(ctx):
    _case("determinism")
    atoms = tfsynth.make_atoms(77, 700, 0.1, n_bins=4)
    win = tfsynth.regular_window("exp", 0, T, 300, 2 * T, 2 * T, 150)
    aid = ctx.upload_atoms(atoms)
    try:
        r1, m1 = ctx.fmap(aid, win, "fp32", want_map=True)
        r2, m2 = ctx.fmap(aid, win, "fp32", want_map=True)
    finally:
        ctx.free(aid)
    assert r1 == r2
    assert bool((m1 == m2).all())


# ---------------------------------------------------------------------------
# Serving: results alone and in a concurrent mix are identical
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("max_batch,precs", [(16, ("fp32",)), (1, ("fp32",)),
                                             (5, ("fp32", "fp64", "bf16x3", "f16x3"))])
def test_submit_poll_mix_invariance(ctx, max_batch, precs):
    """Twelve uneven requests in flight at once give exactly the results of
    each alone: batched admission (up to 16 or 5 fused), one request per
    slot, and a mix of precisions of which only some can be fused."""
    import time
    _case("serving mix max_batch %d %s" % (max_batch, precs))
    reqs = []
    for i in range(12):
        atoms, win = tfsynth.candidate(i, max_slots=3000, max_grid=400, max_bins=6)
        reqs.append((atoms, win))
    prec = [precs[i % len(precs)] for i in range(len(reqs))]
    ids = [ctx.upload_atoms(a) for a, _ in reqs]
    ctx.serve_config(max_batch)
    try:
        alone = [ctx.fmap(aid, w, p)[0] for aid, (_, w), p in zip(ids, reqs, prec)]
        tickets = [ctx.submit(aid, w, p) for aid, (_, w), p in zip(ids, reqs, prec)]
        pending = dict(enumerate(tickets))
        got = {}
        t_end = time.time() + 60
        while pending and time.time() < t_end:
            for i, t in list(pending.items()):
                r = ctx.poll(t, reqs[i][0].n_bins)
                if r is not None:
                    got[i] = r
                    del pending[i]
            time.sleep(0.001)
        assert not pending, "requests did not finish"
        for i in range(len(reqs)):
            assert got[i] == alone[i], i
        # spot-check parity of a few against the oracle
        for i in (0, 1):
            atoms, win = reqs[i]
            check_results(got[i], oracle.fmap_atoms(atoms, win), win, TOL[prec[i]])
    finally:
        ctx.serve_config(16)
        for aid in ids:
            ctx.free(aid)


def test_cancel_and_errors(ctx):
    from paper_1805_05652_amd import TfstatError, _abi
    _case("errors")
    atoms = tfsynth.make_atoms(3, 100, 0.1)
    aid = ctx.upload_atoms(atoms)
    try:
        bad = tfsynth.list_window("exp", [0, 0], [T])
        with pytest.raises(TfstatError) as e:
            ctx.fmap(aid, bad, "fp32")
        assert e.value.code == _abi.E_GRID
        with pytest.raises(TfstatError) as e:
            ctx.fmap(aid + 1000, tfsynth.regular_window("exp", 0, T, 2, T, T, 2), "fp32")
        assert e.value.code == _abi.E_NOTFOUND
        with pytest.raises(TfstatError) as e:
            ctx.upload(np.array([0, 1000]), [1, 1], [1, 1], [0, 0], np.zeros((2, 2)),
                       np.zeros((2, 2)), 1800)
        assert e.value.code == _abi.E_GRID
        win = tfsynth.regular_window("exp", 0, T, 50, 2 * T, T, 50)
        tickets = [ctx.submit(aid, win, "fp32") for _ in range(6)]
        ctx.cancel(tickets[-1])
        import time
        t_end = time.time() + 30
        states = {}
        while len(states) < len(tickets) and time.time() < t_end:
            for t in tickets:
                if t in states:
                    continue
                try:
                    r = ctx.poll(t, 1)
                    if r is not None:
                        states[t] = "done"
                except TfstatError as err:
                    states[t] = err.code
            time.sleep(0.001)
        assert all(states[t] == "done" for t in tickets[:-1])
        assert states[tickets[-1]] in ("done", _abi.E_CANCELLED)
    finally:
        ctx.free(aid)


def test_arena_too_small():
    import paper_1805_05652_amd as tf
    from paper_1805_05652_amd import TfstatError, _abi
    _case("small arena")
    with tf.Context(0, arena_bytes=2 << 20) as small:
        atoms, win = tfsynth.workload_exp_1bin(n_slots=5000, n_t0=1000, n_tau=1000)
        aid = small.upload_atoms(atoms)
        with pytest.raises(TfstatError) as e:
            small.fmap(aid, win, "fp32")
        assert e.value.code == _abi.E_NOMEM
        small.free(aid)


# ---------------------------------------------------------------------------
# General window shapes through the exponential window's kernels
# ---------------------------------------------------------------------------

def _bump_window(base):
    # an asymmetric rise-and-decay shape, s(x) = x exp(1 - x) on [0, 4]
    x = np.linspace(0.0, 4.0, 257)
    return tfsynth.shape_window(base, x * np.exp(1.0 - x), (4, 1))


@pytest.mark.parametrize("prec", ["fp32", "fp64", "bf16x3", "f16x3"])
def test_shape_window_against_oracle(ctx, prec):
    """t0 100 s after each SFT start (one common offset), ragged taus, bins
    spanning a partial 16-bin column tile for the matrix-core path."""
    _case("shape window " + prec)
    n_bins = 19 if prec in ("bf16x3", "f16x3") else 3
    atoms = tfsynth.make_atoms(501, 420, 0.1, n_bins=n_bins,
                               injections=[tfsynth.Injection(1, "exp", 60 * T, 20 * T, 1.0)])
    rng = np.random.default_rng(7)
    tau = np.unique(np.concatenate([[T // 3, 2 * T], rng.integers(2 * T, 120 * T, size=45)]))
    base = tfsynth.list_window("exp", 100 + T * np.arange(-3, 150, dtype=np.int64), tau)
    run_and_check(ctx, atoms, _bump_window(base), prec)


def test_shape_window_constant_equals_rect(ctx):
    """A constant shape with support 1 gives the rectangular window's map."""
    _case("shape constant vs rect")
    atoms = tfsynth.make_atoms(503, 150, 0.1, n_bins=2)
    base = tfsynth.regular_window("rect", 0, T, 120, T, 700, 90)
    aid = ctx.upload_atoms(atoms)
    try:
        _, rect = ctx.fmap(aid, base, "fp64", want_map=True)
        _, shp = ctx.fmap(aid, tfsynth.shape_window(base, np.ones(5), (1, 1)), "fp64", want_map=True)
        ref = oracle.fmap_atoms(atoms, base)
        check_map(rect.cpu().numpy(), ref, TOL["fp64"])
        check_map(shp.cpu().numpy(), ref, TOL["fp64"])
    finally:
        ctx.free(aid)


def test_shape_window_errors(ctx):
    import paper_1805_05652_amd as tf
    _case("shape window errors")
    atoms = tfsynth.make_atoms(505, 100, 0.0)
    aid = ctx.upload_atoms(atoms)
    try:
        uneven = tfsynth.shape_window(tfsynth.list_window("exp", [0, T + 5], [3 * T]), np.ones(3))
        with pytest.raises(tf.TfstatError) as e:
            ctx.fmap(aid, uneven, "fp32")
        assert e.value.code == tf._abi.E_GRID
        ok = tfsynth.shape_window(tfsynth.list_window("exp", [0, T], [3 * T]), np.ones(3))
        with pytest.raises(tf.TfstatError) as e:
            ctx.fmap(aid, ok, "recur64")
        assert e.value.code == tf._abi.E_INVAL
        bad = tfsynth.shape_window(tfsynth.list_window("exp", [0, T], [3 * T]), np.array([1.0, np.nan]))
        with pytest.raises(tf.TfstatError) as e:
            ctx.fmap(aid, bad, "fp32")
        assert e.value.code == tf._abi.E_INVAL
    finally:
        ctx.free(aid)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_window_odds_against_oracle(ctx, prec):
    """Rect against exp on the same atoms (section 5: window models compared
    through their Bayes factors): per-bin log odds logB_exp - logB_rect
    against the oracle's two logB values, within the sum of the two logB
    tolerances; different grids for the two models; bin 1 holds a loud
    exponential transient, which the exponential model must favour."""
    from checks import LOGB_TOL
    _case("window odds " + prec)
    atoms = tfsynth.make_atoms(511, 600, 0.1, n_bins=3,
                               injections=[tfsynth.Injection(1, "exp", 100 * T, 40 * T, 3.0)])
    w_exp = tfsynth.regular_window("exp", 0, 2 * T, 250, 2 * T, 3 * T, 120)
    w_rect = tfsynth.regular_window("rect", 0, T, 480, 2 * T, 5 * T, 110)
    aid = ctx.upload_atoms(atoms)
    try:
        got = ctx.window_odds(aid, w_exp, w_rect, prec)
        _, _, lb_e = oracle.reduce(oracle.fmap_atoms(atoms, w_exp))
        _, _, lb_r = oracle.reduce(oracle.fmap_atoms(atoms, w_rect))
        ref = lb_e - lb_r
        assert np.all(np.abs(got - ref) <= 2 * LOGB_TOL), (got, ref)
        assert ref[1] > 0.0 and got[1] > 0.0, (got, ref)
        back = ctx.window_odds(aid, w_rect, w_exp, prec)
        assert np.array_equal(back, -got)
    finally:
        ctx.free(aid)
