"""GPU parity of the uneven batch (tfstat_batch_*): many maps of different
candidates, grids, bin counts and window types in one captured graph with
one persistent fused launch.

Each map of a batch is checked two ways:
  * against the FP64 CPU oracle (per-bin max 2F, argmax, logB) with the
    tolerances of the single-map tests (2F 1e-4 relative in FP32 and 1e-9 in
    FP64, logB 1e-3 absolute, argmax exact or a near-tie);
  * against tfstat_fmap of the same map: the batch's default variant keeps
    each map's own tile shape, so its results are bit-identical.
"""
import numpy as np
import pytest

import oracle
import tfsynth

pytestmark = pytest.mark.gpu

T = tfsynth.T_SFT
from checks import TOL, check_results  # noqa: E402


def _case(msg):
    print("case:", msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import paper_1805_05652_amd as tf
    c = tf.Context(0, arena_bytes=3 << 30)
    yield c
    c.close()


def small_candidates(n=8, seed_base=7100):
    """Uneven candidates at sizes the oracle maps in well under a second."""
    return [tfsynth.candidate(i, seed_base=seed_base, max_slots=600, max_grid=150, max_bins=6)
            for i in range(n)]


def check_against_oracle(res, atoms, win, tol):
    check_results(res, oracle.fmap_atoms(atoms, win), win, tol)


def same_results(a, b):
    assert len(a) == len(b)
    for x, y in zip(a, b):
        assert (x["max2F"], x["logB"], x["m"], x["n"]) == (y["max2F"], y["logB"], y["m"], y["n"]), (x, y)


def upload_all(ctx, cands):
    return [ctx.upload_atoms(a) for a, _ in cands]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_small_batch_against_oracle_and_fmap(ctx, prec):
    _case("small uneven batch " + prec)
    cands = small_candidates()
    kinds = {w.kind for _, w in cands}
    assert kinds == {"rect", "exp"}
    ids = upload_all(ctx, cands)
    try:
        with ctx.batch(list(zip(ids, [w for _, w in cands])), prec) as b:
            st = b.stats()
            assert st["variant"] == ("mixed" if prec == "fp32" else "fp64_r4")
            assert st["n_results"] == sum(a.n_bins for a, _ in cands)
            got = b.run()
        for (atoms, win), aid, res in zip(cands, ids, got):
            check_against_oracle(res, atoms, win, TOL[prec])
            single, _ = ctx.fmap(aid, win, prec)
            same_results(res, single)
    finally:
        for aid in ids:
            ctx.free(aid)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_sparse_row_batch(ctx, prec):
    """Candidates with few t0 rows over long data (64-row tiles that span
    more slots than an LDS stage holds) mixed with rect maps."""
    _case("sparse-row batch " + prec)
    cands = [tfsynth.candidate(i, seed_base=7600, max_slots=4000, max_grid=120, max_bins=6) for i in range(6)]
    ids = upload_all(ctx, cands)
    try:
        with ctx.batch(list(zip(ids, [w for _, w in cands])), prec) as b:
            got = b.run()
        for (atoms, win), aid, res in zip(cands, ids, got):
            check_against_oracle(res, atoms, win, TOL[prec])
            single, _ = ctx.fmap(aid, win, prec)
            same_results(res, single)
    finally:
        for aid in ids:
            ctx.free(aid)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_runs_form(ctx, prec):
    """Every exponential map of the batch on the runs form (tiling threshold
    0): against the oracle, and bit-identical to tfstat_fmap of the same map
    planned the same way."""
    _case("batch runs form " + prec)
    cands = small_candidates(8, seed_base=7700)
    ids = upload_all(ctx, cands)
    try:
        ctx.tiling_config(0)
        with ctx.batch(list(zip(ids, [w for _, w in cands])), prec) as b:
            got = b.run()
        for (atoms, win), aid, res in zip(cands, ids, got):
            check_against_oracle(res, atoms, win, TOL[prec])
            single, _ = ctx.fmap(aid, win, prec)
            same_results(res, single)
    finally:
        ctx.tiling_config(-1)
        for aid in ids:
            ctx.free(aid)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_split_form(ctx, prec):
    """Maps of 8 to 13 bins (FP32: the split form, an A/B/C pre-pass and
    F_a/F_b-only tiles in the persistent launch; FP64: plain tiles) mixed
    with rect maps: against the oracle and bit-identical to tfstat_fmap."""
    _case("batch split form " + prec)
    cands = []
    for i in range(6):
        atoms = tfsynth.make_atoms(7800 + i, 300 + 90 * i, 0.1 * (i % 3), n_bins=8 + i,
                                   injections=[tfsynth.Injection(i % 4, "exp", 50 * T, 20 * T, 1.0)])
        kind = "rect" if i % 3 == 2 else "exp"
        win = tfsynth.regular_window(kind, 3 * T + 7 * i, T, 70 + 20 * i, 2 * T,
                                     2 * T + 13 * i, 31 + 7 * i)
        cands.append((atoms, win))
    ids = upload_all(ctx, cands)
    try:
        with ctx.batch(list(zip(ids, [w for _, w in cands])), prec) as b:
            got = b.run()
            again = b.run()
        for (atoms, win), aid, res, res2 in zip(cands, ids, got, again):
            check_against_oracle(res, atoms, win, TOL[prec])
            single, _ = ctx.fmap(aid, win, prec)
            same_results(res, single)
            same_results(res, res2)
    finally:
        for aid in ids:
            ctx.free(aid)


def test_graph_replays_with_eager_work_between(ctx):
    """Every replay of the captured graph gives the first run's results, with
    the library's own eager launches and synchronisations in between."""
    _case("batch graph replays")
    cands = small_candidates(6, seed_base=7200)
    ids = upload_all(ctx, cands)
    try:
        with ctx.batch(list(zip(ids, [w for _, w in cands])), "fp32") as b:
            first = b.run()
            for rep in range(4):
                ctx.fmap(ids[rep % len(ids)], cands[rep % len(ids)][1], "fp32")
                again = b.run()
                for x, y in zip(first, again):
                    same_results(x, y)
    finally:
        for aid in ids:
            ctx.free(aid)


def test_autotuned_batch(ctx):
    """The autotuner times every tile shape and width and keeps one; the
    chosen plan matches the oracle, and a batch of the same shape reuses the
    choice without tuning again."""
    _case("autotuned batch")
    cands = small_candidates(6, seed_base=7300)
    ids = upload_all(ctx, cands)
    items = list(zip(ids, [w for _, w in cands]))
    try:
        with ctx.batch(items, "fp32", tune=True) as b:
            st = b.stats()
            assert st["tune_ms"] > 0.0
            assert st["variant"].replace("_lowocc", "") in ("fp32_r8", "fp32_r4_b2", "fp32_r4_b4", "mixed")
            assert st["groups"] >= 1
            got = b.run()
        for (atoms, win), res in zip(cands, got):
            check_against_oracle(res, atoms, win, TOL["fp32"])
        with ctx.batch(items, "fp32", tune=True) as b2:
            st2 = b2.stats()
            assert st2["tune_ms"] == 0.0
            assert (st2["variant"], st2["groups"]) == (st["variant"], st["groups"])
    finally:
        for aid in ids:
            ctx.free(aid)


def test_batch_holds_atoms_and_rejects_bad_input(ctx):
    import paper_1805_05652_amd as tf
    _case("batch errors")
    cands = small_candidates(2, seed_base=7400)
    ids = upload_all(ctx, cands)
    items = list(zip(ids, [w for _, w in cands]))
    b = ctx.batch(items, "fp32")
    with pytest.raises(tf.TfstatError) as e:
        ctx.free(ids[0])
    assert e.value.code == tf._abi.E_BUSY
    b.close()
    with pytest.raises(tf.TfstatError) as e:
        ctx.batch(items, "recur64")
    assert e.value.code == tf._abi.E_INVAL
    with pytest.raises(tf.TfstatError) as e:
        ctx.batch([(987654, cands[0][1])], "fp32")
    assert e.value.code == tf._abi.E_NOTFOUND
    for aid in ids:
        ctx.free(aid)


def _variant_maps():
    """Maps that reach every tile kind of the fused kernel: one-bin, five-bin
    (four-bin group + one-bin tail) and six-bin (+ bin-pair tail) dense
    maps, a nine-bin map (split form in FP32), a map whose rows are far
    apart (runs form) and a rectangular map."""
    maps = []
    for i, nb in enumerate((1, 5, 6, 9)):
        atoms = tfsynth.make_atoms(7900 + i, 420 + 60 * i, 0.1, n_bins=nb)
        maps.append((atoms, tfsynth.regular_window("exp", 3 * T + 11, T, 90 + 7 * i, 2 * T, 3 * T, 33)))
    atoms = tfsynth.make_atoms(7910, 1500, 0.12, n_bins=3)
    maps.append((atoms, tfsynth.regular_window("exp", 0, 9 * T, 100, 2 * T, 5 * T, 40)))
    atoms = tfsynth.make_atoms(7911, 500, 0.1, n_bins=2)
    maps.append((atoms, tfsynth.regular_window("rect", 0, T, 150, 2 * T, T, 120)))
    return maps


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_every_fused_variant(ctx, prec):
    """Each build of the persistent kernel (every tile shape, each at the
    stand-alone waves per SIMD and one fewer) forced on one batch of maps
    that reaches every tile kind: each map matches the oracle."""
    _case("every fused variant " + prec)
    import paper_1805_05652_amd._abi as abi
    maps = _variant_maps()
    refs = []
    for atoms, win in maps:
        ref = oracle.fmap_atoms(atoms, win)
        refs.append((ref, oracle.reduce(ref)))
    ids = upload_all(ctx, maps)
    names = ["fp64_r4"] if prec == "fp64" else ["fp32_r8", "fp32_r4_b2", "fp32_r4_b4", "mixed"]
    names = names + [v + "_lowocc" for v in names]
    try:
        for name in names:
            assert name in abi.BATCH_VARIANTS
            with ctx.batch(list(zip(ids, [w for _, w in maps])), prec, variant=name) as b:
                assert b.stats()["variant"] == name
                got = b.run()
            for (atoms, win), (ref, (mx, am, lb)), res in zip(maps, refs, got):
                assert len(res) == atoms.n_bins
                for bn, r in enumerate(res):
                    assert abs(r["logB"] - lb[bn]) <= 1e-3, (name, bn, r["logB"], lb[bn])
                    assert abs(r["max2F"] - mx[bn]) <= TOL[prec] * max(mx[bn], 1.0), (name, bn, r["max2F"], mx[bn])
                    idx = r["m"] * win.n_tau + r["n"]
                    assert idx == am[bn] or ref[bn].ravel()[idx] >= (1 - 1e-4) * mx[bn], (name, bn, idx, am[bn])
        with pytest.raises(RuntimeError):
            ctx.batch(list(zip(ids, [w for _, w in maps])), prec,
                      variant="fp32_r8" if prec == "fp64" else "fp64_r4")
    finally:
        for aid in ids:
            ctx.free(aid)


def test_full_uneven_batch_64_candidates():
    """The 64-candidate uneven batch at full size, in the launch
    configuration the benchmark times (autotuned): the tuner keeps each map's
    own tile shape, so every map is bit-identical to the single-map path.
    Agreement with the oracle is checked for all 64 maps in
    test_full_uneven_batch_against_oracle."""
    import paper_1805_05652_amd as tf
    _case("full uneven batch, 64 candidates")
    cands = [tfsynth.candidate(i) for i in range(64)]
    c = tf.Context(0, arena_bytes=16 << 30)
    try:
        ids = [c.upload_atoms(a) for a, _ in cands]
        with c.batch(list(zip(ids, [w for _, w in cands])), "fp32", tune=True) as b:
            got = b.run()
            assert b.stats()["variant"] in ("mixed", "mixed_lowocc")
        for (atoms, win), aid, res in zip(cands, ids, got):
            single, _ = c.fmap(aid, win, "fp32")
            same_results(res, single)
    finally:
        c.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_composition_invariance(ctx, prec):
    """One map in two different autotuned batches and alone: bit-identical
    results each time (a result never depends on the other maps)."""
    _case("batch composition invariance " + prec)
    cands = small_candidates(10, seed_base=7300)
    ids = upload_all(ctx, cands)
    wins = [w for _, w in cands]
    try:
        probe = [i for i, (_, w) in enumerate(cands) if w.kind == "exp"][:2] + \
                [i for i, (_, w) in enumerate(cands) if w.kind == "rect"][:1]
        first = list(range(0, 6))
        second = [i for i in range(10) if i % 2 == 1 or i in probe][::-1]
        got = {}
        for members in (first, second):
            with ctx.batch([(ids[i], wins[i]) for i in members], prec, tune=True) as b:
                assert b.stats()["variant"] in (("mixed", "mixed_lowocc") if prec == "fp32"
                                                else ("fp64_r4", "fp64_r4_lowocc"))
                for i, res in zip(members, b.run()):
                    got.setdefault(i, []).append(res)
        for i in probe:
            alone, _ = ctx.fmap(ids[i], wins[i], prec)
            for res in got[i]:
                same_results(res, alone)
    finally:
        for aid in ids:
            ctx.free(aid)


def test_timed_run_matches_graph_run(ctx):
    """The direct launches of a timed run give the graph replay's results and
    a positive fused-kernel time."""
    _case("batch timed run")
    cands = small_candidates(4, seed_base=7500)
    ids = upload_all(ctx, cands)
    try:
        with ctx.batch(list(zip(ids, [w for _, w in cands])), "fp32") as b:
            g = b.run()
            t = b.run(timed=True)
            st = b.stats()
            assert 0.0 < st["last_fused_ms"] <= st["last_ms"]
            for x, y in zip(g, t):
                same_results(x, y)
    finally:
        for aid in ids:
            ctx.free(aid)


@pytest.mark.parametrize("prec", ["f16x3", "bf16x3"])
def test_matrix_batch_against_oracle_and_fmap(ctx, prec):
    """A matrix-core batch of uneven candidates (1-24 bins: exponential maps
    of 2 or more bins on the matrix cores, one-bin maps on FP32 tiles; rect maps; linspace
    grids): every map against the oracle and bit-identical to tfstat_fmap of
    the same map in the same precision, autotuned and forced to the default
    build."""
    _case(prec + " batch")
    cands = [tfsynth.candidate(i, seed_base=7700, max_slots=1500, max_grid=170, max_bins=24)
             for i in range(10)]
    assert any(a.n_bins >= 4 and w.kind == "exp" for a, w in cands)
    ids = upload_all(ctx, cands)
    try:
        for tune in (True, False):
            with ctx.batch(list(zip(ids, [w for _, w in cands])), prec, tune=tune) as b:
                assert b.stats()["variant"] in ("mixed", "mixed_lowocc")
                got = b.run()
                again = b.run()
            for (atoms, win), aid, res, res2 in zip(cands, ids, got, again):
                same_results(res, res2)
                check_against_oracle(res, atoms, win, TOL[prec])
                single, _ = ctx.fmap(aid, win, prec)
                same_results(res, single)
    finally:
        for aid in ids:
            ctx.free(aid)
