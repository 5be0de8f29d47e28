"""Full-size parity of the uneven batch and of a served request stream
against the FP64 CPU oracle (tolerances in checks.py).

  * Uneven batch: the 64 follow-up candidates (slots log-uniform in
    [500, 8000], gaps U[0, 0.3], grids U{100..1500}^2, 1-16 bins, rect and
    exp alternating) in the benchmark's autotuned launch configuration.
    Batches in FP32, F16X3 and BF16X3 (matrix cores for maps of 4 or more
    bins).
    Every map's per-bin results (max 2F, argmax, logB) are compared with the
    oracle's full map, and every cell of the single-map path's 2F map
    (bit-identical results, see test_gpu_batch) with the oracle's cells.
    The oracle work (2.7e11 cells*SFTs*bins) is split over four tests.
  * Served stream: 106 requests of the serving workload's distribution
    (Poisson 200/s for 0.6 s; slots log-uniform [200, 10000], grids up to
    2000^2, 1-64 bins, window type random), submitted at their arrival
    times in FP32, F16X3 and BF16X3 in turn.  Each served result
    equals tfstat_fmap alone (bitwise); the 40
    requests of least oracle work are compared with the oracle's full map;
    the other 66 (the 10 largest among them) on sampled cells plus every
    bin's argmax cell.
"""
import time

import numpy as np
import pytest

import oracle
import tfsynth
from checks import TOL, check_map, check_results, check_sampled

pytestmark = pytest.mark.gpu


def _case(msg):
    print("case:", msg, flush=True)


def _same(a, b):
    assert len(a) == len(b)
    for x, y in zip(a, b):
        assert (x["max2F"], x["logB"], x["m"], x["n"]) == (y["max2F"], y["logB"], y["m"], y["n"]), (x, y)


PRECS = ("fp32", "f16x3", "bf16x3")


@pytest.fixture(scope="module")
def batch64():
    """The 64-candidate batch, autotuned, run once in FP32 and once in
    BF16X3; the context stays open for the single-map maps of the quarter
    tests."""
    import paper_1805_05652_amd as tf
    cands = [tfsynth.candidate(i) for i in range(64)]
    c = tf.Context(0, arena_bytes=24 << 30)
    ids = [c.upload_atoms(a) for a, _ in cands]
    got = {}
    for prec in PRECS:
        _case("uneven batch %s: plan, tune and run" % prec)
        with c.batch(list(zip(ids, [w for _, w in cands])), prec, tune=True) as b:
            got[prec] = b.run()
            assert b.stats()["variant"] in ("mixed", "mixed_lowocc")
    yield c, cands, ids, got
    c.close()


@pytest.mark.parametrize("quarter", [0, 1, 2, 3])
def test_full_uneven_batch_against_oracle(batch64, quarter):
    """A quarter of the 64 maps: per-bin results of both batches against the
    oracle's full map, and every cell of the single-map maps (whose results
    the batches reproduce bit for bit)."""
    c, cands, ids, got = batch64
    worst = {p: 0.0 for p in PRECS}
    for i in range(quarter, 64, 4):
        atoms, win = cands[i]
        _case("uneven batch map %d: %s, %d slots, %d bins, %d x %d"
              % (i, win.kind, atoms.n_slots, atoms.n_bins, win.n_t0, win.n_tau))
        ref = oracle.fmap_atoms(atoms, win)
        for prec in PRECS:
            check_results(got[prec][i], ref, win, TOL[prec])
            single, twoF = c.fmap(ids[i], win, prec, want_map=True)
            _same(got[prec][i], single)
            worst[prec] = max(worst[prec], check_map(twoF.cpu().numpy(), ref, TOL[prec]))
            del twoF
    print("uneven batch quarter %d: max rel err %s" % (quarter, worst), flush=True)


def _oracle_work(atoms, win):
    """cells*present SFTs*bins of a map (the oracle's direct-summation work)."""
    ts = atoms.timestamps
    span = win.tau if win.kind == "rect" else 3 * win.tau
    tot = 0
    for t0 in win.t0.tolist():
        tot += int((np.searchsorted(ts, t0 + span, "left") - np.searchsorted(ts, t0, "left")).sum())
    return tot * atoms.n_bins


def test_served_stream_against_alone_and_oracle():
    import paper_1805_05652_amd as tf
    import torch
    reqs = tfsynth.request_stream(4000, 200.0, 0.6)
    assert len(reqs) >= 100
    _case("served stream: %d requests" % len(reqs))
    c = tf.Context(0, arena_bytes=24 << 30)
    try:
        ids, wins, nbs = [], [], []
        for r in reqs:
            atoms, win = tfsynth.request_atoms(r)
            ids.append(c.upload_atoms(atoms))
            wins.append(win)
            nbs.append(atoms.n_bins)
        # requests in FP32, F16X3 and BF16X3 in turn (each fused with its kind)
        precs = [("fp32", "f16x3", "bf16x3")[k % 3] for k in range(len(reqs))]
        c.serve_config(16)
        served = {}
        pending = {}
        t_start = time.perf_counter()
        i = 0
        deadline = t_start + 120.0
        while (i < len(reqs) or pending) and time.perf_counter() < deadline:
            now = time.perf_counter() - t_start
            while i < len(reqs) and reqs[i]["arrival"] <= now:
                pending[c.submit(ids[i], wins[i], precs[i])] = i
                i += 1
            for t, k in list(pending.items()):
                r = c.poll(t, nbs[k])
                if r is not None:
                    served[k] = r
                    del pending[t]
            time.sleep(0.0005)
        assert len(served) == len(reqs), "requests did not finish"
        _case("served stream: results alone")
        for k in range(len(reqs)):
            alone, _ = c.fmap(ids[k], wins[k], precs[k])
            _same(served[k], alone)
        order = sorted(range(len(reqs)), key=lambda k: _oracle_work(*tfsynth.request_atoms(reqs[k])))
        full, sampled = order[:40], order[40:]
        worst_full = worst_sampled = 0.0
        for k in full:
            atoms, win = tfsynth.request_atoms(reqs[k])
            _case("served request %d (full oracle): %s %d slots %d bins %d x %d"
                  % (k, win.kind, atoms.n_slots, atoms.n_bins, win.n_t0, win.n_tau))
            ref = oracle.fmap_atoms(atoms, win)
            check_results(served[k], ref, win, TOL[precs[k]])
            _, twoF = c.fmap(ids[k], win, precs[k], want_map=True)
            worst_full = max(worst_full, check_map(twoF.cpu().numpy(), ref, TOL[precs[k]]))
            del twoF
        rng = np.random.default_rng(4001)
        for k in sampled:
            atoms, win = tfsynth.request_atoms(reqs[k])
            _case("served request %d (sampled): %s %d slots %d bins %d x %d"
                  % (k, win.kind, atoms.n_slots, atoms.n_bins, win.n_t0, win.n_tau))
            res, twoF = c.fmap(ids[k], win, precs[k], want_map=True)
            _same(served[k], res)
            worst_sampled = max(worst_sampled, check_sampled(twoF, res, atoms, win, TOL[precs[k]], rng))
            del twoF
            torch.cuda.empty_cache()
        print("served stream: %d requests, max rel err %.3e (full maps), %.3e (sampled)"
              % (len(reqs), worst_full, worst_sampled), flush=True)
    finally:
        c.close()
