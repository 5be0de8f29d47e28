"""Allocation-free logB of stored maps (tfstat_logB_noalloc) through the C
ABI: two calls in a row, the second on fewer and smaller maps, each against
tfstat_logB on the same maps (bit for bit: the same kernels) and against the
oracle's reduction of the same float32 values; a call above the static
workspace's limit fails with E_INVAL before any device work."""
import numpy as np
import pytest

import oracle
import tfsynth

pytestmark = pytest.mark.gpu


def _case(msg):
    print("case:", msg, flush=True)


def test_logB_noalloc_two_calls_against_logB():
    import torch
    import paper_1805_05652_amd as tf
    T = tfsynth.T_SFT
    atoms = tfsynth.make_atoms(17, 400, 0.1, n_bins=5,
                               injections=[tfsynth.Injection(2, "exp", 40 * T, 12 * T, 1.0)])
    with tf.Context(0, arena_bytes=256 << 20) as c:
        aid = c.upload_atoms(atoms)
        # 140 x 150 cells: two 16384-cell reduction tiles, the second ragged;
        # then 3 maps of 30 x 40 cells (one tile) into the same workspace
        calls = [("exp", 140, 150, 5), ("rect", 30, 40, 3)]
        for kind, n_t0, n_tau, n_maps in calls:
            _case("logB_noalloc %s %d maps of %d x %d" % (kind, n_maps, n_t0, n_tau))
            win = tfsynth.regular_window(kind, 0, 2 * T, n_t0, 2 * T, T, n_tau)
            _, twoF = c.fmap(aid, win, "fp32", want_map=True)
            maps = twoF[:n_maps].contiguous()
            out = torch.full((n_maps,), float("nan"), dtype=torch.float64, device=maps.device)
            c.logB_noalloc(maps, out)
            c.stream.synchronize()
            got = out.cpu().numpy()
            want = c.logB(maps)
            assert np.array_equal(got, want), (got, want)
            _, _, lb = oracle.reduce(maps.cpu().numpy().astype(np.float64))
            assert np.max(np.abs(got - lb)) <= 1e-9, (got, lb)
        c.free(aid)


def test_logB_noalloc_rejects_workspace_above_limit():
    import torch
    import paper_1805_05652_amd as tf
    from paper_1805_05652_amd import _abi
    # 10923 maps of 128 x 2048 cells need 10923 * 16 partials of 24 bytes
    # plus 24 bytes per map: just over 4 MiB.  The maps are really there, so
    # nothing could read past them even if the call went ahead.
    n_maps, n_t0, n_tau = 10923, 128, 2048
    with tf.Context(0, arena_bytes=16 << 20) as c:
        maps = torch.zeros((n_maps, n_t0, n_tau), dtype=torch.float32, device="cuda")
        out = torch.zeros((n_maps,), dtype=torch.float64, device="cuda")
        with pytest.raises(_abi.TfstatError) as e:
            c.logB_noalloc(maps, out)
        assert e.value.code == _abi.E_INVAL
        assert "workspace" in str(e.value)
        del maps
