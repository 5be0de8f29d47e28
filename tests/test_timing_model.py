"""The timing model of appendix A: effective summation counts against their
closed forms, and the three-step fit recovering known constants."""
import numpy as np
import pytest

from paper_1805_05652_amd import timing_model as tm

T = tm.T_SFT


def test_nsums_exp_embedded_closed_form():
    """Embedded case: N_sums^e = 3 N_t0 sum_n tau_n / T_sft
    = 3 N_t0 N_tau (tau_min + 0.5 dtau') / T_sft for a regular tau grid."""
    t_data = 10000 * T
    t0 = np.arange(40) * 7 * T
    tau = (2 + np.arange(30)) * 11 * T
    got = tm.n_sums_exp(t0, tau, t_data)
    assert got == pytest.approx(3 * len(t0) * tau.sum() / T)
    mean_tau = tau.mean()
    assert got == pytest.approx(3 * len(t0) * len(tau) * mean_tau / T)


def test_nsums_rect_embedded_and_timing_grid():
    """Embedded: N_t0 tau_max / T_sft.  The timing grid of section 4.1
    (N_t0 dt0 = N_tau dtau = T_data - 2 T_sft, t0 from the data start):
    about 0.5 N_t0 tau_max / T_sft."""
    t_data = 5000 * T
    t0 = np.arange(100) * T
    tau = np.arange(2, 50) * T
    assert tm.n_sums_rect(t0, tau, t_data) == pytest.approx(100 * 49)
    k = 3000
    t_data = k * T
    n = 2000
    t0 = np.linspace(0, t_data - 2 * T, n)
    tau = np.linspace(2 * T, t_data, n)
    assert tm.n_sums_rect(t0, tau, t_data) == pytest.approx(0.5 * n * tau.max() / T, rel=0.01)


def test_nsums_truncated_windows_count_less():
    t_data = 100 * T
    t0 = np.array([0, 90 * T])
    tau = np.array([50 * T])
    assert tm.n_sums_rect(t0, tau, t_data) == pytest.approx(50 + 10)
    assert tm.n_sums_exp(t0, tau, t_data) == pytest.approx(100 + 10)


def _synthetic_runs(c, rng, noise=0.0, offset=0.0, short_pure=False):
    runs = []
    for k in (8, 16, 24, 48, 96, 480, 2000, 5000):
        for n_t0, n_tau in ((2, 2), (3, 3), (10, 10), (50, 20), (100, 100), (300, 300)):
            for kind in ("rect", "exp"):
                n_t0_, n_tau_ = min(n_t0, k - 2), min(n_tau, k - 2)
                t0 = np.linspace(0, (k - 2) * T, n_t0_)
                tau = np.linspace(2 * T, k * T, n_tau_)
                ns = tm.n_sums_rect(t0, tau, k * T) if kind == "rect" else tm.n_sums_exp(t0, tau, k * T)
                cs = c["c_sums_rect"] if kind == "rect" else c["c_sums_exp"]
                t = offset + c["c_SFTs"] * k + cs * ns + c["c_F"] * n_t0_ * n_tau_
                if short_pure and ns <= 100:
                    t = offset + c["c_SFTs"] * k
                t *= 1.0 + noise * rng.standard_normal()
                runs.append({"kind": kind, "n_sft": k, "n_sums": ns, "n_cells": n_t0_ * n_tau_, "t": t})
    return runs


def test_paper_fit_recovers_constants():
    """Timings that follow the model, with the short runs (N_sums <= 100)
    carrying only the N_SFT term as step 1 assumes: the three steps return
    the paper's i5 constants."""
    c = {"c_SFTs": 2.80e-8, "c_sums_rect": 0.96e-8, "c_F": 5.59e-8, "c_sums_exp": 3.55e-8}
    runs = _synthetic_runs(c, np.random.default_rng(0), short_pure=True)
    fit = tm.fit_paper(runs)
    for k, v in c.items():
        assert fit[k][0] == pytest.approx(v, rel=1e-6), k


def test_paper_fit_step_order():
    """Step 1 sees only short runs: changing a long run's time moves the
    later constants but never c_SFTs."""
    c = {"c_SFTs": 2.80e-8, "c_sums_rect": 0.96e-8, "c_F": 5.59e-8, "c_sums_exp": 3.55e-8}
    runs = _synthetic_runs(c, np.random.default_rng(0), short_pure=True)
    base = tm.fit_paper(runs)
    for r in runs:
        if r["kind"] == "exp" and r["n_sums"] > 100:
            r["t"] *= 1.5
    moved = tm.fit_paper(runs)
    assert moved["c_SFTs"][0] == base["c_SFTs"][0]
    assert moved["c_F"][0] == base["c_F"][0] and moved["c_sums_rect"][0] == base["c_sums_rect"][0]
    assert moved["c_sums_exp"][0] > 1.2 * base["c_sums_exp"][0]


def test_offset_fit_recovers_constants_and_offset():
    c = {"c_SFTs": 1.0e-9, "c_sums_rect": 2.0e-12, "c_F": 3.0e-11, "c_sums_exp": 5.0e-13}
    runs = _synthetic_runs(c, np.random.default_rng(1), noise=0.0, offset=4e-5, short_pure=True)
    fit = tm.fit_with_offset(runs)
    assert fit["c_0"][0] == pytest.approx(4e-5, rel=1e-6)
    for k, v in c.items():
        assert fit[k][0] == pytest.approx(v, rel=1e-5), k


def test_pgm_conversion_embedded_limit():
    """eq. cost-exp-convert: c_exp^PGM ~ 3 c_sums^e when N_tau >> 1 and the
    N_SFT and c_F terms are negligible; eq. cost-rect-convert: c_rect^PGM ~
    c_sums^r + c_F for N_t0 ~ N_SFT and N_tau T_sft ~ tau_max."""
    fit = {"c_SFTs": (0.0, 0.0), "c_F": (1e-8, 0.0), "c_sums_rect": (2e-8, 0.0), "c_sums_exp": (3e-8, 0.0)}
    day = 86400
    got = tm.pgm_constants(fit, n_sft=17532, n_t0=17532, n_tau=10000, tau_min=0.5 * day,
                           tau_max=10000 * T, dtau=T)
    assert got["c_exp_PGM"] == pytest.approx(9e-8, rel=0.01)
    assert got["c_rect_PGM"] == pytest.approx(3e-8, rel=0.01)
