"""Pins of the FP64 CPU oracle against facts fixed by the paper and by the
mathematics, each by a route that does not reuse the oracle's own formula:

  * exact rational arithmetic of the likelihood maximisation (Fractions);
  * the ordinary (non-transient) F-statistic over all atoms via a 2x2
    complex linear solve (section 2: the persistent case sums all atoms);
  * the real four-parameter quadratic form of eq. F_xMx via a 4x4 solve;
  * numerical maximisation of the per-SFT log-likelihood ratio over the
    complex amplitudes (the definition of F as a maximised likelihood ratio,
    eq. F_OSG), independent of the closed form eq. F_FaFb;
  * closed-form geometric sums of the exponential window (eq. winexp);
  * the Lagrange identity for the determinant D = A B - C^2;
  * prefix-sum rectangular sums (the running-sum reuse of section 3);
  * the long-tau limit of the exponential window;
  * invariances of the map under amplitude scaling, polarisation rotation and
    time shifts;
  * chi-square with 4 degrees of freedom of 2F in Gaussian noise, and the
    non-central mean 4 + lambda for injected signals;
  * closed forms of the marginalised log Bayes factor;
  * the selected-cell entry points (cells, cells_shape), which the
    full-size GPU tests use as their reference, against the full map at the
    same cells and against numerical likelihood maximisation.
"""
from fractions import Fraction

import numpy as np
import pytest
from scipy import optimize, special, stats

import oracle
import tfsynth

T = tfsynth.T_SFT


def _sums(kind, atoms, t0, tau):
    return oracle.cell_sums(kind, atoms.timestamps, atoms.a2, atoms.b2, atoms.ab,
                            atoms.fa, atoms.fb, t0, tau)


def _map(kind, atoms, t0, tau):
    return oracle.fmap(kind, atoms.timestamps, atoms.a2, atoms.b2, atoms.ab,
                       atoms.fa, atoms.fb, t0, tau)


# ---------------------------------------------------------------------------
# Exact arithmetic on a hand-sized example
# ---------------------------------------------------------------------------

def test_exact_rational_three_sfts():
    """Three SFTs with small rational atoms; F computed exactly with Fractions
    by maximising 2 Re(conj(alpha) Fa + conj(beta) Fb) - theta^H M theta, i.e.
    by solving M theta = v exactly and evaluating v^H theta."""
    a = [Fraction(1, 2), Fraction(1, 4), Fraction(-1, 8)]
    b = [Fraction(1, 8), Fraction(1, 2), Fraction(3, 8)]
    x = [(Fraction(1), Fraction(-1, 2)), (Fraction(3, 4), Fraction(1, 4)),
         (Fraction(-1, 2), Fraction(5, 4))]
    ts = np.array([0, T, 2 * T], dtype=np.int64)
    # windowed (rectangular, all three SFTs) sums, exactly
    A = sum(ai * ai for ai in a)
    B = sum(bi * bi for bi in b)
    C = sum(ai * bi for ai, bi in zip(a, b))
    Fa = (sum(ai * xr for ai, (xr, _) in zip(a, x)), sum(ai * xi for ai, (_, xi) in zip(a, x)))
    Fb = (sum(bi * xr for bi, (xr, _) in zip(b, x)), sum(bi * xi for bi, (_, xi) in zip(b, x)))
    # solve [[A, C], [C, B]] theta = v for the real and imaginary parts
    det = A * B - C * C
    th_re = ((B * Fa[0] - C * Fb[0]) / det, (A * Fb[0] - C * Fa[0]) / det)
    th_im = ((B * Fa[1] - C * Fb[1]) / det, (A * Fb[1] - C * Fa[1]) / det)
    F_exact = Fa[0] * th_re[0] + Fb[0] * th_re[1] + Fa[1] * th_im[0] + Fb[1] * th_im[1]
    fa = np.array([[[float(ai * xr), float(ai * xi)] for ai, (xr, xi) in zip(a, x)]])
    fb = np.array([[[float(bi * xr), float(bi * xi)] for bi, (xr, xi) in zip(b, x)]])
    a2 = np.array([float(ai * ai) for ai in a])
    b2 = np.array([float(bi * bi) for bi in b])
    ab = np.array([float(ai * bi) for ai, bi in zip(a, b)])
    got = oracle.fmap("rect", ts, a2, b2, ab, fa, fb, [0], [3 * T])[0, 0, 0]
    assert got == pytest.approx(float(2 * F_exact), rel=1e-14)
    # [0, 3T - 1) still holds the SFT starting at 2T
    got2 = oracle.fmap("rect", ts, a2, b2, ab, fa, fb, [0], [3 * T - 1])[0, 0, 0]
    assert got2 == got
    # exp window over the same SFTs: weights w_j = exp(-j T / tau) exactly
    tau = 5 * T
    w = [np.exp(-j * T / tau) for j in range(3)]
    Aw = sum(wj * wj * float(ai * ai) for wj, ai in zip(w, a))
    Bw = sum(wj * wj * float(bi * bi) for wj, bi in zip(w, b))
    Cw = sum(wj * wj * float(ai * bi) for wj, ai, bi in zip(w, a, b))
    v = np.array([sum(wj * complex(float(ai * xr), float(ai * xi)) for wj, ai, (xr, xi) in zip(w, a, x)),
                  sum(wj * complex(float(bi * xr), float(bi * xi)) for wj, bi, (xr, xi) in zip(w, b, x))])
    M = np.array([[Aw, Cw], [Cw, Bw]])
    F = np.real(np.conj(v) @ np.linalg.solve(M, v))
    got3 = oracle.fmap("exp", ts, a2, b2, ab, fa, fb, [0], [tau])[0, 0, 0]
    assert got3 == pytest.approx(2 * F, rel=1e-13)


# ---------------------------------------------------------------------------
# Ordinary F-statistic and the four-parameter form
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [1, 2, 3])
def test_full_span_rect_equals_ordinary_F(seed):
    atoms = tfsynth.make_atoms(seed, 60, 0.2, n_bins=3)
    t0 = int(atoms.timestamps[0])
    got = _map("rect", atoms, [t0], [atoms.t_data])[:, 0, 0]
    A = atoms.a2.sum()
    B = atoms.b2.sum()
    C = atoms.ab.sum()
    M = np.array([[A, C], [C, B]])
    for bin_ in range(3):
        fa = atoms.fa[bin_, :, 0] + 1j * atoms.fa[bin_, :, 1]
        fb = atoms.fb[bin_, :, 0] + 1j * atoms.fb[bin_, :, 1]
        v = np.array([fa.sum(), fb.sum()])
        F = np.real(np.conj(v) @ np.linalg.solve(M.astype(complex), v))
        assert got[bin_] == pytest.approx(2 * F, rel=1e-11)


@pytest.mark.parametrize("kind", ["rect", "exp"])
def test_four_parameter_quadratic_form(kind):
    """eq. F_xMx: F = 1/2 x^T Minv x over four real amplitude parameters,
    with x = 2 (Re Fa, Re Fb, Im Fa, Im Fb) and the 4x4 antenna matrix
    2 blockdiag(M, M) (normalisation fixed by the maximised likelihood)."""
    atoms = tfsynth.make_atoms(7, 80, 0.1, n_bins=2)
    rng = np.random.default_rng(5)
    for _ in range(10):
        t0 = int(rng.integers(0, 60)) * T + int(rng.integers(0, T))
        tau = int(rng.integers(2 * T, 40 * T))
        A, B, C, Fa, Fb = _sums(kind, atoms, t0, tau)
        M = np.array([[A, C], [C, B]])
        M4 = 2 * np.block([[M, np.zeros((2, 2))], [np.zeros((2, 2)), M]])
        got = _map(kind, atoms, [t0], [tau])[:, 0, 0]
        for k in range(2):
            x = 2 * np.array([Fa[k].real, Fb[k].real, Fa[k].imag, Fb[k].imag])
            F = 0.5 * x @ np.linalg.solve(M4, x)
            assert got[k] == pytest.approx(2 * F, rel=1e-10)


# ---------------------------------------------------------------------------
# Brute force: numerical maximisation of the per-SFT likelihood ratio
# ---------------------------------------------------------------------------

def _window_weights(kind, ts, t0, tau):
    """Window of section 2 evaluated directly from its definition."""
    span = tau if kind == "rect" else 3 * tau
    inside = (ts >= t0) & (ts < t0 + span)
    if kind == "rect":
        return inside.astype(float)
    return np.where(inside, np.exp(-(ts - t0) / tau), 0.0)


def _brute_force_2F(kind, atoms, bin_, t0, tau):
    w = _window_weights(kind, atoms.timestamps, t0, tau)
    fa = atoms.fa[bin_, :, 0] + 1j * atoms.fa[bin_, :, 1]
    fb = atoms.fb[bin_, :, 0] + 1j * atoms.fb[bin_, :, 1]

    def neg_loglr(p):
        al = p[0] + 1j * p[1]
        be = p[2] + 1j * p[3]
        # per SFT: 2 Re(conj(s_j) x_j) - |s_j|^2 with s_j = w_j (al a_j + be b_j)
        cross = 2 * w * np.real(np.conj(al) * fa + np.conj(be) * fb)
        power = w * w * (abs(al) ** 2 * atoms.a2 + abs(be) ** 2 * atoms.b2
                         + 2 * np.real(np.conj(al) * be) * atoms.ab)
        return -(cross - power).sum()

    best = None
    for start in ([0, 0, 0, 0], [1, -1, 0.5, 0.2]):
        r = optimize.minimize(neg_loglr, np.array(start, float), method="BFGS",
                              options=dict(gtol=1e-12, maxiter=2000))
        if best is None or r.fun < best.fun:
            best = r
    return -2 * best.fun


@pytest.mark.parametrize("kind", ["rect", "exp"])
def test_brute_force_tiny_grid(kind):
    atoms = tfsynth.make_atoms(11, 8, 0.0, n_bins=2,
                               injections=[tfsynth.Injection(1, kind, 2 * T, 3 * T, 1.5)])
    t0s = np.arange(0, 6 * T + 1, T, dtype=np.int64)
    taus = np.array([2 * T, 3 * T, 4 * T + 7, 8 * T], dtype=np.int64)
    got = _map(kind, atoms, t0s, taus)
    for m, t0 in enumerate(t0s):
        for n, tau in enumerate(taus):
            w = _window_weights(kind, atoms.timestamps, int(t0), int(tau))
            if (w > 0).sum() < 2:
                assert got[0, m, n] == 0.0
                continue
            for k in range(2):
                bf = _brute_force_2F(kind, atoms, k, int(t0), int(tau))
                assert got[k, m, n] == pytest.approx(bf, rel=1e-6, abs=1e-8)


# ---------------------------------------------------------------------------
# Exponential window: closed-form geometric sums
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("tau_s,L", [(2 * T, 6), (2 * T + 1, 7), (2 * T - 1, 6),
                                     (10 * T, 30), (7 * T + 600, 22)])
def test_exp_window_geometric_closed_form(tau_s, L):
    """Regular slots, a^2 = alpha^2, b^2 = beta^2, ab = 0, Fa_j = 1, Fb_j = 0.
    Then A = alpha^2 S2, B = beta^2 S2 with S2 = sum_{d<L} r^(2d), C = 0,
    Fa = S1 = sum_{d<L} r^d with r = exp(-T/tau), and 2F = 2 S1^2 / (alpha^2 S2).
    L is the number of SFT starts in [t0, t0 + 3 tau)."""
    n = 80
    ts = np.arange(n, dtype=np.int64) * T
    alpha2, beta2 = 0.3, 0.7
    a2 = np.full(n, alpha2)
    b2 = np.full(n, beta2)
    ab = np.zeros(n)
    fa = np.zeros((1, n, 2))
    fa[0, :, 0] = 1.0
    fb = np.zeros((1, n, 2))
    r = np.exp(-T / tau_s)
    S1 = (1 - r ** L) / (1 - r)
    S2 = (1 - r ** (2 * L)) / (1 - r * r)
    expect = 2 * S1 * S1 / (alpha2 * S2)
    got = oracle.fmap("exp", ts, a2, b2, ab, fa, fb, [5 * T], [tau_s])[0, 0, 0]
    assert got == pytest.approx(expect, rel=1e-12)
    # same through the window sums
    A, B, C, Fa, Fb = oracle.cell_sums("exp", ts, a2, b2, ab, fa, fb, 5 * T, tau_s)
    assert A == pytest.approx(alpha2 * S2, rel=1e-13)
    assert B == pytest.approx(beta2 * S2, rel=1e-13)
    assert C == 0.0
    assert Fa[0].real == pytest.approx(S1, rel=1e-13)


def test_window_edges_and_truncation():
    """Half-open windows on SFT start times and truncation at the data end."""
    n = 10
    ts = np.arange(n, dtype=np.int64) * T
    ones = np.ones(n)
    fa = np.zeros((1, n, 2))
    fa[0, :, 0] = 1.0
    fb = np.zeros((1, n, 2))
    cases = [
        ("rect", 0, 3 * T, 3),          # starts 0, T, 2T
        ("rect", 0, 3 * T + 1, 4),      # 3T < 3T + 1
        ("rect", 1, 3 * T, 3),          # [1, 3T + 1): T, 2T, 3T
        ("rect", 1, 3 * T - 1, 2),      # [1, 3T): T, 2T
        ("rect", 7 * T, 10 * T, 3),     # truncated at the data end
        ("rect", 10 * T, 5 * T, 0),     # entirely after the data
        ("exp", 0, T, 3),               # [0, 3T)
        ("exp", 0, T + 1, 4),
        ("exp", 8 * T, 5 * T, 2),       # truncated
    ]
    for kind, t0, tau, count in cases:
        A, B, C, Fa, Fb = oracle.cell_sums(kind, ts, ones, ones, 0 * ones, fa, fb, t0, tau)
        if kind == "rect":
            assert A == count and Fa[0].real == count
        else:
            d = (ts[(ts >= t0) & (ts < t0 + 3 * tau)] - t0) / tau
            assert len(d) == count
            assert A == pytest.approx(np.exp(-2 * d).sum(), rel=1e-15)


# ---------------------------------------------------------------------------
# Determinant, prefix sums, long-tau limit
# ---------------------------------------------------------------------------

def test_lagrange_identity_for_D():
    atoms = tfsynth.make_atoms(21, 120, 0.15)
    rng = np.random.default_rng(3)
    ts = atoms.timestamps
    for kind in ("rect", "exp"):
        for _ in range(20):
            t0 = int(rng.integers(0, 100)) * T
            tau = int(rng.integers(2, 16)) * T
            A, B, C, _, _ = _sums(kind, atoms, t0, tau)
            w = _window_weights(kind, ts, t0, tau)
            idx = np.nonzero(w)[0]
            D_lag = 0.0
            for i in range(len(idx)):
                for j in range(i + 1, len(idx)):
                    p, q = idx[i], idx[j]
                    D_lag += (w[p] * w[q]) ** 2 * (atoms.a[p] * atoms.b[q] - atoms.a[q] * atoms.b[p]) ** 2
            assert A * B - C * C == pytest.approx(D_lag, rel=1e-9, abs=1e-12 * A * B)


def test_rect_prefix_sums_equal_direct_sums():
    atoms = tfsynth.make_atoms(31, 300, 0.2, n_bins=2)
    K = atoms.n_slots
    slot = (atoms.timestamps // T).astype(int)
    dense = np.zeros((K, 3 + 8))
    dense[slot, 0] = atoms.a2
    dense[slot, 1] = atoms.b2
    dense[slot, 2] = atoms.ab
    for k in range(2):
        dense[slot, 3 + 4 * k + 0] = atoms.fa[k, :, 0]
        dense[slot, 3 + 4 * k + 1] = atoms.fa[k, :, 1]
        dense[slot, 3 + 4 * k + 2] = atoms.fb[k, :, 0]
        dense[slot, 3 + 4 * k + 3] = atoms.fb[k, :, 1]
    P = np.vstack([np.zeros((1, dense.shape[1])), np.cumsum(dense, axis=0)])
    rng = np.random.default_rng(4)
    for _ in range(50):
        t0 = int(rng.integers(0, K * T))
        tau = int(rng.integers(1, K * T))
        lo = min(K, -(-t0 // T))             # first slot with start >= t0
        hi = min(K, -(-(t0 + tau) // T))     # first slot with start >= t0 + tau
        hi = max(hi, lo)
        ref = P[hi] - P[lo]
        A, B, C, Fa, Fb = _sums("rect", atoms, t0, tau)
        got = np.array([A, B, C, Fa[0].real, Fa[0].imag, Fb[0].real, Fb[0].imag,
                        Fa[1].real, Fa[1].imag, Fb[1].real, Fb[1].imag])
        assert np.allclose(got, ref, rtol=1e-10, atol=1e-10)


def test_long_tau_exp_approaches_rect_to_data_end():
    atoms = tfsynth.make_atoms(41, 200, 0.1, n_bins=2)
    t0s = np.array([0, 10 * T, 50 * T + 300], dtype=np.int64)
    big = 10_000 * atoms.t_data
    e = _map("exp", atoms, t0s, [big])[:, :, 0]
    r = _map("rect", atoms, t0s, [atoms.t_data])[:, :, 0]
    # weights differ from 1 by at most T_data / tau = 1e-4
    assert np.allclose(e, r, rtol=5e-4, atol=1e-6)
    assert not np.array_equal(e, r)


# ---------------------------------------------------------------------------
# Invariances
# ---------------------------------------------------------------------------

def _atoms_from_ab(ts, a, b, x):
    fa = (a[None] * x).astype(np.complex128)
    fb = (b[None] * x).astype(np.complex128)
    return (a * a, b * b, a * b, np.stack([fa.real, fa.imag], -1),
            np.stack([fb.real, fb.imag], -1))


@pytest.mark.parametrize("kind", ["rect", "exp"])
def test_invariances(kind):
    rng = np.random.default_rng(8)
    atoms = tfsynth.make_atoms(51, 90, 0.1)
    ts, a, b = atoms.timestamps, atoms.a, atoms.b
    x = (rng.standard_normal((2, len(ts))) + 1j * rng.standard_normal((2, len(ts)))) / np.sqrt(2)
    t0 = np.array([0, 3 * T, 20 * T + 5, 41 * T], dtype=np.int64)
    tau = np.array([2 * T, 5 * T + 11, 17 * T, 60 * T], dtype=np.int64)
    base = oracle.fmap(kind, ts, *_atoms_from_ab(ts, a, b, x), t0, tau)
    # amplitude scaling of (a, b) with the data x fixed
    scaled = oracle.fmap(kind, ts, *_atoms_from_ab(ts, 3.7 * a, 3.7 * b, x), t0, tau)
    assert np.allclose(scaled, base, rtol=1e-10, atol=1e-12)
    # polarisation rotation of (a, b)
    psi = 0.83
    ar = a * np.cos(psi) - b * np.sin(psi)
    br = a * np.sin(psi) + b * np.cos(psi)
    rot = oracle.fmap(kind, ts, *_atoms_from_ab(ts, ar, br, x), t0, tau)
    assert np.allclose(rot, base, rtol=1e-9, atol=1e-10)
    # a common time shift of data and grid
    shift = 987_654_321
    shifted = oracle.fmap(kind, ts + shift, *_atoms_from_ab(ts, a, b, x), t0 + shift, tau)
    assert np.array_equal(shifted, base)
    # a phase rotation of the data
    ph = oracle.fmap(kind, ts, *_atoms_from_ab(ts, a, b, x * np.exp(0.6j)), t0, tau)
    assert np.allclose(ph, base, rtol=1e-10, atol=1e-12)


# ---------------------------------------------------------------------------
# Statistics in Gaussian noise and with injections
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind,t0,tau", [("rect", 5 * T, 12 * T), ("exp", 5 * T, 4 * T),
                                         ("exp", 0, 30 * T + 123), ("rect", 17, 2 * T + 40)])
def test_noise_is_chi2_4(kind, t0, tau):
    """2F over many independent noise bins follows chi-square with 4 dof."""
    atoms = tfsynth.make_atoms(61, 120, 0.1, n_bins=4000)
    vals = _map(kind, atoms, [t0], [tau])[:, 0, 0]
    assert vals.mean() == pytest.approx(4.0, abs=4 * np.sqrt(8 / len(vals)))
    assert vals.var() == pytest.approx(8.0, rel=0.15)
    ks = stats.kstest(vals, stats.chi2(4).cdf)
    assert ks.pvalue > 1e-3


def test_injection_noncentral_mean():
    """E[2F] = 4 + lambda with lambda = 2 h^2 (A + B) for a matched window."""
    n_bins = 3000
    t0, tau, h = 10 * T, 6 * T, 0.6
    inj = [tfsynth.Injection(k, "exp", t0, tau, h, chi=0.1 * k) for k in range(n_bins)]
    atoms = tfsynth.make_atoms(71, 100, 0.1, n_bins=n_bins, injections=inj)
    vals = _map("exp", atoms, [t0], [tau])[:, 0, 0]
    A, B, _, _, _ = _sums("exp", atoms, t0, tau)
    lam = 2 * h * h * (A + B)
    sd = np.sqrt(2 * (4 + 2 * lam) / n_bins)
    assert vals.mean() == pytest.approx(4 + lam, abs=4 * sd)
    ks = stats.kstest(vals, stats.ncx2(4, lam).cdf)
    assert ks.pvalue > 1e-3


def test_degenerate_cells_are_zero():
    atoms = tfsynth.make_atoms(81, 20, 0.0)
    # a single SFT in the window, and an empty window
    got = _map("rect", atoms, [3 * T, 100 * T], [T, 5 * T])
    assert got[0, 0, 0] == 0.0
    assert got[0, 1, 0] == 0.0 and got[0, 1, 1] == 0.0
    assert got[0, 0, 1] > 0.0
    # collinear antenna patterns: D = 0 for every window
    a = atoms.a
    ts = atoms.timestamps
    x = np.ones((1, len(ts)), dtype=complex)
    a2, b2, ab, fa, fb = _atoms_from_ab(ts, a, 2 * a, x)
    col = oracle.fmap("exp", ts, a2, b2, ab, fa, fb, [0, 2 * T], [2 * T, 4 * T])
    assert np.all(col == 0.0)


# ---------------------------------------------------------------------------
# Marginalised Bayes factor and argmax
# ---------------------------------------------------------------------------

def test_logB_closed_forms():
    c = 3.25
    mx, am, lb = oracle.reduce(np.full((1, 7, 9), 2 * c))
    assert lb[0] == pytest.approx(c, abs=1e-14)
    assert am[0] == 0 and mx[0] == 2 * c
    rng = np.random.default_rng(9)
    m2 = rng.chisquare(4, size=(3, 40, 50))
    mx, am, lb = oracle.reduce(m2)
    for k in range(3):
        F = m2[k].ravel() / 2
        ref = special.logsumexp(F) - np.log(F.size)
        assert lb[k] == pytest.approx(ref, abs=1e-12)
        assert F.max() - np.log(F.size) <= lb[k] <= F.max()
        assert am[k] == int(np.argmax(m2[k]))
    # overflow guard: values whose exponentials overflow a double
    big = np.full((1, 4, 4), 0.0)
    big[0, 1, 2] = 2 * 1000.0
    mx, am, lb = oracle.reduce(big)
    assert np.isfinite(lb[0])
    assert lb[0] == pytest.approx(1000.0 - np.log(16.0), abs=1e-9)
    assert am[0] == 6


def test_argmax_first_in_row_major_order():
    m = np.zeros((1, 3, 4))
    m[0, 2, 1] = 5.0
    m[0, 1, 3] = 5.0
    _, am, _ = oracle.reduce(m)
    assert am[0] == 1 * 4 + 3


def test_loud_injection_found():
    """A loud matched injection (lambda ~ 260) is the map's argmax."""
    t0, tau = 40 * T, 25 * T
    atoms = tfsynth.make_atoms(91, 150, 0.1, injections=[
        tfsynth.Injection(0, "rect", t0, tau, 4.5, 0.4)])
    win = tfsynth.regular_window("rect", 0, T, 100, 2 * T, T, 140)
    twoF = oracle.fmap_atoms(atoms, win)
    res = oracle.results(atoms, win, twoF)[0]
    assert res["max2F"] > 150
    assert abs(res["t0"] - t0) <= 2 * T and abs(res["tau"] - tau) <= 3 * T


# ---------------------------------------------------------------------------
# General window shapes (section 5: other window functions follow the
# exponential window's setup)
# ---------------------------------------------------------------------------

def _shape_map(atoms, win):
    return oracle.fmap_atoms(atoms, win)


def test_shape_constant_is_rect():
    """A constant shape over [0, 1) tau is the rectangular window, exactly."""
    atoms = tfsynth.make_atoms(41, 60, 0.1, n_bins=2)
    base = tfsynth.regular_window("rect", -T // 2, T // 3, 70, T - 5, 700, 40)
    rect = oracle.fmap_atoms(atoms, base)
    shp = tfsynth.shape_window(base, np.ones(2), (1, 1))
    assert np.array_equal(_shape_map(atoms, shp), rect)


def _shape_brute(atoms, t0, tau, weight_fn, end):
    ts = atoms.timestamps
    inside = (ts >= t0) & (ts < end)
    w = np.where(inside, weight_fn((ts - t0) / tau), 0.0)
    return w


@pytest.mark.parametrize("support,tau", [((2, 1), 3 * T + 7), ((5, 2), 3 * T + 1), ((5, 2), 2 * T)])
def test_shape_linear_ramp_brute_force(support, tau):
    """A linear ramp s(x) = 1 - x / S over [0, S) tau, sampled at its ends
    and midpoint (linear interpolation is exact for it), against numerical
    maximisation of the likelihood with weights taken from the definition,
    including the integer window end floor(tau * num / den)."""
    num, den = support
    S = num / den
    atoms = tfsynth.make_atoms(43, 14, 0.0, n_bins=1,
                               injections=[tfsynth.Injection(0, "rect", 2 * T, 6 * T, 1.2)])
    base = tfsynth.list_window("rect", np.array([0, T, 2 * T + 300], dtype=np.int64),
                               np.array([tau], dtype=np.int64))
    win = tfsynth.shape_window(base, np.array([1.0, 0.5, 0.0]), support)
    got = _shape_map(atoms, win)
    for m, t0 in enumerate(base.t0):
        end = int(t0) + tau * num // den
        w = _shape_brute(atoms, int(t0), tau, lambda x: 1.0 - x / S, end)
        if (w > 0).sum() < 2:
            assert got[0, m, 0] == 0.0
            continue
        bf = _brute_force_2F_weights(atoms, 0, w)
        assert got[0, m, 0] == pytest.approx(bf, rel=1e-6, abs=1e-8)


def _brute_force_2F_weights(atoms, bin_, w):
    fa = atoms.fa[bin_, :, 0] + 1j * atoms.fa[bin_, :, 1]
    fb = atoms.fb[bin_, :, 0] + 1j * atoms.fb[bin_, :, 1]

    def neg_loglr(p):
        al = p[0] + 1j * p[1]
        be = p[2] + 1j * p[3]
        cross = 2 * w * np.real(np.conj(al) * fa + np.conj(be) * fb)
        power = w * w * (abs(al) ** 2 * atoms.a2 + abs(be) ** 2 * atoms.b2
                         + 2 * np.real(np.conj(al) * be) * atoms.ab)
        return -(cross - power).sum()

    best = None
    for start in ([0, 0, 0, 0], [1, -1, 0.5, 0.2]):
        r = optimize.minimize(neg_loglr, np.array(start, float), method="BFGS",
                              options=dict(gtol=1e-12, maxiter=2000))
        if best is None or r.fun < best.fun:
            best = r
    return -2 * best.fun


def test_shape_sampled_exponential_approaches_exp_window():
    """exp(-x) sampled finely over [0, 3] with support 3: linear
    interpolation is within h^2/8 of the exponential (h = 1e-4), so the map
    agrees with the exponential window's to about 1e-8 relative."""
    atoms = tfsynth.make_atoms(47, 200, 0.1, n_bins=2,
                               injections=[tfsynth.Injection(0, "exp", 20 * T, 15 * T, 0.8)])
    base = tfsynth.regular_window("exp", 0, 2 * T, 60, 2 * T, 3 * T + 11, 25)
    x = np.linspace(0.0, 3.0, 30001)
    shp = tfsynth.shape_window(base, np.exp(-x), (3, 1))
    ref = oracle.fmap_atoms(atoms, base)
    got = _shape_map(atoms, shp)
    assert np.all((got == 0) == (ref == 0))
    assert np.max(np.abs(got - ref) / np.maximum(ref, 1.0)) < 1e-6


# ---------------------------------------------------------------------------
# Selected cells: the reference of the full-size GPU tests
# ---------------------------------------------------------------------------

def _cell_sample(rng, win, n):
    m = rng.integers(0, win.n_t0, size=n)
    k = rng.integers(0, win.n_tau, size=n)
    m = np.concatenate([m, [0, 0, win.n_t0 - 1, win.n_t0 - 1]])
    k = np.concatenate([k, [0, win.n_tau - 1, 0, win.n_tau - 1]])
    return m.astype(np.int32), k.astype(np.int32)


@pytest.mark.parametrize("kind", ["rect", "exp", "shape"])
def test_cells_equal_full_map_at_same_cells(kind):
    """oracle.cells / oracle.cells_shape return exactly the full map's value
    at every selected (m, n), for every bin, on a ragged grid (t0 before,
    inside and after the data, off the slot grid; tau below one SFT and past
    the data) with an injection and gaps."""
    atoms = tfsynth.make_atoms(61, 240, 0.15, n_bins=5,
                               injections=[tfsynth.Injection(3, "exp", 50 * T, 20 * T, 1.5)])
    rng = np.random.default_rng(62)
    t0 = np.unique(np.concatenate([[-3 * T - 5, 0, 7], rng.integers(0, 240 * T, size=70),
                                   [240 * T + 11]]))
    tau = np.unique(np.concatenate([[T - 1, 2 * T], rng.integers(2 * T, 150 * T, size=40),
                                    [300 * T]]))
    base = tfsynth.list_window("rect" if kind == "rect" else "exp", t0, tau)
    if kind == "shape":
        x = np.linspace(0.0, 4.0, 129)
        # every t0 one offset from the slot grid is not needed by the oracle
        base = tfsynth.shape_window(base, x * np.exp(1.0 - x), (4, 1))
    full = oracle.fmap_atoms(atoms, base)
    mi, ni = _cell_sample(rng, base, 300)
    sel = oracle.cells_atoms(atoms, base, mi, ni)
    assert sel.shape == (atoms.n_bins, mi.shape[0])
    assert np.array_equal(sel, full[:, mi, ni])
    # threads change no arithmetic
    assert np.array_equal(oracle.cells_atoms(atoms, base, mi, ni, n_threads=1), sel)


def test_cells_against_likelihood_maximisation():
    """A few selected cells of each window type against numerical
    maximisation of the per-SFT likelihood ratio (weights from the
    definition), independent of the closed form."""
    atoms = tfsynth.make_atoms(63, 16, 0.0, n_bins=2,
                               injections=[tfsynth.Injection(1, "rect", 3 * T, 6 * T, 1.3)])
    t0s = np.array([0, T, 3 * T + 200, 5 * T], dtype=np.int64)
    taus = np.array([2 * T + 5, 4 * T, 9 * T], dtype=np.int64)
    mi = np.array([0, 1, 2, 3, 2], dtype=np.int32)
    ni = np.array([2, 0, 1, 2, 2], dtype=np.int32)
    for kind in ("rect", "exp", "shape"):
        if kind == "shape":
            win = tfsynth.shape_window(tfsynth.list_window("exp", t0s, taus),
                                       np.array([1.0, 0.5, 0.0]), (2, 1))
        else:
            win = tfsynth.list_window(kind, t0s, taus)
        got = oracle.cells_atoms(atoms, win, mi, ni)
        for i, (m, n) in enumerate(zip(mi, ni)):
            t0, tau = int(t0s[m]), int(taus[n])
            if kind == "shape":
                w = _shape_brute(atoms, t0, tau, lambda x: 1.0 - x / 2.0, t0 + 2 * tau)
            else:
                w = _window_weights(kind, atoms.timestamps, t0, tau)
            for b in range(2):
                if (w > 0).sum() < 2:
                    assert got[b, i] == 0.0
                    continue
                bf = _brute_force_2F_weights(atoms, b, w)
                assert got[b, i] == pytest.approx(bf, rel=1e-6, abs=1e-8), (kind, m, n, b)


def test_cells_reject_out_of_range_indices():
    atoms = tfsynth.make_atoms(65, 20, 0.0)
    win = tfsynth.regular_window("exp", 0, T, 4, 2 * T, T, 3)
    for mi, ni in (([4], [0]), ([0], [3]), ([-1], [0])):
        with pytest.raises(ValueError):
            oracle.cells_atoms(atoms, win, np.array(mi), np.array(ni))
