/*
 * Plain FP64 CPU oracle for the transient F-statistic map.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library, and it is deliberately slow:
 * every cell is computed by direct summation over the SFT list, in the order
 * the paper states the method (section 2, "Formalism"):
 *
 *   1. window membership of each SFT start time t_j (eq. winrect, eq. winexp);
 *   2. window weight w_j: 1 for the rectangular window, exp(-(t_j - t0)/tau)
 *      for the exponential window (libm exp, not a lookup table; section 4.3
 *      reports that a table-based exponential changes F by up to ~10%), and
 *      for a general window shape (section 5 names other window functions)
 *      the caller's samples of s((t_j - t0)/tau), linearly interpolated;
 *   3. windowed antenna sums A, B, C over a^2, b^2, ab with weight w^2 and
 *      windowed data sums F_a, F_b with weight w (the windowed quantities that
 *      enter eq. F_FaFb);
 *   4. D = A B - C^2 and F from eq. F_FaFb; the stored value is 2F;
 *   5. the marginalised Bayes factor over the map, max-shifted log-sum-exp of
 *      F with a flat prior over the grid cells (the exponent of eq. F_OSG is F).
 *
 * Readings where the paper is silent (shared with the GPU library by
 * specification, not by code):
 *   - windows are half-open on SFT start times: [t0, t0 + tau) for rect and
 *     [t0, t0 + 3 tau) for exp, decided in integer seconds;
 *   - windows that reach past the end of the data are truncated, never
 *     renormalised (appendix A, data-end truncation);
 *   - a cell with D <= 1e-10 * A * B (empty, single-SFT or rank-one windows)
 *     gets 2F = 0;
 *   - logB = ln( (1 / (N_t0 N_tau)) * sum_mn exp(F_mn) ), degenerate cells
 *     included with F = 0;
 *   - the argmax is the first maximum of 2F in row-major (m, n) order.
 *
 * Sums are sequential in ascending SFT index, in FP64 with round-to-nearest.
 * The (bin, t0-row) loop is parallelised with OpenMP; that changes no
 * arithmetic.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TFO_RECT 0
#define TFO_EXP 1
#define TFO_SHAPE 2

#define TFO_DEGENERATE_RTOL 1e-10

/*
 * A window: rectangular, exponential, or a general shape w = s((t - t0)/tau)
 * given as samples (the other window functions named in section 5).  A shape
 * window covers [t0, t0 + floor(tau * num / den)) and s is linear between
 * n_shape samples spaced evenly over [0, num / den] in units of tau.
 */
typedef struct {
    int type;
    const double *shape;
    int n_shape;
    int64_t num, den;
} tfo_win;

/* Window membership of an SFT starting at t (eq. winrect / eq. winexp, read
 * as half-open intervals on SFT start times). */
static int tfo_in_window(const tfo_win *w, int64_t t, int64_t t0, int64_t tau)
{
    int64_t end;
    if (w->type == TFO_RECT)
        end = t0 + tau;
    else if (w->type == TFO_EXP)
        end = t0 + 3 * tau;
    else
        end = t0 + tau * w->num / w->den;
    return t >= t0 && t < end;
}

/* Window weight of an SFT inside the window (eq. winrect / eq. winexp; for
 * a shape window, linear interpolation of the samples). */
static double tfo_weight(const tfo_win *w, int64_t t, int64_t t0, int64_t tau)
{
    double u, frac;
    int64_t i;
    if (w->type == TFO_RECT)
        return 1.0;
    if (w->type == TFO_EXP)
        return exp(-(double)(t - t0) / (double)tau);
    /* position in sample intervals: ((t - t0) / tau) / (num / den) * (n - 1) */
    u = ((double)(t - t0) / (double)tau) * ((double)(w->n_shape - 1) * (double)w->den / (double)w->num);
    i = (int64_t)floor(u);
    if (i < 0)
        i = 0;
    if (i > w->n_shape - 2)
        i = w->n_shape - 2;
    frac = u - (double)i;
    return w->shape[i] + frac * (w->shape[i + 1] - w->shape[i]);
}

/* Index of the first SFT with start time >= t0 (timestamps ascending). */
static int tfo_first_at_or_after(const int64_t *ts, int n, int64_t t0)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = lo + (hi - lo) / 2;
        if (ts[mid] < t0)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

/*
 * Windowed sums for one cell (t0, tau) and every bin.
 *   sums_abc[3]          = A, B, C                       (weights w^2)
 *   sums_f[bin*4 + 0..3] = Re F_a, Im F_a, Re F_b, Im F_b (weights w)
 * fa, fb are [n_bins][n_sft][2] (re, im).
 */
static void tfo_window_sums(const tfo_win *win, int n_sft, const int64_t *ts,
                            const double *a2, const double *b2, const double *ab,
                            int n_bins, const double *fa, const double *fb,
                            int64_t t0, int64_t tau,
                            double *sums_abc, double *sums_f)
{
    int j, bin;
    sums_abc[0] = sums_abc[1] = sums_abc[2] = 0.0;
    for (bin = 0; bin < 4 * n_bins; bin++)
        sums_f[bin] = 0.0;
    for (j = tfo_first_at_or_after(ts, n_sft, t0); j < n_sft; j++) {
        double w;
        if (!tfo_in_window(win, ts[j], t0, tau))
            break; /* ascending start times: every later SFT is outside too */
        w = tfo_weight(win, ts[j], t0, tau);
        sums_abc[0] += (w * w) * a2[j];
        sums_abc[1] += (w * w) * b2[j];
        sums_abc[2] += (w * w) * ab[j];
        for (bin = 0; bin < n_bins; bin++) {
            const double *pa = fa + ((size_t)bin * n_sft + j) * 2;
            const double *pb = fb + ((size_t)bin * n_sft + j) * 2;
            sums_f[bin * 4 + 0] += w * pa[0];
            sums_f[bin * 4 + 1] += w * pa[1];
            sums_f[bin * 4 + 2] += w * pb[0];
            sums_f[bin * 4 + 3] += w * pb[1];
        }
    }
}

/* 2F from windowed sums (eq. F_FaFb), with the degenerate-window rule. */
static double tfo_twoF(const double *abc, const double *f)
{
    double A = abc[0], B = abc[1], C = abc[2];
    double D = A * B - C * C;
    double fa_re = f[0], fa_im = f[1], fb_re = f[2], fb_im = f[3];
    double F;
    if (D <= TFO_DEGENERATE_RTOL * A * B)
        return 0.0;
    F = (B * (fa_re * fa_re + fa_im * fa_im)
         + A * (fb_re * fb_re + fb_im * fb_im)
         - 2.0 * C * (fa_re * fb_re + fa_im * fb_im)) / D;
    return 2.0 * F;
}

static int tfo_check(const tfo_win *w, int n_sft, const int64_t *ts, int n_bins,
                     int n_t0, const int64_t *t0, int n_tau, const int64_t *tau)
{
    int i;
    if (w->type != TFO_RECT && w->type != TFO_EXP && w->type != TFO_SHAPE)
        return -1;
    if (w->type == TFO_SHAPE) {
        if (!w->shape || w->n_shape < 2 || w->num < 1 || w->den < 1 || w->num > 1024 || w->den > 1024)
            return -1;
        for (i = 0; i < n_tau; i++)
            if (tau[i] > ((int64_t)1 << 50))
                return -1;
    }
    if (n_sft < 1 || n_bins < 1 || n_t0 < 1 || n_tau < 1)
        return -1;
    for (i = 1; i < n_sft; i++)
        if (ts[i] <= ts[i - 1])
            return -1;
    for (i = 0; i < n_tau; i++)
        if (tau[i] <= 0)
            return -1;
    (void)t0;
    return 0;
}

/*
 * Full 2F map: twoF[bin][m][n] (row-major), FP64.
 * Returns 0, or -1 on invalid arguments.
 */
static int tfo_fmap_win(const tfo_win *win, int n_sft, const int64_t *ts,
                        const double *a2, const double *b2, const double *ab,
                        int n_bins, const double *fa, const double *fb,
                        int n_t0, const int64_t *t0, int n_tau, const int64_t *tau,
                        int n_threads, double *twoF)
{
    int m;
    if (tfo_check(win, n_sft, ts, n_bins, n_t0, t0, n_tau, tau))
        return -1;
#ifdef _OPENMP
    if (n_threads > 0)
        omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel for schedule(static)
    for (m = 0; m < n_t0; m++) {
        double abc[3];
        double *f = (double *)malloc(sizeof(double) * 4 * (size_t)n_bins);
        int n, bin;
        for (n = 0; n < n_tau; n++) {
            tfo_window_sums(win, n_sft, ts, a2, b2, ab, n_bins, fa, fb,
                            t0[m], tau[n], abc, f);
            for (bin = 0; bin < n_bins; bin++)
                twoF[((size_t)bin * n_t0 + m) * n_tau + n] = tfo_twoF(abc, f + 4 * bin);
        }
        free(f);
    }
    return 0;
}

int tfo_fmap(int type, int n_sft, const int64_t *ts,
             const double *a2, const double *b2, const double *ab,
             int n_bins, const double *fa, const double *fb,
             int n_t0, const int64_t *t0, int n_tau, const int64_t *tau,
             int n_threads, double *twoF)
{
    tfo_win w = {type, NULL, 0, 1, 1};
    if (type == TFO_SHAPE)
        return -1;
    return tfo_fmap_win(&w, n_sft, ts, a2, b2, ab, n_bins, fa, fb, n_t0, t0, n_tau, tau,
                        n_threads, twoF);
}

/*
 * Full 2F map for a shape window: shape[n_shape] samples of s(x) on
 * [0, num / den] (see tfo_win).
 */
int tfo_fmap_shape(const double *shape, int n_shape, int64_t num, int64_t den,
                   int n_sft, const int64_t *ts,
                   const double *a2, const double *b2, const double *ab,
                   int n_bins, const double *fa, const double *fb,
                   int n_t0, const int64_t *t0, int n_tau, const int64_t *tau,
                   int n_threads, double *twoF)
{
    tfo_win w = {TFO_SHAPE, shape, n_shape, num, den};
    return tfo_fmap_win(&w, n_sft, ts, a2, b2, ab, n_bins, fa, fb, n_t0, t0, n_tau, tau,
                        n_threads, twoF);
}

/*
 * Selected cells only: twoF_sel[bin][i] for cells (m_idx[i], n_idx[i]).
 */
static int tfo_cells_win(const tfo_win *win, int n_sft, const int64_t *ts,
                         const double *a2, const double *b2, const double *ab,
                         int n_bins, const double *fa, const double *fb,
                         int n_t0, const int64_t *t0, int n_tau, const int64_t *tau,
                         int n_sel, const int32_t *m_idx, const int32_t *n_idx,
                         int n_threads, double *twoF_sel)
{
    int i;
    if (tfo_check(win, n_sft, ts, n_bins, n_t0, t0, n_tau, tau))
        return -1;
    for (i = 0; i < n_sel; i++)
        if (m_idx[i] < 0 || m_idx[i] >= n_t0 || n_idx[i] < 0 || n_idx[i] >= n_tau)
            return -1;
#ifdef _OPENMP
    if (n_threads > 0)
        omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel for schedule(dynamic, 16)
    for (i = 0; i < n_sel; i++) {
        double abc[3];
        double *f = (double *)malloc(sizeof(double) * 4 * (size_t)n_bins);
        int bin;
        tfo_window_sums(win, n_sft, ts, a2, b2, ab, n_bins, fa, fb,
                        t0[m_idx[i]], tau[n_idx[i]], abc, f);
        for (bin = 0; bin < n_bins; bin++)
            twoF_sel[(size_t)bin * n_sel + i] = tfo_twoF(abc, f + 4 * bin);
        free(f);
    }
    return 0;
}

int tfo_cells(int type, int n_sft, const int64_t *ts,
              const double *a2, const double *b2, const double *ab,
              int n_bins, const double *fa, const double *fb,
              int n_t0, const int64_t *t0, int n_tau, const int64_t *tau,
              int n_sel, const int32_t *m_idx, const int32_t *n_idx,
              int n_threads, double *twoF_sel)
{
    tfo_win w = {type, NULL, 0, 1, 1};
    if (type == TFO_SHAPE)
        return -1;
    return tfo_cells_win(&w, n_sft, ts, a2, b2, ab, n_bins, fa, fb, n_t0, t0, n_tau, tau,
                         n_sel, m_idx, n_idx, n_threads, twoF_sel);
}

int tfo_cells_shape(const double *shape, int n_shape, int64_t num, int64_t den,
                    int n_sft, const int64_t *ts,
                    const double *a2, const double *b2, const double *ab,
                    int n_bins, const double *fa, const double *fb,
                    int n_t0, const int64_t *t0, int n_tau, const int64_t *tau,
                    int n_sel, const int32_t *m_idx, const int32_t *n_idx,
                    int n_threads, double *twoF_sel)
{
    tfo_win w = {TFO_SHAPE, shape, n_shape, num, den};
    return tfo_cells_win(&w, n_sft, ts, a2, b2, ab, n_bins, fa, fb, n_t0, t0, n_tau, tau,
                         n_sel, m_idx, n_idx, n_threads, twoF_sel);
}

/*
 * Windowed sums of one cell, for tests of the individual steps:
 * out[0..2] = A, B, C; out[3 + 4*bin + 0..3] = Re F_a, Im F_a, Re F_b, Im F_b.
 */
int tfo_cell_sums(int type, int n_sft, const int64_t *ts,
                  const double *a2, const double *b2, const double *ab,
                  int n_bins, const double *fa, const double *fb,
                  int64_t t0, int64_t tau, double *out)
{
    int64_t one_t0 = t0, one_tau = tau;
    tfo_win w = {type, NULL, 0, 1, 1};
    if (type == TFO_SHAPE || tfo_check(&w, n_sft, ts, n_bins, 1, &one_t0, 1, &one_tau))
        return -1;
    tfo_window_sums(&w, n_sft, ts, a2, b2, ab, n_bins, fa, fb, t0, tau,
                    out, out + 3);
    return 0;
}

/*
 * Reductions over n_maps maps of n_cells cells each (twoF[map][cell]):
 * max 2F, first row-major argmax, and
 *   logB = F_max + ln sum_c exp(F_c - F_max) - ln(n_cells),  F = 2F / 2.
 */
int tfo_reduce(const double *twoF, int n_maps, int64_t n_cells,
               double *max2F, int64_t *argmax, double *logB)
{
    int k;
    if (n_maps < 1 || n_cells < 1)
        return -1;
    for (k = 0; k < n_maps; k++) {
        const double *map = twoF + (size_t)k * (size_t)n_cells;
        double best = map[0];
        int64_t best_i = 0, c;
        double fmax, s = 0.0;
        for (c = 1; c < n_cells; c++) {
            if (map[c] > best) {
                best = map[c];
                best_i = c;
            }
        }
        fmax = 0.5 * best;
        for (c = 0; c < n_cells; c++)
            s += exp(0.5 * map[c] - fmax);
        max2F[k] = best;
        argmax[k] = best_i;
        logB[k] = fmax + log(s) - log((double)n_cells);
    }
    return 0;
}
