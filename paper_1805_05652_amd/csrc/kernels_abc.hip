// Antenna sums A, B, C of exponential windows by a recurrence over t0 rows.
//
// For one tau and one channel y (a^2, b^2 or ab; section 2, eq. F_FaFb with
// the window of eq. winexp) the sum of a cell is
//   S_m = e^(-2 delta_m / tau) G_m,   G_m = sum_{k in [k0_m, e_m)} u^(k - k0_m) y_k,
// with u = e^(-2 T_sft / tau), k0_m the first slot at or after t0_m,
// delta_m = t_{k0_m} - t0_m and e_m the window's end slot, clipped at the
// data end (slots outside [0, K) hold no data).  Rows are in ascending t0,
// so k0_m <= k0_{m+1}, and G of a row follows from the next row's:
//   G_m = u^D G_{m+1} + sum_{[k0_m, k0_{m+1})} u^(k - k0_m) y_k
//         + sum_{[e_{m+1}, e_m)} ... - sum_{[e_m, e_{m+1})} ...,   D = k0_{m+1} - k0_m,
// (only one of the last two ranges is non-empty).  The factor u^D <= 1
// damps what earlier steps left in G, so the recurrence runs from the last
// row down; a row whose window does not reach the next row's start is
// summed directly.  The work per tau is O(slots + rows) instead of
// O(rows x window length): the paper finds no such reuse across tau
// (section 3), but along t0 at fixed tau the exponential window allows it.
//
// Lane layout: one lane per (tau, segment of rows); each segment starts
// with one direct sum, so segments run in parallel at the price of that
// sum (the planner keeps it a fraction of the recurrence's work).  All arithmetic is
// FP64; the output is A, B, C of every cell, row scale and exact band
// included, as the matrix-core and F-only tiles read them.
#include "tfstat_device.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace tfs {

namespace {

// Running sums of the three antenna channels.
struct Sum3 {
    double a, b, c;
};

// g + sum_{k in [lo, hi)} f u^(k - lo) y_k, k clipped to [0, K) (f is the
// weight of slot lo, sign included; c2 = ln u).  Eight slots' atoms are
// loaded before they are summed, so that the loads of a group are in flight
// together.  Out of line (it is the rare path) and by value, so that the
// caller's sums stay in registers.
__device__ __attribute__((noinline)) Sum3 add_run(Sum3 acc, const double *abc, int32_t K, int64_t lo, int64_t hi,
                                                  double f, double u, double c2) {
    double g[3] = {acc.a, acc.b, acc.c};
    if (lo < 0) {
        f *= exp(c2 * (double)(-lo));
        lo = 0;
    }
    hi = hi > K ? K : hi;
    if (lo >= hi) return acc;
    int64_t k = lo;
    for (; k + 8 <= hi; k += 8) {
        double2 ab[8];
        double c[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            ab[i] = *reinterpret_cast<const double2 *>(abc + (k + i) * 4);
            c[i] = abc[(k + i) * 4 + 2];
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            g[0] = fma(f, ab[i].x, g[0]);
            g[1] = fma(f, ab[i].y, g[1]);
            g[2] = fma(f, c[i], g[2]);
            f *= u;
        }
    }
    for (; k < hi; ++k) {
        const double *y = abc + k * 4;
        g[0] = fma(f, y[0], g[0]);
        g[1] = fma(f, y[1], g[1]);
        g[2] = fma(f, y[2], g[2]);
        f *= u;
    }
    return Sum3{g[0], g[1], g[2]};
}

// Atoms (a^2, b^2, ab) of slot k, zero outside [0, K).
__device__ inline void load_slot(const double *abc, int32_t K, int64_t k, double y[3]) {
    if (k < 0 || k >= K) {
        y[0] = y[1] = y[2] = 0.0;
        return;
    }
    const double2 ab = *reinterpret_cast<const double2 *>(abc + k * 4);
    y[0] = ab.x;
    y[1] = ab.y;
    y[2] = abc[k * 4 + 2];
}

constexpr int kRecurChunk = 8;   // rows whose atoms are fetched together

template <typename PP>
__device__ __attribute__((always_inline)) inline void abc_recur_lane(PP &p, int n, int seg) {
    if (n >= p.n_tau) return;
    const int m_lo = seg * p.seg_rows;
    const int m_hi = min(m_lo + p.seg_rows, p.n_t0);
    if (m_lo >= m_hi) return;
    const int64_t T = p.t_sft;
    const int64_t tau_i = p.tau[n];
    const double tau = (double)tau_i;
    const double c2 = -2.0 * (double)T / tau;   // ln u
    const double u = exp(c2);
    const int64_t span = 3 * tau_i;
    const int32_t K = p.K;
    // a window holds lmax = ceil(span / T) slots at delta = 0 and lmax or
    // lmax - 1 at any other delta: u^len from two precomputed powers
    const int64_t lmax = (span + T - 1) / T;
    const double u_lm1 = lmax >= 1 ? exp(c2 * (double)(lmax - 1)) : 1.0;
    const double u_lmax = u_lm1 * u;
    double g[3] = {0.0, 0.0, 0.0};
    int64_t kn = 0, en = 0, lenn = 0;   // the next row's first slot, window end and length
    int32_t last_delta = -1;
    double s2 = 1.0;          // e^(-2 delta / tau) of the last delta seen
    for (int mc = m_hi - 1; mc >= m_lo; mc -= kRecurChunk) {
        const int nr = min(kRecurChunk, mc - m_lo + 1);
        // the chunk's rows (mc down to mc - nr + 1) and, when every step is
        // a recurrence step with at most one head and one tail slot, their
        // atoms, all loaded before any is summed
        // (slots fit in int32: k0 in [-2^30, K], window ends clipped at K;
        // lengths are only used unclipped, below K)
        int32_t k0s[kRecurChunk], es[kRecurChunk], lens[kRecurChunk], ds[kRecurChunk];
        bool simple = true;
        {
            int64_t kp = kn, ep = en;
            for (int i = 0; i < kRecurChunk; ++i) {
                if (i >= nr) break;
                const RowPlan r = p.rows[mc - i];
                const int64_t len = span > r.delta ? (span - r.delta + T - 1) / T : 0;
                const int64_t e = min((int64_t)r.k0 + len, (int64_t)K);
                k0s[i] = r.k0;
                ds[i] = r.delta;
                lens[i] = (int32_t)min(len, (int64_t)INT32_MAX);
                es[i] = (int32_t)e;
                const bool first = (mc - i == m_hi - 1);
                const int64_t D = kp - r.k0;
                const int64_t dt = e - ep;
                simple = simple && !first && kp < es[i] && D <= 1 && dt >= -1 && dt <= 1 && ep < K && es[i] < K;
                kp = r.k0;
                ep = es[i];
            }
        }
        double hy[kRecurChunk][3], ty[kRecurChunk][3];
        if (simple) {
            int64_t kp = kn, ep = en;
#pragma unroll
            for (int i = 0; i < kRecurChunk; ++i) {
                if (i < nr) {
                    load_slot(p.abc, K, kp > k0s[i] ? k0s[i] : -1, hy[i]);
                    load_slot(p.abc, K, es[i] != ep ? min(es[i], ep) : -1, ty[i]);
                    kp = k0s[i];
                    ep = es[i];
                }
            }
        }
#pragma unroll
        for (int i = 0; i < kRecurChunk; ++i) {
            if (i >= nr) break;
            const int m = mc - i;
            const int64_t k0 = k0s[i], e = es[i];
            if (simple) {
                // one step: G = u^D G' + head - or + one tail slot
                const double uD = kn > k0 ? u : 1.0;
                g[0] *= uD;
                g[1] *= uD;
                g[2] *= uD;
                g[0] += hy[i][0];   // head weight u^0 (zero when D = 0)
                g[1] += hy[i][1];
                g[2] += hy[i][2];
                if (e != en) {
                    // tail at en (added, weight u^(D + len')) or at e
                    // (removed, weight u^len)
                    const double f = e > en ? uD * (lenn == lmax ? u_lmax : u_lm1)
                                            : -(lens[i] == lmax ? u_lmax : u_lm1);
                    g[0] = fma(f, ty[i][0], g[0]);
                    g[1] = fma(f, ty[i][1], g[1]);
                    g[2] = fma(f, ty[i][2], g[2]);
                }
            } else if (m == m_hi - 1 || kn >= e) {
                const Sum3 r = add_run(Sum3{0.0, 0.0, 0.0}, p.abc, K, k0, e, 1.0, u, c2);
                g[0] = r.a;
                g[1] = r.b;
                g[2] = r.c;
            } else {
                // u^D by products for short steps, the exponential otherwise
                const int64_t D = kn - k0;
                double uD = 1.0;
                if (D <= 8) {
                    for (int64_t q = 0; q < D; ++q) uD *= u;
                } else {
                    uD = exp(c2 * (double)D);
                }
                Sum3 r = add_run(Sum3{g[0] * uD, g[1] * uD, g[2] * uD}, p.abc, K, k0, kn, 1.0, u, c2);
                if (e != en) {
                    const int64_t lo = e > en ? en : e;
                    const double sign = e > en ? 1.0 : -1.0;
                    r = add_run(r, p.abc, K, lo, e > en ? e : en, sign * exp(c2 * (double)(lo - k0)), u, c2);
                }
                g[0] = r.a;
                g[1] = r.b;
                g[2] = r.c;
            }
            kn = k0;
            en = e;
            lenn = lens[i];
            if (ds[i] != last_delta) {
                s2 = exp(-2.0 * (double)ds[i] / tau);
                last_delta = ds[i];
            }
            double *o = p.abc_out + ((size_t)m * p.abc_pitch + n) * 3;
            o[0] = s2 * g[0];
            o[1] = s2 * g[1];
            o[2] = s2 * g[2];
        }
    }
}

// Lane (tau, segment) from a linear index: taus (rounded up to 64) run
// fastest, so a workgroup's 256 lanes are consecutive taus of one segment
// when the map has that many.
template <typename PP>
__device__ __attribute__((always_inline)) inline void abc_recur_index(PP &p, int64_t idx) {
    const int64_t n64 = (p.n_tau + 63) / 64 * 64;
    abc_recur_lane(p, (int)(idx % n64), (int)(idx / n64));
}

__global__ __launch_bounds__(256, 2) void abc_recur_kernel(AbcRecurParams p) {
    abc_recur_index(p, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

// Many maps: entry e is {map, block of 256 lanes of that map}.
__global__ __launch_bounds__(256, 2) void abc_recur_batch_kernel(AbcRecurBatchParams b) {
    const int e = blockIdx.x;
    const AbcRecurParams &p = b.jobs[b.entries[2 * e + 0]];
    abc_recur_index(p, (int64_t)b.entries[2 * e + 1] * 256 + threadIdx.x);
}

}  // namespace

hipError_t launch_abc_recur(const AbcRecurParams &p, hipStream_t s) {
    if (p.n_tau <= 0 || p.n_t0 <= 0) return hipSuccess;
    if (p.seg_rows < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(abc_recur_kernel, dim3((unsigned)abc_recur_blocks(p)), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_abc_recur_batch(const AbcRecurBatchParams &p, hipStream_t s) {
    if (p.n_entries <= 0) return hipSuccess;
    hipLaunchKernelGGL(abc_recur_batch_kernel, dim3((unsigned)p.n_entries), dim3(256), 0, s, p);
    return hipGetLastError();
}

}  // namespace tfs
