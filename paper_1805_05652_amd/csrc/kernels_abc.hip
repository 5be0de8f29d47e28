// Antenna sums A, B, C of exponential windows by a recurrence over t0 rows,
// evaluated as a parallel scan.
//
// For one tau and one channel y (a^2, b^2 or ab; section 2, eq. F_FaFb with
// the window of eq. winexp) the sum of a cell is
//   S_m = e^(-2 delta_m / tau) G_m,   G_m = sum_{k in [k0_m, e_m)} u^(k - k0_m) y_k,
// with u = e^(-2 T_sft / tau), k0_m the first slot at or after t0_m,
// delta_m = t_{k0_m} - t0_m and e_m the window's end slot, clipped at the
// data end (slots outside [0, K) hold no data).  Rows are in ascending t0,
// so k0_m <= k0_{m+1}, and G of a row follows from the next row's by an
// affine step
//   G_m = a_m G_{m+1} + b_m,   a_m = u^D,  D = k0_{m+1} - k0_m,
//   b_m = sum_{[k0_m, k0_{m+1})} u^(k - k0_m) y_k
//         + sum_{[e_{m+1}, e_m)} ... - sum_{[e_m, e_{m+1})} ...
// (only one of the last two ranges is non-empty); a row whose window ends
// before the next row's start has a_m = 0 and b_m its whole window.  The
// factor a_m <= 1 damps what later rows contribute, so the composition of
// these steps from the last row down is stable, and being associative it is
// computed by a scan: one wave per (tau, segment of rows), lane = row, 64
// rows at a time from the segment's end down, each lane composing its step
// with those of the rows above it in log2(64) shuffle rounds and applying
// the result to the carry (G of the row after the chunk).  The segment's
// last row is summed directly by the whole wave.  The work per tau is
// O(slots + rows) instead of O(rows x window length): the paper finds no
// such reuse across tau (section 3), but along t0 at fixed tau the
// exponential window allows it.  All arithmetic is FP64; the output is A,
// B, C of every cell, row scale and exact band included, as the
// matrix-core and F-only tiles read them.
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

// Atoms (a^2, b^2, ab) of slot k, zero outside [0, K).
__device__ inline Sum3 load_slot(const double *abc, int32_t K, int64_t k) {
    if (k < 0 || k >= K) return Sum3{0.0, 0.0, 0.0};
    const double2 ab = *reinterpret_cast<const double2 *>(abc + k * 4);
    return Sum3{ab.x, ab.y, abc[k * 4 + 2]};
}

// acc + sum_{k in [lo, hi)} f u^(k - lo) y_k, k clipped to [0, K) (f is the
// weight of slot lo, sign included; c2 = ln u).  Eight slots' atoms are
// loaded before they are summed, so that the loads of a group are in flight
// together.
__device__ inline Sum3 add_run(Sum3 acc, const double *abc, int32_t K, int64_t lo, int64_t hi, double f,
                               double u, double c2) {
    if (lo < 0) {
        f *= exp(c2 * (double)(-lo));
        lo = 0;
    }
    hi = hi > K ? K : hi;
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
            acc.a = fma(f, ab[i].x, acc.a);
            acc.b = fma(f, ab[i].y, acc.b);
            acc.c = fma(f, c[i], acc.c);
            f *= u;
        }
    }
    for (; k < hi; ++k) {
        const Sum3 y = load_slot(abc, K, k);
        acc.a = fma(f, y.a, acc.a);
        acc.b = fma(f, y.b, acc.b);
        acc.c = fma(f, y.c, acc.c);
        f *= u;
    }
    return acc;
}

// Wave sum of a lane's three partial sums (every lane gets the total).
__device__ inline Sum3 wave_sum(Sum3 s) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        s.a += __shfl_xor(s.a, o, 64);
        s.b += __shfl_xor(s.b, o, 64);
        s.c += __shfl_xor(s.c, o, 64);
    }
    return s;
}

// One wave: tau n, rows [m_lo, m_hi) of segment seg.
template <typename PP>
__device__ __attribute__((always_inline)) inline void abc_scan_wave(PP &p, int n, int seg) {
    const int lane = threadIdx.x & 63;
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
    // window of row m: first slot k0 and end slot e (clipped at K)
    auto window = [&](int m, int64_t &k0, int64_t &e) {
        const RowPlan r = p.rows[m];
        const int64_t len = span > r.delta ? (span - r.delta + T - 1) / T : 0;
        k0 = r.k0;
        e = min((int64_t)r.k0 + len, (int64_t)K);
    };

    // G of the segment's last row, summed by the whole wave: lane i takes
    // slots k0 + i, k0 + i + 64, ...
    Sum3 g_last{0.0, 0.0, 0.0};
    {
        int64_t k0, e;
        window(m_hi - 1, k0, e);
        const double u64 = exp(64.0 * c2);
        double f = exp(c2 * (double)lane);
        Sum3 s{0.0, 0.0, 0.0};
        for (int64_t k = k0 + lane; k < e; k += 64) {
            const Sum3 y = load_slot(p.abc, K, k);
            s.a = fma(f, y.a, s.a);
            s.b = fma(f, y.b, s.b);
            s.c = fma(f, y.c, s.c);
            f *= u64;
        }
        g_last = wave_sum(s);
    }

    // chunks of 64 rows from the segment's end down; lane l holds row
    // cb - 63 + l, and carry is G of row cb + 1
    Sum3 carry{0.0, 0.0, 0.0};
    for (int cb = m_hi - 1; cb >= m_lo; cb -= 64) {
        const int m = cb - 63 + lane;
        // this row's step G_m = a G_{m+1} + b (identity for rows outside
        // the segment, the direct sum for its last row)
        double a = 1.0;
        Sum3 b{0.0, 0.0, 0.0};
        if (m == m_hi - 1) {
            a = 0.0;
            b = g_last;
        } else if (m >= m_lo) {
            int64_t k0, e, kn, en;
            window(m, k0, e);
            window(m + 1, kn, en);
            if (kn >= e) {
                // the next row starts at or past this window's end
                a = 0.0;
                b = add_run(b, p.abc, K, k0, e, 1.0, u, c2);
            } else {
                const int64_t D = kn - k0;
                if (D <= 8) {
                    for (int64_t q = 0; q < D; ++q) a *= u;
                } else {
                    a = exp(c2 * (double)D);
                }
                b = add_run(b, p.abc, K, k0, kn, 1.0, u, c2);
                if (e != en) {
                    const int64_t lo = e > en ? en : e;
                    const double sign = e > en ? 1.0 : -1.0;
                    b = add_run(b, p.abc, K, lo, e > en ? e : en, sign * exp(c2 * (double)(lo - k0)), u, c2);
                }
            }
        }
        // suffix scan: lane l composes its step with those of the lanes
        // above it in the chunk, (a, b) o (a', b') = (a a', b + a b')
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const double a2 = __shfl_down(a, o, 64);
            const double ba = __shfl_down(b.a, o, 64);
            const double bb = __shfl_down(b.b, o, 64);
            const double bc = __shfl_down(b.c, o, 64);
            if (lane + o < 64) {
                b.a = fma(a, ba, b.a);
                b.b = fma(a, bb, b.b);
                b.c = fma(a, bc, b.c);
                a *= a2;
            }
        }
        const Sum3 g{fma(a, carry.a, b.a), fma(a, carry.b, b.b), fma(a, carry.c, b.c)};
        if (m >= m_lo && m < m_hi) {
            const double s2 = exp(-2.0 * (double)p.rows[m].delta / tau);
            double *o = p.abc_out + ((size_t)m * p.abc_pitch + n) * 3;
            o[0] = s2 * g.a;
            o[1] = s2 * g.b;
            o[2] = s2 * g.c;
        }
        // G of the chunk's first row: the next chunk's carry
        carry.a = __shfl(g.a, 0, 64);
        carry.b = __shfl(g.b, 0, 64);
        carry.c = __shfl(g.c, 0, 64);
    }
}

// Wave (tau, segment) from a linear wave index: taus run fastest.
template <typename PP>
__device__ __attribute__((always_inline)) inline void abc_scan_index(PP &p, int64_t w) {
    abc_scan_wave(p, (int)(w % p.n_tau), (int)(w / p.n_tau));
}

__global__ __launch_bounds__(256) void abc_recur_kernel(AbcRecurParams p) {
    abc_scan_index(p, (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6));
}

// Many maps: entry e is {map, block of 4 waves of that map}.
__global__ __launch_bounds__(256) void abc_recur_batch_kernel(AbcRecurBatchParams b) {
    const int e = blockIdx.x;
    const AbcRecurParams &p = b.jobs[b.entries[2 * e + 0]];
    abc_scan_index(p, (int64_t)b.entries[2 * e + 1] * 4 + (threadIdx.x >> 6));
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
