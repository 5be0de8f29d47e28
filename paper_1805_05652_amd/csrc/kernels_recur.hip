// Exponential-window sums by an exact recurrence along t0 (FP64).
//
// For one tau the window weights of consecutive t0 rows differ by a fixed
// factor when the rows advance by a fixed number s of slots with one common
// offset delta (section 2, eq. winexp: w = exp(-(t - t0)/tau) on
// [t0, t0 + 3 tau)).  With rho = exp(-T_sft/tau), band length L and
//   U_m = sum_{d<L} rho^d x[k_m + d],   k_{m+1} = k_m + s,
// every channel obeys
//   U_m = sum_{d<s} rho^d x[k_m + d] + rho^s U_{m+1} - sum_{d=L}^{L+s-1} rho^d x[k_m + d],
// so a map costs O(N_t0 + L) per channel instead of the O(N_t0 L) direct
// sums that section 3 describes (the paper finds no reuse of the sums
// across tau; along t0 there is one).  A, B, C use rho^2, F_a, F_b use rho; the common row
// scale exp(-delta/tau) (squared for A, B, C) is applied at the end.
//
// One wave per (tau, group of BG bins).  Lane j owns a segment of G rows.
// The recurrence is first run with a zero boundary to get each segment's
// affine map U_start = a_j U_end + b_j; a suffix scan of the maps over the
// lanes (shuffles) gives every segment its true boundary from the window
// sum at the virtual row after the grid, which the wave computes directly.
// The recurrence is stable (|rho| < 1): rounding errors are damped by rho
// per step, so FP64 keeps the sums near 1e-13 relative.
#include "tfstat_device.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace tfs {

namespace {

struct Red {
    double f;
    double s;
    long long i;
};

__device__ inline Red red_empty() { return Red{-INFINITY, 0.0, 0x7fffffffffffffffLL}; }

__device__ inline Red red_combine(const Red &a, const Red &b) {
    Red r;
    r.f = fmax(a.f, b.f);
    if (r.f == -INFINITY) return red_empty();
    const double sa = (a.f == -INFINITY) ? 0.0 : a.s * exp(a.f - r.f);
    const double sb = (b.f == -INFINITY) ? 0.0 : b.s * exp(b.f - r.f);
    r.s = sa + sb;
    r.i = (a.f > b.f) ? a.i : (b.f > a.f) ? b.i : (a.i < b.i ? a.i : b.i);
    return r;
}

__device__ inline double twoF_cell(double A, double B, double C, double far_, double fai,
                                   double fbr, double fbi) {
    const double D = A * B - C * C;
    if (D <= kDegenerateRtol * A * B) return 0.0;
    const double num = B * (far_ * far_ + fai * fai) + A * (fbr * fbr + fbi * fbi)
                       - 2.0 * C * (far_ * fbr + fai * fbi);
    return 2.0 * (num / D);
}

// Channel values of one slot: 3 antenna channels, then 4 per bin of the group.
template <int BG>
struct Slot {
    double a[3];
    double x[BG][4];
};

template <int BG>
__device__ inline Slot<BG> load_slot(const RecurParams &p, int64_t k, int bin0) {
    Slot<BG> v;
    if (k < 0 || k >= p.K) {
#pragma unroll
        for (int c = 0; c < 3; ++c) v.a[c] = 0.0;
#pragma unroll
        for (int b = 0; b < BG; ++b)
#pragma unroll
            for (int c = 0; c < 4; ++c) v.x[b][c] = 0.0;
        return v;
    }
    const double *ab = p.abc + (size_t)k * 4;
    v.a[0] = ab[0];
    v.a[1] = ab[1];
    v.a[2] = ab[2];
#pragma unroll
    for (int b = 0; b < BG; ++b) {
        const int bin = bin0 + b < p.n_bins ? bin0 + b : p.n_bins - 1;
        const double *xp = p.x64 + ((size_t)k * p.n_bins + bin) * 4;
#pragma unroll
        for (int c = 0; c < 4; ++c) v.x[b][c] = xp[c];
    }
    return v;
}

template <int BG>
struct Acc {
    double a[3];
    double x[BG][4];
    __device__ inline void zero() {
#pragma unroll
        for (int c = 0; c < 3; ++c) a[c] = 0.0;
#pragma unroll
        for (int b = 0; b < BG; ++b)
#pragma unroll
            for (int c = 0; c < 4; ++c) x[b][c] = 0.0;
    }
    // this += wa * slot.a, wx * slot.x
    __device__ inline void add(const Slot<BG> &v, double wa, double wx) {
#pragma unroll
        for (int c = 0; c < 3; ++c) a[c] = fma(wa, v.a[c], a[c]);
#pragma unroll
        for (int b = 0; b < BG; ++b)
#pragma unroll
            for (int c = 0; c < 4; ++c) x[b][c] = fma(wx, v.x[b][c], x[b][c]);
    }
    __device__ inline void scale(double fa, double fx) {
#pragma unroll
        for (int c = 0; c < 3; ++c) a[c] *= fa;
#pragma unroll
        for (int b = 0; b < BG; ++b)
#pragma unroll
            for (int c = 0; c < 4; ++c) x[b][c] *= fx;
    }
};

template <int BG>
__global__ __launch_bounds__(256) void exp_recur_kernel(RecurParams p) {
    __shared__ Red wred[4][BG];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int n = blockIdx.x * 4 + wave;          // tau column
    const int bin0 = blockIdx.y * BG;
    const bool col_ok = n < p.n_tau;
    const int nn = col_ok ? n : p.n_tau - 1;
    const int M = p.n_t0;
    const int S = p.stride;                       // slots between rows
    const int64_t T = p.t_sft;
    const double tau = (double)p.tau[nn];
    const double lrho = -(double)T / tau;         // log rho
    const int64_t span = 3 * p.tau[nn];
    const int64_t L = span > p.delta ? (span - p.delta + T - 1) / T : 0;   // band (slots)
    const double rho = exp(lrho);
    const double rhoS = exp(lrho * S);
    const double rhoS2 = rhoS * rhoS;
    const double rhoL = exp(lrho * (double)L);
    const double scale = p.delta ? exp(-(double)p.delta / tau) : 1.0;

    // 1. window sums at the virtual row M (k = k0 + M S), lanes stride 64 over d
    Acc<BG> bnd;
    bnd.zero();
    {
        const int64_t kM = (int64_t)p.k0_first + (int64_t)M * S;
        const int64_t lim = min(L, max((int64_t)0, (int64_t)p.K - kM));
        double w = exp(lrho * lane);
        const double w64 = exp(lrho * 64);
        for (int64_t d = lane; d < lim; d += 64) {
            const Slot<BG> v = load_slot<BG>(p, kM + d, bin0);
            bnd.add(v, w * w, w);
            w *= w64;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
            for (int c = 0; c < 3; ++c) bnd.a[c] += __shfl_xor(bnd.a[c], o, 64);
#pragma unroll
            for (int b = 0; b < BG; ++b)
#pragma unroll
                for (int c = 0; c < 4; ++c) bnd.x[b][c] += __shfl_xor(bnd.x[b][c], o, 64);
        }
    }

    // 2. each lane's segment with a zero boundary: U_start = a U_end + b
    const int G = (M + 63) / 64;
    const int r_begin = min(lane * G, M);
    const int r_end = min(r_begin + G, M);
    auto row_step = [&](Acc<BG> &u, int m) {
        // u holds U_{m+1}; returns U_m
        const int64_t k = (int64_t)p.k0_first + (int64_t)m * S;
        u.scale(rhoS2, rhoS);
        double w = 1.0;
        for (int d = 0; d < S; ++d) {
            const Slot<BG> v = load_slot<BG>(p, k + d, bin0);
            u.add(v, w * w, w);
            w *= rho;
        }
        double wl = rhoL;
        for (int d = 0; d < S; ++d) {
            const Slot<BG> v = load_slot<BG>(p, k + L + d, bin0);
            u.add(v, -wl * wl, -wl);
            wl *= rho;
        }
    };
    Acc<BG> seg;
    seg.zero();
    for (int m = r_end - 1; m >= r_begin; --m) row_step(seg, m);
    double aA = exp(2.0 * lrho * S * (double)(r_end - r_begin));   // rho^(2 S rows)
    double aX = exp(lrho * S * (double)(r_end - r_begin));

    // 3. suffix scan of the affine maps over lanes: lane j ends with the map
    //    from U at the grid end (row M) to U at its segment start
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double naA = __shfl_down(aA, o, 64);
        const double naX = __shfl_down(aX, o, 64);
        Acc<BG> nb;
#pragma unroll
        for (int c = 0; c < 3; ++c) nb.a[c] = __shfl_down(seg.a[c], o, 64);
#pragma unroll
        for (int b = 0; b < BG; ++b)
#pragma unroll
            for (int c = 0; c < 4; ++c) nb.x[b][c] = __shfl_down(seg.x[b][c], o, 64);
        if (lane + o < 64) {
#pragma unroll
            for (int c = 0; c < 3; ++c) seg.a[c] = fma(aA, nb.a[c], seg.a[c]);
#pragma unroll
            for (int b = 0; b < BG; ++b)
#pragma unroll
                for (int c = 0; c < 4; ++c) seg.x[b][c] = fma(aX, nb.x[b][c], seg.x[b][c]);
            aA *= naA;
            aX *= naX;
        }
    }
    // value at this lane's segment start, then the next lane's = this lane's end
    Acc<BG> start;
#pragma unroll
    for (int c = 0; c < 3; ++c) start.a[c] = fma(aA, bnd.a[c], seg.a[c]);
#pragma unroll
    for (int b = 0; b < BG; ++b)
#pragma unroll
        for (int c = 0; c < 4; ++c) start.x[b][c] = fma(aX, bnd.x[b][c], seg.x[b][c]);
    Acc<BG> u;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double nx = __shfl_down(start.a[c], 1, 64);
        u.a[c] = lane == 63 ? bnd.a[c] : nx;
    }
#pragma unroll
    for (int b = 0; b < BG; ++b)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double nx = __shfl_down(start.x[b][c], 1, 64);
            u.x[b][c] = lane == 63 ? bnd.x[b][c] : nx;
        }

    // 4. rerun the segment from its true boundary: finalize every row.  A
    //    window holding fewer than two SFTs (exact integer count) is summed
    //    directly, so that empty and single-SFT windows get exactly the
    //    direct sums and not the recurrence's rounding residue.
    Red red[BG];
#pragma unroll
    for (int b = 0; b < BG; ++b) red[b] = red_empty();
    const double s2 = scale * scale;
    for (int m = r_end - 1; m >= r_begin; --m) {
        row_step(u, m);
        if (!col_ok) continue;
        const int64_t k = (int64_t)p.k0_first + (int64_t)m * S;
        const int64_t lo = min(max(k, (int64_t)0), (int64_t)p.K);
        const int64_t hi = min(max(k + L, (int64_t)0), (int64_t)p.K);
        const int cnt = p.npref[hi] - p.npref[lo];
        Acc<BG> w1;
        if (cnt == 1) {
            // the single present slot: first k' in [lo, hi) with npref[k'+1] > npref[lo]
            int64_t a0 = lo, a1 = hi - 1;
            const int base = p.npref[lo];
            while (a0 < a1) {
                const int64_t mid = (a0 + a1) / 2;
                if (p.npref[mid + 1] > base) a1 = mid; else a0 = mid + 1;
            }
            const double wd = exp(lrho * (double)(a0 - k));
            w1.zero();
            w1.add(load_slot<BG>(p, a0, bin0), wd * wd, wd);
        }
        const Acc<BG> &uu = cnt == 1 ? w1 : u;
#pragma unroll
        for (int b = 0; b < BG; ++b) {
            const int bin = bin0 + b;
            if (bin >= p.n_bins) continue;
            const double v = cnt == 0 ? 0.0
                : twoF_cell(s2 * uu.a[0], s2 * uu.a[1], s2 * uu.a[2], scale * uu.x[b][0],
                            scale * uu.x[b][1], scale * uu.x[b][2], scale * uu.x[b][3]);
            if (p.twoF) p.twoF[((size_t)bin * M + m) * p.n_tau + n] = (float)v;
            red[b] = red_combine(red[b], Red{0.5 * v, 1.0, (long long)m * p.n_tau + n});
        }
    }
#pragma unroll
    for (int b = 0; b < BG; ++b) {
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            Red w;
            w.f = __shfl_xor(red[b].f, o, 64);
            w.s = __shfl_xor(red[b].s, o, 64);
            w.i = __shfl_xor(red[b].i, o, 64);
            red[b] = red_combine(red[b], w);
        }
        if (lane == 0 && col_ok && bin0 + b < p.n_bins) {
            Partial &o = p.part[(size_t)(bin0 + b) * p.n_tiles + n];
            o.fmax = red[b].f;
            o.s = red[b].s;
            o.idx = red[b].i;
        }
    }
}

}  // namespace

hipError_t launch_exp_recur(const RecurParams &p, int BG, hipStream_t s) {
    const dim3 grid((unsigned)((p.n_tau + 3) / 4), (unsigned)((p.n_bins + BG - 1) / BG));
    if (BG == 1)
        hipLaunchKernelGGL(exp_recur_kernel<1>, grid, dim3(256), 0, s, p);
    else if (BG == 2)
        hipLaunchKernelGGL(exp_recur_kernel<2>, grid, dim3(256), 0, s, p);
    else if (BG == 4)
        hipLaunchKernelGGL(exp_recur_kernel<4>, grid, dim3(256), 0, s, p);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace tfs
