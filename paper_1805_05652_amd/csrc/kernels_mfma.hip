// Exponential-window F_a, F_b sums for many frequency bins on bf16 matrix
// cores (gfx950 v_mfma_f32_16x16x32_bf16).
//
// For one tau_n the window sums over all t0 rows m and data columns c
// (Re F_a, Im F_a, Re F_b, Im F_b of every bin) form a banded product
//   F[m][c] = s_n * sum_k W_n[m][k] X[k][c],   W_n[m][k] = g_n[k - k0_m],
// with g_n[d] = exp(-d T_sft / tau_n) on the band 0 <= d < L_n (section 2,
// eq. winexp; section 3: every cell of the exponential map sums its own
// window).  The antenna atoms a^2, b^2, ab are shared by all bins, so the
// data columns of all bins share one weight matrix: a dense contraction.
//
// Both operands are split into bf16 hi + lo parts (x = hi + lo + O(2^-16 x))
// and three products W_hi X_hi + W_hi X_lo + W_lo X_hi are accumulated in
// FP32.  A, B, C (FP64) come from the VALU kernel in its A/B/C-only mode.
//
// Work item: 64 consecutive t0 rows x 16 bins (64 data columns) x 8 taus.
// Wave w owns rows 16w..16w+15; its four 16x16 output tiles per tau are the
// four data components of the same 16 bins, so every lane ends with all four
// components of (row, bin) cells and finalizes them in place.
#include "tfstat_device.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace tfs {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kNT = 8;        // taus per work item (== VALU block width)
constexpr int kSK = 256;      // band slots per staged weight window
constexpr int kTW = kSK + 64; // staged weight window width

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

__device__ inline Red red_shfl_xor(const Red &v, int o) {
    Red w;
    w.f = __shfl_xor(v.f, o, 64);
    w.s = __shfl_xor(v.s, o, 64);
    w.i = __shfl_xor(v.i, o, 64);
    return w;
}

__device__ inline double twoF_cell(double A, double B, double C, double far_, double fai,
                                   double fbr, double fbi) {
    const double D = A * B - C * C;
    if (D <= kDegenerateRtol * A * B) return 0.0;
    const double num = B * (far_ * far_ + fai * fai) + A * (fbr * fbr + fbi * fbi)
                       - 2.0 * C * (far_ * fbr + fai * fbi);
    return 2.0 * (num / D);
}

// Round-to-nearest-even FP32 -> bf16 bits (inputs are finite).
__device__ inline unsigned int bf16_bits(float x) {
    const unsigned int u = __float_as_uint(x);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

__device__ inline float bf16_value(unsigned int b) { return __uint_as_float(b << 16); }

// Packs hi in the low and lo in the high 16 bits.
__device__ inline unsigned int split_pack(float x) {
    const unsigned int h = bf16_bits(x);
    const unsigned int l = bf16_bits(x - bf16_value(h));
    return h | (l << 16);
}

template <typename T>
__device__ inline T bitcast4(u32x4 v) {
    return __builtin_bit_cast(T, v);
}

__global__ __launch_bounds__(256) void exp_mfma_kernel(ExpMfmaParams p) {
    __shared__ unsigned int tab[kNT][kTW];
    __shared__ Red wred[4][16];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    // task decode: (block rank q, row tile, column tile); block ranks are
    // dealt round-robin to the 8 XCDs (workgroup b runs on XCD b % 8), the
    // tasks of one block stay on one XCD.
    const int per_block = p.n_row_tiles * p.n_col_tiles;
    const int bid = blockIdx.x;
    const int xcd = bid & 7;
    const int slot = bid >> 3;
    const int q = (slot / per_block) * 8 + xcd;
    if (q >= p.n_blocks) return;
    const int rem = slot % per_block;
    const int row_tile = rem / p.n_col_tiles;
    const int col_tile = rem % p.n_col_tiles;
    const int nb = p.blk_list[q];
    const int tile = nb * p.n_row_tiles + row_tile;

    const int m_first = row_tile * 64;
    const int m_last = min(m_first + 63, p.n_t0 - 1);
    const int k_first = p.k0_first + m_first;           // rows are consecutive slots
    const int k_last = p.k0_first + m_last;
    const int k_nom = k_first + 63;                      // slot of the tile's nominal last row
    const int lblk = p.lblk[nb];
    const int kb_begin = k_first & ~31;
    const int kb_end = min((k_last + lblk + 31) & ~31, p.kp_data);
    const int64_t off = p.blk_off[nb];

    // lane geometry
    const int lrow = lane & 15;           // A row / C column within a 16 tile
    const int kg = lane >> 4;             // K group of 8
    const int my_row = 16 * wave + lrow;  // A operand row within the 64-row tile
    const int bin = col_tile * 16 + lrow; // B / C column -> bin

    f32x4 acc[kNT][4];
#pragma unroll
    for (int t = 0; t < kNT; ++t)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};

    const unsigned short *xhi = p.xhi;
    const unsigned short *xlo = p.xlo;
    const size_t plane_col = (size_t)p.kp;   // elements per (component, bin) row

    for (int ks = kb_begin; ks < kb_end; ks += kSK) {
        // Stage weights for d in [d_lo, d_lo + kTW) with d_lo = ks - k_nom:
        // every row of the tile (also rows past n_t0, whose outputs are
        // discarded) reads inside the window.
        const int d_lo = ks - k_nom;
        __syncthreads();
        for (int i = tid; i < kNT * kTW; i += 256) {
            const int t = i / kTW;
            const int dd = i - t * kTW;
            const int d = d_lo + dd;
            float g = 0.f;
            if (d >= 0 && d < lblk) g = p.g32[off + (int64_t)d * kNT + t];
            tab[t][dd] = split_pack(g);
        }
        __syncthreads();
        const int ke = min(ks + kSK, kb_end);
        for (int kb = ks; kb < ke; kb += 32) {
            // B operands: 8 consecutive slots of one bin column, 4 components
            bf16x8 bh[4], bl[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const size_t o = ((size_t)(c * p.bins16 + bin)) * plane_col + kb + 8 * kg;
                bh[c] = bitcast4<bf16x8>(*reinterpret_cast<const u32x4 *>(xhi + o));
                bl[c] = bitcast4<bf16x8>(*reinterpret_cast<const u32x4 *>(xlo + o));
            }
            // A operand index: d = kb + 8 kg + j - k0(row) relative to d_lo
            const int base = (kb - ks) + (63 - my_row) + 8 * kg;
#pragma unroll
            for (int t = 0; t < kNT; ++t) {
                unsigned int w[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) w[j] = tab[t][base + j];
                u32x4 hv, lv;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    hv[j] = __builtin_amdgcn_perm(w[2 * j + 1], w[2 * j], 0x05040100u);
                    lv[j] = __builtin_amdgcn_perm(w[2 * j + 1], w[2 * j], 0x07060302u);
                }
                const bf16x8 ah = bitcast4<bf16x8>(hv);
                const bf16x8 al = bitcast4<bf16x8>(lv);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[c], acc[t][c], 0, 0, 0);
                    acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[c], acc[t][c], 0, 0, 0);
                    acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[c], acc[t][c], 0, 0, 0);
                }
            }
        }
    }

    // Finalize: lane holds rows 16w + 4 kg + r (r < 4) of bin `bin`.
    Red red = red_empty();
    const bool bin_ok = bin < p.n_bins;
#pragma unroll
    for (int t = 0; t < kNT; ++t) {
        const int n = nb * kNT + t;
        if (n >= p.n_tau) continue;
        const double tau = (double)p.tau[n];
        const double s = p.delta ? exp(-(double)p.delta / tau) : 1.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = m_first + 16 * wave + 4 * kg + r;
            if (m >= p.n_t0 || !bin_ok) continue;
            const double *abc = p.abc_cell + ((size_t)m * p.n_tau + n) * 3;
            const double v = twoF_cell(abc[0], abc[1], abc[2], s * (double)acc[t][0][r],
                                       s * (double)acc[t][1][r], s * (double)acc[t][2][r],
                                       s * (double)acc[t][3][r]);
            if (p.twoF) p.twoF[((size_t)bin * p.n_t0 + m) * p.n_tau + n] = (float)v;
            red = red_combine(red, Red{0.5 * v, 1.0, (long long)m * p.n_tau + n});
        }
    }
    // lanes sharing a bin: xor 16, 32; then the four waves in order
    red = red_combine(red, red_shfl_xor(red, 16));
    red = red_combine(red, red_shfl_xor(red, 32));
    if (lane < 16) wred[wave][lane] = red;
    __syncthreads();
    if (tid < 16) {
        const int b = col_tile * 16 + tid;
        if (b < p.n_bins) {
            Red tt = wred[0][tid];
            for (int w = 1; w < 4; ++w) tt = red_combine(tt, wred[w][tid]);
            Partial &o = p.part[(size_t)b * p.n_tiles + tile];
            o.fmax = tt.f;
            o.s = tt.s;
            o.idx = tt.i;
        }
    }
}

// bf16 hi / lo planes [4][bins16][kp] from the FP32 atoms x32 [K+1][bins][4].
__global__ __launch_bounds__(256) void build_planes_kernel(const float *x32, int32_t K, int32_t n_bins,
                                                           int32_t bins16, int32_t kp,
                                                           unsigned short *xhi, unsigned short *xlo) {
    const int64_t total = (int64_t)4 * bins16 * kp;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const int64_t k = i % kp;
        const int64_t cb = i / kp;
        const int bin = (int)(cb % bins16);
        const int c = (int)(cb / bins16);
        float x = 0.f;
        if (k < K && bin < n_bins) x = x32[((size_t)k * n_bins + bin) * 4 + c];
        const unsigned int pk = split_pack(x);
        xhi[i] = (unsigned short)(pk & 0xffffu);
        xlo[i] = (unsigned short)(pk >> 16);
    }
}

}  // namespace

hipError_t launch_exp_mfma(const ExpMfmaParams &p, hipStream_t s) {
    if (p.n_blocks <= 0) return hipSuccess;
    const int groups = (p.n_blocks + 7) / 8;
    const unsigned grid = (unsigned)(8 * groups * p.n_row_tiles * p.n_col_tiles);
    hipLaunchKernelGGL(exp_mfma_kernel, dim3(grid), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_build_planes(const float *x32, int32_t K, int32_t n_bins, int32_t bins16, int32_t kp,
                               unsigned short *xhi, unsigned short *xlo, hipStream_t s) {
    const int64_t total = (int64_t)4 * bins16 * kp;
    int64_t g = (total + 255) / 256;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(build_planes_kernel, dim3((unsigned)g), dim3(256), 0, s, x32, K, n_bins, bins16,
                       kp, xhi, xlo);
    return hipGetLastError();
}

}  // namespace tfs
