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
// Both operands are split into bf16 (or half-precision) hi + lo parts
// (x = hi + lo + O(2^-16 x)) and three products W_hi X_hi + W_hi X_lo +
// W_lo X_hi are accumulated in FP32.
//
// Three kernels share this file.  Shape windows whose rows lie on
// consecutive slots (exp_mfma_kernel) take the work item 64 consecutive t0
// rows x 16 bins (64 data columns) x 8 taus, in two passes of 4 taus: wave
// w owns rows 16w..16w+15, its four 16x16 output tiles per tau are the four
// data components of the same 16 bins, so every lane ends with all four
// components of (row, bin) cells and finalizes them in place; their A, B, C
// (FP64) come from the VALU kernel in its A/B/C-only mode.  Exponential
// windows on any t0 grid take the transposed work item (maps of 2 to 48
// bins, mfma_cells_tile) or the shared-weight one (49 or more bins,
// mfma_rows_tile_sw), described below, with A, B, C from the A/B/C scan.
#include "tfstat_device.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

namespace tfs {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kBlk = 8;       // taus per block (shared with the VALU tiling)
constexpr int kNT = 4;        // taus per matrix-core pass (two passes per block)
constexpr int kSK = kMfmaSK;  // band slots per staged weight window
static_assert(kSK % 64 == 0, "windows hold an even number of 32-slot K steps");
constexpr int kTW = kMfmaTW;  // staged window width (multiple of 8; sets the LDS pitch)
constexpr int kPad = kMfmaPad;  // zero entries in front of every shifted table
constexpr int kShifts = kMfmaShifts;  // shifted copies per (tau, part)
constexpr int kRowChunks = kTW / 8;                 // 16-byte chunks per table row
constexpr int kTabChunks = kNT * 2 * kShifts * kRowChunks;   // chunks per staged window
constexpr int kTabInstr = (kTabChunks + 63) / 64;   // 64-lane copies per window
constexpr int kAbcChunks = 64 * kBlk * 3 / 2;       // A/B/C of the tile, 16-byte chunks
// s_waitcnt operand (gfx9 encoding) that waits for LDS / scalar memory only:
// vmcnt 63, expcnt 7, lgkmcnt 0
constexpr int kWaitLgkm0 = 0xC07F;

struct Red {
    double f;
    double s;
    long long i;
};

__device__ inline Red red_empty() { return Red{-INFINITY, 0.0, 0x7fffffffffffffffLL}; }

// Max-shifted merge of two partial sums of exp(F); the scale factors
// exp(f - max) <= 1 are taken in FP32 (relative error ~1e-7 on the sum).
__device__ inline Red red_combine(const Red &a, const Red &b) {
    Red r;
    r.f = fmax(a.f, b.f);
    if (r.f == -INFINITY) return red_empty();
    const double sa = (a.f == -INFINITY) ? 0.0 : a.s * (double)__expf((float)(a.f - r.f));
    const double sb = (b.f == -INFINITY) ? 0.0 : b.s * (double)__expf((float)(b.f - r.f));
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

// 2F = (2 / D) (B |F_a|^2 + A |F_b|^2 - 2 C Re(F_a F_b*)), D = A B - C^2
// (section 2), with F = s acc: the factor k = 2 s^2 / D is folded into the
// cell's A, B, C once per (row, tau) and shared by all bins of the tile.
// Degenerate cells (D <= rtol A B) get zero coefficients, hence 2F = 0.
__device__ inline void fold_abc(double *abc, double s) {
    const double A = abc[0], B = abc[1], C = abc[2];
    const double D = A * B - C * C;
    double k = 0.0;
    if (D > kDegenerateRtol * A * B) k = 2.0 * s * s / D;
    abc[0] = k * A;
    abc[1] = k * B;
    abc[2] = 2.0 * k * C;
}

__device__ inline double twoF_folded(const double *abc, double far_, double fai, double fbr, double fbi) {
    return abc[1] * (far_ * far_ + fai * fai) + abc[0] * (fbr * fbr + fbi * fbi)
           - abc[2] * (far_ * fbr + fai * fbi);
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

// Shifted bf16 weight tables, built once per map: for block nb, tau t,
// part (0 = hi, 1 = lo) and shift s < 4, entry x holds part(g_t[x - kPad + s])
// (zero outside 0 <= d < lblk), so that 8 weights starting anywhere are two
// aligned 8-byte reads from the copy matching their start modulo 4.
__global__ __launch_bounds__(256) void shift_tables_kernel(ShiftTableParams p) {
    const int nb = p.blk_list[blockIdx.y];
    const int lblk = p.lblk[nb];
    const int lg = p.lg[nb];
    const int64_t src = p.blk_off[nb];
    unsigned short *dst = p.gsh + p.gsh_off[nb];
    const int64_t total = (int64_t)kBlk * 2 * kShifts * lg;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const int x = (int)(i % lg);
        const int64_t r = i / lg;
        const int sh = (int)(r % kShifts);
        const int part = (int)((r / kShifts) % 2);
        const int t = (int)(r / (2 * kShifts));
        const int d = x - kPad + sh;
        float g = 0.f;
        if (d >= 0 && d < lblk) g = p.g32[src + (int64_t)d * kBlk + t];
        const unsigned int pk = split_pack(g);
        dst[i] = (unsigned short)(part ? (pk >> 16) : (pk & 0xffffu));
    }
}

// Copies 16 bytes per lane from global memory straight into LDS: lane l of
// the wave writes dst + 16 l (gfx950 global_load_lds_dwordx4).
__device__ inline void copy16_to_lds(const void *src, void *dst_wave_base) {
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)dst_wave_base, 16, 0,
                                     0);
}

#ifndef TFS_MFMA_WAVES
#define TFS_MFMA_WAVES 2       // waves per SIMD the register budget targets
#endif
#ifndef TFS_MFMA_APREFETCH
#define TFS_MFMA_APREFETCH 1   // 1: weights read from LDS one K step ahead
#endif


__global__ __launch_bounds__(256, TFS_MFMA_WAVES) void exp_mfma_kernel(ExpMfmaParams p) {
    // two weight windows: flat 16-byte chunks, row (t, part, shift) by row
    // two weight-window buffers as two objects, so that the compiler can see
    // that reads of one do not wait for the direct-to-LDS copies into the other
    __shared__ __attribute__((aligned(16))) unsigned short tab0[kTabInstr * 64 * 8];
    __shared__ __attribute__((aligned(16))) unsigned short tab1[kTabInstr * 64 * 8];
    __shared__ __attribute__((aligned(16))) double abcs[64][kBlk][3];
    __shared__ Red wred[4][16];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    // Task decode.  Workgroup b runs on XCD b % 8, and each XCD has its own
    // L2.  With 8 or more column tiles (16 bins each), the column tiles are
    // dealt round-robin to the XCDs, so an XCD streams only its own bins'
    // bf16 planes; its tasks run block by block (largest band first), row
    // tile by row tile, so one block's weight tables are reused while hot.
    // With fewer column tiles, the blocks are the units of unit_decode.
    const int bid = blockIdx.x;
    const int xcd = bid & 7;
    const int slot = bid >> 3;
    int q, row_tile, col_tile;
    if (p.n_col_tiles >= 8) {
        const int cpx = (p.n_col_tiles + 7) / 8;          // column tiles per XCD
        const int per_block = p.n_row_tiles * cpx;
        q = slot / per_block;
        const int rem = slot % per_block;
        row_tile = rem / cpx;
        col_tile = (rem % cpx) * 8 + xcd;
        if (q >= p.n_blocks || col_tile >= p.n_col_tiles) return;
    } else {
        int rem;
        unit_decode(bid, p.n_blocks, p.n_row_tiles * p.n_col_tiles, q, rem);
        if (q >= p.n_blocks) return;
        row_tile = rem / p.n_col_tiles;
        col_tile = rem % p.n_col_tiles;
    }
    const int nb = p.blk_list[q];
    const int tile = nb * p.n_row_tiles + row_tile;

    const int m_first = row_tile * 64;
    const int m_last = min(m_first + 63, p.n_t0 - 1);
    const int k_first = p.k0_first + m_first;           // rows are consecutive slots
    const int k_last = p.k0_first + m_last;
    const int k_nom = k_first + 63;                      // slot of the tile's nominal last row
    const int lblk = p.lblk[nb];
    const int lg = p.lg[nb];
    const int kb_begin = k_first & ~31;
    // K steps of 32 slots from kb_begin; their number is rounded up to even
    // (columns kp_data .. kp of the B planes are zero)
    const int kb_data_end = min((k_last + lblk + 31) & ~31, p.kp_data);
    const int kb_end = kb_data_end > kb_begin ? kb_begin + ((kb_data_end - kb_begin + 63) & ~63) : kb_begin;
    const unsigned short *gsh = p.gsh + p.gsh_off[nb];

    // lane geometry
    const int lrow = lane & 15;           // A row / C column within a 16 tile
    const int kg = lane >> 4;             // K group of 8
    const int my_row = 16 * wave + lrow;  // A operand row within the 64-row tile
    const int bin = col_tile * 16 + lrow; // B / C column -> bin
    const bool bin_ok = bin < p.n_bins;

    // planes [4][kp / 32][bins16][32]: lane's 8 slots of step kb for its bin
    const unsigned short *bh_base = p.xhi + (size_t)bin * 32 + 8 * kg;
    const unsigned short *bl_base = p.xlo + (size_t)bin * 32 + 8 * kg;
    const size_t comp_stride = (size_t)p.bins16 * p.kp;
    const size_t step_stride = (size_t)p.bins16 * 32;
    auto load_b = [&](int kb, u32x4 *h, u32x4 *l) {
        const size_t so = (size_t)(kb >> 5) * step_stride;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            h[c] = *reinterpret_cast<const u32x4 *>(bh_base + c * comp_stride + so);
            l[c] = *reinterpret_cast<const u32x4 *>(bl_base + c * comp_stride + so);
        }
    };

    // A, B, C of the tile's 64 rows x 8 taus into LDS (rows past n_t0 read a
    // valid row; rows of abc_cell hold whole blocks and start 16-byte aligned).
    for (int i = wave; i < (kAbcChunks + 63) / 64; i += 4) {
        int f = i * 64 + lane;
        if (f >= kAbcChunks) f = 0;
        const int row = f / (kBlk * 3 / 2);
        const int ch = f - row * (kBlk * 3 / 2);
        const int m = min(m_first + row, p.n_t0 - 1);
        copy16_to_lds(p.abc_cell + ((size_t)m * p.abc_pitch + (size_t)nb * kBlk) * 3 + 2 * ch,
                      reinterpret_cast<double *>(abcs) + (size_t)i * 64 * 2);
    }

    Red red = red_empty();

#pragma unroll 1
    for (int half = 0; half < kBlk / kNT; ++half) {
        const int t0 = half * kNT;        // first tau of this pass within the block
        f32x4 acc[kNT][4];
#pragma unroll
        for (int t = 0; t < kNT; ++t)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};

        // Windows of weights: in window w, copy s, position x holds
        // g[d_lo(w) + x + s] with d_lo(w) = floor8(kb_begin + w kSK - k_nom),
        // a straight aligned copy of the global shifted tables from entry
        // d_lo(w) + kPad.  Window w + 1 is copied into the other buffer while
        // window w is in use.
        auto issue = [&](int w, unsigned short *dst) {
            const int dl = (kb_begin + w * kSK - k_nom) & ~7;
            const unsigned short *src0 = gsh + (size_t)t0 * 2 * kShifts * lg + (dl + kPad);
            for (int i = wave; i < kTabInstr; i += 4) {
                int f = i * 64 + lane;
                if (f >= kTabChunks) f = 0;     // padding chunks: any valid source
                const int row = f / kRowChunks;
                const int ch = f - row * kRowChunks;
                copy16_to_lds(src0 + (size_t)row * lg + 8 * ch, dst + i * 64 * 8);
            }
        };
        const int n_win = (kb_end - kb_begin + kSK - 1) / kSK;
        int ks = kb_begin;
        int d_lo = (kb_begin - k_nom) & ~7;
        auto enter_window = [&](int w, unsigned short *nxt) {
            // window w has landed and every wave is done with window w - 1
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            ks = kb_begin + w * kSK;
            d_lo = (ks - k_nom) & ~7;
            if (w + 1 < n_win) issue(w + 1, nxt);
        };
        // Lane's weights for the K step at kb: g[kb + 8 kg - k0(row) .. + 8)
        // from copy u % kShifts of the staged window.
        auto load_a = [&](const unsigned short *cur, int kb, bf16x8 *ah, bf16x8 *al) {
            const int u = kb + 8 * kg - (k_first + my_row) - d_lo;
            const int sh = u & (kShifts - 1);
            const int q0 = u - sh;
            const unsigned short *tl = cur + sh * kTW + q0;   // (t, part) rows stride kShifts kTW
#pragma unroll
            for (int t = 0; t < kNT; ++t) {
                const unsigned short *th = tl + (t * 2 + 0) * kShifts * kTW;
                const unsigned short *tw = tl + (t * 2 + 1) * kShifts * kTW;
                if constexpr (kShifts == 8) {
                    ah[t] = bitcast4<bf16x8>(*reinterpret_cast<const u32x4 *>(th));
                    al[t] = bitcast4<bf16x8>(*reinterpret_cast<const u32x4 *>(tw));
                } else {
                    const uint64_t *ph = reinterpret_cast<const uint64_t *>(th);
                    const uint64_t *pl = reinterpret_cast<const uint64_t *>(tw);
                    u32x4 h, l;
                    const uint64_t h0 = ph[0], h1 = ph[1], l0 = pl[0], l1 = pl[1];
                    h[0] = (unsigned)h0; h[1] = (unsigned)(h0 >> 32); h[2] = (unsigned)h1; h[3] = (unsigned)(h1 >> 32);
                    l[0] = (unsigned)l0; l[1] = (unsigned)(l0 >> 32); l[2] = (unsigned)l1; l[3] = (unsigned)(l1 >> 32);
                    ah[t] = bitcast4<bf16x8>(h);
                    al[t] = bitcast4<bf16x8>(l);
                }
            }
        };
        // 48 products of one K step.  The three products run one after the
        // other over all 16 accumulators, so dependent matrix-core ops on one
        // accumulator are 16 apart.
        auto mfma_step = [&](const bf16x8 *ah, const bf16x8 *al, const u32x4 *ch, const u32x4 *cl) {
#pragma unroll
            for (int t = 0; t < kNT; ++t)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[t], bitcast4<bf16x8>(ch[c]), acc[t][c], 0, 0, 0);
#pragma unroll
            for (int t = 0; t < kNT; ++t)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[t], bitcast4<bf16x8>(cl[c]), acc[t][c], 0, 0, 0);
#pragma unroll
            for (int t = 0; t < kNT; ++t)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[t], bitcast4<bf16x8>(ch[c]), acc[t][c], 0, 0, 0);
        };
        // Software pipeline: while the products of step kb run, the B
        // operands of step kb + 32 (global) and the weights of step kb + 32
        // (LDS, same window) are already on their way.  Every window holds an
        // even number of K steps (kSK is a multiple of 64 and the pass end is
        // rounded up to one, over zero B columns), so the loop body is two
        // steps with no branch; a prefetch past the window or the pass end
        // re-reads an in-range step and is discarded.
        u32x4 bh[4], bl[4], nh[4], nl[4];
        bf16x8 ah[kNT], al[kNT], mh[kNT], ml[kNT];
        if (kb_begin < kb_end) {
            __syncthreads();   // the previous pass is done with both buffers
            issue(0, tab0);
            load_b(kb_begin, bh, bl);
        }
        // Two K steps from kb (kb + 32 < kw_end always holds).
        auto pair = [&](const unsigned short *cur, int kb, int ka_last) {
            load_b(kb + 32, nh, nl);
            load_a(cur, kb + 32, mh, ml);
            if constexpr (!TFS_MFMA_APREFETCH) load_a(cur, kb, ah, al);
            __builtin_amdgcn_sched_barrier(0);
            mfma_step(ah, al, bh, bl);
            __builtin_amdgcn_sched_barrier(0);
            load_b(min(kb + 64, kb_end - 32), bh, bl);
            if constexpr (TFS_MFMA_APREFETCH) load_a(cur, min(kb + 64, ka_last), ah, al);
            __builtin_amdgcn_sched_barrier(0);
            mfma_step(mh, ml, nh, nl);
            __builtin_amdgcn_sched_barrier(0);
        };
        auto run_window = [&](int w, const unsigned short *cur, unsigned short *nxt) {
            enter_window(w, nxt);
            const int kw_end = min(ks + kSK, kb_end);
            const int ka_last = ks + kSK - 32;      // last K step this window's weights cover
            if constexpr (TFS_MFMA_APREFETCH) load_a(cur, ks, ah, al);
            // Only the weights just read are waited for here; without this the
            // loop's first products would also wait for every B prefetch.
            __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
            // The first pair is peeled off: while the next window's direct
            // copies are in flight, B loads can only be waited for all at once,
            // and the peeled pair takes that wait once per window instead of
            // once per loop trip.
            pair(cur, ks, ka_last);
#pragma unroll 1
            for (int kb = ks + 64; kb < kw_end; kb += 64) pair(cur, kb, ka_last);
        };
#pragma unroll 1
        for (int w = 0; w < n_win; w += 2) {
            run_window(w, tab0, tab1);
            if (w + 1 < n_win) run_window(w + 1, tab1, tab0);
        }

        if (half == 0) {   // A/B/C copies have landed (also with no K steps):
                           // fold the window scale and 1 / D into them
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            for (int e = tid; e < 64 * kBlk; e += 256) {
                const int n = nb * kBlk + (e % kBlk);
                const double tau = (double)p.tau[n < p.n_tau ? n : p.n_tau - 1];
                fold_abc(abcs[e / kBlk][e % kBlk], p.delta ? exp(-(double)p.delta / tau) : 1.0);
            }
            __syncthreads();
        }
        // Finalize this pass: lane holds rows 16w + 4 kg + r (r < 4) of bin
        // `bin`; 2F in FP64, then max, first argmax and sum of exp(F - max).
        double v2[kNT][4];
        double fmx = -INFINITY;
        long long imx = 0x7fffffffffffffffLL;
#pragma unroll
        for (int t = 0; t < kNT; ++t) {
            const int n = nb * kBlk + t0 + t;
            const bool n_ok = n < p.n_tau;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m_first + 16 * wave + 4 * kg + r;
                v2[t][r] = -INFINITY;
                if (!n_ok || m >= p.n_t0 || !bin_ok) continue;
                const double v = twoF_folded(abcs[m - m_first][t0 + t], (double)acc[t][0][r],
                                             (double)acc[t][1][r], (double)acc[t][2][r],
                                             (double)acc[t][3][r]);
                if (p.twoF) p.twoF[((size_t)bin * p.n_t0 + m) * p.n_tau + n] = (float)v;
                v2[t][r] = v;
                const long long idx = (long long)m * p.n_tau + n;
                if (v > fmx || (v == fmx && idx < imx)) {
                    fmx = v;
                    imx = idx;
                }
            }
        }
        if (fmx != -INFINITY) {
            double sum = 0.0;
#pragma unroll
            for (int t = 0; t < kNT; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (v2[t][r] != -INFINITY) sum += (double)__expf((float)(0.5 * (v2[t][r] - fmx)));
            red = red_combine(red, Red{0.5 * fmx, sum, imx});
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

// ---------------------------------------------------------------------------
// Any t0 grid: weights computed in registers.
//
// Eight weights of one K step of a lane are
//   w_j = exp(-(t_{k+j} - t0_m) / tau) = 2^((d + j) c_T + c_delta),
//   d = k - k0_m, c_T = -T log2(e) / tau, c_delta = -delta_m log2(e) / tau,
// zero outside the row's window (0 <= d + j < L_m: the SFT start times in
// [t0_m, t0_m + 3 tau)), generated as one exp2 and 7 products by
// exp(-T / tau), then split into hi + lo parts.  A, B, C (FP64, the same
// weights squared) come from the A/B/C scan.
// ---------------------------------------------------------------------------

// The lane's 8 weights of one K step as hi and lo parts (lo = part(w - hi),
// w - hi exact before its own rounding): bf16 (round to nearest even) or,
// for F16, IEEE half precision (round toward zero; lo then keeps 11 of the
// 13 remaining bits) of w * 2^kF16WeightExp (the caller folds the
// factor into cD; it keeps the lo parts of the smallest weights, e^-3 * 2^-11,
// out of the half-precision subnormal range).  The exponential is the
// hardware base-2 one: within a window its argument is in (-3 log2(e), 0]
// (plus the F16 offset), far from the range where it would flush to zero.
// EDGE: the step may hold slots outside the lane's window [0, L), which
// weigh 0.
// w - h with h the low (sub_half_lo) or high (sub_half_hi) IEEE half of the
// packed pair hb: one v_fma_mix_f32 (h * -1 + w, the half widened exactly).
__device__ inline float sub_half_lo(float w, unsigned hb) {
    float r;
    asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(hb), "v"(w));
    return r;
}
__device__ inline float sub_half_hi(float w, unsigned hb) {
    float r;
    asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(hb), "v"(w));
    return r;
}

template <bool EDGE, bool F16>
__device__ __attribute__((always_inline)) inline void rows_weights(int d0, float cT, float cD, float rho, int L,
                                                                 u32x4 &h, u32x4 &l) {
    // hi and lo must split one rounded FP32 weight: a product fused into
    // the lo subtraction but not into the hi conversion would leave hi + lo
    // one hi ulp (2^-11 in half precision) away from the weight
#pragma clang fp contract(off)
    float w[8];
    w[0] = __builtin_amdgcn_exp2f(fmaf((float)d0, cT, cD));
#pragma unroll
    for (int j = 1; j < 8; ++j) w[j] = w[j - 1] * rho;
    if constexpr (EDGE) {
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if ((unsigned)(d0 + j) >= (unsigned)L) w[j] = 0.f;
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        if constexpr (F16) {
            // hi by the packing conversion (round toward zero); w - hi, exact
            // in FP32, from the packed half and the same rounded weight in
            // one mixed-precision FMA each; lo its packing conversion
            const auto h2 = __builtin_amdgcn_cvt_pkrtz(w[2 * p], w[2 * p + 1]);
            const unsigned hb = __builtin_bit_cast(unsigned, h2);
            const auto l2 = __builtin_amdgcn_cvt_pkrtz(sub_half_lo(w[2 * p], hb), sub_half_hi(w[2 * p + 1], hb));
            h[p] = hb;
            l[p] = __builtin_bit_cast(unsigned, l2);
        } else {
            typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
            const bf16x2 h2 = {(__bf16)w[2 * p], (__bf16)w[2 * p + 1]};
            const unsigned u = __builtin_bit_cast(unsigned, h2);
            // hi parts as floats: the low half moved up (a byte permute, so
            // that the compiler does not convert w again) and the high half
            // masked
            const float h0 = __uint_as_float(__builtin_amdgcn_perm(0u, u, 0x01000c0cu));
            const float h1 = __uint_as_float(u & 0xffff0000u);
            const bf16x2 l2 = {(__bf16)(w[2 * p] - h0), (__bf16)(w[2 * p + 1] - h1)};
            h[p] = u;
            l[p] = __builtin_bit_cast(unsigned, l2);
        }
    }
}

// One 16x16x32 product of the part type (bf16 or half), FP32 accumulate.
template <bool F16>
__device__ __attribute__((always_inline)) inline f32x4 mfma_part(u32x4 a, u32x4 b, f32x4 c) {
    if constexpr (F16)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(bitcast4<f16x8>(a), bitcast4<f16x8>(b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(bitcast4<bf16x8>(a), bitcast4<bf16x8>(b), c, 0, 0, 0);
}

// Buffer resource of `bytes` bytes at `base` (raw buffer: stride 0, offsets
// in bytes; reads past the end return zero).
__device__ inline __amdgpu_buffer_rsrc_t plane_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}

// ---------------------------------------------------------------------------
// Maps of fewer than kSwMinColTiles column tiles: the transposed product.
// For one bin, one tau and data component c,
//   F_c[m] = s_m sum_d g[d] x_c[k0_m + d],   g[d] = exp(-d T_sft / tau),
//   s_m = exp(-delta_m / tau),
// with k0_m the row's first slot on the slot grid (extended before the
// data, so that delta_m lies in [0, T_sft)).  The weights g depend on the
// tau and the lag only, so they are the B operand (32 lags x 16 taus per
// K step) that a wave shares among all its rows, and the A operand gathers
// the data: row i of 16-row tile c is component c of the wave's cell i
// (t0 row m = first + i), and its 8 lags of a K step are the 8 slots from
// k0_m + d; the accumulators then give each lane all four components of
// its cells, and the rows of one load instruction read one plane, where
// nearby rows share cache lines.  A window
// holds the lags below L_m = ceil((3 tau - delta_m) / T_sft), which is
// L = ceil(3 tau / T_sft) or L - 1; B holds the lags below L, and a cell
// whose band is L - 1 has the product of lag L - 1 taken off in the
// finalize.  Every product's columns are taus and its rows cells, so the
// matrix cores do no work on absent bins, and a weight is made once per
// 16 cells.
//
// Work item: 64 rows (16 per wave, one 16-row tile per component) x one
// bin x kCellsBlocks blocks of 8 taus (kCellsNT tiles of 16 taus; the
// blocks of one item are consecutive in the block list, which runs from
// the longest band down, and a tile sits out the K steps past its own
// longest band).  Data planes: [copy kCellsCopies][component 4][bin][kpc],
// slot k of copy r at element k + 16 - r, so that the 8 slots from any k
// are one 16-byte load from copy k mod kCellsCopies at an address aligned
// to 2 kCellsCopies bytes (two copies: 4-byte aligned, which the loads
// need; eight copies, 16-byte aligned, measured no faster); slots outside
// [0, K) read as zero (the elements in front and the pad behind K are
// zero, and loads that would start more than 8 slots before the data or at
// or after K are sent beyond the buffer's end, which reads zero).
// ---------------------------------------------------------------------------
struct CellsSmem {
    Red wred[4];
};

template <bool F16, typename PP>
__device__ __attribute__((always_inline)) inline void mfma_cells_tile(PP &p, CellsSmem &sm, int g, int row_tile,
                                                                    int bin) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lrow = lane & 15;   // A row / B and C column within the 16 tile
    const int kg = lane >> 4;     // K group of 8; C rows 4 kg .. 4 kg + 3
    const int n_t0 = p.n_t0;
    const int K = p.K;
    const int m_w = row_tile * 64 + 16 * wave;   // first row of this wave
    const int q0 = g * kCellsBlocks;
    const int nblk = min(kCellsBlocks, p.n_blocks - q0);
    const int64_t T = p.t_sft;

    // B side: the lane's tau (column lrow) of each 16-tau tile; a column
    // without a tau has weights exp2(-inf) = 0
    float cT[kCellsNT], cD[kCellsNT], rho[kCellsNT];
    int L[kCellsNT];
    int Lt[kCellsNT];        // the tile's longest band (wave-uniform; 0: no tau)
    int Ls[kCellsNT];        // the tile's shortest band (wave-uniform)
    // the lane's tau of tile t (-1: none)
    auto tau_of = [&](int t) {
        const int qb = 2 * t + (lrow >> 3);
        int n = -1;
        if (qb < nblk) {
            n = p.blk_list[q0 + qb] * kBlk + (lrow & 7);
            if (n >= p.n_tau) n = -1;
        }
        return n;
    };
#pragma unroll
    for (int t = 0; t < kCellsNT; ++t) {
        const int n = tau_of(t);
        if (n >= 0) {
            const int64_t tau = p.tau[n];
            const double inv = 1.4426950408889634 / (double)tau;
            cT[t] = (float)(-(double)T * inv);
            cD[t] = F16 ? (float)kF16WeightExp : 0.f;
            rho[t] = exp2f(cT[t]);
            L[t] = (int)min((3 * tau + T - 1) / T, (int64_t)1 << 30);
        } else {
            cT[t] = 0.f;
            cD[t] = -INFINITY;
            rho[t] = 0.f;
            L[t] = 0;
        }
        int lt = L[t];
        int ls = n >= 0 ? L[t] : 1 << 30;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            lt = max(lt, __shfl_xor(lt, o, 64));
            ls = min(ls, __shfl_xor(ls, o, 64));
        }
        Lt[t] = __builtin_amdgcn_readfirstlane(lt);
        Ls[t] = __builtin_amdgcn_readfirstlane(ls);
    }

    // A side: 16-row tile c holds component c of the wave's 16 cells, the
    // lane's cell being row m_w + lrow; element of its slot k0 in its copy
    // (rows past the grid repeat the last one; never written)
    const int a_k0 = p.rows[min(m_w + lrow, n_t0 - 1)].k0;
    int a_base[4];
    {
        const int r = a_k0 & (kCellsCopies - 1);
#pragma unroll
        for (int c = 0; c < 4; ++c) a_base[c] = ((r * 4 + c) * p.n_bins + bin) * p.kpc + 16 - r + a_k0;
    }
    int k0lo = a_k0, k0hi = a_k0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        k0lo = min(k0lo, __shfl_xor(k0lo, o, 64));
        k0hi = max(k0hi, __shfl_xor(k0hi, o, 64));
    }
    k0lo = __builtin_amdgcn_readfirstlane(k0lo);
    k0hi = __builtin_amdgcn_readfirstlane(k0hi);
    int lmax = 0;
#pragma unroll
    for (int t = 0; t < kCellsNT; ++t) lmax = max(lmax, Lt[t]);
    // lags with data for some row: below K - k0lo; an even number of steps
    const int kend = min(lmax, K - k0lo);
    const int kb_end = kend > 0 ? (kend + 31) & ~31 : 0;
    // steps whose loads all fall in [-8, K) (no per-lane check)
    const int kd_lo = -8 - k0lo, kd_hi = K - 24 - k0hi;

    const uint32_t bytes = (uint32_t)(kCellsCopies * 4 * p.n_bins) * (uint32_t)p.kpc * 2u;
    const __amdgpu_buffer_rsrc_t rh = plane_rsrc(p.chi, bytes);
    const __amdgpu_buffer_rsrc_t rl = plane_rsrc(p.clo, bytes);
    auto load_a = [&](int kb, u32x4 *h, u32x4 *l) {
        const int d0 = kb + 8 * kg;
        const bool edge = kb < kd_lo || kb >= kd_hi;
        const int s = a_k0 + d0;
        const bool out = edge && (s < -8 || s >= K);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint32_t off = out ? 0x80000000u : (uint32_t)(a_base[c] + d0) * 2u;
            h[c] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rh, (int)off, 0, 0));
            l[c] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rl, (int)off, 0, 0));
        }
    };

    f32x4 acc[4][kCellsNT];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int t = 0; t < kCellsNT; ++t) acc[mt][t] = f32x4{0.f, 0.f, 0.f, 0.f};

    // one K step: per tau tile still inside its band, the lane's weights
    // (masked past a band only where one of the tile's bands may end in
    // the step), then 12 products (three of each 16-row tile)
    auto step = [&](int kb, const u32x4 *ah, const u32x4 *al) {
        const int d0 = kb + 8 * kg;
#pragma unroll
        for (int t = 0; t < kCellsNT; ++t) {
            if (kb >= Lt[t]) continue;
            u32x4 bh, bl;
            if (kb + 32 > Ls[t])
                rows_weights<true, F16>(d0, cT[t], cD[t], rho[t], L[t], bh, bl);
            else
                rows_weights<false, F16>(d0, cT[t], cD[t], rho[t], L[t], bh, bl);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) acc[mt][t] = mfma_part<F16>(ah[mt], bh, acc[mt][t]);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) acc[mt][t] = mfma_part<F16>(ah[mt], bl, acc[mt][t]);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) acc[mt][t] = mfma_part<F16>(al[mt], bh, acc[mt][t]);
        }
    };
    // one step's loads at a time: the registers of a second set would cost
    // a wave per SIMD, and three waves hide the loads' latency better
#pragma unroll 1
    for (int kb = 0; kb < kb_end; kb += 32) {
        u32x4 ah[4], al[4];
        load_a(kb, ah, al);
        step(kb, ah, al);
    }

    // finalize: lane holds cells 4 kg + r (rows m_w + 4 kg + r, r < 4) for
    // the tau of its column, component c in acc[c][t][r].  Half precision
    // sums carry the powers of two of the weights and of their data
    // column, removed exactly here.
    double sc[4] = {1.0, 1.0, 1.0, 1.0};
    if constexpr (F16) {
#pragma unroll
        for (int c = 0; c < 4; ++c) sc[c] = ldexp(1.0, -(kF16WeightExp + p.colexp[c * p.bins16 + bin]));
    }
    Red red = red_empty();
#pragma unroll
    for (int t = 0; t < kCellsNT; ++t) {
        const int n = tau_of(t);
        if (n < 0) continue;
        const int64_t tau = p.tau[n];
        const float cI = (float)(1.4426950408889634 / (double)tau);
        double v2[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
        double fmx = -INFINITY;
        long long imx = 0x7fffffffffffffffLL;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const int m = m_w + 4 * kg + mt;
            if (m >= n_t0) continue;
            const RowPlan rp = p.rows[m];
            double f[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) f[c] = sc[c] * (double)acc[c][t][mt];
            // the band of this row: L or L - 1; the last lag's product off
            const int64_t span = 3 * tau - rp.delta;
            const int64_t Lm = span > 0 ? min((span + T - 1) / T, (int64_t)1 << 30) : 0;
            const int sf = rp.k0 + L[t] - 1;
            if (Lm < L[t] && sf >= 0 && sf < K) {
                // the weight of lag L - 1 as the K steps made it
                const int dl = L[t] - 1;
                float w = __builtin_amdgcn_exp2f(fmaf((float)(dl & ~7), cT[t], cD[t]));
                for (int j = 0; j < (dl & 7); ++j) w *= rho[t];
                const double wq = F16 ? ldexp((double)w, -kF16WeightExp) : (double)w;
                const float4 x = *reinterpret_cast<const float4 *>(p.x32 + ((size_t)sf * p.n_bins + bin) * 4);
                f[0] -= wq * (double)x.x;
                f[1] -= wq * (double)x.y;
                f[2] -= wq * (double)x.z;
                f[3] -= wq * (double)x.w;
            }
            const double *src = p.abc_cell + ((size_t)m * p.abc_pitch + n) * 3;
            double abc[3] = {src[0], src[1], src[2]};
            fold_abc(abc, (double)exp2f(-(float)rp.delta * cI));
            const double v = twoF_folded(abc, f[0], f[1], f[2], f[3]);
            if (p.twoF) p.twoF[((size_t)bin * n_t0 + m) * p.n_tau + n] = (float)v;
            v2[mt] = v;
            const long long idx = (long long)m * p.n_tau + n;
            if (v > fmx || (v == fmx && idx < imx)) {
                fmx = v;
                imx = idx;
            }
        }
        if (fmx != -INFINITY) {
            double sum = 0.0;
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
                if (v2[mt] != -INFINITY) sum += (double)__expf((float)(0.5 * (v2[mt] - fmx)));
            red = red_combine(red, Red{0.5 * fmx, sum, imx});
        }
    }

    // the wave's lanes, then the four waves in order
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) red = red_combine(red, red_shfl_xor(red, o));
    if (lane == 0) sm.wred[wave] = red;
    __syncthreads();
    if (tid < nblk) {
        Red tt = red_empty();
        if (tid == 0)
            for (int w = 0; w < 4; ++w) tt = red_combine(tt, sm.wred[w]);
        // the item's cells count in its first block's slot; the others empty
        Partial &o = p.part[(size_t)bin * p.n_tiles + (size_t)p.blk_list[q0 + tid] * p.n_row_tiles + row_tile];
        o.fmax = tt.f;
        o.s = tt.s;
        o.idx = tt.i;
    }
}

// ---------------------------------------------------------------------------
// Maps of kSwMinColTiles or more 16-bin column tiles: one work item is 64 t0
// rows x 4 column tiles (64 bins) x 8 taus.  The four waves take the rows 16
// at a time, all four on the same rows, and split the bins (wave w: column
// tile 4 g + w); the 8 taus are one pass, so that each B load of a wave
// feeds 8 taus' products.  In every K step each wave makes the weights of two
// taus (w and w + 4) for the shared rows, the row scale and each row's exact
// band end included, and puts their hi and lo parts in LDS; every wave reads the eight
// taus' parts from there.  A weight is thus made once per 64 bins instead of
// once per 16, which leaves the matrix cores most of each wave's issue
// cycles.  The K steps of the four waves are the same (same rows, same
// taus), so they run in step, two LDS buffers of weights and one barrier per
// step.
// ---------------------------------------------------------------------------
#ifndef TFS_SW_NT
#define TFS_SW_NT 8            // taus per pass of the shared-weight work item
#endif
constexpr int kSwNT = TFS_SW_NT;
constexpr int kSwTW = kSwNT / 4;   // taus whose weights each wave makes
static_assert(kSwNT % 4 == 0 && kBlk % kSwNT == 0, "taus of a pass split over the four waves");

struct SwSmem {
    u32x4 a[2][kSwNT][2][64];        // weights of one K step: [buffer][tau][hi, lo][lane]
    double abc[16][kBlk][3];         // the 16 rows' folded A, B, C of the block
    float out[4][16][16][kBlk + 1];  // per wave: 2F of the rows x its 16 bins x 8 taus
};

template <bool F16, typename PP>
__device__ __attribute__((always_inline)) inline void mfma_rows_tile_sw(PP &p, SwSmem &sm, int q, int row_tile,
                                                                      int col_group) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nb = p.blk_list[q];
    const int tile = nb * p.n_row_tiles + row_tile;
    const int n_t0 = p.n_t0;
    const int lrow = lane & 15;   // A row / C column within the 16 tile
    const int kg = lane >> 4;     // K group of 8
    const int col_tile = col_group * 4 + wave;
    const bool col_ok = col_tile < p.n_col_tiles;   // wave-uniform
    const int bin = col_tile * 16 + lrow;
    const bool bin_ok = bin < p.n_bins;
    const int64_t T = p.t_sft;

    // B operand: planes [4][kp / 32][bins16][32], the lane's 8 slots of step
    // kb for its bin.  One buffer resource per component and part (scalar
    // registers), the step's offset in a scalar, the lane's own offset in a
    // vector register: no vector address arithmetic per load (component
    // planes are < 2^31 bytes, which the planner checks).  Waves past the
    // last column tile load nothing; they still make weights and keep the
    // barriers.
    const uint32_t comp_bytes = (uint32_t)p.bins16 * (uint32_t)p.kp * 2u;
    const uint32_t step_bytes = (uint32_t)p.bins16 * 64u;
    const uint32_t lane_off = (uint32_t)(((col_ok ? col_tile : 0) * 16 + lrow) * 32 + 8 * kg) * 2u;
    __amdgpu_buffer_rsrc_t rh[4], rl[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        rh[c] = plane_rsrc(p.xhi + (size_t)c * p.bins16 * p.kp, comp_bytes);
        rl[c] = plane_rsrc(p.xlo + (size_t)c * p.bins16 * p.kp, comp_bytes);
    }
    auto load_b = [&](int kb, u32x4 *h, u32x4 *l) {
        const int so = (int)((uint32_t)(kb >> 5) * step_bytes);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            h[c] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rh[c], (int)lane_off, so, 0));
            l[c] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rl[c], (int)lane_off, so, 0));
        }
    };
    double sc[4] = {1.0, 1.0, 1.0, 1.0};
    if constexpr (F16) {
        if (col_ok) {
#pragma unroll
            for (int c = 0; c < 4; ++c)
                sc[c] = ldexp(1.0, -(kF16WeightExp + p.colexp[c * p.bins16 + col_tile * 16 + lrow]));
        }
    }

    Red red = red_empty();
#pragma unroll 1
    for (int g = 0; g < 4; ++g) {
        const int m_g = row_tile * 64 + 16 * g;   // first row of the group
        if (m_g >= n_t0) break;
        // A, B, C of the group's 16 rows x 8 taus with 2 / D folded in (the
        // previous group's readers are done first)
        __syncthreads();
        if (tid < 16 * kBlk) {
            const int r = tid / kBlk, t = tid % kBlk;
            const int m = min(m_g + r, n_t0 - 1);
            const double *src = p.abc_cell + ((size_t)m * p.abc_pitch + (size_t)nb * kBlk + t) * 3;
            double abc[3] = {src[0], src[1], src[2]};
            fold_abc(abc, 1.0);
            sm.abc[r][t][0] = abc[0];
            sm.abc[r][t][1] = abc[1];
            sm.abc[r][t][2] = abc[2];
        }
        __syncthreads();
        // the lane's A row (rows past the grid repeat the last one; never written)
        const RowPlan ra = p.rows[min(m_g + lrow, n_t0 - 1)];
        const int k_first = __builtin_amdgcn_readfirstlane(p.rows[m_g].k0);
#pragma unroll 1
        for (int half = 0; half < kBlk / kSwNT; ++half) {
            const int t0 = half * kSwNT;
            // this wave's taus (t0 + w + 4 i): their weight constants for the
            // lane's row; the pass's last tau: the K range
            float cT[kSwTW], cD[kSwTW], rho[kSwTW];
            int Lw[kSwTW], Llast;
#pragma unroll
            for (int i = 0; i < kSwTW; ++i) {
                const int n = min(nb * kBlk + t0 + wave + 4 * i, p.n_tau - 1);
                const int64_t tau = p.tau[n];
                const double inv = 1.4426950408889634 / (double)tau;
                cT[i] = (float)(-(double)T * inv);
                cD[i] = (float)(-(double)ra.delta * inv) + (F16 ? (float)kF16WeightExp : 0.f);
                rho[i] = exp2f(cT[i]);
                const int64_t span = 3 * tau;
                Lw[i] = span > ra.delta ? (int)min((span - ra.delta + T - 1) / T, (int64_t)1 << 30) : 0;
            }
            {
                const int64_t span_l = 3 * p.tau[min(nb * kBlk + t0 + kSwNT - 1, p.n_tau - 1)];
                Llast = span_l > ra.delta ? (int)min((span_l - ra.delta + T - 1) / T, (int64_t)1 << 30) : 0;
            }
            // K range: the first row's slot to the furthest band end of the
            // rows (the pass's last tau is its longest), an even number of
            // 32-slot steps
            int kend = (int)min((int64_t)ra.k0 + Llast, (int64_t)p.kp_data);
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) kend = max(kend, __shfl_xor(kend, o, 64));
            kend = __builtin_amdgcn_readfirstlane(kend);
            const int kb_begin = max(k_first, 0) & ~31;
            const int kb_data_end = min((kend + 31) & ~31, p.kp_data);
            const int kb_end = kb_data_end > kb_begin ? kb_begin + ((kb_data_end - kb_begin + 63) & ~63) : kb_begin;

            f32x4 acc[kSwNT][4];
#pragma unroll
            for (int t = 0; t < kSwNT; ++t)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};

            // this wave's weights of step kb into LDS buffer buf (the window
            // mask applied in every step: no branch between the weights and
            // the products, which the compiler may then interleave)
            auto make_w = [&](int kb, int buf) {
#pragma unroll
                for (int i = 0; i < kSwTW; ++i) {
                    u32x4 ah, al;
                    rows_weights<true, F16>(kb + 8 * kg - ra.k0, cT[i], cD[i], rho[i], Lw[i], ah, al);
                    sm.a[buf][wave + 4 * i][0][lane] = ah;
                    sm.a[buf][wave + 4 * i][1][lane] = al;
                }
            };
            // the products of one step (12 per tau), each tau's weights read
            // from LDS buffer buf one tau ahead of its products
            auto mma = [&](int buf, const u32x4 *ch, const u32x4 *cl) {
                u32x4 ah = sm.a[buf][0][0][lane], al = sm.a[buf][0][1][lane];
#pragma unroll
                for (int t = 0; t < kSwNT; ++t) {
                    u32x4 nah = ah, nal = al;
                    if (t + 1 < kSwNT) {
                        nah = sm.a[buf][t + 1][0][lane];
                        nal = sm.a[buf][t + 1][1][lane];
                    }
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[t][c] = mfma_part<F16>(ah, ch[c], acc[t][c]);
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[t][c] = mfma_part<F16>(ah, cl[c], acc[t][c]);
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[t][c] = mfma_part<F16>(al, ch[c], acc[t][c]);
                    ah = nah;
                    al = nal;
                }
            };
            if (kb_begin < kb_end) {
                make_w(kb_begin, 0);
                if (col_ok) {
                    u32x4 bh[4], bl[4], nh[4], nl[4];
                    load_b(kb_begin, bh, bl);
                    __syncthreads();
#pragma unroll 1
                    for (int kb = kb_begin; kb < kb_end; kb += 64) {
                        // step kb from buffer 0 while step kb + 32's weights
                        // go to buffer 1 (kb + 32 < kb_end: the count is even)
                        load_b(kb + 32, nh, nl);
                        make_w(kb + 32, 1);
                        mma(0, bh, bl);
                        __syncthreads();
                        load_b(min(kb + 64, kb_end - 32), bh, bl);
                        // (the last round writes one step again: no branch)
                        make_w(min(kb + 64, kb_end - 32), 0);
                        mma(1, nh, nl);
                        __syncthreads();
                    }
                } else {
                    // no column tile: this wave's weights only
                    __syncthreads();
#pragma unroll 1
                    for (int kb = kb_begin; kb < kb_end; kb += 64) {
                        make_w(kb + 32, 1);
                        __syncthreads();
                        make_w(min(kb + 64, kb_end - 32), 0);
                        __syncthreads();
                    }
                }
            }

            // finalize: lane holds rows 4 kg + r (r < 4) of the group for
            // `bin`; half-precision sums carry the powers of two of the
            // weights and of their data column, removed exactly here
            if (col_ok) {
                double v2[kSwNT][4];
                double fmx = -INFINITY;
                long long imx = 0x7fffffffffffffffLL;
#pragma unroll
                for (int t = 0; t < kSwNT; ++t) {
                    const int n = nb * kBlk + t0 + t;
                    const bool n_ok = n < p.n_tau;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int m = m_g + 4 * kg + r;
                        v2[t][r] = -INFINITY;
                        if (!n_ok || m >= n_t0 || !bin_ok) continue;
                        const double v = twoF_folded(sm.abc[4 * kg + r][t0 + t], sc[0] * (double)acc[t][0][r],
                                                     sc[1] * (double)acc[t][1][r], sc[2] * (double)acc[t][2][r],
                                                     sc[3] * (double)acc[t][3][r]);
                        if (p.twoF) sm.out[wave][4 * kg + r][lrow][t0 + t] = (float)v;
                        v2[t][r] = v;
                        const long long idx = (long long)m * p.n_tau + n;
                        if (v > fmx || (v == fmx && idx < imx)) {
                            fmx = v;
                            imx = idx;
                        }
                    }
                }
                if (fmx != -INFINITY) {
                    double sum = 0.0;
#pragma unroll
                    for (int t = 0; t < kSwNT; ++t)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (v2[t][r] != -INFINITY) sum += (double)__expf((float)(0.5 * (v2[t][r] - fmx)));
                    red = red_combine(red, Red{0.5 * fmx, sum, imx});
                }
            }
        }

        // the group's map cells of this wave's bins, 8 taus of one (bin,
        // row) at a time
        if (p.twoF && col_ok) {
            __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
            __builtin_amdgcn_wave_barrier();
            const int n0 = nb * kBlk;
            const int nt = min(kBlk, p.n_tau - n0);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int pr = lane + 64 * j;
                const int r = pr >> 4, bl = pr & 15;
                const int m = m_g + r, b = col_tile * 16 + bl;
                if (m < n_t0 && b < p.n_bins) {
                    float *dst = p.twoF + ((size_t)b * n_t0 + m) * p.n_tau + n0;
                    const float *src = sm.out[wave][r][bl];
                    if (nt == kBlk) {
#pragma unroll
                        for (int t = 0; t < kBlk; ++t) dst[t] = src[t];
                    } else {
                        for (int t = 0; t < nt; ++t) dst[t] = src[t];
                    }
                }
            }
        }
    }

    // lanes sharing a bin: xor 16, 32; each wave owns its bins' partials
    red = red_combine(red, red_shfl_xor(red, 16));
    red = red_combine(red, red_shfl_xor(red, 32));
    if (col_ok && lane < 16 && bin_ok) {
        Partial &o = p.part[(size_t)bin * p.n_tiles + tile];
        o.fmax = red.f;
        o.s = red.s;
        o.idx = red.i;
    }
}

#ifndef TFS_ROWS_WAVES
#define TFS_ROWS_WAVES 2       // waves per SIMD the register budget targets
#endif
#ifndef TFS_CELLS_WAVES
#define TFS_CELLS_WAVES 3      // the same for the transposed form's kernels
#endif

// Work item of launch block bid of a map, in an XCD-aware order: column
// items dealt to the XCDs when there are at least 8 of them, one per XCD
// when there are 2 or 4, otherwise the units (tau blocks, or groups of them
// in the transposed form) as the units of unit_decode.  False: no item.
__device__ inline bool rows_task(const ExpMfmaRowsParams &p, int bid, int &q, int &row_tile, int &col_item) {
    const int xcd = bid & 7;
    const int slot = bid >> 3;
    const int n_col = mfma_col_items(p.n_col_tiles, p.n_bins);
    const int n_units = mfma_units(p.n_blocks, p.n_col_tiles);
    if (n_col >= 8) {
        const int cpx = (n_col + 7) / 8;
        const int per_block = p.n_row_tiles * cpx;
        q = slot / per_block;
        const int rem = slot % per_block;
        row_tile = rem / cpx;
        col_item = (rem % cpx) * 8 + xcd;
        return q < n_units && col_item < n_col;
    }
    if (n_col == 2 || n_col == 4) {
        // each XCD one column item (its share of the data planes stays in
        // the XCD's L2) and every (8 / n_col)-th unit
        const int r = 8 / n_col;
        col_item = xcd % n_col;
        q = (slot / p.n_row_tiles) * r + xcd / n_col;
        row_tile = slot % p.n_row_tiles;
        return q < n_units;
    }
    int rem;
    unit_decode(bid, n_units, p.n_row_tiles * n_col, q, rem);
    row_tile = rem / n_col;
    col_item = rem % n_col;
    return q < n_units;
}

// Maps of kSwMinColTiles or more column tiles (the shared-weight item).
template <bool F16>
__global__ __launch_bounds__(256, TFS_ROWS_WAVES) void exp_mfma_rows_kernel(ExpMfmaRowsParams p) {
    __shared__ SwSmem sm;
    int q, row_tile, col_item;
    if (rows_task(p, blockIdx.x, q, row_tile, col_item)) mfma_rows_tile_sw<F16>(p, sm, q, row_tile, col_item);
}

// Maps of fewer column tiles (the transposed item).
template <bool F16>
__global__ __launch_bounds__(256, TFS_CELLS_WAVES) void exp_mfma_cells_kernel(ExpMfmaRowsParams p) {
    __shared__ CellsSmem sm;
    int q, row_tile, col_item;
    if (rows_task(p, blockIdx.x, q, row_tile, col_item)) mfma_cells_tile<F16>(p, sm, q, row_tile, col_item);
}

// Matrix-core work items of many maps (one entry per workgroup): the
// transposed form's entries [0, n_cells), the others after them.
template <bool F16>
__global__ __launch_bounds__(256, TFS_CELLS_WAVES) void mfma_cells_batch_kernel(MfmaBatchParams b) {
    __shared__ CellsSmem sm;
    const int32_t *en = b.entries + 4 * (size_t)blockIdx.x;
    mfma_cells_tile<F16>(*reinterpret_cast<const __attribute__((address_space(4))) ExpMfmaRowsParams *>(
                             reinterpret_cast<uintptr_t>(b.jobs + en[0])),
                         sm, en[1], en[2], en[3]);
}

template <bool F16>
__global__ __launch_bounds__(256, TFS_ROWS_WAVES) void mfma_batch_kernel(MfmaBatchParams b) {
    __shared__ SwSmem sm;
    const int32_t *en = b.entries + 4 * ((size_t)b.n_cells + blockIdx.x);
    mfma_rows_tile_sw<F16>(*reinterpret_cast<const __attribute__((address_space(4))) ExpMfmaRowsParams *>(
                               reinterpret_cast<uintptr_t>(b.jobs + en[0])),
                           sm, en[1], en[2], en[3]);
}

// Per data column (component c, bin) of the FP32 atoms x32 [K+1][bins][4],
// the power of two e with max_k |x| * 2^e in [2^13, 2^14) (0 for an
// all-zero column), so that the half-precision hi parts stay below the
// format's largest value and the lo parts of all but tiny entries stay
// normal; colexp is [4][bins16].
__global__ __launch_bounds__(256) void col_exp_kernel(const float *x32, int32_t K, int32_t n_bins,
                                                      int32_t bins16, int32_t *colexp) {
    const int col = blockIdx.x * 256 + threadIdx.x;   // bin * 4 + c
    if (col >= 4 * bins16) return;
    const int bin = col >> 2, c = col & 3;
    float mx = 0.f;
    if (bin < n_bins)
        for (int32_t k = 0; k < K; ++k) mx = fmaxf(mx, fabsf(x32[(size_t)k * n_bins * 4 + col]));
    int e = 0;
    if (mx > 0.f) {
        int ex;
        (void)frexpf(mx, &ex);   // mx in [2^(ex-1), 2^ex)
        e = 14 - ex;
    }
    colexp[c * bins16 + bin] = e;
}

// hi / lo planes from the FP32 atoms x32 [K+1][bins][4], laid out
// [4 components][kp / 32 steps][bins16][32 slots]: the B operand of one K
// step for 16 bins is one contiguous kilobyte.  bf16 (round to nearest
// even), or half precision of x * 2^colexp (exact scaling).
template <bool F16>
__global__ __launch_bounds__(256) void build_planes_kernel(const float *x32, int32_t K, int32_t n_bins,
                                                           int32_t bins16, int32_t kp, const int32_t *colexp,
                                                           unsigned short *xhi, unsigned short *xlo) {
    const int64_t total = (int64_t)4 * bins16 * kp;
    const int64_t per_c = (int64_t)bins16 * kp;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const int c = (int)(i / per_c);
        const int64_t r = i - c * per_c;
        const int64_t step = r / ((int64_t)bins16 * 32);
        const int64_t r2 = r - step * bins16 * 32;
        const int bin = (int)(r2 / 32);
        const int64_t k = step * 32 + (r2 % 32);
        float x = 0.f;
        if (k < K && bin < n_bins) x = x32[((size_t)k * n_bins + bin) * 4 + c];
        if constexpr (F16) {
#pragma clang fp contract(off)
            x = ldexpf(x, colexp[c * bins16 + bin]);
            const _Float16 h = (_Float16)x;
            const _Float16 l = (_Float16)(x - (float)h);
            xhi[i] = __builtin_bit_cast(unsigned short, h);
            xlo[i] = __builtin_bit_cast(unsigned short, l);
        } else {
            const unsigned int pk = split_pack(x);
            xhi[i] = (unsigned short)(pk & 0xffffu);
            xlo[i] = (unsigned short)(pk >> 16);
        }
    }
}

// Column planes of the transposed form: the parts build_planes_kernel
// makes, laid out [copy kCellsCopies][4 components][n_bins][kpc] with slot
// k of copy r at element k + 16 - r (zero outside [0, K)).
template <bool F16>
__global__ __launch_bounds__(256) void build_cplanes_kernel(const float *x32, int32_t K, int32_t n_bins,
                                                            int32_t bins16, int32_t kpc, const int32_t *colexp,
                                                            unsigned short *chi, unsigned short *clo) {
    const int64_t per_c = (int64_t)n_bins * kpc;
    const int64_t per_copy = 4 * per_c;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < kCellsCopies * per_copy;
         i += (int64_t)gridDim.x * 256) {
        const int cp = (int)(i / per_copy);
        const int64_t r = i - cp * per_copy;
        const int c = (int)(r / per_c);
        const int64_t r2 = r - c * per_c;
        const int bin = (int)(r2 / kpc);
        const int64_t k = r2 - (int64_t)bin * kpc - 16 + cp;
        float x = 0.f;
        if (k >= 0 && k < K) x = x32[((size_t)k * n_bins + bin) * 4 + c];
        if constexpr (F16) {
#pragma clang fp contract(off)
            x = ldexpf(x, colexp[c * bins16 + bin]);
            const _Float16 h = (_Float16)x;
            const _Float16 l = (_Float16)(x - (float)h);
            chi[i] = __builtin_bit_cast(unsigned short, h);
            clo[i] = __builtin_bit_cast(unsigned short, l);
        } else {
            const unsigned int pk = split_pack(x);
            chi[i] = (unsigned short)(pk & 0xffffu);
            clo[i] = (unsigned short)(pk >> 16);
        }
    }
}

}  // namespace

hipError_t launch_build_cplanes(const float *x32, int32_t K, int32_t n_bins, int32_t bins16, int32_t kpc,
                                const int32_t *colexp, unsigned short *chi, unsigned short *clo, hipStream_t s) {
    const int64_t total = (int64_t)kCellsCopies * 4 * n_bins * kpc;
    int64_t g = (total + 255) / 256;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    if (colexp)
        hipLaunchKernelGGL(build_cplanes_kernel<true>, dim3((unsigned)g), dim3(256), 0, s, x32, K, n_bins, bins16,
                           kpc, colexp, chi, clo);
    else
        hipLaunchKernelGGL(build_cplanes_kernel<false>, dim3((unsigned)g), dim3(256), 0, s, x32, K, n_bins, bins16,
                           kpc, colexp, chi, clo);
    return hipGetLastError();
}

hipError_t launch_exp_mfma(const ExpMfmaParams &p, hipStream_t s) {
    if (p.n_blocks <= 0) return hipSuccess;
    if (p.kp < p.kp_data + 32) return hipErrorInvalidValue;   // even-step padding reads up to kp_data + 32
    unsigned grid;
    if (p.n_col_tiles >= 8) {
        const int cpx = (p.n_col_tiles + 7) / 8;
        grid = (unsigned)(8 * p.n_blocks * p.n_row_tiles * cpx);
    } else {
        grid = (unsigned)unit_grid(p.n_blocks, p.n_row_tiles * p.n_col_tiles);
    }
    hipLaunchKernelGGL(exp_mfma_kernel, dim3(grid), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_exp_mfma_rows(const ExpMfmaRowsParams &p, hipStream_t s) {
    if (p.n_blocks <= 0) return hipSuccess;
    if (p.kp < p.kp_data + 32) return hipErrorInvalidValue;   // even-step padding reads up to kp_data + 32
    const bool cells = mfma_cells_form(p.n_col_tiles);
    if (cells && (p.chi == nullptr || p.clo == nullptr || p.x32 == nullptr)) return hipErrorInvalidValue;
    unsigned grid;
    const int n_col = mfma_col_items(p.n_col_tiles, p.n_bins);
    const int n_units = mfma_units(p.n_blocks, p.n_col_tiles);
    if (n_col >= 8) {
        const int cpx = (n_col + 7) / 8;
        grid = (unsigned)(8 * n_units * p.n_row_tiles * cpx);
    } else if (n_col == 2 || n_col == 4) {
        const int r = 8 / n_col;
        grid = (unsigned)(8 * ((n_units + r - 1) / r) * p.n_row_tiles);
    } else {
        grid = (unsigned)unit_grid(n_units, p.n_row_tiles * n_col);
    }
    if (cells) {
        if (p.f16)
            hipLaunchKernelGGL(exp_mfma_cells_kernel<true>, dim3(grid), dim3(256), 0, s, p);
        else
            hipLaunchKernelGGL(exp_mfma_cells_kernel<false>, dim3(grid), dim3(256), 0, s, p);
    } else {
        if (p.f16)
            hipLaunchKernelGGL(exp_mfma_rows_kernel<true>, dim3(grid), dim3(256), 0, s, p);
        else
            hipLaunchKernelGGL(exp_mfma_rows_kernel<false>, dim3(grid), dim3(256), 0, s, p);
    }
    return hipGetLastError();
}

hipError_t launch_mfma_batch(const MfmaBatchParams &p, hipStream_t s) {
    if (p.n_entries <= 0) return hipSuccess;
    if (p.n_cells < 0 || p.n_cells > p.n_entries) return hipErrorInvalidValue;
    if (p.n_cells > 0) {
        if (p.f16)
            hipLaunchKernelGGL(mfma_cells_batch_kernel<true>, dim3((unsigned)p.n_cells), dim3(256), 0, s, p);
        else
            hipLaunchKernelGGL(mfma_cells_batch_kernel<false>, dim3((unsigned)p.n_cells), dim3(256), 0, s, p);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int n_rest = p.n_entries - p.n_cells;
    if (n_rest > 0) {
        if (p.f16)
            hipLaunchKernelGGL(mfma_batch_kernel<true>, dim3((unsigned)n_rest), dim3(256), 0, s, p);
        else
            hipLaunchKernelGGL(mfma_batch_kernel<false>, dim3((unsigned)n_rest), dim3(256), 0, s, p);
    }
    return hipGetLastError();
}

hipError_t launch_shift_tables(const ShiftTableParams &p, int64_t max_entries, hipStream_t s) {
    if (p.n_blocks <= 0) return hipSuccess;
    int64_t gx = (max_entries + 255) / 256;
    if (gx < 1) gx = 1;
    if (gx > 1024) gx = 1024;
    hipLaunchKernelGGL(shift_tables_kernel, dim3((unsigned)gx, (unsigned)p.n_blocks), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_build_planes(const float *x32, int32_t K, int32_t n_bins, int32_t bins16, int32_t kp,
                               int32_t *colexp, unsigned short *xhi, unsigned short *xlo, hipStream_t s) {
    const int64_t total = (int64_t)4 * bins16 * kp;
    int64_t g = (total + 255) / 256;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    if (colexp) {
        hipLaunchKernelGGL(col_exp_kernel, dim3((unsigned)((4 * bins16 + 255) / 256)), dim3(256), 0, s, x32, K,
                           n_bins, bins16, colexp);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(build_planes_kernel<true>, dim3((unsigned)g), dim3(256), 0, s, x32, K, n_bins, bins16,
                           kp, (const int32_t *)colexp, xhi, xlo);
    } else {
        hipLaunchKernelGGL(build_planes_kernel<false>, dim3((unsigned)g), dim3(256), 0, s, x32, K, n_bins,
                           bins16, kp, (const int32_t *)nullptr, xhi, xlo);
    }
    return hipGetLastError();
}

}  // namespace tfs
