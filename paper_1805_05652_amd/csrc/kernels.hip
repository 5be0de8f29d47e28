// HIP kernels of the transient F-statistic map for gfx950 (MI355X).
//
// Method: Keitel & Ashton, arXiv:1805.05652, section 2 (windows eq. winrect
// and eq. winexp, F from windowed atom sums eq. F_FaFb, the map eq. Fmn) and
// section 3 (running-sum reuse for rectangular windows, per-cell sums for
// exponential windows, D and F evaluated in the kernel).  The marginalised
// Bayes factor (appendix A footnote) is reduced from per-tile partials.
//
// Layout of resident atoms (slot grid, zero-filled gaps, row K all zeros):
//   abc [K+1][4]          FP64 a^2, b^2, ab, 0
//   x64 [K+1][bins][4]    FP64 Re Fa, Im Fa, Re Fb, Im Fb
//   x32 [K+1][bins][4]    FP32 copy of x64
#include "tfstat_device.h"

#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <stdint.h>

namespace tfs {

namespace {

constexpr int kLanes = 64;
constexpr int kWaves = 4;
constexpr int kThreads = kLanes * kWaves;
#ifndef TFS_KDC
#define TFS_KDC 256
#endif
constexpr int kDC = TFS_KDC;      // band slots staged per round (at most)
constexpr int kMinDC = kExpMinStageRound;   // fewest band slots per round worth staging

// Slots one LDS stage holds (exp_stage_len): a 64-row tile whose rows span
// `spread` slots stages spread + dn slots per round, dn = min(kDC, stage -
// spread) >= kMinDC.  The FP32 one-bin shape keeps 4 workgroups per CU
// (40 KB of LDS each) with a 1008-slot stage.
template <typename XT, int BG>
constexpr int stage_len() {
    return exp_stage_len(sizeof(XT) == 8 ? 0 : 1, BG);
}

// ---------------------------------------------------------------------------
// Reduction state: (F max, sum exp(F - fmax), first index of the max).
// ---------------------------------------------------------------------------
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

// Adds one cell (F = 2F / 2 and its linear index) to a lane's running
// state: one exponential per cell, FP32 arguments (exp(F - fmax) <= 1).
__device__ inline void red_add(Red &r, double F, long long idx) {
    if (F > r.f) {
        r.s = (r.f == -INFINITY) ? 1.0 : r.s * (double)__expf((float)(r.f - F)) + 1.0;
        r.f = F;
        r.i = idx;
    } else {
        r.s += (double)__expf((float)(F - r.f));
        if (F == r.f && idx < r.i) r.i = idx;
    }
}

// Wave reduction: the maximum and its first index by butterfly, then every
// lane's sum rescaled to that maximum (one exponential per lane; FP32
// argument unless EXACT) and added by butterfly; lane 0's result is used.
template <bool EXACT = false>
__device__ inline Red red_wave(Red v) {
    double fm = v.f;
    long long im = v.i;
#pragma unroll
    for (int o = 1; o < kLanes; o <<= 1) {
        const double fo = __shfl_xor(fm, o, kLanes);
        const long long io = __shfl_xor(im, o, kLanes);
        if (fo > fm || (fo == fm && io < im)) {
            fm = fo;
            im = io;
        }
    }
    if (fm == -INFINITY) return red_empty();
    const double e = EXACT ? exp(v.f - fm) : (double)__expf((float)(v.f - fm));
    double sv = (v.f == -INFINITY) ? 0.0 : v.s * e;
#pragma unroll
    for (int o = 1; o < kLanes; o <<= 1) sv += __shfl_xor(sv, o, kLanes);
    return Red{fm, sv, im};
}

// 2F of one cell from windowed sums (eq. F_FaFb), FP64, with the
// degenerate-window rule.
__device__ inline double twoF_cell(double A, double B, double C, double far_,
                                   double fai, double fbr, double fbi) {
    const double D = A * B - C * C;
    if (D <= kDegenerateRtol * A * B) return 0.0;
    const double num = B * (far_ * far_ + fai * fai) + A * (fbr * fbr + fbi * fbi)
                       - 2.0 * C * (far_ * fbr + fai * fbi);
    return 2.0 * (num / D);
}

template <typename T>
struct Q4 {
    T x, y, z, w;
};

__device__ inline Q4<float> load_q4(const float *p) {
    const float4 v = *reinterpret_cast<const float4 *>(p);
    return Q4<float>{v.x, v.y, v.z, v.w};
}
__device__ inline Q4<double> load_q4(const double *p) {
    const double2 a = *reinterpret_cast<const double2 *>(p);
    const double2 b = *reinterpret_cast<const double2 *>(p + 2);
    return Q4<double>{a.x, a.y, b.x, b.y};
}

// Data plane and weight table of the sum type XT; PP is the parameter block,
// possibly in the constant address space.
template <typename XT, typename PP>
__device__ inline const XT *xplane(PP &p) {
    if constexpr (sizeof(XT) == 4) return p.at.x32;
    else return p.at.x64;
}
template <typename XT, typename PP>
__device__ inline const XT *wplane(PP &p) {
    if constexpr (sizeof(XT) == 4) return p.g32;
    else return p.g64;
}

// A parameter block that the kernel never writes, read with scalar loads
// from the constant address space wherever a field is used.
template <typename T>
using ConstParams = const __attribute__((address_space(4))) T;

template <typename T>
__device__ inline ConstParams<T> &const_params(const T *p) {
    return *reinterpret_cast<ConstParams<T> *>(reinterpret_cast<uintptr_t>(p));
}

// ---------------------------------------------------------------------------
// Exponential-window sums and finalize, VALU form.
//
// Workgroup = one (64-row t0 tile, R-column tau block) task.  Lane l owns
// row m = tile*64 + l; the R taus of the block share every atom the lane
// loads.  Window weights w = exp(-(delta_m + d T)/tau_n) factor into a
// per-row scale s = exp(-delta_m/tau) and a table g_n[d] = exp(-d T/tau_n)
// that is uniform across the wave (scalar loads).  The band d is split into
// four contiguous quarters per staged chunk, one per wave, and the four
// partial sums are combined through LDS in a fixed order.
// ---------------------------------------------------------------------------
template <typename XT, int R, int BG>
struct ExpSmem {
    union {
        struct {
            double a2[stage_len<XT, BG>()];
            double b2[stage_len<XT, BG>()];
            double ab[stage_len<XT, BG>()];
            Q4<XT> x[BG][stage_len<XT, BG>()];
        } stage;
        struct {
            double abc[1][R][3][kLanes];
            XT f[1][R][BG][4][kLanes];
        } comb;
    } u;
    Red wred[kWaves][BG];
};

// What an exponential tile sums: everything, A/B/C only (FP64, for the
// matrix-core form), or F_a/F_b only (A/B/C read from abc_out).
constexpr int kModeAll = 0;
constexpr int kModeAbc = 1;
constexpr int kModeF = 2;

template <typename XT, int R, int BG, int MODE = kModeAll>
struct ExpAcc {
    double A[R], B[R], C[R];
    XT f[R][BG][4];

    __device__ inline void zero() {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            A[r] = 0.0; B[r] = 0.0; C[r] = 0.0;
#pragma unroll
            for (int b = 0; b < BG; ++b)
#pragma unroll
                for (int c = 0; c < 4; ++c) f[r][b][c] = XT(0);
        }
    }

    __device__ inline void step(const XT *__restrict__ gw, const double *__restrict__ gq,
                                double a2, double b2, double ab, const Q4<XT> *x) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if constexpr (MODE != kModeF) {
                const double q = gq[r];
                A[r] = fma(q, a2, A[r]);
                B[r] = fma(q, b2, B[r]);
                C[r] = fma(q, ab, C[r]);
            }
            if constexpr (MODE == kModeAbc) continue;
            const XT g = gw[r];
#pragma unroll
            for (int b = 0; b < BG; ++b) {
                f[r][b][0] = fma(g, x[b].x, f[r][b][0]);
                f[r][b][1] = fma(g, x[b].y, f[r][b][1]);
                f[r][b][2] = fma(g, x[b].z, f[r][b][2]);
                f[r][b][3] = fma(g, x[b].w, f[r][b][3]);
            }
        }
    }

    template <typename SM>
    __device__ inline void store(SM &sm, int j, int lane) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if constexpr (MODE != kModeF) {
                sm.u.comb.abc[j][r][0][lane] = A[r];
                sm.u.comb.abc[j][r][1][lane] = B[r];
                sm.u.comb.abc[j][r][2][lane] = C[r];
            }
            if constexpr (MODE == kModeAbc) continue;
#pragma unroll
            for (int b = 0; b < BG; ++b)
#pragma unroll
                for (int c = 0; c < 4; ++c) sm.u.comb.f[j][r][b][c][lane] = f[r][b][c];
        }
    }

    template <typename SM>
    __device__ inline void add(const SM &sm, int j, int lane) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if constexpr (MODE != kModeF) {
                A[r] += sm.u.comb.abc[j][r][0][lane];
                B[r] += sm.u.comb.abc[j][r][1][lane];
                C[r] += sm.u.comb.abc[j][r][2][lane];
            }
            if constexpr (MODE == kModeAbc) continue;
#pragma unroll
            for (int b = 0; b < BG; ++b)
#pragma unroll
                for (int c = 0; c < 4; ++c) f[r][b][c] += sm.u.comb.f[j][r][b][c][lane];
        }
    }
};

// s_waitcnt operand (gfx9 encoding) that waits for LDS / scalar memory only:
// vmcnt 63, expcnt 7, lgkmcnt 0
constexpr int kWaitLgkm0 = 0xC07F;

// Operands of one band step of the staged form: the R weights and squared
// weights of slot offset d (uniform: scalar registers) and the lane's atoms.
template <typename XT, int R, int BG>
struct StepOps {
    XT w[R];
    double q[R];
    double a2, b2, ab;
    Q4<XT> x[BG];
};

// The weight tables are read through the constant address space: the
// explicit waits of the pipelined loops would otherwise keep the compiler
// from proving them unwritten, and it would load them into vector registers.
template <typename T>
__device__ inline ConstParams<T> *const_ptr(const T *p) {
    return reinterpret_cast<ConstParams<T> *>(reinterpret_cast<uintptr_t>(p));
}

template <int MODE, typename SM, typename XT, int R, int BG>
__device__ __attribute__((always_inline)) inline void fetch_step(const SM &sm, const XT *__restrict__ gw_base,
                                                                 const double *__restrict__ gq_base, int my,
                                                                 int d0, int dd, StepOps<XT, R, BG> &o) {
    const int li = my + dd;
    const size_t d = (size_t)(d0 + dd);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        o.w[r] = gw_base[d * R + r];
        o.q[r] = gq_base[d * R + r];
    }
    if constexpr (MODE != kModeF) {
        o.a2 = sm.u.stage.a2[li];
        o.b2 = sm.u.stage.b2[li];
        o.ab = sm.u.stage.ab[li];
    }
    if constexpr (MODE != kModeAbc) {
#pragma unroll
        for (int b = 0; b < BG; ++b) o.x[b] = sm.u.stage.x[b][li];
    }
}

// Shapes whose staged band loop is software-pipelined: bit 1 FP64, 2 FP32
// R = 8, 4 FP32 R = 4 BG = 2, 8 FP32 R = 4 BG = 4, 16 A/B/C only, 32 F
// only, 64 FP32 R = 4 BG = 1.  The four-bin shape and the A/B/C pass have the registers for a
// second operand set at their occupancy (measured: the four-bin shape
// faster in the fused batch kernel and about even alone, the A/B/C pass a
// third faster); this set is fetched with vector loads (weights included).
#ifndef TFS_PIPE_MASK
#define TFS_PIPE_MASK 24
#endif
template <typename XT, int R, int BG, int MODE>
constexpr int exp_shape_bit() {
    return MODE == kModeAbc ? 16 : MODE == kModeF ? 32 : sizeof(XT) == 8 ? 1 : R == 8 ? 2 : BG == 1 ? 64 : BG == 2 ? 4 : 8;
}
template <typename XT, int R, int BG, int MODE>
constexpr bool exp_pipe() {
    return (TFS_PIPE_MASK & exp_shape_bit<XT, R, BG, MODE>()) != 0;
}
// Shapes (same bits) whose weights alone are fetched one step ahead, into
// scalar registers: no vector registers beyond the unpipelined loop, which
// waits for each step's scalar loads together with its LDS reads.  Measured:
// the one-bin FP32 map 7% faster, FP64 even, the batch 1% faster; the F-only
// and four-bin shapes slower in the fused batch kernel.
#ifndef TFS_SPIPE_MASK
#define TFS_SPIPE_MASK 71
#endif
template <typename XT, int R, int BG, int MODE>
constexpr bool exp_spipe() {
    return !exp_pipe<XT, R, BG, MODE>() && (TFS_SPIPE_MASK & exp_shape_bit<XT, R, BG, MODE>()) != 0;
}

// The weights of one band step (wave-uniform: scalar registers).
template <typename XT, int R>
struct StepW {
    XT w[R];
    double q[R];
};

template <int MODE, typename XT, int R>
__device__ __attribute__((always_inline)) inline void fetch_w(const XT *__restrict__ gw_base,
                                                              const double *__restrict__ gq_base, int d,
                                                              StepW<XT, R> &o) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if constexpr (MODE != kModeAbc) o.w[r] = const_ptr(gw_base)[(size_t)d * R + r];
        if constexpr (MODE != kModeF) o.q[r] = const_ptr(gq_base)[(size_t)d * R + r];
    }
}

// One (64-row tile, R-tau block, BG-bin group) task of the exponential map:
// q indexes p.blk_list.  Every thread of the workgroup calls it.
template <typename XT, int R, int BG, int MODE = kModeAll, typename PP>
__device__ __attribute__((always_inline)) inline void exp_tile(PP &p,
                                                               ExpSmem<XT, R, BG> &sm, int q,
                                                               int row_tile, int bin_group) {
    const int tid = threadIdx.x;
    const int lane = tid & (kLanes - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nb = p.blk_list[q];
    const int tile = nb * p.n_row_tiles + row_tile;
    const int bin0 = p.bin_base + bin_group * BG;
    const int n_bins = p.at.n_bins;
    const int K = p.at.K;

    const int m_first = row_tile * kLanes;
    const int m_last = min(m_first + kLanes - 1, p.n_t0 - 1);
    const bool row_ok = m_first + lane < p.n_t0;
    const int m = min(m_first + lane, p.n_t0 - 1);
    const RowPlan rp = p.rows[m];
    const int k_lo = p.rows[m_first].k0;
    const int k_hi = p.rows[m_last].k0;
    const int spread = k_hi - k_lo;
    const int lblk = p.lblk[nb];
    const int dwg = min(lblk, K - k_lo);
    const int64_t off = p.blk_off[nb];
    const XT *__restrict__ gw_base = wplane<XT>(p) + off;
    const double *__restrict__ gq_base = p.gsq + off;
    const XT *__restrict__ xg = xplane<XT>(p);
    const double *__restrict__ abc = p.at.abc;

    ExpAcc<XT, R, BG, MODE> acc;
    acc.zero();

    constexpr int kStageLen = stage_len<XT, BG>();
    if (spread <= kStageLen - kMinDC) {
        const int my = rp.k0 - k_lo;
        const int dc = min(kDC, kStageLen - spread);
        for (int d0 = 0; d0 < dwg; d0 += dc) {
            const int dn = min(dc, dwg - d0);
            const int width = spread + dn;
            __syncthreads();
            for (int i = tid; i < width; i += kThreads) {
                const int k = k_lo + d0 + i;
                const bool in = (unsigned)k < (unsigned)K;
                if constexpr (MODE != kModeF) {
                    double a2 = 0.0, b2 = 0.0, ab = 0.0;
                    if (in) {
                        const double2 v = *reinterpret_cast<const double2 *>(abc + (size_t)k * 4);
                        a2 = v.x;
                        b2 = v.y;
                        ab = abc[(size_t)k * 4 + 2];
                    }
                    sm.u.stage.a2[i] = a2;
                    sm.u.stage.b2[i] = b2;
                    sm.u.stage.ab[i] = ab;
                }
                if constexpr (MODE != kModeAbc) {
#pragma unroll
                    for (int b = 0; b < BG; ++b) {
                        Q4<XT> x{XT(0), XT(0), XT(0), XT(0)};
                        if (in && bin0 + b < n_bins)
                            x = load_q4(xg + ((size_t)k * n_bins + bin0 + b) * 4);
                        sm.u.stage.x[b][i] = x;
                    }
                }
            }
            __syncthreads();
            const int per = (dn + kWaves - 1) / kWaves;
            const int ds = wave * per;
            const int de = min(dn, ds + per);
            if constexpr (exp_pipe<XT, R, BG, MODE>()) {
                // Software pipeline: the operands of step dd + 1 (weights by
                // scalar loads, atoms from LDS) are fetched while the sums of
                // step dd run.  Scalar loads complete out of order, so the
                // wait for one step's operands is taken explicitly at the top
                // of each half-iteration, before the next step's fetch.
                if (ds < de) {
                    StepOps<XT, R, BG> a, b;
                    fetch_step<MODE>(sm, gw_base, gq_base, my, d0, ds, a);
                    int dd = ds;
#pragma unroll 1
                    for (; dd + 2 <= de; dd += 2) {
                        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
                        __builtin_amdgcn_sched_barrier(0);
                        fetch_step<MODE>(sm, gw_base, gq_base, my, d0, dd + 1, b);
                        __builtin_amdgcn_sched_barrier(0);
                        acc.step(a.w, a.q, a.a2, a.b2, a.ab, a.x);
                        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
                        __builtin_amdgcn_sched_barrier(0);
                        fetch_step<MODE>(sm, gw_base, gq_base, my, d0, min(dd + 2, de - 1), a);
                        __builtin_amdgcn_sched_barrier(0);
                        acc.step(b.w, b.q, b.a2, b.b2, b.ab, b.x);
                    }
                    if (dd < de) acc.step(a.w, a.q, a.a2, a.b2, a.ab, a.x);
                }
            } else if constexpr (exp_spipe<XT, R, BG, MODE>()) {
                // Weights one step ahead: the scalar loads of step dd + 1 are
                // issued once the LDS operands of step dd have landed (so the
                // wait for those never waits for scalar loads, which complete
                // out of order) and complete while the sums of step dd run.
                if (ds < de) {
                    StepW<XT, R> wa, wb;
                    fetch_w<MODE>(gw_base, gq_base, d0 + ds, wa);
// One step dd with the weights in CUR; the next step's (DN) go to NXT.
#define TFS_SPIPE_STEP(CUR, NXT, DD, DN)                                             \
    {                                                                                \
        const int li = my + (DD);                                                    \
        double a2 = 0.0, b2 = 0.0, ab = 0.0;                                         \
        Q4<XT> x[BG];                                                                \
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);                                      \
        __builtin_amdgcn_sched_barrier(0);                                           \
        if constexpr (MODE != kModeF) {                                              \
            a2 = sm.u.stage.a2[li];                                                  \
            b2 = sm.u.stage.b2[li];                                                  \
            ab = sm.u.stage.ab[li];                                                  \
        }                                                                            \
        if constexpr (MODE != kModeAbc) {                                            \
            _Pragma("unroll") for (int b = 0; b < BG; ++b) x[b] = sm.u.stage.x[b][li]; \
        }                                                                            \
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);                                      \
        __builtin_amdgcn_sched_barrier(0);                                           \
        fetch_w<MODE>(gw_base, gq_base, d0 + (DN), NXT);                             \
        __builtin_amdgcn_sched_barrier(0);                                           \
        acc.step(CUR.w, CUR.q, a2, b2, ab, x);                                       \
    }
                    int dd = ds;
#pragma unroll 1
                    for (; dd + 2 <= de; dd += 2) {
                        TFS_SPIPE_STEP(wa, wb, dd, dd + 1)
                        TFS_SPIPE_STEP(wb, wa, dd + 1, min(dd + 2, de - 1))
                    }
                    if (dd < de) TFS_SPIPE_STEP(wa, wb, dd, dd)
#undef TFS_SPIPE_STEP
                }
            } else {
                for (int dd = ds; dd < de; ++dd) {
                    const int li = my + dd;
                    Q4<XT> x[BG];
                    if constexpr (MODE != kModeAbc) {
#pragma unroll
                        for (int b = 0; b < BG; ++b) x[b] = sm.u.stage.x[b][li];
                    }
                    const int d = d0 + dd;
                    acc.step(gw_base + (size_t)d * R, gq_base + (size_t)d * R,
                             sm.u.stage.a2[li], sm.u.stage.b2[li], sm.u.stage.ab[li], x);
                }
            }
        }
    } else {
        // Rows too far apart to stage one band: each lane reads its own
        // slots through the caches, kU slots' loads in flight before their
        // sums (the order of the sums is unchanged).
        const int per = (max(dwg, 0) + kWaves - 1) / kWaves;
        const int ds = wave * per;
        const int de = min(dwg, ds + per);
        auto load_slot = [&](int d, double &a2, double &b2, double &ab, Q4<XT> *x) {
            const int k = rp.k0 + d;
            const int kk = ((unsigned)k < (unsigned)K) ? k : K;   // row K is zero
            const double2 v = *reinterpret_cast<const double2 *>(abc + (size_t)kk * 4);
            a2 = v.x;
            b2 = v.y;
            ab = abc[(size_t)kk * 4 + 2];
            if constexpr (MODE != kModeAbc) {
#pragma unroll
                for (int b = 0; b < BG; ++b)
                    x[b] = (bin0 + b < n_bins) ? load_q4(xg + ((size_t)kk * n_bins + bin0 + b) * 4)
                                               : Q4<XT>{XT(0), XT(0), XT(0), XT(0)};
            }
        };
        constexpr int kU = (BG == 1 && sizeof(XT) == 4) ? 4 : 2;
        int d = ds;
        for (; d + kU <= de; d += kU) {
            double a2[kU], b2[kU], ab[kU];
            Q4<XT> x[kU][BG];
#pragma unroll
            for (int u = 0; u < kU; ++u) load_slot(d + u, a2[u], b2[u], ab[u], x[u]);
#pragma unroll
            for (int u = 0; u < kU; ++u)
                acc.step(gw_base + (size_t)(d + u) * R, gq_base + (size_t)(d + u) * R, a2[u], b2[u], ab[u], x[u]);
        }
        for (; d < de; ++d) {
            double a2, b2, ab;
            Q4<XT> x[BG];
            load_slot(d, a2, b2, ab, x);
            acc.step(gw_base + (size_t)d * R, gq_base + (size_t)d * R, a2, b2, ab, x);
        }
    }

    // Combine the four waves' partial sums as (((w3 + w2) + w1) + w0) through
    // one LDS slot; the total is left in that slot.
    __syncthreads();
    if (wave == kWaves - 1) acc.store(sm, 0, lane);
#pragma unroll 1
    for (int w = kWaves - 2; w >= 0; --w) {
        __syncthreads();
        if (wave == w) {
            acc.add(sm, 0, lane);
            acc.store(sm, 0, lane);
        }
    }
    __syncthreads();

    // Finalize, one tau column per wave at a time: exact band end, row
    // scale, D, 2F, map, reductions.
    const int64_t T = p.at.t_sft;
    Red red[BG];
#pragma unroll
    for (int b = 0; b < BG; ++b) red[b] = red_empty();
#pragma unroll 1
    for (int r = wave; r < R; r += kWaves) {
        const int n = nb * R + r;
        const bool ok = row_ok && n < p.n_tau;
        const int nn = min(n, p.n_tau - 1);
        const int64_t tau = p.tau[nn];
        const int64_t span = 3 * tau;
        const int64_t lmn = span > rp.delta ? (span - rp.delta + T - 1) / T : 0;
        const int lc = p.lcol[nn];
        double A = 0.0, B = 0.0, C = 0.0;
        if constexpr (MODE != kModeF) {
            A = sm.u.comb.abc[0][r][0][lane];
            B = sm.u.comb.abc[0][r][1][lane];
            C = sm.u.comb.abc[0][r][2][lane];
        }
        double f[BG][4];
#pragma unroll
        for (int b = 0; b < BG; ++b)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                f[b][c] = MODE == kModeAbc ? 0.0 : (double)sm.u.comb.f[0][r][b][c][lane];
        // The table holds the shortest band over all rows of the grid; a row
        // whose band reaches further (smaller delta) adds its last terms
        // here, in FP64, with weights exp(-d T / tau).  (Shape windows have
        // one delta for all rows, hence no such terms.)
        const int64_t dend = p.scale_rows ? min(lmn, (int64_t)K - rp.k0) : 0;
        for (int64_t d = lc; d < dend; ++d) {
            const int64_t k = (int64_t)rp.k0 + d;
            if (k < 0) continue;
            const double gd = exp(-(double)(d * T) / (double)tau);
            if constexpr (MODE != kModeF) {
                const double qd = gd * gd;
                A += qd * abc[k * 4 + 0];
                B += qd * abc[k * 4 + 1];
                C += qd * abc[k * 4 + 2];
            }
#pragma unroll
            for (int b = 0; b < BG; ++b) {
                if (MODE == kModeAbc || bin0 + b >= n_bins) continue;
                const Q4<XT> x = load_q4(xg + ((size_t)k * n_bins + bin0 + b) * 4);
                f[b][0] += gd * (double)x.x;
                f[b][1] += gd * (double)x.y;
                f[b][2] += gd * (double)x.z;
                f[b][3] += gd * (double)x.w;
            }
        }
        if (p.scale_rows && rp.delta != 0) {
            const double s = exp(-(double)rp.delta / (double)tau);
            const double s2 = s * s;
            A *= s2; B *= s2; C *= s2;
#pragma unroll
            for (int b = 0; b < BG; ++b)
#pragma unroll
                for (int c = 0; c < 4; ++c) f[b][c] *= s;
        }
        if constexpr (MODE == kModeAbc) {
            if (ok) {
                double *o = p.abc_out + ((size_t)m * p.abc_pitch + n) * 3;
                o[0] = A;
                o[1] = B;
                o[2] = C;
            }
            continue;
        }
        if constexpr (MODE == kModeF) {
            // A, B, C of the cell (scaled, exact band) from the A/B/C-only pass
            const double *o = p.abc_out + ((size_t)m * p.abc_pitch + nn) * 3;
            A = o[0];
            B = o[1];
            C = o[2];
        }
#pragma unroll
        for (int b = 0; b < BG; ++b) {
            const int bin = bin0 + b;
            if (!ok || bin >= n_bins) continue;
            const double v = twoF_cell(A, B, C, f[b][0], f[b][1], f[b][2], f[b][3]);
            if (p.twoF) p.twoF[((size_t)bin * p.n_t0 + m) * p.n_tau + n] = (float)v;
            red_add(red[b], 0.5 * v, (long long)m * p.n_tau + n);
        }
    }
    if constexpr (MODE == kModeAbc) return;
#pragma unroll
    for (int b = 0; b < BG; ++b) {
        const Red w = red_wave(red[b]);
        if (lane == 0) sm.wred[wave][b] = w;
    }
    __syncthreads();
    if (tid < BG && bin0 + tid < n_bins) {
        Red t = sm.wred[0][tid];
        for (int w = 1; w < kWaves; ++w) t = red_combine(t, sm.wred[w][tid]);
        Partial &o = p.part[(size_t)(bin0 + tid) * p.n_tiles + tile];
        o.fmax = t.f;
        o.s = t.s;
        o.idx = t.i;
    }
}

// Waves per SIMD each exponential tile shape is built for.
template <typename XT, int R, int BG, int MODE>
constexpr int exp_waves() {
    return MODE == kModeAbc ? 5
           : MODE == kModeF ? 3
           : (sizeof(XT) == 8 ? 5 : (R == 8 ? 4 : (BG == 4 ? 3 : 5)));
}

template <typename XT, int R, int BG, int MODE = kModeAll>
__global__ __launch_bounds__(kThreads, (exp_waves<XT, R, BG, MODE>())) void exp_valu_kernel(ExpValuParams p) {
    __shared__ ExpSmem<XT, R, BG> sm;
    // XCD-aware task order (unit_decode): blocks of tau (sorted largest band
    // first), each with its row tiles, so a block's weight table is fetched
    // into one L2 only
    int q, row_tile;
    unit_decode(blockIdx.x, p.n_list, p.n_row_tiles, q, row_tile);
    if (q >= p.n_list) return;
    exp_tile<XT, R, BG, MODE>(p, sm, q, row_tile, blockIdx.y);
}

// ---------------------------------------------------------------------------
// Exponential-window sums for t0 rows far apart in slot space ("runs" form).
//
// When the 64 rows of a tile start many slots apart, the union of their
// bands is far wider than one LDS stage, and each staged slot feeds only a
// few rows.  Here each row gets its own run of kG consecutive slots per
// round, loaded with coalesced reads into LDS, and the four waves of the
// workgroup sum four different tau blocks (R taus each, blk_list positions
// q0 .. q0 + 3) over the same runs, so that every staged slot feeds 4R taus
// of its row.  The loads of the next round are in flight while the current
// round is summed.  Each wave sums the whole band of its block (the other
// form splits it over the four waves) and finalizes the block alone.
// ---------------------------------------------------------------------------
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// G: slots per run and round.  The stand-alone kernel stages 8 (fewer
// barriers per sum); the persistent kernel 4 (fewer prefetch registers
// beside its other tile shapes).  The order of the sums does not depend on
// it.
template <typename XT, int BG, int G>
struct RunCfg {
    static constexpr int kCpb = (int)sizeof(XT) / 4;        // 16-byte chunks per bin and slot
    static constexpr int kNC = 2 + BG * kCpb;               // chunk arrays: (a2, b2), (ab, 0), data
    static constexpr int kG = G;                            // slots per run and round
    static constexpr int kSh = G == 8 ? 1 : 2;              // LDS swizzle: rows per rotation step
    static constexpr int kPer = kLanes * kG * kNC / kThreads;   // chunks each thread loads per round
    static_assert(kLanes * kG * kNC % kThreads == 0, "whole chunks per thread");
    static_assert(kThreads % kG == 0, "a thread keeps its slot within the run");
};

// One round: the runs (16-byte chunks) of the round's kG slots and, unless
// SW, each wave's weights g[d][r], g^2[d][r] for them.  The weights are
// wave-uniform: with SW they come from scalar loads one step ahead instead
// (no LDS reads for them; the scalar registers limit the one-bin shape).
template <typename XT, int R, int BG, int G, bool SW>
struct RunSmem {
    u32x4 c[RunCfg<XT, BG, G>::kNC][kLanes * G];
    XT g[SW ? 1 : kWaves][G][R] __attribute__((aligned(16)));
    double q[SW ? 1 : kWaves][G][R] __attribute__((aligned(16)));
};

// Element of row r, slot j of a run: rows of kG elements, rotated by r >> kSh
// so that the 16 lanes of a quarter wave reading one slot hit 16 distinct
// 16-byte bank groups.
template <typename XT, int BG, int G>
__device__ inline int run_index(int r, int j) {
    using C = RunCfg<XT, BG, G>;
    return r * C::kG + ((j + (r >> C::kSh)) & (C::kG - 1));
}

template <typename XT, int R, int BG, int G, bool SW, typename PP>
__device__ __attribute__((always_inline)) inline void exp_runs_tile(PP &p, RunSmem<XT, R, BG, G, SW> &sm, int q0,
                                                                    int row_tile, int bin_group) {
    using C = RunCfg<XT, BG, G>;
    const int tid = threadIdx.x;
    const int lane = tid & (kLanes - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int bin0 = p.bin_base + bin_group * BG;
    const int n_bins = p.at.n_bins;
    const int K = p.at.K;
    const int m_first = row_tile * kLanes;
    const int k_lo = p.rows[m_first].k0;

    // this wave's block; the workgroup's band is the longest of its blocks
    const int q = q0 + wave;
    const bool has_blk = q < p.n_list;
    const int nb = has_blk ? p.blk_list[q] : p.blk_list[q0];
    const int kmax = K - k_lo;
    const int dw = has_blk ? max(min(p.lblk[nb], kmax), 0) : 0;
    int dall = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w)
        if (q0 + w < p.n_list) dall = max(dall, min(p.lblk[p.blk_list[q0 + w]], kmax));
    const int64_t off = p.blk_off[nb];
    const XT *__restrict__ gw_base = wplane<XT>(p) + off;
    const double *__restrict__ gq_base = p.gsq + off;
    const XT *__restrict__ xg = xplane<XT>(p);
    const double *__restrict__ abc = p.at.abc;

    // This thread always loads slot js of its runs, for row rr and, with
    // kG = 8, row rr + 32: chunk i of a round is array i / kRep, row
    // rr + (i % kRep) * (kThreads / kG).
    constexpr int kRep = kLanes * C::kG / kThreads;
    const int js = tid % C::kG;
    const int rr = tid / C::kG;
    int kr[kRep];
    int sidx[kRep];
#pragma unroll
    for (int h = 0; h < kRep; ++h) {
        const int r = rr + h * (kThreads / C::kG);
        kr[h] = p.rows[min(m_first + r, p.n_t0 - 1)].k0 + js;
        sidx[h] = run_index<XT, BG, G>(r, js);
    }
    u32x4 buf[C::kPer];
    // chunk sources of one round: slot k of array a (k outside the data
    // reads row K, which is zero)
#define TFS_RUNS_LOAD(D0)                                                                       \
    _Pragma("unroll") for (int i = 0; i < C::kPer; ++i) {                                       \
        const int a = i / kRep;                                                                 \
        int k = kr[i % kRep] + (D0);                                                            \
        if ((unsigned)k >= (unsigned)K) k = K;                                                  \
        if (a < 2) {                                                                            \
            buf[i] = *reinterpret_cast<const u32x4 *>(abc + (size_t)k * 4 + 2 * a);            \
        } else {                                                                                \
            const int b = (a - 2) / C::kCpb;                                                    \
            const bool bin_ok = bin0 + b < n_bins;                                              \
            const size_t e = ((size_t)(bin_ok ? k : K) * n_bins + (bin_ok ? bin0 + b : 0)) * 4; \
            buf[i] = reinterpret_cast<const u32x4 *>(xg + e)[(a - 2) % C::kCpb];                \
        }                                                                                       \
    }

    // Without SW, the wave's weights of one round: lane l < kWc copies one
    // 16-byte chunk of rows d0 .. d0 + kG - 1 of its block's tables (rows
    // past the band repeat the last one; a wave without rows copies the zero
    // atom row).
    constexpr int kCg = R * (int)sizeof(XT) / 16;    // chunks per g row
    constexpr int kCq = R * 8 / 16;                  // chunks per g^2 row
    constexpr int kWc = C::kG * (kCg + kCq);
    static_assert(kWc <= kLanes && R * sizeof(XT) % 16 == 0, "one weight chunk per lane");
    const int lb = has_blk ? p.lblk[nb] : 0;
    const bool wl = !SW && lane < kWc;
    const int wj = lane < C::kG * kCg ? lane / kCg : (lane - C::kG * kCg) / kCq;
    const int wc = lane < C::kG * kCg ? lane % kCg : (lane - C::kG * kCg) % kCq;
    u32x4 *const wdst = lane < C::kG * kCg ? reinterpret_cast<u32x4 *>(&sm.g[SW ? 0 : wave][wj][0]) + wc
                                           : reinterpret_cast<u32x4 *>(&sm.q[SW ? 0 : wave][wj][0]) + wc;
    u32x4 wbuf;
#define TFS_RUNS_WLOAD(D0)                                                                      \
    if constexpr (!SW) {                                                                        \
        const int d = min((D0) + wj, lb - 1);                                                   \
        const u32x4 *src = reinterpret_cast<const u32x4 *>(abc + (size_t)K * 4);               \
        if (wl && d >= 0)                                                                       \
            src = lane < C::kG * kCg ? reinterpret_cast<const u32x4 *>(gw_base + (size_t)d * R) + wc \
                                     : reinterpret_cast<const u32x4 *>(gq_base + (size_t)d * R) + wc; \
        wbuf = *src;                                                                            \
    }

    ExpAcc<XT, R, BG> acc;
    acc.zero();
    // With SW, the wave's weights of step d, one step ahead in scalar registers: the
    // scalar loads of the next step are issued once this step's LDS operands
    // have landed (both count on one counter; scalar loads complete out of
    // order) and complete while this step's sums run.  Waves without a block
    // run no steps and load no weights.
    StepW<XT, R> wa, wb;
    if (SW && dw > 0) fetch_w<kModeAll>(gw_base, gq_base, 0, wa);
    // step j of the round from d0 with the weights in CUR; those of step DN
    // (clamped into the band) go to NXT
#define TFS_RUNS_STEP(CUR, NXT, J, DN)                                                          \
    {                                                                                           \
        const int e = run_index<XT, BG, G>(lane, (J));                                          \
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);                                                 \
        __builtin_amdgcn_sched_barrier(0);                                                      \
        const double2 v = *reinterpret_cast<const double2 *>(&cur[0][e]);                       \
        const double ab = *reinterpret_cast<const double *>(&cur[1][e]);                        \
        Q4<XT> x[BG];                                                                           \
        _Pragma("unroll") for (int b = 0; b < BG; ++b) {                                        \
            if constexpr (sizeof(XT) == 4) {                                                    \
                const u32x4 u = cur[2 + b][e];                                                  \
                x[b] = Q4<XT>{__uint_as_float(u.x), __uint_as_float(u.y), __uint_as_float(u.z), \
                              __uint_as_float(u.w)};                                            \
            } else {                                                                            \
                const double2 lo = *reinterpret_cast<const double2 *>(&cur[2 + 2 * b][e]);      \
                const double2 hi = *reinterpret_cast<const double2 *>(&cur[3 + 2 * b][e]);      \
                x[b] = Q4<XT>{lo.x, lo.y, hi.x, hi.y};                                          \
            }                                                                                   \
        }                                                                                       \
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);                                                 \
        __builtin_amdgcn_sched_barrier(0);                                                      \
        fetch_w<kModeAll>(gw_base, gq_base, min((DN), dw - 1), NXT);                            \
        __builtin_amdgcn_sched_barrier(0);                                                      \
        acc.step(CUR.w, CUR.q, v.x, v.y, ab, x);                                                \
    }
    TFS_RUNS_LOAD(0)
    TFS_RUNS_WLOAD(0)
#pragma unroll 1
    for (int d0 = 0; d0 < dall; d0 += C::kG) {
        __syncthreads();   // every wave is done with the previous round
        auto &cur = sm.c;
#pragma unroll
        for (int i = 0; i < C::kPer; ++i) cur[i / kRep][sidx[i % kRep]] = buf[i];
        if (wl) *wdst = wbuf;
        __syncthreads();
        // next round (past the band this reads zero rows or unused slots;
        // an unconditional load keeps buf in registers)
        TFS_RUNS_LOAD(d0 + C::kG)
        TFS_RUNS_WLOAD(d0 + C::kG)
        const int jn = min(C::kG, dw - d0);
        if constexpr (!SW) {
            // every operand from LDS (in-order completion lets the loads of
            // one step overlap the products of the previous one)
#pragma unroll 2
            for (int j = 0; j < jn; ++j) {
                const int e = run_index<XT, BG, G>(lane, j);
                const double2 v = *reinterpret_cast<const double2 *>(&cur[0][e]);
                const double ab = *reinterpret_cast<const double *>(&cur[1][e]);
                Q4<XT> x[BG];
#pragma unroll
                for (int b = 0; b < BG; ++b) {
                    if constexpr (sizeof(XT) == 4) {
                        const u32x4 u = cur[2 + b][e];
                        x[b] = Q4<XT>{__uint_as_float(u.x), __uint_as_float(u.y), __uint_as_float(u.z),
                                      __uint_as_float(u.w)};
                    } else {
                        const double2 lo = *reinterpret_cast<const double2 *>(&cur[2 + 2 * b][e]);
                        const double2 hi = *reinterpret_cast<const double2 *>(&cur[3 + 2 * b][e]);
                        x[b] = Q4<XT>{lo.x, lo.y, hi.x, hi.y};
                    }
                }
                acc.step(&sm.g[SW ? 0 : wave][j][0], &sm.q[SW ? 0 : wave][j][0], v.x, v.y, ab, x);
            }
            continue;
        }
        int j = 0;
#pragma unroll 1
        for (; j + 2 <= jn; j += 2) {
            TFS_RUNS_STEP(wa, wb, j, d0 + j + 1)
            TFS_RUNS_STEP(wb, wa, j + 1, d0 + j + 2)
        }
        if (j < jn) {
            TFS_RUNS_STEP(wa, wb, j, d0 + j + 1)
            wa = wb;
        }
    }
#undef TFS_RUNS_STEP
#undef TFS_RUNS_LOAD
#undef TFS_RUNS_WLOAD
    if (!has_blk) return;

    // Finalize the wave's block: exact band end, row scale, D, 2F, map,
    // reductions (as in exp_tile).
    const bool row_ok = m_first + lane < p.n_t0;
    const int m = min(m_first + lane, p.n_t0 - 1);
    const RowPlan rp = p.rows[m];
    const int64_t T = p.at.t_sft;
    Red red[BG];
#pragma unroll
    for (int b = 0; b < BG; ++b) red[b] = red_empty();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int n = nb * R + r;
        const bool ok = row_ok && n < p.n_tau;
        const int nn = min(n, p.n_tau - 1);
        const int64_t tau = p.tau[nn];
        const int64_t span = 3 * tau;
        const int64_t lmn = span > rp.delta ? (span - rp.delta + T - 1) / T : 0;
        const int lc = p.lcol[nn];
        double A = acc.A[r], B = acc.B[r], Cc = acc.C[r];
        double f[BG][4];
#pragma unroll
        for (int b = 0; b < BG; ++b)
#pragma unroll
            for (int c = 0; c < 4; ++c) f[b][c] = (double)acc.f[r][b][c];
        const int64_t dend = p.scale_rows ? min(lmn, (int64_t)K - rp.k0) : 0;
        for (int64_t d = lc; d < dend; ++d) {
            const int64_t k = (int64_t)rp.k0 + d;
            if (k < 0) continue;
            const double gd = exp(-(double)(d * T) / (double)tau);
            const double qd = gd * gd;
            A += qd * abc[k * 4 + 0];
            B += qd * abc[k * 4 + 1];
            Cc += qd * abc[k * 4 + 2];
#pragma unroll
            for (int b = 0; b < BG; ++b) {
                if (bin0 + b >= n_bins) continue;
                const Q4<XT> x = load_q4(xg + ((size_t)k * n_bins + bin0 + b) * 4);
                f[b][0] += gd * (double)x.x;
                f[b][1] += gd * (double)x.y;
                f[b][2] += gd * (double)x.z;
                f[b][3] += gd * (double)x.w;
            }
        }
        if (p.scale_rows && rp.delta != 0) {
            const double s = exp(-(double)rp.delta / (double)tau);
            const double s2 = s * s;
            A *= s2; B *= s2; Cc *= s2;
#pragma unroll
            for (int b = 0; b < BG; ++b)
#pragma unroll
                for (int c = 0; c < 4; ++c) f[b][c] *= s;
        }
#pragma unroll
        for (int b = 0; b < BG; ++b) {
            const int bin = bin0 + b;
            if (!ok || bin >= n_bins) continue;
            const double v = twoF_cell(A, B, Cc, f[b][0], f[b][1], f[b][2], f[b][3]);
            if (p.twoF) p.twoF[((size_t)bin * p.n_t0 + m) * p.n_tau + n] = (float)v;
            red_add(red[b], 0.5 * v, (long long)m * p.n_tau + n);
        }
    }
    const int tile = nb * p.n_row_tiles + row_tile;
#pragma unroll
    for (int b = 0; b < BG; ++b) {
        const Red w = red_wave(red[b]);
        if (lane == 0 && bin0 + b < n_bins) {
            Partial &o = p.part[(size_t)(bin0 + b) * p.n_tiles + tile];
            o.fmax = w.f;
            o.s = w.s;
            o.idx = w.i;
        }
    }
}

// Waves per SIMD the runs form is built for (the four-bin shape needs more
// registers per lane).
template <typename XT, int R, int BG>
constexpr int runs_waves() {
    return BG == 4 ? 2 : 3;
}

// Weights of the stand-alone runs kernel (rounds of 8 slots): scalar loads
// for FP64 sums, LDS for FP32 (measured: FP64 maps 5-9% faster with scalar
// loads, FP32 bin pairs 2-9% and the one-bin shape 35% slower).  The
// persistent kernel (rounds of 4) takes scalar loads for every shape.
template <typename XT, int R, int BG>
constexpr bool runs_sw() {
    return sizeof(XT) == 8;
}

template <typename XT, int R, int BG>
__global__ __launch_bounds__(kThreads, (runs_waves<XT, R, BG>())) void exp_runs_kernel(ExpValuParams p) {
    __shared__ RunSmem<XT, R, BG, 8, runs_sw<XT, R, BG>()> sm;
    // groups of four tau blocks as the units of the XCD-aware order
    int g, row_tile;
    unit_decode(blockIdx.x, (p.n_list + kWaves - 1) / kWaves, p.n_row_tiles, g, row_tile);
    if (g * kWaves >= p.n_list) return;
    exp_runs_tile<XT, R, BG, 8, runs_sw<XT, R, BG>()>(p, sm, g * kWaves, row_tile, blockIdx.y);
}

// ---------------------------------------------------------------------------
// Exponential weight tables g_n[d] = exp(-d T / tau_n) for d < lcol[n],
// blocked [block][d][R] and zero-padded to the block's longest band.
// ---------------------------------------------------------------------------
template <typename PP>
__device__ inline void weights_block(PP &p, int nb, int chunk, int n_chunks) {
    const int R = p.R;
    const int64_t cnt = (int64_t)p.lblk[nb] * R;
    const int64_t off = p.blk_off[nb];
    for (int64_t i = (int64_t)chunk * 256 + threadIdx.x; i < cnt; i += (int64_t)n_chunks * 256) {
        const int64_t d = i / R;
        const int r = (int)(i - d * R);
        const int n = nb * R + r;
        double g = 0.0;
        if (n < p.n_tau && d < p.lcol[n]) {
            if (p.shape == nullptr) {
                g = exp(-(double)(d * p.t_sft) / (double)p.tau[n]);
            } else {
                // s(x) at x = (delta + d T) / tau, linear between the samples
                const double u = ((double)(p.delta + d * p.t_sft) / (double)p.tau[n]) *
                                 ((double)(p.n_shape - 1) * (double)p.shape_den / (double)p.shape_num);
                int64_t i = (int64_t)floor(u);
                i = i < 0 ? 0 : (i > p.n_shape - 2 ? p.n_shape - 2 : i);
                const double f = u - (double)i;
                g = p.shape[i] + f * (p.shape[i + 1] - p.shape[i]);
            }
        }
        p.g32[off + i] = (float)g;
        p.gsq[off + i] = g * g;
        if (p.want64) p.g64[off + i] = g;
    }
}

__global__ __launch_bounds__(256) void weights_kernel(WeightParams p) {
    weights_block(p, blockIdx.y, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void weights_batch_kernel(WeightBatchParams p) {
    const int e = blockIdx.x;
    weights_block(const_params(p.jobs + p.job[e]), p.blk[e], blockIdx.y, gridDim.y);
}

// ---------------------------------------------------------------------------
// FP32 plane of the data atoms.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void build_x32_kernel(const double *x64, float *x32, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        x32[i] = (float)x64[i];
}

// ---------------------------------------------------------------------------
// Exclusive prefix sums over slots (rectangular windows: section 3's running
// sums turned into O(1) differences per cell), carried as unevaluated
// double-double pairs so that a window's difference keeps full FP64 accuracy
// relative to the window sum itself, however long the prefix.  Channels come
// in groups of four (a^2, b^2, ab, 0; or the four data components of one
// bin); group g's prefixes are laid out [g][K+1][8]: the four hi terms,
// then the four lo terms, hi + lo = sum_{j<k} in[j][c], so that one window
// end of one group is one contiguous 64-byte read.
// Lane = channel, wave = slot segment.
// ---------------------------------------------------------------------------
constexpr int kScanWaves = 16;

struct DD {
    double h, l;
};

// Error-free sum of two doubles (Knuth's TwoSum).
__device__ inline DD two_sum(double a, double b) {
    const double s = a + b;
    const double bb = s - a;
    const double e = (a - (s - bb)) + (b - bb);
    return DD{s, e};
}

__device__ inline DD dd_add(DD x, double v) {
    const DD t = two_sum(x.h, v);
    return DD{t.h, x.l + t.l};
}

__device__ inline DD dd_add(DD x, DD y) {
    const DD t = two_sum(x.h, y.h);
    return DD{t.h, x.l + y.l + t.l};
}

__device__ __attribute__((always_inline)) inline void scan_chunk(const double *__restrict__ in,
                                                                 int64_t stride, double *__restrict__ out,
                                                                 int32_t K, int32_t C, int chunk,
                                                                 DD (*tot)[64]) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int c = chunk * 64 + lane;
    const int seg = (K + kScanWaves - 1) / kScanWaves;
    const int kb = min(K, wave * seg);
    const int ke = min(K, kb + seg);
    constexpr size_t row = 8;
    double *o = out + (size_t)(c >> 2) * ((size_t)K + 1) * 8 + (c & 3);   // this channel's hi terms
    // kSU slots' loads are issued before their (sequential) sums
    constexpr int kSU = 8;
    DD sum{0.0, 0.0};
    if (c < C) {
        int k = kb;
        for (; k + kSU <= ke; k += kSU) {
            double v[kSU];
#pragma unroll
            for (int u = 0; u < kSU; ++u) v[u] = in[(size_t)(k + u) * stride + c];
#pragma unroll
            for (int u = 0; u < kSU; ++u) sum = dd_add(sum, v[u]);
        }
        for (; k < ke; ++k) sum = dd_add(sum, in[(size_t)k * stride + c]);
    }
    tot[wave][lane] = sum;
    __syncthreads();
    DD run{0.0, 0.0};
    for (int w = 0; w < wave; ++w) run = dd_add(run, tot[w][lane]);
    if (c < C) {
        if (wave == 0) {
            o[0] = 0.0;
            o[4] = 0.0;
        }
        int k = kb;
        for (; k + kSU <= ke; k += kSU) {
            double v[kSU];
#pragma unroll
            for (int u = 0; u < kSU; ++u) v[u] = in[(size_t)(k + u) * stride + c];
#pragma unroll
            for (int u = 0; u < kSU; ++u) {
                run = dd_add(run, v[u]);
                o[(size_t)(k + u + 1) * row] = run.h;
                o[(size_t)(k + u + 1) * row + 4] = run.l;
            }
        }
        for (; k < ke; ++k) {
            run = dd_add(run, in[(size_t)k * stride + c]);
            o[(size_t)(k + 1) * row] = run.h;
            o[(size_t)(k + 1) * row + 4] = run.l;
        }
    }
}

__global__ __launch_bounds__(kScanWaves * 64) void scan_kernel(const double *__restrict__ in,
                                                               int64_t stride, double *__restrict__ out,
                                                               int32_t K, int32_t C) {
    __shared__ DD tot[kScanWaves][64];
    scan_chunk(in, stride, out, K, C, blockIdx.x, tot);
}

__global__ __launch_bounds__(kScanWaves * 64) void scan_batch_kernel(const ScanJob *jobs) {
    __shared__ DD tot[kScanWaves][64];
    const ScanJob j = jobs[blockIdx.x];
    scan_chunk(j.in, j.stride, j.out, j.K, j.C, j.chunk, tot);
}

// ---------------------------------------------------------------------------
// Rectangular windows: window sums from compensated prefixes, D, 2F, the
// optional map, per-tile reduction.  Tile = kRectRows rows x 64 taus x
// kRectBins bins: lane = tau, the waves take every fourth row; A, B, C and
// 2 / D of a cell are formed once for its bins, and each lane keeps a
// running (max, sum, first argmax) per bin, so the tile reduces once.
//
// Window ends hi = ceil((t0 - T0 + tau) / T_sft) grow with t0 and tau, so a
// tile's ends lie between those of its first cell and its last.  When that
// range fits kRectStage slots (tiles of a grid at about one slot per step),
// STAGE copies the range's prefixes of the tile's bins and of the antenna
// sums into LDS once, laid out [channel][slot] as (hi, lo) pairs so that the
// 64 lanes' reads of consecutive slots are conflict-free 16-byte accesses;
// the cells then read their end prefixes from LDS instead of addressing 80
// bytes per cell and bin through the texture path.  Window starts are one
// per row, wave-uniform, read through the scalar path either way.
// ---------------------------------------------------------------------------
constexpr int kRectStage = 128;                 // staged window-end slots
constexpr int kRectStageCh = 4 * kRectBins + 3;  // data (4 per bin) and antenna channels

struct RectStage {
    double2 v[kRectStageCh][kRectStage];
};

template <bool STAGE, typename PP>
__device__ __attribute__((always_inline)) inline void rect_block(PP &p, Red (*wred)[kRectBins], RectStage *st,
                                                                 int bx, int by, int bg) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n = bx * 64 + lane;
    const bool n_ok = n < p.n_tau;
    const int nn = min(n, p.n_tau - 1);
    const int64_t tau = p.tau[nn];
    const int64_t T = p.t_sft;
    const int64_t K = p.K;
    const int bin0 = bg * kRectBins;
    const int nbg = min(kRectBins, p.n_bins - bin0);
    const size_t bin_stride = ((size_t)K + 1) * 8;   // prefixes of one bin: [K+1][8]
    const double *pxb = p.px + (size_t)bin0 * bin_stride;
    // Window of a row for tau = q T + r (0 <= r < T): the SFT starts in
    // [t0, t0 + tau) are slots k0 .. k0 + L - 1 with L = ceil((tau - delta) / T)
    // (0 when tau <= delta); as the row offset delta lies in [0, T), that is
    // L = q + (r > delta), so the division is made once per tau, not per cell.
    auto window_qr = [&](const RowPlan &rp, int64_t q_t, int64_t r_t, int64_t &lo, int64_t &hi) {
        const int64_t L = q_t + (r_t > rp.delta ? 1 : 0);
        lo = min(max((int64_t)rp.k0, (int64_t)0), K);
        hi = min(max((int64_t)rp.k0 + L, (int64_t)0), K);
    };
    auto window = [&](const RowPlan &rp, int64_t tau_c, int64_t &lo, int64_t &hi) {
        window_qr(rp, tau_c / T, tau_c % T, lo, hi);
    };
    const int64_t tau_q = tau / T, tau_r = tau % T;
    bool staged = false;
    int64_t s0 = 0;
    if constexpr (STAGE) {
        const int m_last = min(by * kRectRows + kRectRows - 1, p.n_t0 - 1);
        const int n_last = min(bx * 64 + 63, p.n_tau - 1);
        int64_t lo_a, hi_a, lo_b, hi_b;
        window(p.rows[by * kRectRows], p.tau[bx * 64], lo_a, hi_a);
        window(p.rows[m_last], p.tau[n_last], lo_b, hi_b);
        s0 = hi_a;
        staged = hi_b - hi_a < kRectStage;
        if (staged) {
            const int ns = (int)(hi_b - hi_a + 1);
            for (int e = threadIdx.x; e < kRectStageCh * ns; e += 256) {
                const int ch = e / ns, sl = e - ch * ns;
                const int64_t k = s0 + sl;
                const double *src;
                int c;
                if (ch < 4 * kRectBins) {
                    const int b = ch >> 2;
                    c = ch & 3;
                    src = pxb + min(b, nbg - 1) * bin_stride + k * 8;
                } else {
                    c = ch - 4 * kRectBins;
                    src = p.pabc + k * 8;
                }
                st->v[ch][sl] = double2{src[c], src[4 + c]};
            }
            __syncthreads();
        }
    }
    Red r[kRectBins];
#pragma unroll
    for (int b = 0; b < kRectBins; ++b) r[b] = red_empty();
#pragma unroll 2
    for (int i = 0; i < kRectRows / kWaves; ++i) {
        const int m = by * kRectRows + i * kWaves + wave;
        if (m >= p.n_t0) break;
        const RowPlan rp = p.rows[m];
        int64_t lo, hi;
        window_qr(rp, tau_q, tau_r, lo, hi);
        // window sums from compensated prefixes: (hi_h - lo_h) + (hi_l - lo_l)
        const double *a_lo = p.pabc + lo * 8;
        double A, B, C;
        if (STAGE && staged) {
            const int sl = (int)(hi - s0);
            const double2 ha = st->v[4 * kRectBins + 0][sl], hb = st->v[4 * kRectBins + 1][sl],
                          hc = st->v[4 * kRectBins + 2][sl];
            A = (ha.x - a_lo[0]) + (ha.y - a_lo[4]);
            B = (hb.x - a_lo[1]) + (hb.y - a_lo[5]);
            C = (hc.x - a_lo[2]) + (hc.y - a_lo[6]);
        } else {
            const double *a_hi = p.pabc + hi * 8;
            A = (a_hi[0] - a_lo[0]) + (a_hi[4] - a_lo[4]);
            B = (a_hi[1] - a_lo[1]) + (a_hi[5] - a_lo[5]);
            C = (a_hi[2] - a_lo[2]) + (a_hi[6] - a_lo[6]);
        }
        // 2F = (2 / D) (B |F_a|^2 + A |F_b|^2 - 2 C Re(F_a F_b*)) (eq. F_FaFb);
        // a degenerate window (D <= rtol A B) gets 2F = 0
        const double D = A * B - C * C;
        const double k = D > kDegenerateRtol * A * B ? 2.0 / D : 0.0;
        const double kA = k * A, kB = k * B, kC = 2.0 * k * C;
        const long long idx = (long long)m * p.n_tau + n;
#pragma unroll
        for (int b = 0; b < kRectBins; ++b) {
            if (b >= nbg) break;
            const double *x_lo = pxb + b * bin_stride + lo * 8;
            double f[4];
            if (STAGE && staged) {
                const int sl = (int)(hi - s0);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const double2 h = st->v[4 * b + c][sl];
                    f[c] = (h.x - x_lo[c]) + (h.y - x_lo[4 + c]);
                }
            } else {
                const double *x_hi = pxb + b * bin_stride + hi * 8;
#pragma unroll
                for (int c = 0; c < 4; ++c) f[c] = (x_hi[c] - x_lo[c]) + (x_hi[4 + c] - x_lo[4 + c]);
            }
            const double v = kB * (f[0] * f[0] + f[1] * f[1]) + kA * (f[2] * f[2] + f[3] * f[3])
                             - kC * (f[0] * f[2] + f[1] * f[3]);
            if (n_ok) {
                if (p.twoF) p.twoF[((size_t)(bin0 + b) * p.n_t0 + m) * p.n_tau + n] = (float)v;
                red_add(r[b], 0.5 * v, idx);
            }
        }
    }
#pragma unroll
    for (int b = 0; b < kRectBins; ++b) {
        if (b >= nbg) break;
        const Red w = red_wave(r[b]);
        if (lane == 0) wred[wave][b] = w;
    }
    __syncthreads();
    if (threadIdx.x < nbg) {
        const int b = threadIdx.x;
        Red t = wred[0][b];
        for (int w = 1; w < kWaves; ++w) t = red_combine(t, wred[w][b]);
        Partial &o = p.part[(size_t)(bin0 + b) * p.n_tiles + by * p.n_tiles_n + bx];
        o.fmax = t.f;
        o.s = t.s;
        o.idx = t.i;
    }
}

__global__ __launch_bounds__(256) void rect_kernel(RectParams p) {
    __shared__ Red wred[kWaves][kRectBins];
    __shared__ RectStage st;
    rect_block<true>(p, wred, &st, blockIdx.x, blockIdx.y, blockIdx.z);
}

// ---------------------------------------------------------------------------
// Per-map merge of tile partials in a fixed order -> max 2F, argmax, logB.
// ---------------------------------------------------------------------------
template <typename PP>
__device__ __attribute__((always_inline)) inline void merge_map(PP &p, int map,
                                                                Red *sred) {
    const Partial *part = p.part + (size_t)map * p.n_tiles;
    Red r = red_empty();
    for (int t = threadIdx.x; t < p.n_tiles; t += 256) {
        const Partial q = part[t];
        r = red_combine(r, Red{q.fmax, q.s, q.idx});
    }
    sred[threadIdx.x] = r;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sred[threadIdx.x] = red_combine(sred[threadIdx.x], sred[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const Red t = sred[0];
        BinResultDev o;
        o.max2F = 2.0 * t.f;
        o.logB = t.f + log(t.s) - log((double)p.n_cells);
        o.idx = t.i;
        p.out[map] = o;
        if (p.logB_out) p.logB_out[map] = o.logB;
    }
}

__global__ __launch_bounds__(256) void merge_kernel(MergeParams p) {
    __shared__ Red sred[256];
    merge_map(p, blockIdx.x, sred);
}

__global__ __launch_bounds__(256) void merge_batch_kernel(MergeBatchParams p) {
    __shared__ Red sred[256];
    const int e = blockIdx.x;
    merge_map(const_params(p.jobs + p.job[e]), p.map[e], sred);
}

// A/B/C pre-pass of a batch: one (64-row tile, tau block) per workgroup.
__global__ __launch_bounds__(kThreads, (exp_waves<float, 8, 1, kModeAbc>())) void abc_batch_kernel(AbcBatchParams p) {
    __shared__ ExpSmem<float, 8, 1> sm;
    const int e = blockIdx.x;
    exp_tile<float, 8, 1, kModeAbc>(const_params(p.jobs + p.job[e]), sm, p.x[e], p.y[e], 0);
}

__global__ __launch_bounds__(256) void fill_i32_kernel(int32_t *dst, int32_t n, int32_t value) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) dst[i] = value;
}

// ---------------------------------------------------------------------------
// Persistent fused kernel of an uneven batch.  Each workgroup takes the next
// tile of the shared list (largest expected cost first) until the list is
// exhausted, so that maps of very different sizes and both window types
// keep every CU busy in one launch.  Every workgroup leaves once the counter
// has passed the end of the list.
// ---------------------------------------------------------------------------
// Slots per run and round in the persistent kernel's runs tiles (8 measured
// even on the uneven batch once the weights moved to scalar registers).
#ifndef TFS_FUSED_RUNS_G
#define TFS_FUSED_RUNS_G 4
#endif
constexpr int kFusedRunsG = TFS_FUSED_RUNS_G;

template <int V>
struct FusedSmem {
    static constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }
    // FP32 variants also run F_a/F_b-only tiles (8 taus, bin pairs: the
    // same sums as the stand-alone kernel's four bins per lane, in fewer
    // registers)
    static constexpr size_t fonly = V == kShapeD41 ? 0 : sizeof(ExpSmem<float, 8, 2>);
    static constexpr size_t exp_bytes = cmax(
        fonly, V == kShapeD41   ? sizeof(ExpSmem<double, 4, 1>)
               : V == kShapeF81 ? sizeof(ExpSmem<float, 8, 1>)
               : V == kShapeF42 ? sizeof(ExpSmem<float, 4, 2>)
               : V == kShapeF44 ? cmax(sizeof(ExpSmem<float, 4, 4>), sizeof(ExpSmem<float, 4, 1>))
                                : cmax(cmax(sizeof(ExpSmem<float, 4, 4>), sizeof(ExpSmem<float, 4, 1>)),
                                       sizeof(ExpSmem<double, 4, 1>)));
    // runs tiles: FP64 (R = 4) or FP32 one bin (R = 8) and bin pairs (R = 4)
    static constexpr size_t runs_bytes = V == kShapeD41 ? sizeof(RunSmem<double, 4, 1, kFusedRunsG, true>)
                                         : cmax(sizeof(RunSmem<float, 8, 1, kFusedRunsG, true>),
                                                sizeof(RunSmem<float, 4, 2, kFusedRunsG, true>));
    static constexpr size_t bytes = cmax(cmax(exp_bytes, runs_bytes), sizeof(Red) * kWaves * kRectBins);
};


// Loads a descriptor that the kernel never writes, whose address is the same
// in every lane, and keeps it in scalar registers.
template <typename T>
__device__ __attribute__((always_inline)) inline T load_uniform(const T *src) {
    static_assert(sizeof(T) % 4 == 0, "dword-sized descriptor");
    T out;
    const int *s = reinterpret_cast<const int *>(src);
    int *d = reinterpret_cast<int *>(&out);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) d[i] = __builtin_amdgcn_readfirstlane(s[i]);
    return out;
}

// Runs tiles come in three shapes: maps with four-bin groups run their
// runs tiles as bin pairs (same sums, fewer registers per lane).
template <int SHAPE, typename PP>
__device__ __attribute__((always_inline)) inline void fused_runs(PP &p, char *smem,
                                                                 const BatchTile &t) {
    if constexpr (SHAPE == kShapeD41)
        exp_runs_tile<double, 4, 1, kFusedRunsG, true>(p, *reinterpret_cast<RunSmem<double, 4, 1, kFusedRunsG, true> *>(smem), t.x, t.y, t.z);
    else if constexpr (SHAPE == kShapeF81)
        exp_runs_tile<float, 8, 1, kFusedRunsG, true>(p, *reinterpret_cast<RunSmem<float, 8, 1, kFusedRunsG, true> *>(smem), t.x, t.y, t.z);
    else
        exp_runs_tile<float, 4, 2, kFusedRunsG, true>(p, *reinterpret_cast<RunSmem<float, 4, 2, kFusedRunsG, true> *>(smem), t.x, t.y, t.z);
}

template <int SHAPE, typename PP>
__device__ __attribute__((always_inline)) inline void fused_exp(PP &p, char *smem,
                                                                const BatchTile &t) {
    if constexpr (SHAPE == kShapeD41)
        exp_tile<double, 4, 1>(p, *reinterpret_cast<ExpSmem<double, 4, 1> *>(smem), t.x, t.y, t.z);
    else if constexpr (SHAPE == kShapeF81)
        exp_tile<float, 8, 1>(p, *reinterpret_cast<ExpSmem<float, 8, 1> *>(smem), t.x, t.y, t.z);
    else if constexpr (SHAPE == kShapeF42)
        exp_tile<float, 4, 2>(p, *reinterpret_cast<ExpSmem<float, 4, 2> *>(smem), t.x, t.y, t.z);
    else if constexpr (SHAPE == kShapeF41)
        exp_tile<float, 4, 1>(p, *reinterpret_cast<ExpSmem<float, 4, 1> *>(smem), t.x, t.y, t.z);
    else
        exp_tile<float, 4, 4>(p, *reinterpret_cast<ExpSmem<float, 4, 4> *>(smem), t.x, t.y, t.z);
}

// Waves per SIMD each variant is built for: those of the stand-alone
// exponential kernel of the same shape (M = 0), or one fewer, which leaves
// the compiler more registers per wave (M = 1).
template <int V, int M>
constexpr int fused_waves() {
    return (V == kShapeF81 ? 4 : V == kShapeF44 ? 3 : V == kShapeMixed ? 3 : 5) - M;
}

template <int V, int M>
__global__ __launch_bounds__(kThreads, (fused_waves<V, M>())) void fused_kernel(FusedParams p) {
    __shared__ __attribute__((aligned(16))) char smem[FusedSmem<V>::bytes];
    __shared__ int s_next;
#pragma unroll 1
    for (;;) {
        __syncthreads();   // the previous tile is finished with smem and s_next
        if (threadIdx.x == 0) s_next = atomicAdd(p.counter, 1);
        __syncthreads();
        const int ti = __builtin_amdgcn_readfirstlane(s_next);
        if (ti >= p.n_tiles) break;
        const BatchTile t = load_uniform(p.tiles + ti);   // one tile, held in scalar registers
        if (t.kind == 1) {
            auto &rp = const_params(p.rect_jobs + t.job);
            rect_block<false>(rp, reinterpret_cast<Red (*)[kRectBins]>(smem), nullptr, t.x, t.y, t.z);
            continue;
        }
        auto &ep = const_params(p.exp_jobs + t.job);
        if constexpr (V != kShapeD41) {
            if (t.kind == 3) {
                exp_tile<float, 8, 2, kModeF>(ep, *reinterpret_cast<ExpSmem<float, 8, 2> *>(smem), t.x, t.y, t.z);
                continue;
            }
        }
        if (t.kind == 2) {
            if constexpr (V == kShapeMixed) {
                switch (t.shape) {
                case kShapeD41: fused_runs<kShapeD41>(ep, smem, t); break;
                case kShapeF81: fused_runs<kShapeF81>(ep, smem, t); break;
                default: fused_runs<kShapeF42>(ep, smem, t); break;
                }
            } else {
                fused_runs<V>(ep, smem, t);
            }
            continue;
        }
        if constexpr (V == kShapeMixed) {
            switch (t.shape) {
            case kShapeD41: fused_exp<kShapeD41>(ep, smem, t); break;
            case kShapeF81: fused_exp<kShapeF81>(ep, smem, t); break;
            case kShapeF42: fused_exp<kShapeF42>(ep, smem, t); break;
            case kShapeF41: fused_exp<kShapeF41>(ep, smem, t); break;
            default: fused_exp<kShapeF44>(ep, smem, t); break;
            }
        } else if constexpr (V == kShapeF44) {
            if (t.shape == kShapeF42) fused_exp<kShapeF42>(ep, smem, t);        // tail bin pair
            else if (t.shape == kShapeF41) fused_exp<kShapeF41>(ep, smem, t);   // tail bin
            else fused_exp<V>(ep, smem, t);
        } else {
            fused_exp<V>(ep, smem, t);
        }
    }
}

// ---------------------------------------------------------------------------
// Tile partials of an existing FP32 2F map (logB of a stored map).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void map_reduce_kernel(MapReduceParams p) {
    __shared__ Red wred[kWaves];
    const int map = blockIdx.y;
    const int tile = blockIdx.x;
    const int64_t c0 = (int64_t)tile * p.cells_per_tile;
    const int64_t c1 = min(p.n_cells, c0 + p.cells_per_tile);
    const float *src = p.twoF + (size_t)map * p.n_cells;
    Red r = red_empty();
    for (int64_t c = c0 + threadIdx.x; c < c1; c += 256) {
        const double F = 0.5 * (double)src[c];
        if (F > r.f) {
            r.s = (r.f == -INFINITY) ? 1.0 : r.s * exp(r.f - F) + 1.0;
            r.f = F;
            r.i = c;
        } else {
            r.s += exp(F - r.f);
        }
    }
    r = red_wave<true>(r);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) wred[wave] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        Red t = wred[0];
        for (int w = 1; w < kWaves; ++w) t = red_combine(t, wred[w]);
        Partial &o = p.part[(size_t)map * p.n_tiles + tile];
        o.fmax = t.f;
        o.s = t.s;
        o.idx = t.i;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
void exp_valu_config(int prec, int n_bins, int *R, int *BG) {
    if (prec == 0) {
        *R = 4;
        *BG = 1;
    } else if (n_bins >= 4) {
        *R = 4;
        *BG = 4;
    } else if (n_bins >= 2) {
        *R = 4;
        *BG = 2;
    } else {
        *R = 8;
        *BG = 1;
    }
}

hipError_t launch_exp_abc(const ExpValuParams &p, hipStream_t s) {
    if (p.n_list <= 0) return hipSuccess;
    const dim3 grid((unsigned)unit_grid(p.n_list, p.n_row_tiles), 1u);
    hipLaunchKernelGGL((exp_valu_kernel<float, 8, 1, kModeAbc>), grid, dim3(kThreads), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_exp_fonly(const ExpValuParams &p, int n_groups, hipStream_t s) {
    if (p.n_list <= 0 || n_groups <= 0) return hipSuccess;
    if (p.bin_base + (n_groups - 1) * 4 >= p.at.n_bins || !p.abc_out) return hipErrorInvalidValue;
    const dim3 grid((unsigned)unit_grid(p.n_list, p.n_row_tiles), (unsigned)n_groups);
    hipLaunchKernelGGL((exp_valu_kernel<float, 8, 4, kModeF>), grid, dim3(kThreads), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_exp_valu(const ExpValuParams &p, int prec, int R, int BG, int n_groups, hipStream_t s) {
    if (p.n_list <= 0 || n_groups <= 0) return hipSuccess;
    if (p.bin_base + (n_groups - 1) * BG >= p.at.n_bins) return hipErrorInvalidValue;
    const dim3 grid((unsigned)unit_grid(p.n_list, p.n_row_tiles), (unsigned)n_groups);
    if (prec == 0 && R == 4 && BG == 1)
        hipLaunchKernelGGL((exp_valu_kernel<double, 4, 1>), grid, dim3(kThreads), 0, s, p);
    else if (prec == 1 && R == 8 && BG == 1)
        hipLaunchKernelGGL((exp_valu_kernel<float, 8, 1>), grid, dim3(kThreads), 0, s, p);
    else if (prec == 1 && R == 4 && BG == 2)
        hipLaunchKernelGGL((exp_valu_kernel<float, 4, 2>), grid, dim3(kThreads), 0, s, p);
    else if (prec == 1 && R == 4 && BG == 1)
        hipLaunchKernelGGL((exp_valu_kernel<float, 4, 1>), grid, dim3(kThreads), 0, s, p);
    else if (prec == 1 && R == 4 && BG == 4)
        hipLaunchKernelGGL((exp_valu_kernel<float, 4, 4>), grid, dim3(kThreads), 0, s, p);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_exp_runs(const ExpValuParams &p, int prec, int R, int BG, int n_groups, hipStream_t s) {
    if (p.n_list <= 0 || n_groups <= 0) return hipSuccess;
    if (p.bin_base + (n_groups - 1) * BG >= p.at.n_bins) return hipErrorInvalidValue;
    const int n_q = (p.n_list + kWaves - 1) / kWaves;
    const dim3 grid((unsigned)unit_grid(n_q, p.n_row_tiles), (unsigned)n_groups);
    if (prec == 0 && R == 4 && BG == 1)
        hipLaunchKernelGGL((exp_runs_kernel<double, 4, 1>), grid, dim3(kThreads), 0, s, p);
    else if (prec == 1 && R == 8 && BG == 1)
        hipLaunchKernelGGL((exp_runs_kernel<float, 8, 1>), grid, dim3(kThreads), 0, s, p);
    else if (prec == 1 && R == 4 && BG == 2)
        hipLaunchKernelGGL((exp_runs_kernel<float, 4, 2>), grid, dim3(kThreads), 0, s, p);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_weights(const WeightParams &p, int64_t max_per_block, hipStream_t s) {
    int64_t gx = (max_per_block + 255) / 256;
    if (gx < 1) gx = 1;
    if (gx > 4096) gx = 4096;
    hipLaunchKernelGGL(weights_kernel, dim3((unsigned)gx, (unsigned)p.n_blocks), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_build_x32(const double *x64, float *x32, int64_t n, hipStream_t s) {
    int64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(build_x32_kernel, dim3((unsigned)g), dim3(256), 0, s, x64, x32, n);
    return hipGetLastError();
}

hipError_t launch_scan(const double *in, int64_t stride, double *out, int32_t K, int32_t C,
                       hipStream_t s) {
    hipLaunchKernelGGL(scan_kernel, dim3((unsigned)((C + 63) / 64)), dim3(kScanWaves * 64), 0, s,
                       in, stride, out, K, C);
    return hipGetLastError();
}

hipError_t launch_rect(const RectParams &p, hipStream_t s) {
    const dim3 grid((unsigned)p.n_tiles_n, (unsigned)((p.n_t0 + kRectRows - 1) / kRectRows),
                    (unsigned)((p.n_bins + kRectBins - 1) / kRectBins));
    hipLaunchKernelGGL(rect_kernel, grid, dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_merge(const MergeParams &p, hipStream_t s) {
    hipLaunchKernelGGL(merge_kernel, dim3((unsigned)p.n_maps), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_weights_batch(const WeightBatchParams &p, hipStream_t s) {
    if (p.n_entries <= 0) return hipSuccess;
    if (p.chunks < 1 || p.chunks > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(weights_batch_kernel, dim3((unsigned)p.n_entries, (unsigned)p.chunks), dim3(256), 0,
                       s, p);
    return hipGetLastError();
}

hipError_t launch_abc_batch(const AbcBatchParams &p, hipStream_t s) {
    if (p.n_entries <= 0) return hipSuccess;
    hipLaunchKernelGGL(abc_batch_kernel, dim3((unsigned)p.n_entries), dim3(kThreads), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_scan_batch(const ScanJob *jobs, int32_t n_jobs, hipStream_t s) {
    if (n_jobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(scan_batch_kernel, dim3((unsigned)n_jobs), dim3(kScanWaves * 64), 0, s, jobs);
    return hipGetLastError();
}

hipError_t launch_merge_batch(const MergeBatchParams &p, hipStream_t s) {
    if (p.n_entries <= 0) return hipSuccess;
    hipLaunchKernelGGL(merge_batch_kernel, dim3((unsigned)p.n_entries), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *dst, int32_t n, int32_t value, hipStream_t s) {
    const int g = std::max(1, std::min((n + 255) / 256, 1024));
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)g), dim3(256), 0, s, dst, n, value);
    return hipGetLastError();
}

namespace {
// variant = shape + kShapeCount1 * M, shape in [0, kShapeMixed], M in {0, 1}
constexpr int kShapeCount1 = kShapeMixed + 1;

template <int V, int M>
const void *fused_fn() {
    return reinterpret_cast<const void *>(&fused_kernel<V, M>);
}

template <int M>
const void *fused_variant_m(int v) {
    switch (v) {
    case kShapeD41: return fused_fn<kShapeD41, M>();
    case kShapeF81: return fused_fn<kShapeF81, M>();
    case kShapeF42: return fused_fn<kShapeF42, M>();
    case kShapeF44: return fused_fn<kShapeF44, M>();
    case kShapeMixed: return fused_fn<kShapeMixed, M>();
    default: return nullptr;
    }
}

const void *fused_variant(int variant) {
    if (variant < 0 || variant >= 2 * kShapeCount1) return nullptr;
    return variant < kShapeCount1 ? fused_variant_m<0>(variant) : fused_variant_m<1>(variant - kShapeCount1);
}
}  // namespace

int fused_groups_per_cu(int variant) {
    const void *fn = fused_variant(variant);
    if (!fn) return 0;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, kThreads, 0) != hipSuccess) return 0;
    return n;
}

hipError_t launch_fused(const FusedParams &p, int variant, int n_groups, hipStream_t s) {
    if (p.n_tiles <= 0) return hipSuccess;
    if (n_groups < 1) return hipErrorInvalidValue;
    const void *fn = fused_variant(variant);
    if (!fn) return hipErrorInvalidValue;
    void *args[] = {const_cast<FusedParams *>(&p)};
    return hipLaunchKernel(fn, dim3(n_groups), dim3(kThreads), args, 0, s);
}

hipError_t launch_map_reduce(const MapReduceParams &p, hipStream_t s) {
    hipLaunchKernelGGL(map_reduce_kernel, dim3((unsigned)p.n_tiles, (unsigned)p.n_maps), dim3(256),
                       0, s, p);
    return hipGetLastError();
}

}  // namespace tfs
