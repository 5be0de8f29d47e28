// Host runtime and C ABI of the tfstat library: device-arena sub-allocator,
// resident atom store, integer grid planner, job execution on HIP streams,
// a continuous-batching request loop, and per-kernel timing.
//
// The problem statement follows Keitel & Ashton (arXiv:1805.05652),
// section 3: the inputs are per-SFT atoms plus a window type and a {t0, tau}
// grid; the output is the transient map F_mn (eq. Fmn) and, per the
// appendix A footnote, its marginalised Bayes factor.
#include "../../include/tfstat.h"
#include "tfstat_device.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

struct Failure {
    int code;
    std::string msg;
};

[[noreturn]] void raise(int code, const std::string &msg) { throw Failure{code, msg}; }

void hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess) raise(TFSTAT_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int64_t floor_div(int64_t a, int64_t b) {
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
    return q;
}
int64_t ceil_div(int64_t a, int64_t b) { return -floor_div(-a, b); }

// ---------------------------------------------------------------------------
// First-fit sub-allocator over the caller's device arena (host bookkeeping
// only; no device allocation).  256-byte granularity, coalescing frees.
// ---------------------------------------------------------------------------
class Arena {
  public:
    void init(void *base, size_t size) {
        base_ = static_cast<char *>(base);
        size_ = size;
        free_.clear();
        used_.clear();
        free_[0] = size;
        in_use_ = 0;
    }
    void *alloc(size_t bytes) {
        bytes = round_up(std::max<size_t>(bytes, 1), 256);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, sz = it->second;
            free_.erase(it);
            if (sz > bytes) free_[off + bytes] = sz - bytes;
            used_[off] = bytes;
            in_use_ += bytes;
            return base_ + off;
        }
        return nullptr;
    }
    void release(void *p) {
        if (!p) return;
        const size_t off = static_cast<char *>(p) - base_;
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t sz = u->second;
        used_.erase(u);
        in_use_ -= sz;
        size_t start = off;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && next->first == off + sz) {
            sz += next->second;
            free_.erase(next);
        }
        auto it = free_.lower_bound(off);
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == off) {
                start = prev->first;
                sz += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = sz;
    }
    size_t capacity() const { return size_; }
    size_t in_use() const { return in_use_; }
    size_t largest_free() const {
        size_t m = 0;
        for (auto &kv : free_) m = std::max(m, kv.second);
        return m;
    }

  private:
    char *base_ = nullptr;
    size_t size_ = 0;
    size_t in_use_ = 0;
    std::map<size_t, size_t> free_;
    std::unordered_map<size_t, size_t> used_;
};

// Pool of pinned host buffers (staging of tables and results).
class PinnedPool {
  public:
    ~PinnedPool() {
        for (auto &kv : free_) (void)hipHostFree(kv.second);
    }
    void *get(size_t bytes, size_t *got) {
        size_t want = 4096;
        while (want < bytes) want <<= 1;
        {
            std::lock_guard<std::mutex> g(mu_);
            auto it = free_.lower_bound(want);
            if (it != free_.end()) {
                void *p = it->second;
                *got = it->first;
                free_.erase(it);
                return p;
            }
        }
        void *p = nullptr;
        hip_check(hipHostMalloc(&p, want, hipHostMallocDefault), "hipHostMalloc");
        *got = want;
        return p;
    }
    void put(void *p, size_t size) {
        if (!p) return;
        std::lock_guard<std::mutex> g(mu_);
        free_.emplace(size, p);
    }

  private:
    std::mutex mu_;
    std::multimap<size_t, void *> free_;
};

struct AtomsSet {
    int32_t K = 0, n_bins = 0, n_sft = 0;
    int64_t T0 = 0, t_sft = 0;
    void *mem = nullptr;
    size_t bytes = 0;
    double *abc = nullptr;
    double *x64 = nullptr;
    float *x32 = nullptr;
    int32_t *npref = nullptr;   // [K+1] present SFTs in slots [0, k)
    // bf16 hi / lo planes for the matrix-core path, built on first use
    void *planes = nullptr;
    unsigned short *xhi = nullptr, *xlo = nullptr;
    // half-precision hi / lo planes of the scaled columns and the columns'
    // scale exponents (F16X3), built on first use
    void *planes16 = nullptr;
    unsigned short *xhi16 = nullptr, *xlo16 = nullptr;
    int32_t *colexp = nullptr;
    int32_t bins16 = 0, kp = 0;
    // column planes of the transposed matrix-core form (maps of fewer than
    // 64 bins): bf16 and half-precision parts, in the allocations above
    unsigned short *chi = nullptr, *clo = nullptr, *chi16 = nullptr, *clo16 = nullptr;
    int32_t kpc = 0;
    int busy = 0;
    tfs::AtomsView view() const {
        tfs::AtomsView v;
        v.K = K;
        v.n_bins = n_bins;
        v.t_sft = t_sft;
        v.abc = abc;
        v.x64 = x64;
        v.x32 = x32;
        return v;
    }
};

struct WindowOwned {
    int32_t type = 0;
    std::vector<int64_t> t0, tau;
    std::vector<double> shape;          // shape windows: samples of s(x)
    int32_t num = 1, den = 1;           // their support [0, num/den] in units of tau
};

// Banded windows run the exponential window's kernels.
inline bool banded(int32_t type) { return type == TFSTAT_WIN_EXP || type == TFSTAT_WIN_SHAPE; }

// Precisions whose long-band exponential sums run on the matrix cores.
inline bool matrix_prec(int32_t prec) { return prec == TFSTAT_PREC_BF16X3 || prec == TFSTAT_PREC_F16X3; }

WindowOwned copy_window(const tfstat_window *w) {
    if (!w) raise(TFSTAT_E_INVAL, "window is null");
    if (w->type != TFSTAT_WIN_RECT && w->type != TFSTAT_WIN_EXP && w->type != TFSTAT_WIN_SHAPE)
        raise(TFSTAT_E_INVAL, "unknown window type");
    if (w->reserved != 0 || w->reserved2 != 0) raise(TFSTAT_E_INVAL, "window.reserved fields must be 0");
    if (w->n_t0 < 1 || w->n_tau < 1) raise(TFSTAT_E_GRID, "n_t0 and n_tau must be >= 1");
    WindowOwned o;
    o.type = w->type;
    o.t0.resize(w->n_t0);
    o.tau.resize(w->n_tau);
    if (w->t0_list) {
        std::memcpy(o.t0.data(), w->t0_list, sizeof(int64_t) * w->n_t0);
    } else {
        if (w->dt0 < 1) raise(TFSTAT_E_GRID, "dt0 must be >= 1");
        for (int32_t i = 0; i < w->n_t0; ++i) o.t0[i] = w->t0_min + (int64_t)i * w->dt0;
    }
    if (w->tau_list) {
        std::memcpy(o.tau.data(), w->tau_list, sizeof(int64_t) * w->n_tau);
    } else {
        if (w->dtau < 1) raise(TFSTAT_E_GRID, "dtau must be >= 1");
        for (int32_t i = 0; i < w->n_tau; ++i) o.tau[i] = w->tau_min + (int64_t)i * w->dtau;
    }
    for (size_t i = 1; i < o.t0.size(); ++i)
        if (o.t0[i] <= o.t0[i - 1]) raise(TFSTAT_E_GRID, "t0 grid must be strictly increasing");
    for (size_t i = 0; i < o.tau.size(); ++i) {
        if (o.tau[i] < 1) raise(TFSTAT_E_GRID, "tau values must be >= 1");
        if (o.tau[i] > ((int64_t)1 << 58)) raise(TFSTAT_E_GRID, "tau too large");
        if (i && o.tau[i] <= o.tau[i - 1]) raise(TFSTAT_E_GRID, "tau grid must be strictly increasing");
    }
    if (w->type == TFSTAT_WIN_SHAPE) {
        if (!w->shape || w->n_shape < 2 || w->n_shape > 65536)
            raise(TFSTAT_E_INVAL, "shape windows need 2..65536 samples");
        if (w->support_num < 1 || w->support_num > 1024 || w->support_den < 1 || w->support_den > 1024)
            raise(TFSTAT_E_INVAL, "shape support num/den must be in 1..1024");
        o.shape.assign(w->shape, w->shape + w->n_shape);
        for (double v : o.shape)
            if (!std::isfinite(v)) raise(TFSTAT_E_INVAL, "shape samples must be finite");
        o.num = w->support_num;
        o.den = w->support_den;
        for (int64_t t : o.tau)
            if (t > ((int64_t)1 << 50)) raise(TFSTAT_E_GRID, "tau too large for a shape window");
    }
    return o;
}

enum { NK = TFSTAT_K_COUNT };

constexpr int kMfmaTaus = 8;       // taus per matrix-core work item
inline int32_t abc_pitch(int32_t n_tau) { return (n_tau + kMfmaTaus - 1) / kMfmaTaus * kMfmaTaus; }
constexpr int kMfmaMinBand = 64;      // BF16X3: shorter bands stay on the VALU path
constexpr int kMfmaMinBandF16 = 24;   // F16X3: the same for its finer parts
// Exponential one-bin maps run the FP32 path: there each wave-uniform weight
// serves 64 rows' sums (about 0.35 ns per cell*SFT on the 1-bin workload),
// while the matrix-core form makes a weight per row, tau and slot (about
// 0.44 ns per cell*SFT for any bin count up to 16 on the uneven batch); from
// two bins on the matrix cores are faster.
constexpr int kMfmaMinBins = 2;
// Tiling threshold of the exponential VALU sums (tfstat_tiling_config):
// kRunsAuto sends a map to the runs form when its median 64-row tile spans
// more slots than one LDS stage can stage in rounds of kExpMinStageRound.
constexpr int32_t kRunsAuto = -1;
// FP32 maps with at least this many bins (and rows close enough for the band
// stage) take the split form: A/B/C pass, then F_a/F_b-only tiles.
constexpr int32_t kSplitMinBins = 8;

// ---------------------------------------------------------------------------
// One map computation: plan (host, integer), workspace, launches, results.
// ---------------------------------------------------------------------------
struct Job {
    AtomsSet *at = nullptr;
    WindowOwned win;
    int prec = TFSTAT_PREC_FP32;
    float *twoF = nullptr;

    // plan
    std::vector<tfs::RowPlan> rows;
    std::vector<int32_t> lcol, lblk, order;
    std::vector<int64_t> blk_off;
    int R = 0, BG = 0, NB = 0, n_row_tiles = 0, n_tiles = 0, n_tiles_n = 0;
    int force_R = 0, force_BG = 0;   // exponential VALU tile shape chosen by the caller
    int32_t runs_min_spread = kRunsAuto;   // see tfstat_tiling_config
    bool runs = false;         // VALU blocks by the runs form (t0 rows far apart)
    int32_t split_min_bins = kSplitMinBins;     // see tfstat_tiling_config
    // A/B/C once per cell in an FP64 pass, then F_a, F_b only with four bins
    // per lane (FP32 maps with many bins and rows close together)
    bool split = false;
    // bin groups of BG bins; with four-bin groups and one or two bins left
    // over, those take one two-bin group after the n_groups full ones
    int n_groups = 0;
    bool tail2 = false;
    int64_t wtot = 0, max_blk = 0;
    bool use_recur = false;    // RECUR64: exponential sums by the t0 recurrence
    int32_t recur_stride = 0, recur_k0 = 0, recur_bg = 1;
    bool use_mfma = false;     // BF16X3 on matrix cores for long bands
    // matrix-core form: true = weights computed per row (exponential
    // windows, any t0 grid); false = shifted weight tables (shape windows
    // with rows on consecutive slots)
    bool mfma_rows = false;
    int n_valu = 0, n_mfma = 0;  // block lists: order[0..n_valu) VALU, then MFMA
    std::vector<int32_t> lg;     // shifted bf16 table length per block (MFMA blocks)
    std::vector<int64_t> gsh_off;
    int64_t gsh_total = 0, gsh_max = 0;

    // memory
    size_t ws_bytes = 0;
    void *ws = nullptr;
    void *pin = nullptr;
    size_t pin_bytes = 0;
    size_t off_rows = 0, off_tau = 0, off_lcol = 0, off_lblk = 0, off_boff = 0, off_order = 0,
           tables_bytes = 0;
    size_t off_g32 = 0, off_gsq = 0, off_g64 = 0, off_pabc = 0, off_px = 0, off_part = 0,
           off_res = 0, off_abc = 0, off_lg = 0, off_gshoff = 0, off_gsh = 0, off_shape = 0;

    // timing
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> timed;
    hipEvent_t done = nullptr;
};

void plan_job(Job &j) {
    const AtomsSet &at = *j.at;
    const int64_t T = at.t_sft;
    const int n_t0 = (int)j.win.t0.size();
    const int n_tau = (int)j.win.tau.size();
    j.rows.resize(n_t0);
    int64_t k0_min = INT64_MAX;
    for (int m = 0; m < n_t0; ++m) {
        const int64_t diff = j.win.t0[m] - at.T0;
        if (diff > ((int64_t)1 << 58) || diff < -((int64_t)1 << 58))
            raise(TFSTAT_E_GRID, "t0 too far from the data");
        int64_t k0 = ceil_div(diff, T);
        const int64_t delta = at.T0 + k0 * T - j.win.t0[m];
        if (k0 > at.K) k0 = at.K;
        if (k0 < -((int64_t)1 << 30)) raise(TFSTAT_E_GRID, "t0 too far before the data");
        j.rows[m].k0 = (int32_t)k0;
        j.rows[m].delta = (int32_t)delta;
        k0_min = std::min(k0_min, k0);
    }
    const bool is_exp = banded(j.win.type);
    const bool is_shape = j.win.type == TFSTAT_WIN_SHAPE;
    if (is_shape) {
        if (j.prec == TFSTAT_PREC_RECUR64) raise(TFSTAT_E_INVAL, "RECUR64 applies to exponential windows only");
        for (int m = 1; m < n_t0; ++m)
            if (j.rows[m].delta != j.rows[0].delta)
                raise(TFSTAT_E_GRID, "shape windows need every t0 at one offset from the SFT start grid");
    }
    // Table length per tau: the shortest band over all rows (the row with
    // the largest delta), capped where no row can reach data any more.
    // Rows with longer bands add their extra terms in the finalize step.
    int64_t delta_max = 0;
    for (int m = 0; m < n_t0; ++m) delta_max = std::max<int64_t>(delta_max, j.rows[m].delta);
    j.lcol.assign(n_tau, 0);
    const int64_t cap = std::max<int64_t>(0, (int64_t)at.K - k0_min);
    for (int n = 0; n < n_tau; ++n) {
        const int64_t span = is_shape ? j.win.tau[n] * j.win.num / j.win.den
                             : (is_exp ? 3 * j.win.tau[n] : j.win.tau[n]);
        const int64_t shortest = span > delta_max ? ceil_div(span - delta_max, T) : 0;
        j.lcol[n] = (int32_t)std::min(shortest, cap);
    }
    j.n_row_tiles = (n_t0 + 63) / 64;
    // Recurrence path: RECUR64 on a regular t0 grid whose step is a whole
    // number of slots (then every row has the same delta).
    j.use_recur = false;
    if (j.win.type == TFSTAT_WIN_EXP && j.prec == TFSTAT_PREC_RECUR64) {
        bool ok = true;
        int64_t step = n_t0 > 1 ? j.win.t0[1] - j.win.t0[0] : T;
        for (int m = 1; m < n_t0 && ok; ++m) ok = j.win.t0[m] - j.win.t0[m - 1] == step;
        ok = ok && step % T == 0 && step / T <= 64;
        const int64_t k0 = ceil_div(j.win.t0[0] - at.T0, T);
        const int64_t klast = k0 + (int64_t)(n_t0 - 1) * (step / T);
        ok = ok && k0 > -((int64_t)1 << 30) && klast < ((int64_t)1 << 30);
        if (ok) {
            j.use_recur = true;
            j.recur_stride = (int32_t)(step / T);
            j.recur_k0 = (int32_t)k0;
            j.recur_bg = at.n_bins >= 4 ? 4 : (at.n_bins >= 2 ? 2 : 1);
        }
    }
    // Matrix-core path (BF16X3).  Exponential windows: any t0 grid, maps of
    // at least kMfmaMinBins bins whose bf16 component planes stay under
    // 2^31 bytes.  Shape windows: rows on consecutive slots with one delta.
    // Either needs a block of 8 taus whose shortest band is long enough (the
    // band grows with tau, so block b's shortest is that of its first tau).
    j.use_mfma = false;
    j.mfma_rows = false;
    if (is_exp && matrix_prec(j.prec)) {
        bool ok;
        if (is_shape) {
            // the shifted bf16 tables; F16X3 shape windows run the FP32 sums
            ok = j.prec == TFSTAT_PREC_BF16X3 && j.rows[0].k0 >= 0;
            for (int m = 1; m < n_t0 && ok; ++m)
                ok = j.rows[m].k0 == j.rows[0].k0 + m && j.rows[m].delta == j.rows[0].delta;
        } else {
            const int64_t bins16 = (at.n_bins + 15) / 16 * 16;
            const int64_t kp = ((int64_t)at.K + 31) / 32 * 32 + 32;
            ok = at.n_bins >= kMfmaMinBins && bins16 * kp * 2 < ((int64_t)1 << 31);
            if (tfs::mfma_cells_form((int)(bins16 / 16)))
                ok = ok && (int64_t)8 * tfs::kCellsCopies * at.n_bins * tfs::cells_plane_pitch(at.K) <
                               ((int64_t)1 << 31);
            j.mfma_rows = ok;
        }
        bool long_block = false;
        for (int n = 0; n < n_tau && ok && !long_block; n += kMfmaTaus) long_block = j.lcol[n] >= kMfmaMinBand;
        j.use_mfma = ok && long_block;
        if (!j.use_mfma) j.mfma_rows = false;
    }
    if (is_exp && j.use_recur) {
        j.NB = 0;
        j.n_tiles = n_tau;
    } else if (is_exp) {
        const int prec = (j.prec == TFSTAT_PREC_FP64 || j.prec == TFSTAT_PREC_RECUR64) ? 0 : 1;
        // median slot span of the 64-row tiles (tile form choice below)
        int64_t med;
        {
            std::vector<int64_t> spread(j.n_row_tiles);
            for (int t = 0; t < j.n_row_tiles; ++t)
                spread[t] = (int64_t)j.rows[std::min(t * 64 + 63, n_t0 - 1)].k0 - j.rows[t * 64].k0;
            std::nth_element(spread.begin(), spread.begin() + j.n_row_tiles / 2, spread.end());
            med = spread[j.n_row_tiles / 2];
        }
        tfs::exp_valu_config(prec, at.n_bins, &j.R, &j.BG);
        if (j.force_R) {
            j.R = j.force_R;
            j.BG = j.force_BG;
        }
        if (j.use_mfma) {
            j.R = kMfmaTaus;
            j.BG = 1;
        }
        // the split form (its own tile shape in every batch variant); an
        // explicit runs threshold that the map reaches takes precedence
        const bool runs_forced = j.runs_min_spread >= 0 && med >= j.runs_min_spread;
        j.split = prec == 1 && !j.use_mfma && !runs_forced && j.split_min_bins > 0 &&
                  at.n_bins >= j.split_min_bins && med <= tfs::exp_stage_len(1, 4) - tfs::kExpMinStageRound;
        if (j.split) {
            j.R = kMfmaTaus;
            j.BG = 4;
        }
        j.NB = (n_tau + j.R - 1) / j.R;
        j.tail2 = j.BG == 4 && !j.split && (at.n_bins % 4 == 1 || at.n_bins % 4 == 2);
        j.n_groups = j.tail2 ? at.n_bins / 4 : (at.n_bins + j.BG - 1) / j.BG;
        j.lblk.assign(j.NB, 0);
        j.blk_off.assign(j.NB, 0);
        int64_t acc = 0;
        j.max_blk = 0;
        for (int b = 0; b < j.NB; ++b) {
            int32_t mx = 0;
            for (int r = 0; r < j.R && b * j.R + r < n_tau; ++r) mx = std::max(mx, j.lcol[b * j.R + r]);
            j.lblk[b] = mx;
            j.blk_off[b] = acc;
            acc += (int64_t)mx * j.R;
            j.max_blk = std::max<int64_t>(j.max_blk, (int64_t)mx * j.R);
        }
        j.wtot = acc;
        j.order.resize(j.NB);
        for (int b = 0; b < j.NB; ++b) j.order[b] = b;
        std::stable_sort(j.order.begin(), j.order.end(),
                         [&](int a, int b) { return j.lblk[a] > j.lblk[b]; });
        j.n_tiles = j.NB * j.n_row_tiles;
        j.n_valu = j.NB;
        j.n_mfma = 0;
        if (!j.split) {
            // automatic: the runs form where the band stage would fall back
            // to per-lane reads through the caches, except for the 8-tau
            // one-bin shape, whose 32-tau runs tiles leave too few
            // workgroups for one map (its per-lane reads are faster there)
            if (j.runs_min_spread >= 0)
                j.runs = med >= j.runs_min_spread;
            else
                j.runs = j.R != 8 && med > tfs::exp_stage_len(prec, j.BG) - tfs::kExpMinStageRound;
            // the runs form takes four-bin maps as bin pairs (the sums of
            // every cell are the same, with fewer registers per lane)
            if (j.runs && j.BG == 4) {
                j.BG = 2;
                j.tail2 = false;
                j.n_groups = (at.n_bins + 1) / 2;
            }
        }
        if (j.use_mfma) {
            // a block with any short band stays on the FP32 VALU path: short
            // windows carry little work and the worst conditioning, which
            // amplifies the error of the split operands (~2^-16 for bf16,
            // ~2^-22 for half precision: on windows of 3-7 SFTs F16X3 2F
            // errors reach 5e-5 against FP32's 7e-6, and from 24 slots on
            // they are at FP32's level)
            const int32_t min_band = j.prec == TFSTAT_PREC_F16X3 ? kMfmaMinBandF16 : kMfmaMinBand;
            std::vector<int32_t> lv, lm;
            for (int32_t b : j.order) {
                int32_t shortest = INT32_MAX;
                for (int r = 0; r < j.R && b * j.R + r < n_tau; ++r)
                    shortest = std::min(shortest, j.lcol[b * j.R + r]);
                (shortest >= min_band ? lm : lv).push_back(b);
            }
            j.n_valu = (int)lv.size();
            j.n_mfma = (int)lm.size();
            j.order = lv;
            j.order.insert(j.order.end(), lm.begin(), lm.end());
            j.lg.assign(j.NB, 0);
            if (j.mfma_rows) lm.clear();   // weights computed in the kernel: no tables
            j.gsh_off.assign(j.NB, 0);
            j.gsh_total = 0;
            j.gsh_max = 0;
            for (int32_t b : lm) {
                j.lg[b] = tfs::shift_table_len(j.lblk[b]);
                j.gsh_off[b] = j.gsh_total;
                const int64_t n = (int64_t)kMfmaTaus * 2 * tfs::kMfmaShifts * j.lg[b];
                j.gsh_total += n;
                j.gsh_max = std::max(j.gsh_max, n);
            }
        }
    } else {
        j.n_tiles_n = (n_tau + 63) / 64;
        j.n_tiles = j.n_tiles_n * ((n_t0 + tfs::kRectRows - 1) / tfs::kRectRows);
    }

    // workspace layout
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at_ = o;
        o = round_up(o + bytes, 256);
        return at_;
    };
    j.off_rows = take(sizeof(tfs::RowPlan) * n_t0);
    j.off_tau = take(sizeof(int64_t) * n_tau);
    j.off_lcol = take(sizeof(int32_t) * n_tau);
    if (is_exp && !j.use_recur) {
        j.off_lblk = take(sizeof(int32_t) * j.NB);
        j.off_boff = take(sizeof(int64_t) * j.NB);
        j.off_order = take(sizeof(int32_t) * j.NB);
        if (j.use_mfma) {
            j.off_lg = take(sizeof(int32_t) * j.NB);
            j.off_gshoff = take(sizeof(int64_t) * j.NB);
        }
        if (is_shape) j.off_shape = take(sizeof(double) * j.win.shape.size());
    }
    j.tables_bytes = o;
    if (is_exp && j.use_recur) {
        // no weight tables
    } else if (is_exp) {
        j.off_g32 = take(sizeof(float) * std::max<int64_t>(j.wtot, 1));
        j.off_gsq = take(sizeof(double) * std::max<int64_t>(j.wtot, 1));
        if (j.prec == TFSTAT_PREC_FP64 || j.prec == TFSTAT_PREC_RECUR64)
            j.off_g64 = take(sizeof(double) * std::max<int64_t>(j.wtot, 1));
        if (j.use_mfma && j.n_mfma > 0) {
            // rows padded to whole blocks: the matrix-core kernel copies them
            j.off_abc = take(sizeof(double) * 3 * (size_t)n_t0 * abc_pitch(n_tau));
            j.off_gsh = take(sizeof(unsigned short) * (size_t)j.gsh_total);
        }
        if (j.split) j.off_abc = take(sizeof(double) * 3 * (size_t)n_t0 * abc_pitch(n_tau));
    } else {
        j.off_pabc = take(sizeof(double) * 8 * ((size_t)at.K + 1));
        j.off_px = take(sizeof(double) * 8 * (size_t)at.n_bins * ((size_t)at.K + 1));
    }
    j.off_part = take(sizeof(tfs::Partial) * (size_t)j.n_tiles * at.n_bins);
    j.off_res = take(sizeof(tfs::BinResultDev) * at.n_bins);
    j.ws_bytes = o;
}

struct EventPool {
    std::mutex mu;
    std::vector<hipEvent_t> free_;
    hipEvent_t get() {
        {
            std::lock_guard<std::mutex> g(mu);
            if (!free_.empty()) {
                hipEvent_t e = free_.back();
                free_.pop_back();
                return e;
            }
        }
        hipEvent_t e;
        hip_check(hipEventCreate(&e), "hipEventCreate");
        return e;
    }
    void put(hipEvent_t e) {
        std::lock_guard<std::mutex> g(mu);
        free_.push_back(e);
    }
    ~EventPool() {
        for (auto e : free_) (void)hipEventDestroy(e);
    }
};

}  // namespace

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
struct tfstat_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    Arena arena;
    std::mutex mu;   // guards arena, atoms, tickets, stats
    std::unordered_map<uint64_t, std::unique_ptr<AtomsSet>> atoms;
    uint64_t next_atoms = 1;
    PinnedPool pinned;
    EventPool events;
    std::atomic<int> profile{0};
    int64_t k_launches[NK] = {0};
    double k_ms[NK] = {0};

    // serving
    struct Ticket {
        uint64_t atoms_id = 0;
        std::unique_ptr<Job> job;
        enum { QUEUED, RUNNING, DONE, FAILED, CANCELLED } state = QUEUED;
        bool cancel_requested = false;
        int err = 0;
        std::string msg;
        std::vector<tfstat_bin_result> res;
        int slot = -1;
    };
    static constexpr int kSlots = 4;
    static constexpr size_t kMaxQueue = 1 << 16;
    std::unordered_map<uint64_t, Ticket> tickets;
    std::deque<uint64_t> queue;
    uint64_t next_ticket = 1;
    hipStream_t slots[kSlots] = {nullptr};
    std::vector<uint64_t> slot_tickets[kSlots];          // requests running on each slot
    std::unique_ptr<tfstat_batch> slot_batch[kSlots];   // their fused batch, if batched
    hipEvent_t slot_done[kSlots] = {nullptr};
    int serve_max_batch = 16;                           // requests fused into one launch at most
    std::atomic<int32_t> runs_min_spread{kRunsAuto};   // see tfstat_tiling_config
    std::atomic<int32_t> split_min_bins{kSplitMinBins};
    std::thread worker;
    std::condition_variable cv;
    bool stop = false;
    bool worker_started = false;

    // uneven batches: their own stream (graphs cannot capture the null
    // stream) and the autotuner's choices by batch shape signature
    hipStream_t batch_stream = nullptr;
    int n_cu = 0;
    std::map<std::string, std::pair<int, int>> tuned;   // signature -> (variant, groups per CU)
};

namespace {

void record_kernel(tfstat_ctx *ctx, Job &j, int kind, hipStream_t s, bool begin) {
    if (!ctx->profile.load()) return;
    if (begin) {
        hipEvent_t a = ctx->events.get();
        hip_check(hipEventRecord(a, s), "hipEventRecord");
        j.timed.push_back({kind, {a, nullptr}});
    } else {
        hipEvent_t b = ctx->events.get();
        hip_check(hipEventRecord(b, s), "hipEventRecord");
        j.timed.back().second.second = b;
    }
}

void collect_timing(tfstat_ctx *ctx, Job &j) {
    for (auto &t : j.timed) {
        float ms = 0.f;
        if (t.second.second && hipEventElapsedTime(&ms, t.second.first, t.second.second) == hipSuccess) {
            std::lock_guard<std::mutex> g(ctx->mu);
            ctx->k_launches[t.first] += 1;
            ctx->k_ms[t.first] += ms;
        }
        ctx->events.put(t.second.first);
        if (t.second.second) ctx->events.put(t.second.second);
    }
    j.timed.clear();
}

// Allocates the workspace from the arena; false when it does not fit now.
bool alloc_job(tfstat_ctx *ctx, Job &j) {
    j.ws = ctx->arena.alloc(j.ws_bytes);
    return j.ws != nullptr;
}

void release_job(tfstat_ctx *ctx, Job &j) {
    if (j.ws) ctx->arena.release(j.ws);
    j.ws = nullptr;
    if (j.pin) ctx->pinned.put(j.pin, j.pin_bytes);
    j.pin = nullptr;
}

template <typename T>
T *ws_ptr(Job &j, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(j.ws) + off);
}

// Host image of the job's planning tables (the first tables_bytes of its
// workspace).
void fill_tables(const Job &j, char *h) {
    const int n_t0 = (int)j.win.t0.size();
    const int n_tau = (int)j.win.tau.size();
    std::memcpy(h + j.off_rows, j.rows.data(), sizeof(tfs::RowPlan) * n_t0);
    std::memcpy(h + j.off_tau, j.win.tau.data(), sizeof(int64_t) * n_tau);
    std::memcpy(h + j.off_lcol, j.lcol.data(), sizeof(int32_t) * n_tau);
    if (banded(j.win.type) && !j.use_recur) {
        if (j.win.type == TFSTAT_WIN_SHAPE)
            std::memcpy(h + j.off_shape, j.win.shape.data(), sizeof(double) * j.win.shape.size());
        std::memcpy(h + j.off_lblk, j.lblk.data(), sizeof(int32_t) * j.NB);
        std::memcpy(h + j.off_boff, j.blk_off.data(), sizeof(int64_t) * j.NB);
        std::memcpy(h + j.off_order, j.order.data(), sizeof(int32_t) * j.NB);
        if (j.use_mfma) {
            std::memcpy(h + j.off_lg, j.lg.data(), sizeof(int32_t) * j.NB);
            std::memcpy(h + j.off_gshoff, j.gsh_off.data(), sizeof(int64_t) * j.NB);
        }
    }
}

bool wants64(const Job &j) { return j.prec == TFSTAT_PREC_FP64 || j.prec == TFSTAT_PREC_RECUR64; }

tfs::WeightParams weight_params(Job &j) {
    tfs::WeightParams wp{};
    wp.n_tau = (int32_t)j.win.tau.size();
    wp.n_blocks = j.NB;
    wp.R = j.R;
    wp.want64 = wants64(j);
    wp.t_sft = j.at->t_sft;
    wp.tau = ws_ptr<int64_t>(j, j.off_tau);
    wp.lcol = ws_ptr<int32_t>(j, j.off_lcol);
    wp.lblk = ws_ptr<int32_t>(j, j.off_lblk);
    wp.blk_off = ws_ptr<int64_t>(j, j.off_boff);
    wp.g32 = ws_ptr<float>(j, j.off_g32);
    wp.gsq = ws_ptr<double>(j, j.off_gsq);
    wp.g64 = wp.want64 ? ws_ptr<double>(j, j.off_g64) : nullptr;
    if (j.win.type == TFSTAT_WIN_SHAPE) {
        wp.shape = ws_ptr<double>(j, j.off_shape);
        wp.n_shape = (int32_t)j.win.shape.size();
        wp.shape_num = j.win.num;
        wp.shape_den = j.win.den;
        wp.delta = j.rows[0].delta;
    }
    return wp;
}

tfs::ExpValuParams exp_params(Job &j) {
    tfs::ExpValuParams p{};
    p.at = j.at->view();
    p.n_t0 = (int32_t)j.win.t0.size();
    p.n_tau = (int32_t)j.win.tau.size();
    p.n_row_tiles = j.n_row_tiles;
    p.n_list = j.n_valu;
    p.n_tiles = j.n_tiles;
    p.rows = ws_ptr<tfs::RowPlan>(j, j.off_rows);
    p.tau = ws_ptr<int64_t>(j, j.off_tau);
    p.lcol = ws_ptr<int32_t>(j, j.off_lcol);
    p.lblk = ws_ptr<int32_t>(j, j.off_lblk);
    p.blk_off = ws_ptr<int64_t>(j, j.off_boff);
    p.blk_list = ws_ptr<int32_t>(j, j.off_order);
    p.g32 = ws_ptr<float>(j, j.off_g32);
    p.g64 = wants64(j) ? ws_ptr<double>(j, j.off_g64) : nullptr;
    p.gsq = ws_ptr<double>(j, j.off_gsq);
    p.twoF = j.twoF;
    p.part = ws_ptr<tfs::Partial>(j, j.off_part);
    p.abc_out = nullptr;
    if (j.split || (j.use_mfma && j.n_mfma > 0)) {
        // A, B, C of every cell from the A/B/C pass (F_a/F_b-only tiles)
        p.abc_out = ws_ptr<double>(j, j.off_abc);
        p.abc_pitch = abc_pitch((int32_t)j.win.tau.size());
    }
    p.scale_rows = j.win.type == TFSTAT_WIN_EXP ? 1 : 0;
    return p;
}

// Matrix-core parameters of a map planned for the per-row weight form;
// blk_list: the device list of its matrix-core blocks.
tfs::ExpMfmaRowsParams mfma_rows_params(Job &j, const int32_t *blk_list) {
    const AtomsSet &at = *j.at;
    tfs::ExpMfmaRowsParams q{};
    q.n_bins = at.n_bins;
    q.bins16 = at.bins16;
    q.kp = at.kp;
    q.kp_data = (at.K + 31) & ~31;
    q.n_t0 = (int32_t)j.win.t0.size();
    q.n_tau = (int32_t)j.win.tau.size();
    q.n_row_tiles = j.n_row_tiles;
    q.n_col_tiles = at.bins16 / 16;
    q.n_blocks = j.n_mfma;
    q.n_tiles = j.n_tiles;
    q.t_sft = at.t_sft;
    q.rows = ws_ptr<tfs::RowPlan>(j, j.off_rows);
    q.tau = ws_ptr<int64_t>(j, j.off_tau);
    q.blk_list = blk_list;
    q.f16 = j.prec == TFSTAT_PREC_F16X3;
    q.xhi = q.f16 ? at.xhi16 : at.xhi;
    q.xlo = q.f16 ? at.xlo16 : at.xlo;
    q.colexp = q.f16 ? at.colexp : nullptr;
    q.abc_cell = ws_ptr<double>(j, j.off_abc);
    q.abc_pitch = abc_pitch(q.n_tau);
    q.twoF = j.twoF;
    q.part = ws_ptr<tfs::Partial>(j, j.off_part);
    q.chi = q.f16 ? at.chi16 : at.chi;
    q.clo = q.f16 ? at.clo16 : at.clo;
    q.x32 = at.x32;
    q.kpc = at.kpc;
    q.K = at.K;
    return q;
}

// Rows per segment of the A/B/C scan: one wave per (tau, segment), which
// sums the segment's last window directly and scans its rows 64 at a time,
// one dependent chunk after another.  More segments mean shorter chains
// and more waves, and more direct sums; a map takes about 1024 waves, in
// segments of whole 64-row chunks (on the 64-candidate batch the scan took
// 0.76, 0.56, 0.49 and 0.45 ms at 8192, 2048, 1024 and 256 waves per map;
// one map alone needs the waves to fill the GPU, and a map's segments, which
// set its rounding, are the same alone and in a batch).
int32_t abc_seg_rows(const Job &j) {
    const int64_t n_t0 = (int64_t)j.win.t0.size();
    const int64_t n_tau = std::max<int64_t>(1, (int64_t)j.win.tau.size());
    const int64_t chunks = std::max<int64_t>(1, (n_t0 + 63) / 64);
    const int64_t n_seg = std::max<int64_t>(1, std::min<int64_t>((1024 + n_tau - 1) / n_tau, chunks));
    return (int32_t)((chunks + n_seg - 1) / n_seg * 64);
}

// A/B/C of every cell of an exponential-window map by the recurrence over
// t0 rows, into the map's abc_cell buffer (shape windows take the VALU
// A/B/C pass: their weights are not exponential).
tfs::AbcRecurParams abc_recur_params(Job &j) {
    tfs::AbcRecurParams q{};
    q.rows = ws_ptr<tfs::RowPlan>(j, j.off_rows);
    q.tau = ws_ptr<int64_t>(j, j.off_tau);
    q.abc = j.at->abc;
    q.abc_out = ws_ptr<double>(j, j.off_abc);
    q.abc_pitch = abc_pitch((int32_t)j.win.tau.size());
    q.n_t0 = (int32_t)j.win.t0.size();
    q.n_tau = (int32_t)j.win.tau.size();
    q.K = j.at->K;
    q.t_sft = j.at->t_sft;
    q.seg_rows = abc_seg_rows(j);
    return q;
}

tfs::RectParams rect_params(Job &j) {
    tfs::RectParams p{};
    p.K = j.at->K;
    p.n_bins = j.at->n_bins;
    p.n_t0 = (int32_t)j.win.t0.size();
    p.n_tau = (int32_t)j.win.tau.size();
    p.t_sft = j.at->t_sft;
    p.n_tiles_n = j.n_tiles_n;
    p.n_tiles = j.n_tiles;
    p.rows = ws_ptr<tfs::RowPlan>(j, j.off_rows);
    p.tau = ws_ptr<int64_t>(j, j.off_tau);
    p.pabc = ws_ptr<double>(j, j.off_pabc);
    p.px = ws_ptr<double>(j, j.off_px);
    p.twoF = j.twoF;
    p.part = ws_ptr<tfs::Partial>(j, j.off_part);
    return p;
}

tfs::MergeParams merge_params(Job &j) {
    tfs::MergeParams mp{};
    mp.n_tiles = j.n_tiles;
    mp.n_maps = j.at->n_bins;
    mp.n_cells = (int64_t)j.win.t0.size() * (int64_t)j.win.tau.size();
    mp.part = ws_ptr<tfs::Partial>(j, j.off_part);
    mp.out = ws_ptr<tfs::BinResultDev>(j, j.off_res);
    return mp;
}

// The matrix-core form with shifted weight tables (shape windows whose rows
// lie on consecutive slots): the tables, then the kernel, on stream s.
void enqueue_mfma_tables(tfstat_ctx *ctx, Job &j, const tfs::WeightParams &wp, const tfs::ExpValuParams &pa,
                     hipStream_t s) {
    const AtomsSet &at = *j.at;
    const int n_t0 = (int)j.win.t0.size();
    const int n_tau = (int)j.win.tau.size();
    tfs::ExpMfmaParams q{};
    q.n_bins = at.n_bins;
    q.bins16 = at.bins16;
    q.kp = at.kp;
    q.kp_data = (at.K + 31) & ~31;
    q.n_t0 = n_t0;
    q.n_tau = n_tau;
    q.n_row_tiles = j.n_row_tiles;
    q.n_col_tiles = at.bins16 / 16;
    q.n_blocks = j.n_mfma;
    q.n_tiles = j.n_tiles;
    q.k0_first = j.rows[0].k0;
    // the row scale exp(-delta / tau) of exponential windows; shape
    // windows carry their offset in the tables
    q.delta = j.win.type == TFSTAT_WIN_EXP ? j.rows[0].delta : 0;
    q.tau = ws_ptr<int64_t>(j, j.off_tau);
    q.lblk = wp.lblk;
    q.blk_off = wp.blk_off;
    q.blk_list = pa.blk_list;
    q.lg = ws_ptr<int32_t>(j, j.off_lg);
    q.gsh_off = ws_ptr<int64_t>(j, j.off_gshoff);
    q.gsh = ws_ptr<unsigned short>(j, j.off_gsh);
    tfs::ShiftTableParams sp{};
    sp.n_blocks = j.n_mfma;
    sp.blk_list = pa.blk_list;
    sp.lblk = wp.lblk;
    sp.lg = q.lg;
    sp.blk_off = wp.blk_off;
    sp.gsh_off = q.gsh_off;
    sp.g32 = wp.g32;
    sp.gsh = ws_ptr<unsigned short>(j, j.off_gsh);
    record_kernel(ctx, j, TFSTAT_K_WEIGHTS, s, true);
    hip_check(tfs::launch_shift_tables(sp, j.gsh_max, s), "shift tables kernel");
    record_kernel(ctx, j, TFSTAT_K_WEIGHTS, s, false);
    q.xhi = at.xhi;
    q.xlo = at.xlo;
    q.abc_cell = pa.abc_out;
    q.abc_pitch = pa.abc_pitch;
    q.twoF = j.twoF;
    q.part = ws_ptr<tfs::Partial>(j, j.off_part);
    record_kernel(ctx, j, TFSTAT_K_MFMA, s, true);
    hip_check(tfs::launch_exp_mfma(q, s), "exp mfma kernel");
    record_kernel(ctx, j, TFSTAT_K_MFMA, s, false);
}

// Enqueues every step of the map on stream s (tables upload, kernels,
// results download into pinned memory).  The workspace must be allocated.
void enqueue_job(tfstat_ctx *ctx, Job &j, hipStream_t s) {
    const AtomsSet &at = *j.at;
    const int n_t0 = (int)j.win.t0.size();
    const int n_tau = (int)j.win.tau.size();
    const bool is_exp = banded(j.win.type);
    const size_t res_bytes = sizeof(tfs::BinResultDev) * at.n_bins;
    if (!j.pin) j.pin = ctx->pinned.get(std::max(j.tables_bytes, res_bytes), &j.pin_bytes);
    char *h = static_cast<char *>(j.pin);
    fill_tables(j, h);
    hip_check(hipMemcpyAsync(j.ws, h, j.tables_bytes, hipMemcpyHostToDevice, s), "upload tables");

    const auto *tau = ws_ptr<int64_t>(j, j.off_tau);
    auto *part = ws_ptr<tfs::Partial>(j, j.off_part);
    auto *res = ws_ptr<tfs::BinResultDev>(j, j.off_res);

    if (is_exp && j.use_recur) {
        tfs::RecurParams rp{};
        rp.K = at.K;
        rp.n_bins = at.n_bins;
        rp.n_t0 = n_t0;
        rp.n_tau = n_tau;
        rp.t_sft = at.t_sft;
        rp.k0_first = j.recur_k0;
        rp.stride = j.recur_stride;
        rp.delta = j.rows[0].delta;
        rp.n_tiles = j.n_tiles;
        rp.tau = tau;
        rp.abc = at.abc;
        rp.x64 = at.x64;
        rp.npref = at.npref;
        rp.twoF = j.twoF;
        rp.part = part;
        record_kernel(ctx, j, TFSTAT_K_RECUR, s, true);
        hip_check(tfs::launch_exp_recur(rp, j.recur_bg, s), "exp recurrence kernel");
        record_kernel(ctx, j, TFSTAT_K_RECUR, s, false);
    } else if (is_exp) {
        tfs::WeightParams wp = weight_params(j);
        record_kernel(ctx, j, TFSTAT_K_WEIGHTS, s, true);
        hip_check(tfs::launch_weights(wp, j.max_blk, s), "weights kernel");
        record_kernel(ctx, j, TFSTAT_K_WEIGHTS, s, false);

        tfs::ExpValuParams p = exp_params(j);
        // with matrix-core blocks, the VALU blocks take A/B/C from the A/B/C
        // pass (which then covers every block) and sum only F_a, F_b
        const bool split_abc = (j.use_mfma && j.n_mfma > 0) || j.split;
        if (j.split) {
            // A, B, C of every cell, then F_a, F_b only, four bins per lane
            tfs::ExpValuParams pa = p;
            pa.twoF = nullptr;
            record_kernel(ctx, j, TFSTAT_K_ABC, s, true);
            if (j.win.type == TFSTAT_WIN_EXP)
                hip_check(tfs::launch_abc_recur(abc_recur_params(j), s), "abc recurrence kernel");
            else
                hip_check(tfs::launch_exp_abc(pa, s), "exp abc kernel");
            record_kernel(ctx, j, TFSTAT_K_ABC, s, false);
            record_kernel(ctx, j, TFSTAT_K_EXP, s, true);
            hip_check(tfs::launch_exp_fonly(p, j.n_groups, s), "exp F kernel");
            record_kernel(ctx, j, TFSTAT_K_EXP, s, false);
        }
        if (j.n_valu > 0 && !split_abc) {
            record_kernel(ctx, j, TFSTAT_K_EXP, s, true);
            auto launch = j.runs ? tfs::launch_exp_runs : tfs::launch_exp_valu;
            const int pr = wants64(j) ? 0 : 1;
            hip_check(launch(p, pr, j.R, j.BG, j.n_groups, s), "exp kernel");
            if (j.tail2) {
                // the one or two bins after the four-bin groups
                tfs::ExpValuParams pt = p;
                pt.bin_base = 4 * j.n_groups;
                hip_check(launch(pt, pr, j.R, j.at->n_bins % 4, 1, s), "exp kernel (tail bins)");
            }
            record_kernel(ctx, j, TFSTAT_K_EXP, s, false);
        }
        if (j.n_mfma > 0) {
            tfs::ExpValuParams pa = p;
            pa.n_list = j.n_valu + j.n_mfma;
            pa.twoF = nullptr;
            pa.abc_out = ws_ptr<double>(j, j.off_abc);
            pa.abc_pitch = abc_pitch(n_tau);
            record_kernel(ctx, j, TFSTAT_K_ABC, s, true);
            if (j.win.type == TFSTAT_WIN_EXP)
                hip_check(tfs::launch_abc_recur(abc_recur_params(j), s), "abc recurrence kernel");
            else
                hip_check(tfs::launch_exp_abc(pa, s), "exp abc kernel");
            record_kernel(ctx, j, TFSTAT_K_ABC, s, false);
            pa.blk_list = p.blk_list + j.n_valu;   // the matrix-core blocks
            pa.n_list = j.n_mfma;
            if (j.n_valu > 0) {
                tfs::ExpValuParams pf = p;
                pf.abc_out = ws_ptr<double>(j, j.off_abc);
                pf.abc_pitch = abc_pitch(n_tau);
                record_kernel(ctx, j, TFSTAT_K_EXP, s, true);
                hip_check(tfs::launch_exp_fonly(pf, (at.n_bins + 3) / 4, s), "exp F kernel");
                record_kernel(ctx, j, TFSTAT_K_EXP, s, false);
            }
            if (j.mfma_rows) {
                tfs::ExpMfmaRowsParams q = mfma_rows_params(j, pa.blk_list);
                record_kernel(ctx, j, TFSTAT_K_MFMA, s, true);
                hip_check(tfs::launch_exp_mfma_rows(q, s), "exp mfma kernel");
                record_kernel(ctx, j, TFSTAT_K_MFMA, s, false);
            } else {
                enqueue_mfma_tables(ctx, j, wp, pa, s);
            }
        }
    } else {
        double *pabc = ws_ptr<double>(j, j.off_pabc);
        double *px = ws_ptr<double>(j, j.off_px);
        record_kernel(ctx, j, TFSTAT_K_SCAN, s, true);
        hip_check(tfs::launch_scan(at.abc, 4, pabc, at.K, 4, s), "scan kernel");
        hip_check(tfs::launch_scan(at.x64, 4 * (int64_t)at.n_bins, px, at.K, 4 * at.n_bins, s),
                  "scan kernel");
        record_kernel(ctx, j, TFSTAT_K_SCAN, s, false);
        tfs::RectParams p = rect_params(j);
        record_kernel(ctx, j, TFSTAT_K_RECT, s, true);
        hip_check(tfs::launch_rect(p, s), "rect kernel");
        record_kernel(ctx, j, TFSTAT_K_RECT, s, false);
    }
    tfs::MergeParams mp = merge_params(j);
    record_kernel(ctx, j, TFSTAT_K_MERGE, s, true);
    hip_check(tfs::launch_merge(mp, s), "merge kernel");
    record_kernel(ctx, j, TFSTAT_K_MERGE, s, false);
    hip_check(hipMemcpyAsync(j.pin, res, res_bytes, hipMemcpyDeviceToHost, s), "download results");
}

// Per-bin results of a job from the device reduction records r.
void convert_results(const Job &j, const tfs::BinResultDev *r, tfstat_bin_result *out) {
    const int64_t n_tau = (int64_t)j.win.tau.size();
    for (int b = 0; b < j.at->n_bins; ++b) {
        tfstat_bin_result o{};
        o.max2F = r[b].max2F;
        o.logB = r[b].logB;
        const int64_t idx = r[b].idx;
        o.m = (int32_t)(idx / n_tau);
        o.n = (int32_t)(idx % n_tau);
        o.t0 = j.win.t0[o.m];
        o.tau = j.win.tau[o.n];
        out[b] = o;
    }
}

void finish_job(tfstat_ctx *ctx, Job &j, tfstat_bin_result *out) {
    collect_timing(ctx, j);
    convert_results(j, static_cast<const tfs::BinResultDev *>(j.pin), out);
}

// hi / lo planes of the data atoms for the matrix-core path (bf16, or for
// F16X3 half precision with per-column scale exponents); built once per
// atoms set and part type on the context stream.  Caller holds ctx->mu.
void ensure_planes(tfstat_ctx *ctx, AtomsSet *at, int32_t prec) {
    const bool f16 = prec == TFSTAT_PREC_F16X3;
    if (f16 ? at->planes16 != nullptr : at->planes != nullptr) return;
    const int32_t bins16 = (at->n_bins + 15) / 16 * 16;
    const int32_t kp = (at->K + 31) / 32 * 32 + 32;
    const size_t plane = sizeof(unsigned short) * 4 * (size_t)bins16 * kp;
    const size_t plane_b = round_up(plane, 256);
    const size_t exp_b = f16 ? round_up(sizeof(int32_t) * 4 * (size_t)bins16, 256) : 0;
    // the transposed form's column planes (kCellsCopies copies, both parts)
    const bool cells = tfs::mfma_cells_form(bins16 / 16);
    const int32_t kpc = tfs::cells_plane_pitch(at->K);
    const size_t cplane_b =
        cells ? round_up(sizeof(unsigned short) * 4 * tfs::kCellsCopies * (size_t)at->n_bins * kpc, 256) : 0;
    void *mem = ctx->arena.alloc(2 * plane_b + exp_b + 2 * cplane_b);
    if (!mem) raise(TFSTAT_E_NOMEM, "arena cannot hold the matrix-core planes");
    try {
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        auto *xhi = static_cast<unsigned short *>(mem);
        auto *xlo = reinterpret_cast<unsigned short *>(static_cast<char *>(mem) + plane_b);
        auto *colexp = f16 ? reinterpret_cast<int32_t *>(static_cast<char *>(mem) + 2 * plane_b) : nullptr;
        hip_check(tfs::launch_build_planes(at->x32, at->K, at->n_bins, bins16, kp, colexp, xhi, xlo,
                                           ctx->stream),
                  "planes kernel");
        unsigned short *chi = nullptr, *clo = nullptr;
        if (cells) {
            char *base = static_cast<char *>(mem) + 2 * plane_b + exp_b;
            chi = reinterpret_cast<unsigned short *>(base);
            clo = reinterpret_cast<unsigned short *>(base + cplane_b);
            hip_check(tfs::launch_build_cplanes(at->x32, at->K, at->n_bins, bins16, kpc, colexp, chi, clo,
                                                ctx->stream),
                      "column planes kernel");
        }
        hip_check(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
        if (f16) {
            at->xhi16 = xhi;
            at->xlo16 = xlo;
            at->colexp = colexp;
            at->chi16 = chi;
            at->clo16 = clo;
        } else {
            at->xhi = xhi;
            at->xlo = xlo;
            at->chi = chi;
            at->clo = clo;
        }
    } catch (...) {
        ctx->arena.release(mem);
        throw;
    }
    (f16 ? at->planes16 : at->planes) = mem;
    at->bins16 = bins16;
    at->kp = kp;
    at->kpc = kpc;
    at->bytes += 2 * plane_b + exp_b + 2 * cplane_b;
}

AtomsSet *find_atoms(tfstat_ctx *ctx, tfstat_atoms_id id) {
    auto it = ctx->atoms.find(id);
    if (it == ctx->atoms.end()) raise(TFSTAT_E_NOTFOUND, "unknown atoms id");
    return it->second.get();
}

template <typename F>
int guarded(F &&f) {
    try {
        return f();
    } catch (const Failure &e) {
        return fail(e.code, e.msg);
    } catch (const std::bad_alloc &) {
        return fail(TFSTAT_E_NOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(TFSTAT_E_INVAL, e.what());
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Uneven batch: all maps in one workspace, one shared tile list, one
// persistent fused launch, replayed as a captured HIP graph.
// ---------------------------------------------------------------------------
struct tfstat_batch {
    int prec = TFSTAT_PREC_FP32;
    int variant = 0;
    int groups = 0;
    std::vector<std::unique_ptr<Job>> owned;   // maps planned by the batch itself
    std::vector<Job *> jobs;                   // every map of the batch, in result order
    std::vector<int32_t> res_off;   // first result of each map
    int n_results = 0;
    int n_tiles = 0;
    void *ws = nullptr;
    void *pin = nullptr;
    size_t pin_bytes = 0;
    tfs::FusedParams fp{};
    tfs::WeightBatchParams wbp{};
    const tfs::ScanJob *scan_jobs = nullptr;
    int n_scan = 0;
    tfs::MergeBatchParams mbp{};
    tfs::AbcBatchParams abp{};       // A/B/C pre-pass of the split-form and matrix-core maps
    tfs::MfmaBatchParams mfp{};      // matrix-core work of the BF16X3 / F16X3 maps
    tfs::AbcRecurBatchParams rap{};  // recurrence A/B/C of exponential split and matrix-core maps
    tfs::BinResultDev *res_dev = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;    // around each graph launch
    hipEvent_t evf0 = nullptr, evf1 = nullptr;  // around the fused launch (timed runs)
    hipEvent_t evm1 = nullptr;                  // after the matrix-core launch (timed runs)
    double tune_ms = 0.0, last_ms = 0.0, last_fused_ms = 0.0, last_mfma_ms = 0.0;
    bool holds_atoms = false;
};

namespace {

// Tile shape of a map in the mixed variant: the widest bin group its bins fill.
int mixed_shape(int prec, int n_bins) {
    if (prec == TFSTAT_PREC_FP64) return tfs::kShapeD41;
    if (n_bins >= 4) return tfs::kShapeF44;
    if (n_bins >= 2) return tfs::kShapeF42;
    return tfs::kShapeF81;
}

void batch_drop_graph(tfstat_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

void batch_release(tfstat_ctx *ctx, tfstat_batch *b) {
    batch_drop_graph(b);
    for (hipEvent_t *e : {&b->ev0, &b->ev1, &b->evf0, &b->evf1, &b->evm1}) {
        if (*e) ctx->events.put(*e);
        *e = nullptr;
    }
    std::lock_guard<std::mutex> g(ctx->mu);
    if (b->ws) ctx->arena.release(b->ws);
    b->ws = nullptr;
    if (b->pin) ctx->pinned.put(b->pin, b->pin_bytes);
    b->pin = nullptr;
    if (b->holds_atoms)
        for (Job *j : b->jobs) j->at->busy -= 1;
    b->holds_atoms = false;
}

// Tile shape of a planned exponential map (from its precision and R, BG).
int job_shape(const Job &j) {
    if (j.prec == TFSTAT_PREC_FP64) return tfs::kShapeD41;
    if (j.R == 8) return tfs::kShapeF81;
    return j.BG == 2 ? tfs::kShapeF42 : tfs::kShapeF44;
}

// Lays out one workspace for the planned maps b->jobs (plain FP32 or FP64
// exponential maps of the batch's variant, or rectangular maps), builds the
// shared tile list and every descriptor, and uploads them on stream s (then
// waits for the stream when sync).  Returns false, with nothing allocated,
// when the arena cannot hold the workspace.  have_lock: the caller holds
// ctx->mu.
bool batch_layout(tfstat_ctx *ctx, tfstat_batch *b, hipStream_t s, bool sync, bool have_lock) {
    const int32_t n = (int32_t)b->jobs.size();
    std::vector<int> shape(n, -1), eidx(n, -1), ridx(n, -1), midx(n, -1);
    int n_exp = 0, n_rect = 0, n_went = 0, n_scan = 0, n_abc = 0, n_mfma_maps = 0, n_rabc_maps = 0;
    size_t n_rabc = 0;   // recurrence A/B/C entries (exponential windows)
    std::vector<int> aidx(n, -1);
    size_t n_mfma_entries = 0, n_cells_entries = 0;   // matrix-core work items (transposed form first)
    int32_t max_chunks = 1;
    b->res_off.assign(n, 0);
    b->n_results = 0;
    for (int32_t i = 0; i < n; ++i) {
        Job &j = *b->jobs[i];
        if (banded(j.win.type)) {
            if (j.use_mfma && !j.mfma_rows)
                raise(TFSTAT_E_INVAL, "a batch runs no matrix-core shape windows (use tfstat_fmap)");
            shape[i] = job_shape(j);
            eidx[i] = n_exp++;
            // weight tables: every block, except the matrix-core blocks of
            // maps whose matrix-core kernels make their weights in registers
            n_went += (j.use_mfma && j.mfma_rows) ? j.n_valu : j.NB;
            // A/B/C of every cell of split and matrix-core maps: the
            // recurrence for exponential windows, the VALU pass (every
            // block) for shape windows
            if (j.split || j.use_mfma) {
                if (j.win.type == TFSTAT_WIN_EXP) {
                    aidx[i] = n_rabc_maps++;
                    tfs::AbcRecurParams q{};
                    q.n_t0 = (int32_t)j.win.t0.size();
                    q.n_tau = (int32_t)j.win.tau.size();
                    q.seg_rows = abc_seg_rows(j);
                    n_rabc += (size_t)tfs::abc_recur_blocks(q);
                } else {
                    n_abc += (j.n_valu + j.n_mfma) * j.n_row_tiles;
                }
            }
            if (j.use_mfma) {
                // matrix-core work of the long-band blocks
                midx[i] = n_mfma_maps++;
                const size_t ne = (size_t)tfs::mfma_units(j.n_mfma, j.at->bins16 / 16) * j.n_row_tiles *
                                  tfs::mfma_col_items(j.at->bins16 / 16, j.at->n_bins);
                n_mfma_entries += ne;
                if (tfs::mfma_cells_form(j.at->bins16 / 16)) n_cells_entries += ne;
            }
            int64_t mb = j.max_blk;   // the largest table this map's entries make
            if (j.use_mfma && j.mfma_rows) {
                mb = 0;
                for (int q = 0; q < j.n_valu; ++q) mb = std::max<int64_t>(mb, (int64_t)j.lblk[j.order[q]] * j.R);
            }
            max_chunks = std::max<int32_t>(max_chunks, (int32_t)std::min<int64_t>((mb + 255) / 256, 4096));
        } else {
            ridx[i] = n_rect++;
            n_scan += 1 + (4 * j.at->n_bins + 63) / 64;
        }
        b->res_off[i] = b->n_results;
        b->n_results += j.at->n_bins;
    }

    // shared tile list, largest expected cost first (per-lane FMA counts):
    // tiles of one (map, tau block) cost the same, so the groups are sorted
    // and then expanded; rect tiles (all alike and short) go last
    struct Group {
        int32_t map, q;
        double cost;
    };
    std::vector<Group> groups_e;
    size_t n_tiles_total = 0;
    for (int32_t i = 0; i < n; ++i) {
        Job &j = *b->jobs[i];
        if (eidx[i] >= 0) {
            // split maps, and the VALU blocks of matrix-core maps:
            // F_a/F_b-only tiles of bin pairs
            const bool fonly = j.split || j.use_mfma;
            const int bgs = fonly ? (j.at->n_bins + 1) / 2 : j.n_groups + (j.tail2 ? 1 : 0);
            const size_t per = (size_t)j.n_row_tiles * bgs;
            // a runs tile takes four blocks, each over its whole band on one
            // wave: about four times the time of one block's tile
            const int step = j.runs ? 4 : 1;
            const int per_step = fonly ? 4 * 2 : 3 + 4 * j.BG;   // FMAs per lane, slot and tau
            for (int q = 0; q < j.n_valu; q += step)
                groups_e.push_back({i, q, (double)(j.lblk[j.order[q]] + 1) * j.R * per_step * step});
            n_tiles_total += per * ((j.n_valu + step - 1) / step);
        } else {
            const int ny = ((int)j.win.t0.size() + tfs::kRectRows - 1) / tfs::kRectRows;
            n_tiles_total += (size_t)ny * j.n_tiles_n * ((j.at->n_bins + tfs::kRectBins - 1) / tfs::kRectBins);
        }
    }
    if (n_tiles_total > (size_t)INT32_MAX / 2 || n_mfma_entries > (size_t)INT32_MAX / 2 ||
        n_rabc > (size_t)INT32_MAX / 2)
        raise(TFSTAT_E_INVAL, "batch has too many tiles");
    std::stable_sort(groups_e.begin(), groups_e.end(),
                     [](const Group &a, const Group &c) { return a.cost > c.cost; });
    std::vector<tfs::BatchTile> tiles;
    tiles.reserve(n_tiles_total);
    for (const Group &g : groups_e) {
        const Job &j = *b->jobs[g.map];
        const bool fonly = j.split || j.use_mfma;
        const int kind = j.runs ? 2 : (fonly ? 3 : 0);
        const int ng = fonly ? (j.at->n_bins + 1) / 2 : j.n_groups;
        for (int rt = 0; rt < j.n_row_tiles; ++rt) {
            for (int gidx = 0; gidx < ng; ++gidx)
                tiles.push_back(tfs::BatchTile{kind, eidx[g.map], g.q, rt, gidx, shape[g.map]});
            // the one or two bins after the four-bin groups: group index in
            // units of the tail's bins per lane
            if (j.tail2) {
                const bool one = j.at->n_bins % 4 == 1;
                tiles.push_back(tfs::BatchTile{kind, eidx[g.map], g.q, rt, (one ? 4 : 2) * j.n_groups,
                                               one ? tfs::kShapeF41 : tfs::kShapeF42});
            }
        }
    }
    for (int32_t i = 0; i < n; ++i) {
        if (ridx[i] < 0) continue;
        const Job &j = *b->jobs[i];
        const int ny = ((int)j.win.t0.size() + tfs::kRectRows - 1) / tfs::kRectRows;
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < j.n_tiles_n; ++x)
                for (int bg = 0; bg < (j.at->n_bins + tfs::kRectBins - 1) / tfs::kRectBins; ++bg)
                    tiles.push_back(tfs::BatchTile{1, ridx[i], x, y, bg, 0});
    }
    b->n_tiles = (int)tiles.size();

    // workspace layout
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at_ = o;
        o = round_up(o + std::max<size_t>(bytes, 1), 256);
        return at_;
    };
    std::vector<size_t> job_off(n);
    for (int32_t i = 0; i < n; ++i) job_off[i] = take(b->jobs[i]->ws_bytes);
    const size_t desc_begin = o;
    const size_t off_ep = take(sizeof(tfs::ExpValuParams) * n_exp);
    const size_t off_rp = take(sizeof(tfs::RectParams) * n_rect);
    const size_t off_wp = take(sizeof(tfs::WeightParams) * n_exp);
    const size_t off_wjob = take(sizeof(int32_t) * n_went);
    const size_t off_wblk = take(sizeof(int32_t) * n_went);
    const size_t off_scan = take(sizeof(tfs::ScanJob) * n_scan);
    const size_t off_mp = take(sizeof(tfs::MergeParams) * n);
    const size_t off_mjob = take(sizeof(int32_t) * b->n_results);
    const size_t off_mmap = take(sizeof(int32_t) * b->n_results);
    const size_t off_tiles = take(sizeof(tfs::BatchTile) * tiles.size());
    const size_t off_ajob = take(sizeof(int32_t) * n_abc);
    const size_t off_ax = take(sizeof(int32_t) * n_abc);
    const size_t off_ay = take(sizeof(int32_t) * n_abc);
    const size_t off_mfp = take(sizeof(tfs::ExpMfmaRowsParams) * n_mfma_maps);
    const size_t off_ment = take(sizeof(int32_t) * 4 * n_mfma_entries);
    const size_t off_rap = take(sizeof(tfs::AbcRecurParams) * n_rabc_maps);
    const size_t off_rent = take(sizeof(int32_t) * 2 * n_rabc);
    const size_t desc_end = o;
    const size_t off_counter = take(sizeof(int32_t));
    const size_t off_res = take(sizeof(tfs::BinResultDev) * b->n_results);
    const size_t ws_bytes = o;
    if (have_lock) {
        b->ws = ctx->arena.alloc(ws_bytes);
    } else {
        std::lock_guard<std::mutex> g(ctx->mu);
        b->ws = ctx->arena.alloc(ws_bytes);
    }
    if (!b->ws) return false;
    char *ws = static_cast<char *>(b->ws);
    for (int32_t i = 0; i < n; ++i) b->jobs[i]->ws = ws + job_off[i];

    // host image of every table and descriptor
    size_t tables_total = 0;
    for (auto &j : b->jobs) tables_total += round_up(j->tables_bytes, 256);
    const size_t desc_bytes = desc_end - desc_begin;
    b->pin = ctx->pinned.get(std::max(tables_total + desc_bytes, sizeof(tfs::BinResultDev) * b->n_results),
                             &b->pin_bytes);
    char *h = static_cast<char *>(b->pin);
    char *hd = h + tables_total;          // descriptors, at ws offset desc_begin
    auto hptr = [&](size_t off) { return hd + (off - desc_begin); };
    auto dptr = [&](size_t off) { return ws + off; };
    auto *ep = reinterpret_cast<tfs::ExpValuParams *>(hptr(off_ep));
    auto *rp = reinterpret_cast<tfs::RectParams *>(hptr(off_rp));
    auto *wp = reinterpret_cast<tfs::WeightParams *>(hptr(off_wp));
    auto *wjob = reinterpret_cast<int32_t *>(hptr(off_wjob));
    auto *wblk = reinterpret_cast<int32_t *>(hptr(off_wblk));
    auto *scan = reinterpret_cast<tfs::ScanJob *>(hptr(off_scan));
    auto *mp = reinterpret_cast<tfs::MergeParams *>(hptr(off_mp));
    auto *mjob = reinterpret_cast<int32_t *>(hptr(off_mjob));
    auto *mmap = reinterpret_cast<int32_t *>(hptr(off_mmap));
    auto *tl = reinterpret_cast<tfs::BatchTile *>(hptr(off_tiles));
    auto *ajob = reinterpret_cast<int32_t *>(hptr(off_ajob));
    auto *ax = reinterpret_cast<int32_t *>(hptr(off_ax));
    auto *ay = reinterpret_cast<int32_t *>(hptr(off_ay));
    auto *mfp = reinterpret_cast<tfs::ExpMfmaRowsParams *>(hptr(off_mfp));
    auto *ment = reinterpret_cast<int32_t *>(hptr(off_ment));
    auto *rap = reinterpret_cast<tfs::AbcRecurParams *>(hptr(off_rap));
    auto *rent = reinterpret_cast<int32_t *>(hptr(off_rent));
    size_t re = 0;
    int we = 0, se = 0, me = 0, ae = 0;
    size_t mfc = 0, mfe = n_cells_entries;   // next transposed-form and other matrix-core entry
    for (int32_t i = 0; i < n; ++i) {
        Job &j = *b->jobs[i];
        if (eidx[i] >= 0) {
            ep[eidx[i]] = exp_params(j);
            wp[eidx[i]] = weight_params(j);
            const bool regs = j.use_mfma && j.mfma_rows;
            for (int q = 0; q < (regs ? j.n_valu : j.NB); ++q) {
                wjob[we] = eidx[i];
                wblk[we] = regs ? j.order[q] : q;
                ++we;
            }
            if (aidx[i] >= 0) {
                rap[aidx[i]] = abc_recur_params(j);
                const int64_t nb = tfs::abc_recur_blocks(rap[aidx[i]]);
                for (int64_t bk = 0; bk < nb; ++bk) {
                    rent[2 * re + 0] = aidx[i];
                    rent[2 * re + 1] = (int32_t)bk;
                    ++re;
                }
            } else if (j.split || j.use_mfma) {
                // longest bands first, as in the tile list (matrix-core maps:
                // every block, the matrix-core ones included)
                for (int q = 0; q < j.n_valu + j.n_mfma; ++q)
                    for (int rt = 0; rt < j.n_row_tiles; ++rt) {
                        ajob[ae] = eidx[i];
                        ax[ae] = q;
                        ay[ae] = rt;
                        ++ae;
                    }
            }
            if (j.use_mfma) {
                const int32_t *blk = reinterpret_cast<const int32_t *>(ws_ptr<char>(j, j.off_order)) + j.n_valu;
                mfp[midx[i]] = mfma_rows_params(j, blk);
                const int n_ct = tfs::mfma_col_items(j.at->bins16 / 16, j.at->n_bins);
                const int n_u = tfs::mfma_units(j.n_mfma, j.at->bins16 / 16);
                // the transposed form's items first (a launch of their own)
                size_t &pos = tfs::mfma_cells_form(j.at->bins16 / 16) ? mfc : mfe;
                for (int q = 0; q < n_u; ++q)
                    for (int rt = 0; rt < j.n_row_tiles; ++rt)
                        for (int ct = 0; ct < n_ct; ++ct) {
                            ment[4 * pos + 0] = midx[i];
                            ment[4 * pos + 1] = q;
                            ment[4 * pos + 2] = rt;
                            ment[4 * pos + 3] = ct;
                            ++pos;
                        }
            }
        } else {
            rp[ridx[i]] = rect_params(j);
            double *pabc = ws_ptr<double>(j, j.off_pabc);
            double *px = ws_ptr<double>(j, j.off_px);
            scan[se++] = tfs::ScanJob{j.at->abc, pabc, 4, j.at->K, 4, 0, 0};
            const int32_t C = 4 * j.at->n_bins;
            for (int c = 0; c < (C + 63) / 64; ++c)
                scan[se++] = tfs::ScanJob{j.at->x64, px, (int64_t)C, j.at->K, C, c, 0};
        }
        mp[i] = merge_params(j);
        mp[i].out = reinterpret_cast<tfs::BinResultDev *>(dptr(off_res)) + b->res_off[i];
        for (int bin = 0; bin < j.at->n_bins; ++bin) {
            mjob[me] = i;
            mmap[me] = bin;
            ++me;
        }
    }
    std::memcpy(tl, tiles.data(), sizeof(tfs::BatchTile) * tiles.size());

    b->fp.exp_jobs = reinterpret_cast<const tfs::ExpValuParams *>(dptr(off_ep));
    b->fp.rect_jobs = reinterpret_cast<const tfs::RectParams *>(dptr(off_rp));
    b->fp.tiles = reinterpret_cast<const tfs::BatchTile *>(dptr(off_tiles));
    b->fp.n_tiles = b->n_tiles;
    b->fp.counter = reinterpret_cast<int32_t *>(dptr(off_counter));
    b->wbp.jobs = reinterpret_cast<const tfs::WeightParams *>(dptr(off_wp));
    b->wbp.job = reinterpret_cast<const int32_t *>(dptr(off_wjob));
    b->wbp.blk = reinterpret_cast<const int32_t *>(dptr(off_wblk));
    b->wbp.n_entries = n_went;
    b->wbp.chunks = max_chunks;
    b->scan_jobs = reinterpret_cast<const tfs::ScanJob *>(dptr(off_scan));
    b->n_scan = n_scan;
    b->abp.jobs = b->fp.exp_jobs;
    b->abp.job = reinterpret_cast<const int32_t *>(dptr(off_ajob));
    b->abp.x = reinterpret_cast<const int32_t *>(dptr(off_ax));
    b->abp.y = reinterpret_cast<const int32_t *>(dptr(off_ay));
    b->abp.n_entries = n_abc;
    b->rap.jobs = reinterpret_cast<const tfs::AbcRecurParams *>(dptr(off_rap));
    b->rap.entries = reinterpret_cast<const int32_t *>(dptr(off_rent));
    b->rap.n_entries = (int32_t)n_rabc;
    b->mfp.jobs = reinterpret_cast<const tfs::ExpMfmaRowsParams *>(dptr(off_mfp));
    b->mfp.entries = reinterpret_cast<const int32_t *>(dptr(off_ment));
    if (mfc != n_cells_entries || mfe != n_mfma_entries) raise(TFSTAT_E_INVAL, "internal: matrix-core entry count");
    b->mfp.n_entries = (int32_t)mfe;
    b->mfp.n_cells = (int32_t)n_cells_entries;
    b->mfp.f16 = b->prec == TFSTAT_PREC_F16X3;
    b->mbp.jobs = reinterpret_cast<const tfs::MergeParams *>(dptr(off_mp));
    b->mbp.job = reinterpret_cast<const int32_t *>(dptr(off_mjob));
    b->mbp.map = reinterpret_cast<const int32_t *>(dptr(off_mmap));
    b->mbp.n_entries = b->n_results;
    b->res_dev = reinterpret_cast<tfs::BinResultDev *>(dptr(off_res));

    size_t ho = 0;
    for (auto &j : b->jobs) {
        fill_tables(*j, h + ho);
        hip_check(hipMemcpyAsync(j->ws, h + ho, j->tables_bytes, hipMemcpyHostToDevice, s), "upload tables");
        ho += round_up(j->tables_bytes, 256);
    }
    hip_check(hipMemcpyAsync(ws + desc_begin, hd, desc_bytes, hipMemcpyHostToDevice, s), "upload descriptors");
    if (sync) hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    for (hipEvent_t *e : {&b->ev0, &b->ev1, &b->evf0, &b->evf1, &b->evm1})
        if (!*e) *e = ctx->events.get();
    return true;
}

// Plans every map with the variant's tile shapes; then lays the batch out.
void batch_build(tfstat_ctx *ctx, tfstat_batch *b, int32_t n, const tfstat_atoms_id *ids,
                 const tfstat_window *wins) {
    const int prec = b->prec;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        for (int32_t i = 0; i < n; ++i) {
            auto j = std::make_unique<Job>();
            j->at = find_atoms(ctx, ids[i]);
            b->owned.push_back(std::move(j));
        }
        for (auto &j : b->owned) {
            j->at->busy += 1;
            b->jobs.push_back(j.get());
        }
        b->holds_atoms = true;
        if (matrix_prec(prec))
            for (auto &j : b->owned) ensure_planes(ctx, j->at, prec);
    }
    for (int32_t i = 0; i < n; ++i) {
        Job &j = *b->jobs[i];
        j.win = copy_window(&wins[i]);
        j.prec = prec;
        if (banded(j.win.type)) {
            const int vs = tfs::fused_shape(b->variant);
            const int sh = vs == tfs::kShapeMixed ? mixed_shape(prec, j.at->n_bins) : vs;
            int sp = 0, R = 0, BG = 0;
            tfs::shape_dims(sh, &sp, &R, &BG);
            if ((sp == 0) != (prec == TFSTAT_PREC_FP64))
                raise(TFSTAT_E_INVAL, "tile shape does not match the precision");
            j.force_R = R;
            j.force_BG = BG;
        }
        j.runs_min_spread = ctx->runs_min_spread.load();
        j.split_min_bins = ctx->split_min_bins.load();
        plan_job(j);
    }
    if (!batch_layout(ctx, b, ctx->batch_stream, true, false))
        raise(TFSTAT_E_NOMEM, "arena cannot hold the batch workspace");
}

// One run of the batch on stream s: counter reset, weight tables, prefix
// sums, the persistent fused launch (bracketed by evf0/evf1 when timed),
// merges, results to host.
hipError_t batch_enqueue(tfstat_batch *b, hipStream_t s, bool timed) {
    hipError_t e = tfs::launch_fill_i32(b->fp.counter, 1, 0, s);
    if (e == hipSuccess) e = tfs::launch_weights_batch(b->wbp, s);
    if (e == hipSuccess) e = tfs::launch_scan_batch(b->scan_jobs, b->n_scan, s);
    if (e == hipSuccess) e = tfs::launch_abc_batch(b->abp, s);
    if (e == hipSuccess) e = tfs::launch_abc_recur_batch(b->rap, s);
    if (e == hipSuccess && timed) e = hipEventRecord(b->evf0, s);
    if (e == hipSuccess) e = tfs::launch_fused(b->fp, b->variant, b->groups, s);
    if (e == hipSuccess && timed) e = hipEventRecord(b->evf1, s);
    if (e == hipSuccess) e = tfs::launch_mfma_batch(b->mfp, s);
    if (e == hipSuccess && timed) e = hipEventRecord(b->evm1, s);
    if (e == hipSuccess) e = tfs::launch_merge_batch(b->mbp, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->pin, b->res_dev, sizeof(tfs::BinResultDev) * b->n_results,
                           hipMemcpyDeviceToHost, s);
    return e;
}

// Captures one run of the batch as a graph.
void batch_capture(tfstat_ctx *ctx, tfstat_batch *b) {
    batch_drop_graph(b);
    hipStream_t s = ctx->batch_stream;
    hip_check(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    const hipError_t e = batch_enqueue(b, s, false);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(s, &g);
    if (e != hipSuccess || ec != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        hip_check(e != hipSuccess ? e : ec, "batch graph capture");
    }
    b->graph = g;
    hip_check(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
}

// The same run launched directly (not from the graph), timing the fused
// launch with HIP events.
void batch_run_timed(tfstat_ctx *ctx, tfstat_batch *b) {
    hipStream_t s = ctx->batch_stream;
    hip_check(hipEventRecord(b->ev0, s), "hipEventRecord");
    hip_check(batch_enqueue(b, s, true), "batch launch");
    hip_check(hipEventRecord(b->ev1, s), "hipEventRecord");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    float ms = 0.f, fms = 0.f, mms = 0.f;
    hip_check(hipEventElapsedTime(&ms, b->ev0, b->ev1), "hipEventElapsedTime");
    hip_check(hipEventElapsedTime(&fms, b->evf0, b->evf1), "hipEventElapsedTime");
    hip_check(hipEventElapsedTime(&mms, b->evf1, b->evm1), "hipEventElapsedTime");
    b->last_ms = ms;
    b->last_fused_ms = fms;
    b->last_mfma_ms = b->mfp.n_entries > 0 ? mms : 0.0;
}

void batch_launch(tfstat_ctx *ctx, tfstat_batch *b) {
    hipStream_t s = ctx->batch_stream;
    hip_check(hipEventRecord(b->ev0, s), "hipEventRecord");
    hip_check(hipGraphLaunch(b->exec, s), "hipGraphLaunch");
    hip_check(hipEventRecord(b->ev1, s), "hipEventRecord");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, b->ev0, b->ev1), "hipEventElapsedTime");
    b->last_ms = ms;
}

std::string batch_signature(tfstat_ctx *ctx, int32_t n, const tfstat_atoms_id *ids,
                            const tfstat_window *wins, int prec) {
    std::string sig = std::to_string(prec);
    std::lock_guard<std::mutex> g(ctx->mu);
    for (int32_t i = 0; i < n; ++i) {
        const AtomsSet *at = find_atoms(ctx, ids[i]);
        sig += "|" + std::to_string(wins[i].type) + "," + std::to_string(at->K) + "," +
               std::to_string(at->n_bins) + "," + std::to_string(wins[i].n_t0) + "," +
               std::to_string(wins[i].n_tau);
    }
    return sig;
}

void ensure_batch_stream(tfstat_ctx *ctx) {
    if (ctx->batch_stream) return;
    hip_check(hipSetDevice(ctx->device), "hipSetDevice");
    hip_check(hipStreamCreateWithFlags(&ctx->batch_stream, hipStreamNonBlocking), "hipStreamCreate");
    hip_check(hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device),
              "hipDeviceGetAttribute");
}

// ---------------------------------------------------------------------------
// Serving loop (continuous batching).  Whenever a stream slot is free, the
// requests at the head of the queue are admitted together -- up to
// serve_max_batch of them, as many as the arena can hold -- and run as one
// fused batch (one persistent launch over all their tiles) on that slot;
// requests that the fused kernel does not cover (matrix-core and recurrence
// precisions) and large requests run alone.  Up to kSlots admissions are in
// flight at once, so
// requests arriving while others run overlap with them on the device.  A
// request's results do not depend on what it was batched with.
// ---------------------------------------------------------------------------
// Requests whose own kernels run longer than about a millisecond gain
// nothing from sharing a launch, and would hold the results of the small
// requests fused with them until they finish: they run alone.  Work is
// counted in window terms (cell x slot x bin, or cell x bin for rect).
constexpr double kServeFuseMaxWork = 2e9;

double est_work(const Job &j) {
    const double cells_bins = (double)j.win.t0.size() * (double)j.at->n_bins;
    if (!banded(j.win.type)) return cells_bins * (double)j.win.tau.size();
    double band = 0.0;   // sum over taus of the band length, from the block tables
    for (int q = 0; q < j.NB; ++q) {
        // matrix-core blocks: about a quarter of the VALU time per term
        const double w = q >= j.n_valu ? 0.25 : 1.0;
        band += w * (double)j.lblk[j.order[q]] * j.R;
    }
    return cells_bins * band;
}

bool fusable(const Job &j) {
    return (j.prec == TFSTAT_PREC_FP32 || j.prec == TFSTAT_PREC_FP64 || matrix_prec(j.prec)) &&
           !(j.use_mfma && !j.mfma_rows) && !j.use_recur && est_work(j) <= kServeFuseMaxWork;
}

void worker_loop(tfstat_ctx *ctx) {
    (void)hipSetDevice(ctx->device);
    std::unique_lock<std::mutex> lk(ctx->mu);
    while (true) {
        bool progressed = false;
        // completions
        for (int s = 0; s < tfstat_ctx::kSlots; ++s) {
            if (ctx->slot_tickets[s].empty()) continue;
            const hipError_t q = hipEventQuery(ctx->slot_done[s]);
            if (q == hipErrorNotReady) continue;
            std::unique_ptr<tfstat_batch> b = std::move(ctx->slot_batch[s]);
            const std::vector<uint64_t> ids = std::move(ctx->slot_tickets[s]);
            ctx->slot_tickets[s].clear();
            for (size_t i = 0; i < ids.size(); ++i) {
                auto &t = ctx->tickets[ids[i]];
                if (q == hipSuccess) {
                    t.res.resize(t.job->at->n_bins);
                    if (b) {
                        convert_results(*t.job, static_cast<const tfs::BinResultDev *>(b->pin) + b->res_off[i],
                                        t.res.data());
                    } else {
                        lk.unlock();
                        finish_job(ctx, *t.job, t.res.data());
                        lk.lock();
                    }
                    t.state = t.cancel_requested ? tfstat_ctx::Ticket::CANCELLED : tfstat_ctx::Ticket::DONE;
                } else {
                    t.state = tfstat_ctx::Ticket::FAILED;
                    t.err = TFSTAT_E_DEVICE;
                    t.msg = std::string("request failed on the device: ") + hipGetErrorString(q);
                }
                t.job->at->busy -= 1;
                if (b)
                    t.job->ws = nullptr;   // inside the batch workspace
                else
                    release_job(ctx, *t.job);
            }
            ctx->events.put(ctx->slot_done[s]);
            ctx->slot_done[s] = nullptr;
            if (b) {
                lk.unlock();
                batch_release(ctx, b.get());
                lk.lock();
            }
            progressed = true;
        }
        // admissions
        while (!ctx->queue.empty()) {
            int slot = -1;
            for (int s = 0; s < tfstat_ctx::kSlots; ++s)
                if (ctx->slot_tickets[s].empty()) {
                    slot = s;
                    break;
                }
            if (slot < 0) break;
            const uint64_t id = ctx->queue.front();
            auto it = ctx->tickets.find(id);
            if (it == ctx->tickets.end() || it->second.cancel_requested) {
                if (it != ctx->tickets.end()) {
                    it->second.state = tfstat_ctx::Ticket::CANCELLED;
                    if (it->second.job) it->second.job->at->busy -= 1;
                }
                ctx->queue.pop_front();
                progressed = true;
                continue;
            }
            auto &t = it->second;
            if (ctx->serve_max_batch > 1 && fusable(*t.job)) {
                // the longest run of compatible requests at the head of the queue
                std::vector<uint64_t> ids;
                for (uint64_t qid : ctx->queue) {
                    if ((int)ids.size() >= ctx->serve_max_batch) break;
                    auto qt = ctx->tickets.find(qid);
                    if (qt == ctx->tickets.end() || qt->second.cancel_requested || !fusable(*qt->second.job) ||
                        qt->second.job->prec != t.job->prec)
                        break;
                    ids.push_back(qid);
                }
                auto b = std::make_unique<tfstat_batch>();
                b->prec = t.job->prec;
                b->variant = tfs::kShapeMixed;
                b->groups = std::max(1, tfs::fused_groups_per_cu(tfs::kShapeMixed)) * ctx->n_cu;
                bool placed = false, popped = false;
                try {
                    while (!ids.empty()) {
                        b->jobs.clear();
                        for (uint64_t qid : ids) b->jobs.push_back(ctx->tickets[qid].job.get());
                        if (batch_layout(ctx, b.get(), ctx->slots[slot], false, true)) {
                            placed = true;
                            break;
                        }
                        ids.pop_back();   // smaller batch
                    }
                    if (!placed) break;   // wait for memory
                    for (size_t i = 0; i < ids.size(); ++i) ctx->queue.pop_front();
                    popped = true;
                    hip_check(batch_enqueue(b.get(), ctx->slots[slot], false), "batch launch");
                    ctx->slot_done[slot] = ctx->events.get();
                    hip_check(hipEventRecord(ctx->slot_done[slot], ctx->slots[slot]), "hipEventRecord");
                    for (uint64_t qid : ids) {
                        auto &qt = ctx->tickets[qid];
                        qt.state = tfstat_ctx::Ticket::RUNNING;
                        qt.slot = slot;
                    }
                    ctx->slot_tickets[slot] = ids;
                    ctx->slot_batch[slot] = std::move(b);
                } catch (const Failure &f) {
                    // the requests fail; the loop goes on with the rest
                    if (ids.empty()) ids.push_back(id);
                    if (!popped)
                        for (size_t i = 0; i < ids.size() && !ctx->queue.empty(); ++i) ctx->queue.pop_front();
                    for (uint64_t qid : ids) {
                        auto &qt = ctx->tickets[qid];
                        qt.state = tfstat_ctx::Ticket::FAILED;
                        qt.err = f.code;
                        qt.msg = f.msg;
                        qt.job->at->busy -= 1;
                        qt.job->ws = nullptr;
                    }
                    if (ctx->slot_done[slot]) {
                        ctx->events.put(ctx->slot_done[slot]);
                        ctx->slot_done[slot] = nullptr;
                    }
                    lk.unlock();
                    batch_release(ctx, b.get());
                    lk.lock();
                }
                progressed = true;
                continue;
            }
            if (!alloc_job(ctx, *t.job)) break;  // wait for memory
            ctx->queue.pop_front();
            try {
                enqueue_job(ctx, *t.job, ctx->slots[slot]);
                ctx->slot_done[slot] = ctx->events.get();
                hip_check(hipEventRecord(ctx->slot_done[slot], ctx->slots[slot]), "hipEventRecord");
                t.state = tfstat_ctx::Ticket::RUNNING;
                t.slot = slot;
                ctx->slot_tickets[slot] = {id};
            } catch (const Failure &f) {
                t.state = tfstat_ctx::Ticket::FAILED;
                t.err = f.code;
                t.msg = f.msg;
                t.job->at->busy -= 1;
                release_job(ctx, *t.job);
                if (ctx->slot_done[slot]) {
                    ctx->events.put(ctx->slot_done[slot]);
                    ctx->slot_done[slot] = nullptr;
                }
            }
            progressed = true;
        }
        bool running = false;
        for (int s = 0; s < tfstat_ctx::kSlots; ++s) running |= !ctx->slot_tickets[s].empty();
        if (ctx->stop && !running && ctx->queue.empty()) break;
        if (ctx->stop && !running) {
            // drain: cancel what never started
            for (uint64_t id : ctx->queue) {
                auto it = ctx->tickets.find(id);
                if (it != ctx->tickets.end()) {
                    it->second.state = tfstat_ctx::Ticket::CANCELLED;
                    it->second.job->at->busy -= 1;
                }
            }
            ctx->queue.clear();
            break;
        }
        if (!running && ctx->queue.empty()) {
            ctx->cv.wait(lk);
        } else if (!progressed) {
            ctx->cv.wait_for(lk, std::chrono::microseconds(20));
        }
    }
}

void ensure_worker(tfstat_ctx *ctx) {
    if (ctx->worker_started) return;
    ensure_batch_stream(ctx);
    for (int s = 0; s < tfstat_ctx::kSlots; ++s)
        hip_check(hipStreamCreateWithFlags(&ctx->slots[s], hipStreamNonBlocking), "hipStreamCreate");
    ctx->worker = std::thread(worker_loop, ctx);
    ctx->worker_started = true;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *tfstat_last_error(void) { return g_err.c_str(); }

const char *tfstat_version(void) { return "tfstat 0.1 (gfx950)"; }

int tfstat_ctx_create(int device, void *arena_dev, size_t arena_bytes, void *hip_stream,
                      tfstat_ctx **out) {
    return guarded([&] {
        if (!out) raise(TFSTAT_E_INVAL, "out is null");
        if (!arena_dev || (reinterpret_cast<uintptr_t>(arena_dev) & 255))
            raise(TFSTAT_E_INVAL, "arena must be non-null and 256-byte aligned");
        if (arena_bytes < (1u << 20)) raise(TFSTAT_E_INVAL, "arena must be at least 1 MiB");
        int n = 0;
        hip_check(hipGetDeviceCount(&n), "hipGetDeviceCount");
        if (device < 0 || device >= n) raise(TFSTAT_E_DEVICE, "no such device");
        hip_check(hipSetDevice(device), "hipSetDevice");
        auto ctx = std::make_unique<tfstat_ctx>();
        ctx->device = device;
        ctx->stream = static_cast<hipStream_t>(hip_stream);
        hip_check(tfs::noalloc_setup(device), "allocation-free workspace address");
        ctx->arena.init(arena_dev, arena_bytes);
        *out = ctx.release();
        return (int)TFSTAT_OK;
    });
}

int tfstat_ctx_destroy(tfstat_ctx *ctx) {
    if (!ctx) return fail(TFSTAT_E_INVAL, "ctx is null");
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        ctx->stop = true;
    }
    ctx->cv.notify_all();
    if (ctx->worker.joinable()) ctx->worker.join();
    for (int s = 0; s < tfstat_ctx::kSlots; ++s)
        if (ctx->slots[s]) (void)hipStreamDestroy(ctx->slots[s]);
    if (ctx->batch_stream) {
        (void)hipStreamSynchronize(ctx->batch_stream);
        (void)hipStreamDestroy(ctx->batch_stream);
    }
    (void)hipStreamSynchronize(ctx->stream);
    delete ctx;
    return TFSTAT_OK;
}

int tfstat_atoms_upload(tfstat_ctx *ctx, const tfstat_atoms_desc *d, tfstat_atoms_id *out) {
    return guarded([&] {
        if (!ctx || !d || !out) raise(TFSTAT_E_INVAL, "null argument");
        if (d->n_sft < 1 || d->n_bins < 1 || d->t_sft < 1)
            raise(TFSTAT_E_INVAL, "n_sft, n_bins and t_sft must be >= 1");
        if (!d->timestamps || !d->a2 || !d->b2 || !d->ab || !d->fa || !d->fb)
            raise(TFSTAT_E_INVAL, "null atom array");
        if (d->t_sft > (1 << 30)) raise(TFSTAT_E_INVAL, "t_sft too large");
        const int64_t T = d->t_sft, T0 = d->timestamps[0];
        for (int32_t i = 1; i < d->n_sft; ++i)
            if (d->timestamps[i] <= d->timestamps[i - 1])
                raise(TFSTAT_E_GRID, "timestamps must be strictly increasing");
        for (int32_t i = 0; i < d->n_sft; ++i)
            if ((d->timestamps[i] - T0) % T != 0)
                raise(TFSTAT_E_GRID, "timestamps must lie on timestamps[0] + k * t_sft");
        const int64_t K64 = (d->timestamps[d->n_sft - 1] - T0) / T + 1;
        if (K64 > (1 << 28)) raise(TFSTAT_E_GRID, "data span too long");
        const int32_t K = (int32_t)K64;
        const int32_t nb = d->n_bins;
        const size_t rows = (size_t)K + 1;
        const size_t abc_b = round_up(sizeof(double) * 4 * rows, 256);
        const size_t x64_b = round_up(sizeof(double) * 4 * nb * rows, 256);
        const size_t x32_b = round_up(sizeof(float) * 4 * nb * rows, 256);
        const size_t np_b = round_up(sizeof(int32_t) * rows, 256);
        auto set = std::make_unique<AtomsSet>();
        set->K = K;
        set->n_bins = nb;
        set->n_sft = d->n_sft;
        set->T0 = T0;
        set->t_sft = T;
        {
            std::lock_guard<std::mutex> g(ctx->mu);
            set->mem = ctx->arena.alloc(abc_b + x64_b + x32_b + np_b);
        }
        if (!set->mem) raise(TFSTAT_E_NOMEM, "arena cannot hold the atoms");
        set->bytes = abc_b + x64_b + x32_b + np_b;
        char *base = static_cast<char *>(set->mem);
        set->abc = reinterpret_cast<double *>(base);
        set->x64 = reinterpret_cast<double *>(base + abc_b);
        set->x32 = reinterpret_cast<float *>(base + abc_b + x64_b);
        set->npref = reinterpret_cast<int32_t *>(base + abc_b + x64_b + x32_b);
        size_t pin_bytes = 0;
        void *pin = ctx->pinned.get(abc_b + x64_b + np_b, &pin_bytes);
        try {
            std::memset(pin, 0, abc_b + x64_b + np_b);
            double *habc = static_cast<double *>(pin);
            double *hx = reinterpret_cast<double *>(static_cast<char *>(pin) + abc_b);
            for (int32_t i = 0; i < d->n_sft; ++i) {
                const int64_t k = (d->timestamps[i] - T0) / T;
                habc[k * 4 + 0] = d->a2[i];
                habc[k * 4 + 1] = d->b2[i];
                habc[k * 4 + 2] = d->ab[i];
                for (int32_t b = 0; b < nb; ++b) {
                    const double *pa = d->fa + ((size_t)b * d->n_sft + i) * 2;
                    const double *pb = d->fb + ((size_t)b * d->n_sft + i) * 2;
                    double *o = hx + ((size_t)k * nb + b) * 4;
                    o[0] = pa[0];
                    o[1] = pa[1];
                    o[2] = pb[0];
                    o[3] = pb[1];
                }
            }
            hip_check(hipSetDevice(ctx->device), "hipSetDevice");
            // present-SFT prefix counts (exact integers)
            int32_t *hnp = reinterpret_cast<int32_t *>(static_cast<char *>(pin) + abc_b + x64_b);
            {
                std::vector<char> present(K, 0);
                for (int32_t i = 0; i < d->n_sft; ++i) present[(d->timestamps[i] - T0) / T] = 1;
                hnp[0] = 0;
                for (int32_t k = 0; k < K; ++k) hnp[k + 1] = hnp[k] + present[k];
            }
            hip_check(hipMemcpyAsync(set->mem, pin, abc_b + x64_b, hipMemcpyHostToDevice, ctx->stream),
                      "upload atoms");
            hip_check(hipMemcpyAsync(set->npref, hnp, sizeof(int32_t) * rows, hipMemcpyHostToDevice,
                                     ctx->stream), "upload counts");
            Job dummy;
            record_kernel(ctx, dummy, TFSTAT_K_UPLOAD, ctx->stream, true);
            hip_check(tfs::launch_build_x32(set->x64, set->x32, (int64_t)4 * nb * rows, ctx->stream),
                      "x32 kernel");
            record_kernel(ctx, dummy, TFSTAT_K_UPLOAD, ctx->stream, false);
            hip_check(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
            collect_timing(ctx, dummy);
        } catch (...) {
            ctx->pinned.put(pin, pin_bytes);
            std::lock_guard<std::mutex> g(ctx->mu);
            ctx->arena.release(set->mem);
            throw;
        }
        ctx->pinned.put(pin, pin_bytes);
        std::lock_guard<std::mutex> g(ctx->mu);
        const uint64_t id = ctx->next_atoms++;
        ctx->atoms[id] = std::move(set);
        *out = id;
        return (int)TFSTAT_OK;
    });
}

int tfstat_atoms_free(tfstat_ctx *ctx, tfstat_atoms_id id) {
    return guarded([&] {
        if (!ctx) raise(TFSTAT_E_INVAL, "ctx is null");
        std::lock_guard<std::mutex> g(ctx->mu);
        AtomsSet *s = find_atoms(ctx, id);
        if (s->busy > 0) raise(TFSTAT_E_BUSY, "atoms are in use by submitted requests");
        ctx->arena.release(s->mem);
        if (s->planes) ctx->arena.release(s->planes);
        if (s->planes16) ctx->arena.release(s->planes16);
        ctx->atoms.erase(id);
        return (int)TFSTAT_OK;
    });
}

int tfstat_atoms_info(tfstat_ctx *ctx, tfstat_atoms_id id, int32_t *n_slots, int32_t *n_bins) {
    return guarded([&] {
        if (!ctx) raise(TFSTAT_E_INVAL, "ctx is null");
        std::lock_guard<std::mutex> g(ctx->mu);
        AtomsSet *s = find_atoms(ctx, id);
        if (n_slots) *n_slots = s->K;
        if (n_bins) *n_bins = s->n_bins;
        return (int)TFSTAT_OK;
    });
}

int tfstat_fmap(tfstat_ctx *ctx, tfstat_atoms_id id, const tfstat_window *win, int32_t precision,
                float *twoF_dev, tfstat_bin_result *res_host) {
    return guarded([&] {
        if (!ctx || !res_host) raise(TFSTAT_E_INVAL, "null argument");
        if (precision < TFSTAT_PREC_FP64 || precision > TFSTAT_PREC_F16X3)
            raise(TFSTAT_E_INVAL, "unknown precision");
        Job j;
        {
            std::lock_guard<std::mutex> g(ctx->mu);
            j.at = find_atoms(ctx, id);
            if (matrix_prec(precision)) ensure_planes(ctx, j.at, precision);
        }
        j.win = copy_window(win);
        j.prec = precision;
        j.twoF = twoF_dev;
        j.runs_min_spread = ctx->runs_min_spread.load();
        j.split_min_bins = ctx->split_min_bins.load();
        plan_job(j);
        {
            std::lock_guard<std::mutex> g(ctx->mu);
            if (!alloc_job(ctx, j)) raise(TFSTAT_E_NOMEM, "arena cannot hold the map workspace");
        }
        try {
            hip_check(hipSetDevice(ctx->device), "hipSetDevice");
            enqueue_job(ctx, j, ctx->stream);
            hip_check(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
            finish_job(ctx, j, res_host);
        } catch (...) {
            std::lock_guard<std::mutex> g(ctx->mu);
            release_job(ctx, j);
            throw;
        }
        std::lock_guard<std::mutex> g(ctx->mu);
        release_job(ctx, j);
        return (int)TFSTAT_OK;
    });
}

int tfstat_logB(tfstat_ctx *ctx, const float *twoF_dev, int32_t n_maps, int32_t n_t0, int32_t n_tau,
                double *logB_host) {
    return guarded([&] {
        if (!ctx || !twoF_dev || !logB_host) raise(TFSTAT_E_INVAL, "null argument");
        if (n_maps < 1 || n_t0 < 1 || n_tau < 1) raise(TFSTAT_E_INVAL, "sizes must be >= 1");
        if (n_maps > 65535) raise(TFSTAT_E_INVAL, "n_maps must be <= 65535");
        const int64_t cells = (int64_t)n_t0 * n_tau;
        const int64_t cpt = 16384;
        if ((cells + cpt - 1) / cpt > 65535) raise(TFSTAT_E_INVAL, "maps of more than 2^30 cells");
        const int32_t n_tiles = (int32_t)((cells + cpt - 1) / cpt);
        const size_t part_b = round_up(sizeof(tfs::Partial) * (size_t)n_tiles * n_maps, 256);
        const size_t res_b = sizeof(tfs::BinResultDev) * n_maps;
        void *ws;
        {
            std::lock_guard<std::mutex> g(ctx->mu);
            ws = ctx->arena.alloc(part_b + res_b);
        }
        if (!ws) raise(TFSTAT_E_NOMEM, "arena cannot hold the reduction workspace");
        size_t pin_b = 0;
        void *pin = nullptr;
        try {
            hip_check(hipSetDevice(ctx->device), "hipSetDevice");
            pin = ctx->pinned.get(res_b, &pin_b);
            tfs::MapReduceParams rp{};
            rp.twoF = twoF_dev;
            rp.n_cells = cells;
            rp.n_maps = n_maps;
            rp.n_tiles = n_tiles;
            rp.cells_per_tile = cpt;
            rp.part = static_cast<tfs::Partial *>(ws);
            hip_check(tfs::launch_map_reduce(rp, ctx->stream), "map reduce kernel");
            tfs::MergeParams mp{};
            mp.n_tiles = n_tiles;
            mp.n_maps = n_maps;
            mp.n_cells = cells;
            mp.part = rp.part;
            mp.out = reinterpret_cast<tfs::BinResultDev *>(static_cast<char *>(ws) + part_b);
            hip_check(tfs::launch_merge(mp, ctx->stream), "merge kernel");
            hip_check(hipMemcpyAsync(pin, mp.out, res_b, hipMemcpyDeviceToHost, ctx->stream),
                      "download results");
            hip_check(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
            const auto *r = static_cast<const tfs::BinResultDev *>(pin);
            for (int32_t k = 0; k < n_maps; ++k) logB_host[k] = r[k].logB;
        } catch (...) {
            if (pin) ctx->pinned.put(pin, pin_b);
            std::lock_guard<std::mutex> g(ctx->mu);
            ctx->arena.release(ws);
            throw;
        }
        ctx->pinned.put(pin, pin_b);
        std::lock_guard<std::mutex> g(ctx->mu);
        ctx->arena.release(ws);
        return (int)TFSTAT_OK;
    });
}

int tfstat_window_odds(tfstat_ctx *ctx, tfstat_atoms_id id, const tfstat_window *win_a,
                       const tfstat_window *win_b, int32_t precision, double *log_odds_host) {
    return guarded([&] {
        if (!ctx || !win_a || !win_b || !log_odds_host) raise(TFSTAT_E_INVAL, "null argument");
        int32_t n_bins = 0;
        {
            std::lock_guard<std::mutex> g(ctx->mu);
            n_bins = find_atoms(ctx, id)->n_bins;
        }
        std::vector<tfstat_bin_result> ra(n_bins), rb(n_bins);
        int rc = tfstat_fmap(ctx, id, win_a, precision, nullptr, ra.data());
        if (rc != TFSTAT_OK) return rc;
        rc = tfstat_fmap(ctx, id, win_b, precision, nullptr, rb.data());
        if (rc != TFSTAT_OK) return rc;
        for (int32_t b = 0; b < n_bins; ++b) log_odds_host[b] = ra[b].logB - rb[b].logB;
        return (int)TFSTAT_OK;
    });
}

int tfstat_logB_noalloc(tfstat_ctx *ctx, const float *twoF_dev, int32_t n_maps, int32_t n_t0,
                        int32_t n_tau, double *logB_dev) {
    return guarded([&] {
        if (!ctx || !twoF_dev || !logB_dev) raise(TFSTAT_E_INVAL, "null argument");
        if (n_maps < 1 || n_t0 < 1 || n_tau < 1) raise(TFSTAT_E_INVAL, "sizes must be >= 1");
        if (n_maps > 65535) raise(TFSTAT_E_INVAL, "n_maps must be <= 65535");
        const int64_t cells = (int64_t)n_t0 * n_tau;
        const int64_t cpt = 16384;
        if ((cells + cpt - 1) / cpt > 65535) raise(TFSTAT_E_INVAL, "maps of more than 2^30 cells");
        const int32_t n_tiles = (int32_t)((cells + cpt - 1) / cpt);
        const size_t part_b = round_up(sizeof(tfs::Partial) * (size_t)n_tiles * n_maps, 256);
        const size_t res_b = sizeof(tfs::BinResultDev) * n_maps;
        if (part_b + res_b > (size_t)TFSTAT_NOALLOC_SCRATCH_BYTES)
            raise(TFSTAT_E_INVAL, "tfstat_logB_noalloc needs " + std::to_string(part_b + res_b) +
                                      " bytes of workspace; its static workspace holds " +
                                      std::to_string((size_t)TFSTAT_NOALLOC_SCRATCH_BYTES));
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        char *ws = static_cast<char *>(tfs::noalloc_scratch(ctx->device));
        if (!ws) raise(TFSTAT_E_DEVICE, "allocation-free workspace not set up on this device");
        tfs::MapReduceParams rp{};
        rp.twoF = twoF_dev;
        rp.n_cells = cells;
        rp.n_maps = n_maps;
        rp.n_tiles = n_tiles;
        rp.cells_per_tile = cpt;
        rp.part = reinterpret_cast<tfs::Partial *>(ws);
        hip_check(tfs::launch_map_reduce(rp, ctx->stream), "map reduce kernel");
        tfs::MergeParams mp{};
        mp.n_tiles = n_tiles;
        mp.n_maps = n_maps;
        mp.n_cells = cells;
        mp.part = rp.part;
        mp.out = reinterpret_cast<tfs::BinResultDev *>(ws + part_b);
        mp.logB_out = logB_dev;
        hip_check(tfs::launch_merge(mp, ctx->stream), "merge kernel");
        return (int)TFSTAT_OK;
    });
}

int tfstat_submit(tfstat_ctx *ctx, tfstat_atoms_id id, const tfstat_window *win, int32_t precision,
                  tfstat_ticket *out) {
    return guarded([&] {
        if (!ctx || !out) raise(TFSTAT_E_INVAL, "null argument");
        if (precision < TFSTAT_PREC_FP64 || precision > TFSTAT_PREC_F16X3)
            raise(TFSTAT_E_INVAL, "unknown precision");
        auto job = std::make_unique<Job>();
        job->win = copy_window(win);
        job->prec = precision;
        std::lock_guard<std::mutex> g(ctx->mu);
        job->at = find_atoms(ctx, id);
        if (matrix_prec(precision)) ensure_planes(ctx, job->at, precision);
        job->runs_min_spread = ctx->runs_min_spread.load();
        job->split_min_bins = ctx->split_min_bins.load();
        plan_job(*job);
        // A request whose workspace cannot fit beside the resident atoms
        // would wait forever: refuse it now.
        size_t resident = 0;
        for (auto &kv : ctx->atoms) resident += kv.second->bytes;
        if (job->ws_bytes + resident > ctx->arena.capacity())
            raise(TFSTAT_E_NOMEM, "request workspace cannot fit beside the resident atoms");
        if (ctx->queue.size() >= tfstat_ctx::kMaxQueue) raise(TFSTAT_E_BUSY, "serving queue is full");
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        ensure_worker(ctx);
        const uint64_t t = ctx->next_ticket++;
        auto &tk = ctx->tickets[t];
        tk.atoms_id = id;
        job->at->busy += 1;
        tk.job = std::move(job);
        ctx->queue.push_back(t);
        ctx->cv.notify_all();
        *out = t;
        return (int)TFSTAT_OK;
    });
}

int tfstat_poll(tfstat_ctx *ctx, tfstat_ticket t, tfstat_bin_result *res_host, int *done) {
    return guarded([&] {
        if (!ctx || !done) raise(TFSTAT_E_INVAL, "null argument");
        std::lock_guard<std::mutex> g(ctx->mu);
        auto it = ctx->tickets.find(t);
        if (it == ctx->tickets.end()) raise(TFSTAT_E_NOTFOUND, "unknown or retired ticket");
        auto &tk = it->second;
        switch (tk.state) {
            case tfstat_ctx::Ticket::DONE:
                if (!res_host) raise(TFSTAT_E_INVAL, "res_host is null");
                std::memcpy(res_host, tk.res.data(), sizeof(tfstat_bin_result) * tk.res.size());
                *done = 1;
                ctx->tickets.erase(it);
                return (int)TFSTAT_OK;
            case tfstat_ctx::Ticket::FAILED: {
                *done = 1;
                const int e = tk.err;
                const std::string m = tk.msg;
                ctx->tickets.erase(it);
                raise(e, m);
            }
            case tfstat_ctx::Ticket::CANCELLED:
                *done = 1;
                ctx->tickets.erase(it);
                raise(TFSTAT_E_CANCELLED, "ticket was cancelled");
            default:
                *done = 0;
                return (int)TFSTAT_OK;
        }
    });
}

int tfstat_cancel(tfstat_ctx *ctx, tfstat_ticket t) {
    return guarded([&] {
        if (!ctx) raise(TFSTAT_E_INVAL, "ctx is null");
        std::lock_guard<std::mutex> g(ctx->mu);
        auto it = ctx->tickets.find(t);
        if (it == ctx->tickets.end()) raise(TFSTAT_E_NOTFOUND, "unknown or retired ticket");
        it->second.cancel_requested = true;
        ctx->cv.notify_all();
        return (int)TFSTAT_OK;
    });
}

int tfstat_batch_create(tfstat_ctx *ctx, int32_t n_maps, const tfstat_atoms_id *ids,
                        const tfstat_window *wins, int32_t precision, int32_t tune,
                        tfstat_batch **out) {
    return guarded([&] {
        if (!ctx || !ids || !wins || !out) raise(TFSTAT_E_INVAL, "null argument");
        if (n_maps < 1) raise(TFSTAT_E_INVAL, "n_maps must be >= 1");
        if (precision != TFSTAT_PREC_FP32 && precision != TFSTAT_PREC_FP64 && !matrix_prec(precision))
            raise(TFSTAT_E_INVAL, "a batch runs in FP32, FP64, BF16X3 or F16X3");
        if (tune > 1 || tune < -2 * (tfs::kShapeMixed + 1))
            raise(TFSTAT_E_INVAL, "tune must be 0, 1 or -1 - variant");
        ensure_batch_stream(ctx);
        const std::string sig = batch_signature(ctx, n_maps, ids, wins, precision);
        // Builds a caller may force (tune = -1 - v): every tile shape of the
        // precision, at the stand-alone waves per SIMD and one fewer.
        std::vector<int> variants;
        for (int m = 0; m < 2; ++m) {
            const int base = m * (tfs::kShapeMixed + 1);
            if (precision == TFSTAT_PREC_FP64) {
                variants.push_back(base + tfs::kShapeD41);
            } else {
                for (int sh : {tfs::kShapeF81, tfs::kShapeF42, tfs::kShapeF44, tfs::kShapeMixed})
                    variants.push_back(base + sh);
            }
        }
        // Builds the autotuner may keep: only those that give every map its
        // own tile shape (the one tfstat_fmap plans), at either occupancy.
        // Their arithmetic per cell is the stand-alone kernel's, so a map's
        // results never depend on which other maps share its batch.
        const int own = precision == TFSTAT_PREC_FP64 ? tfs::kShapeD41 : tfs::kShapeMixed;
        const std::vector<int> tunable = {own, own + tfs::kShapeMixed + 1};
        double tune_ms = 0.0;
        int variant = precision == TFSTAT_PREC_FP64 ? tfs::kShapeD41 : tfs::kShapeMixed;
        int per_cu = 0;
        bool found = false;
        if (tune < 0) {
            // a given variant at its widest launch; the tuning cache is
            // neither read nor written
            variant = -1 - tune;
            if (std::find(variants.begin(), variants.end(), variant) == variants.end())
                raise(TFSTAT_E_INVAL, "variant not built for this precision");
            found = true;
        }
        if (!found) {
            std::lock_guard<std::mutex> g(ctx->mu);
            auto it = ctx->tuned.find(sig);
            if (it != ctx->tuned.end()) {
                variant = it->second.first;
                per_cu = it->second.second;
                found = true;
            }
        }
        if (tune == 1 && !found) {
            // Autotuner: each build that keeps the maps' own tile shapes x
            // every persistent width that fits; the fastest of three graph
            // replays after one warm-up counts.
            const auto t_start = std::chrono::steady_clock::now();
            double best = 1e300;
            for (int v : tunable) {
                const int occ = tfs::fused_groups_per_cu(v);
                if (occ < 1) continue;
                tfstat_batch cand;
                cand.prec = precision;
                cand.variant = v;
                try {
                    batch_build(ctx, &cand, n_maps, ids, wins);
                    for (int g = 1; g <= occ; ++g) {
                        cand.groups = g * ctx->n_cu;
                        batch_capture(ctx, &cand);
                        batch_launch(ctx, &cand);
                        double t = 1e300;
                        for (int r = 0; r < 3; ++r) {
                            batch_launch(ctx, &cand);
                            t = std::min(t, cand.last_ms);
                        }
                        if (t < best) {
                            best = t;
                            variant = v;
                            per_cu = g;
                        }
                    }
                } catch (const Failure &f) {
                    batch_release(ctx, &cand);
                    if (f.code != TFSTAT_E_NOMEM) throw;
                    continue;   // a shape whose tables do not fit is not a candidate
                }
                batch_release(ctx, &cand);
            }
            if (per_cu < 1) raise(TFSTAT_E_NOMEM, "no tile shape fits the arena");
            tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
            std::lock_guard<std::mutex> g(ctx->mu);
            ctx->tuned[sig] = {variant, per_cu};
        }
        if (per_cu < 1) per_cu = tfs::fused_groups_per_cu(variant);
        if (per_cu < 1) raise(TFSTAT_E_DEVICE, "fused kernel does not fit on a CU");
        auto b = std::make_unique<tfstat_batch>();
        b->prec = precision;
        b->variant = variant;
        b->groups = per_cu * ctx->n_cu;
        b->tune_ms = tune_ms;
        try {
            batch_build(ctx, b.get(), n_maps, ids, wins);
            batch_capture(ctx, b.get());
        } catch (...) {
            batch_release(ctx, b.get());
            throw;
        }
        *out = b.release();
        return (int)TFSTAT_OK;
    });
}

int tfstat_batch_run(tfstat_ctx *ctx, tfstat_batch *b, int32_t timed, tfstat_bin_result *res_host) {
    return guarded([&] {
        if (!ctx || !b || !res_host) raise(TFSTAT_E_INVAL, "null argument");
        if (!b->exec) raise(TFSTAT_E_INVAL, "batch has no graph");
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        if (timed)
            batch_run_timed(ctx, b);
        else
            batch_launch(ctx, b);
        const auto *r = static_cast<const tfs::BinResultDev *>(b->pin);
        for (size_t i = 0; i < b->jobs.size(); ++i)
            convert_results(*b->jobs[i], r + b->res_off[i], res_host + b->res_off[i]);
        return (int)TFSTAT_OK;
    });
}

int tfstat_batch_stats_read(const tfstat_batch *b, tfstat_batch_stats *out) {
    return guarded([&] {
        if (!b || !out) raise(TFSTAT_E_INVAL, "null argument");
        out->variant = b->variant;
        out->groups = b->groups;
        out->n_tiles = b->n_tiles;
        out->n_results = b->n_results;
        out->tune_ms = b->tune_ms;
        out->last_ms = b->last_ms;
        out->last_fused_ms = b->last_fused_ms;
        out->last_mfma_ms = b->last_mfma_ms;
        return (int)TFSTAT_OK;
    });
}

int tfstat_batch_destroy(tfstat_ctx *ctx, tfstat_batch *b) {
    return guarded([&] {
        if (!ctx || !b) raise(TFSTAT_E_INVAL, "null argument");
        if (ctx->batch_stream) (void)hipStreamSynchronize(ctx->batch_stream);
        batch_release(ctx, b);
        delete b;
        return (int)TFSTAT_OK;
    });
}

int tfstat_serve_config(tfstat_ctx *ctx, int32_t max_batch) {
    return guarded([&] {
        if (!ctx) raise(TFSTAT_E_INVAL, "ctx is null");
        if (max_batch < 1 || max_batch > 1024) raise(TFSTAT_E_INVAL, "max_batch must be in 1..1024");
        std::lock_guard<std::mutex> g(ctx->mu);
        ctx->serve_max_batch = max_batch;
        return (int)TFSTAT_OK;
    });
}

int tfstat_tiling_config(tfstat_ctx *ctx, int32_t runs_min_spread, int32_t split_min_bins) {
    return guarded([&] {
        if (!ctx) raise(TFSTAT_E_INVAL, "ctx is null");
        ctx->runs_min_spread.store(runs_min_spread < 0 ? kRunsAuto : runs_min_spread);
        ctx->split_min_bins.store(split_min_bins < 0 ? kSplitMinBins : split_min_bins);
        return (int)TFSTAT_OK;
    });
}

int tfstat_profile_enable(tfstat_ctx *ctx, int on) {
    if (!ctx) return fail(TFSTAT_E_INVAL, "ctx is null");
    ctx->profile.store(on ? 1 : 0);
    return TFSTAT_OK;
}

int tfstat_profile_read(tfstat_ctx *ctx, int32_t kind, int64_t *launches, double *total_ms) {
    if (!ctx || kind < 0 || kind >= NK) return fail(TFSTAT_E_INVAL, "bad argument");
    std::lock_guard<std::mutex> g(ctx->mu);
    if (launches) *launches = ctx->k_launches[kind];
    if (total_ms) *total_ms = ctx->k_ms[kind];
    return TFSTAT_OK;
}

int tfstat_profile_reset(tfstat_ctx *ctx) {
    if (!ctx) return fail(TFSTAT_E_INVAL, "ctx is null");
    std::lock_guard<std::mutex> g(ctx->mu);
    for (int k = 0; k < NK; ++k) {
        ctx->k_launches[k] = 0;
        ctx->k_ms[k] = 0.0;
    }
    return TFSTAT_OK;
}

}  // extern "C"
