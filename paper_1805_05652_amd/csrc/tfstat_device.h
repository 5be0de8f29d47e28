// Device-side parameter blocks and kernel launchers of the tfstat library.
// Shared by the kernels (kernels.hip) and the host runtime (runtime.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tfs {

// Threshold of the degenerate-window rule: 2F := 0 when D <= rtol * A * B.
constexpr double kDegenerateRtol = 1e-10;

// One t0 row of the planned grid.  k0 is the first slot whose start time is
// >= t0 (it may lie before slot 0 or after the last slot: such slots hold
// zeros), delta = t_{k0} - t0 in [0, t_sft).
struct RowPlan {
    int32_t k0;
    int32_t delta;
};

// Per-tile reduction partial: running maximum of F = 2F/2, the sum of
// exp(F - fmax) over the tile's cells, and the smallest linear cell index
// (m * n_tau + n) holding the maximum.
struct Partial {
    double fmax;
    double s;
    int64_t idx;
};

// Per-bin reduction result.
struct BinResultDev {
    double max2F;
    double logB;
    int64_t idx;
};

// Resident atoms of one candidate on the slot grid (row K is all zeros).
struct AtomsView {
    int32_t K;            // number of slots
    int32_t n_bins;
    int64_t t_sft;
    const double *abc;    // [K+1][4]: a2, b2, ab, 0
    const double *x64;    // [K+1][n_bins][4]: Re Fa, Im Fa, Re Fb, Im Fb
    const float *x32;     // [K+1][n_bins][4]
};

// Exponential-window sums, VALU form.  A work item is a (t0 tile of 64 rows,
// tau block of R columns) pair; the d-loop over the window band is split
// across the four waves of a workgroup.
struct ExpValuParams {
    AtomsView at;
    int32_t n_t0, n_tau;
    int32_t n_row_tiles;      // ceil(n_t0 / 64)
    int32_t n_list;           // number of tau blocks this launch processes
    int32_t n_tiles;          // partial slots per bin (all blocks x row tiles)
    int32_t bin_base;         // first bin of bin group 0 of a stand-alone launch
    const RowPlan *rows;      // [n_t0]
    const int64_t *tau;       // [n_tau]
    const int32_t *lcol;      // [n_tau] table length per tau: shortest band over rows
    const int32_t *lblk;      // [n_blocks] max lcol over the block
    const int64_t *blk_off;   // [n_blocks] element offset of the block's table
    const int32_t *blk_list;  // [n_list] blocks processed, largest band first
    const float *g32;         // weight tables [blk][d][R]
    const double *g64;        //   (FP64 weights, FP64 mode only)
    const double *gsq;        //   (squared weights, FP64)
    float *twoF;              // optional map [n_bins][n_t0][n_tau]
    Partial *part;            // [n_bins][n_tiles]
    double *abc_out;          // A/B/C-only mode: [n_t0][abc_pitch][3] (scaled, exact band)
    int32_t abc_pitch;        // cells per row of abc_out (n_tau rounded up to 8)
    int32_t scale_rows;       // 1: exponential window (row scale exp(-delta/tau) and band
                              // tails); 0: shape window (one delta, tables hold it)
};

// LDS stage of the band-staged exponential form: slots per stage for a
// precision (0 = FP64 sums, 1 = FP32) and bins per lane, and the fewest band
// slots per round worth staging.  Tiles whose rows span more than
// stage - kExpMinStageRound slots read through the caches instead.
constexpr int kExpMinStageRound = 64;
constexpr int exp_stage_len(int prec, int BG) { return (prec == 1 && BG == 1) ? 1008 : 512; }

// Exponential-window F_a, F_b on bf16 matrix cores for grids whose t0 rows
// are consecutive slots with one common delta.
struct ExpMfmaParams {
    int32_t n_bins, bins16;   // bins, rounded up to 16
    int32_t kp;               // plane pitch (slots), multiple of 32
    int32_t kp_data;          // round_up(K, 32): slots that may hold data
    int32_t n_t0, n_tau;
    int32_t n_row_tiles;      // ceil(n_t0 / 64)
    int32_t n_col_tiles;      // bins16 / 16
    int32_t n_blocks;         // blocks in blk_list
    int32_t n_tiles;          // partial slots per bin
    int32_t k0_first;         // slot of row 0 (>= 0); row m starts at k0_first + m
    int32_t delta;            // t_{k0} - t0, common to all rows
    const int64_t *tau;
    const int32_t *lblk;      // [blocks] band length of the block's table
    const int64_t *blk_off;   // [blocks] table offsets, [blk][d][8] layout
    const int32_t *blk_list;  // [n_blocks]
    const int32_t *lg;        // [blocks] length of each shifted table
    const int64_t *gsh_off;   // [blocks] element offset of the block's shifted tables
    const unsigned short *gsh;  // shifted bf16 tables [blk][t 8][part 2][shift 8][lg]
    const unsigned short *xhi, *xlo;  // bf16 planes [4][kp / 32][bins16][32]
    const double *abc_cell;   // [n_t0][abc_pitch][3]
    int32_t abc_pitch;        // n_tau rounded up to 8 (rows start 16-byte aligned)
    int32_t pad2;
    float *twoF;
    Partial *part;
};

// Exponential-window F_a, F_b on bf16 matrix cores for any t0 grid.  Each
// wave computes the window weights exp(-(t_k - t0_m) / tau) of its own 16
// rows in registers, so rows may start at any slot k0_m with any offset
// delta_m (the row scale and each row's exact band end are in the weights).
struct ExpMfmaRowsParams {
    int32_t n_bins, bins16;   // bins, rounded up to 16
    int32_t kp;               // plane pitch (slots), multiple of 32
    int32_t kp_data;          // round_up(K, 32): slots that may hold data
    int32_t n_t0, n_tau;
    int32_t n_row_tiles;      // ceil(n_t0 / 64)
    int32_t n_col_tiles;      // bins16 / 16
    int32_t n_blocks;         // blocks in blk_list
    int32_t n_tiles;          // partial slots per bin
    int64_t t_sft;
    const RowPlan *rows;      // [n_t0]
    const int64_t *tau;       // [n_tau]
    const int32_t *blk_list;  // [n_blocks] blocks of 8 taus
    const unsigned short *xhi, *xlo;  // bf16 or half planes [4][kp / 32][bins16][32]
    const int32_t *colexp;    // half planes: column scale exponents [4][bins16]
    const double *abc_cell;   // [n_t0][abc_pitch][3] (scaled, exact band)
    int32_t abc_pitch;        // n_tau rounded up to 8
    int32_t f16;              // 1: half-precision parts (F16X3), 0: bf16
    float *twoF;
    Partial *part;
    // transposed form (maps of fewer than kSwMinColTiles column tiles):
    // column planes [kCellsCopies][4][n_bins][kpc] of the same parts, and
    // the FP32 atoms for the band-end correction
    const unsigned short *chi, *clo;
    const float *x32;         // [K + 1][n_bins][4]
    int32_t kpc;              // column plane pitch, cells_plane_pitch(K)
    int32_t K;
};

// XCD-aware task order.  Workgroup b runs on XCD b % 8, and each XCD has its
// own L2.  With 8 or more units of work (tau blocks, or groups of them),
// the units are dealt round-robin to the XCDs and all per_unit tasks of a
// unit (row tiles, column tiles) stay on its XCD, so the unit's tables are
// fetched into one L2; with fewer units that order would leave XCDs idle,
// and the tasks run in plain order instead.
__host__ __device__ inline int64_t unit_grid(int n_units, int per_unit) {
    return n_units >= 8 ? (int64_t)8 * ((n_units + 7) / 8) * per_unit : (int64_t)n_units * per_unit;
}
// Unit and task within the unit of workgroup bid (unit >= n_units: none).
__host__ __device__ inline void unit_decode(int bid, int n_units, int per_unit, int &unit, int &task) {
    if (n_units >= 8) {
        const int slot = bid >> 3;
        unit = (slot / per_unit) * 8 + (bid & 7);
        task = slot % per_unit;
    } else {
        unit = bid / per_unit;
        task = bid % per_unit;
    }
}

// Maps of at least this many 16-bin column tiles take their matrix-core
// work items four column tiles at a time (one wave each, weights shared);
// maps of fewer take the transposed work item: 64 rows x one bin x
// kCellsBlocks blocks of 8 taus (kCellsNT tiles of 16 taus).
constexpr int kSwMinColTiles = 4;
constexpr int kCellsNT = 4;
constexpr int kCellsBlocks = 2 * kCellsNT;
__host__ __device__ inline bool mfma_cells_form(int n_col_tiles) { return n_col_tiles < kSwMinColTiles; }
// Units of a map along its list of matrix-core blocks: one per block, or
// one per kCellsBlocks blocks in the transposed form.
__host__ __device__ inline int mfma_units(int n_blocks, int n_col_tiles) {
    return mfma_cells_form(n_col_tiles) ? (n_blocks + kCellsBlocks - 1) / kCellsBlocks : n_blocks;
}
// Column work items per unit and 64-row tile: one per bin in the
// transposed form, one per four column tiles otherwise.
__host__ __device__ inline int mfma_col_items(int n_col_tiles, int n_bins) {
    return mfma_cells_form(n_col_tiles) ? n_bins : (n_col_tiles + 3) / 4;
}
// Column planes of the transposed form: slot k of component c, bin b, copy
// r at element ((r * 4 + c) * n_bins + b) * kpc + k + 16 - r, one copy per
// residue of k mod kCellsCopies (a power of two up to 8).
constexpr int kCellsCopies = 2;
static_assert(kCellsCopies == 2 || kCellsCopies == 4 || kCellsCopies == 8, "column plane copies");
__host__ __device__ inline int32_t cells_plane_pitch(int32_t K) { return (K + 7) / 8 * 8 + 24; }

// Half-precision matrix-core weights are taken as w * 2^kF16WeightExp.
constexpr int kF16WeightExp = 4;

// Matrix-core work of many maps: entry e is {map, unit (position in the
// map's blk_list, or group of kCellsBlocks of them), 64-row tile, column
// item}; the transposed form's entries come first and take a launch of
// their own.
struct MfmaBatchParams {
    const ExpMfmaRowsParams *jobs;
    const int32_t *entries;   // [n_entries][4]
    int32_t n_entries;
    int32_t f16;              // every job's parts: 1 half, 0 bf16
    int32_t n_cells;          // entries [0, n_cells): transposed form
    int32_t pad0;
};

struct ShiftTableParams {
    int32_t n_blocks;
    int32_t pad0;
    const int32_t *blk_list;  // [n_blocks]
    const int32_t *lblk;
    const int32_t *lg;
    const int64_t *blk_off;   // offsets into g32 ([blk][d][8])
    const int64_t *gsh_off;
    const float *g32;
    unsigned short *gsh;
};

// Exponential-window sums by the t0 recurrence (rows k0_first + m * stride,
// one common delta).  Partials: one tile per tau column.
struct RecurParams {
    int32_t K, n_bins;
    int32_t n_t0, n_tau;
    int64_t t_sft;
    int32_t k0_first, stride;
    int32_t delta;
    int32_t n_tiles;          // partial slots per bin (n_tau)
    const int64_t *tau;
    const double *abc;        // [K+1][4]
    const double *x64;        // [K+1][n_bins][4]
    const int32_t *npref;     // [K+1] SFTs present in slots [0, k)
    float *twoF;
    Partial *part;
};

// Weight tables [blk][d][R] of a banded window: exponential g[d] =
// exp(-d T / tau), or a shape window g[d] = s((delta + d T) / tau) with s
// linear between samples.
struct WeightParams {
    int32_t n_tau;
    int32_t n_blocks;
    int32_t R;
    int32_t want64;
    int64_t t_sft;
    const int64_t *tau;
    const int32_t *lcol;
    const int32_t *lblk;
    const int64_t *blk_off;
    float *g32;
    double *g64;
    double *gsq;
    const double *shape;      // null: exponential window
    int32_t n_shape;
    int32_t shape_num, shape_den;   // support of the samples: [0, num/den] tau
    int32_t delta;            // common offset t_{k0} - t0 of the rows (shape windows)
};

struct RectParams {
    int32_t K, n_bins;
    int32_t n_t0, n_tau;
    int64_t t_sft;
    int32_t n_tiles_n;        // ceil(n_tau / 64)
    int32_t n_tiles;          // per bin
    const RowPlan *rows;
    const int64_t *tau;
    const double *pabc;       // [K+1][8] exclusive prefix: 4 hi then 4 lo terms
    const double *px;         // [n_bins][K+1][8]: per bin, 4 hi then 4 lo terms
    float *twoF;
    Partial *part;
};

struct MergeParams {
    int32_t n_tiles;
    int32_t n_maps;
    int64_t n_cells;
    const Partial *part;      // [n_maps][n_tiles]
    BinResultDev *out;        // [n_maps]
    double *logB_out;         // optional [n_maps]: logB again, as a plain array
};

// ---------------------------------------------------------------------------
// Uneven batch: many maps (different candidates, grids, bins and window
// types) in one persistent launch that draws tiles from a shared list.
// ---------------------------------------------------------------------------

// Tile shapes of the exponential VALU form: (sum type, taus per lane R, bins
// per group BG).
enum ExpShape : int32_t {
    kShapeD41 = 0,   // FP64 sums, R = 4, BG = 1
    kShapeF81 = 1,   // FP32 F_a/F_b, R = 8, BG = 1
    kShapeF42 = 2,   // FP32, R = 4, BG = 2
    kShapeF44 = 3,   // FP32, R = 4, BG = 4
    kShapeCount = 4,
    kShapeMixed = 4,  // fused-kernel variant: each map keeps its own shape
    kShapeF41 = 5     // tile shape only: a four-bin map's one leftover bin
                      // (FP32, R = 4, BG = 1)
};
inline void shape_dims(int shape, int *prec, int *R, int *BG) {
    static const int t[4][3] = {{0, 4, 1}, {1, 8, 1}, {1, 4, 2}, {1, 4, 4}};
    *prec = t[shape][0];
    *R = t[shape][1];
    *BG = t[shape][2];
}

constexpr int kRectRows = 64;   // rows per rect tile (x 64 taus x kRectBins bins)
constexpr int kRectBins = 4;    // bins per rect tile

struct BatchTile {
    int32_t kind;    // 0: exponential, 1: rectangular, 2: exponential, rows far apart,
                     // 3: exponential F_a/F_b only (A, B, C from the A/B/C pre-pass;
                     //    z counts bin pairs)
    int32_t job;     // index into FusedParams::exp_jobs or ::rect_jobs
    int32_t x;       // exp: position in blk_list (kind 2: first of four); rect: tau tile (64 taus)
    int32_t y;       // exp: 64-row tile; rect: kRectRows-row tile
    int32_t z;       // exp: bin group; rect: group of kRectBins bins
    int32_t shape;   // exp: ExpShape of the job (a four-bin map's tail: kShapeF42, kShapeF41)
};

struct FusedParams {
    const ExpValuParams *exp_jobs;
    const RectParams *rect_jobs;
    const BatchTile *tiles;   // largest expected cost first
    int32_t n_tiles;
    int32_t pad;
    int32_t *counter;         // next tile; zeroed before every launch
};

// A/B/C pre-pass of the maps whose tiles sum F_a, F_b only: entry i is
// (64-row tile y[i], position x[i] in blk_list) of job job[i].
struct AbcBatchParams {
    const ExpValuParams *jobs;
    const int32_t *job;
    const int32_t *x;
    const int32_t *y;
    int32_t n_entries;
    int32_t pad;
};

// A, B, C of every cell of an exponential-window map by the recurrence
// over t0 rows (kernels_abc.hip): lanes (tau, segment of seg_rows rows).
struct AbcRecurParams {
    const RowPlan *rows;      // [n_t0], ascending t0
    const int64_t *tau;       // [n_tau]
    const double *abc;        // resident antenna atoms [K+1][4] (a^2, b^2, ab, 0)
    double *abc_out;          // [n_t0][abc_pitch][3] (scaled, exact band)
    int32_t abc_pitch;
    int32_t n_t0, n_tau;
    int32_t K;
    int64_t t_sft;
    int32_t seg_rows;
    int32_t pad;
};

// Many maps: entry e = {map, block of 4 waves of that map}.
struct AbcRecurBatchParams {
    const AbcRecurParams *jobs;
    const int32_t *entries;   // [n_entries][2]
    int32_t n_entries;
    int32_t pad;
};

// Workgroups of 4 waves that cover a map's (tau, segment) waves.
inline int64_t abc_recur_blocks(const AbcRecurParams &p) {
    const int64_t n_seg = (p.n_t0 + p.seg_rows - 1) / p.seg_rows;
    return ((int64_t)p.n_tau * n_seg + 3) / 4;
}

// Weight tables of many maps: entry i is block blk[i] of job job[i].
struct WeightBatchParams {
    const WeightParams *jobs;
    const int32_t *job;
    const int32_t *blk;
    int32_t n_entries;
    int32_t chunks;           // grid.x: 256-element chunks per block
};

// Compensated prefix sums of many channel sets: entry i scans 64 channels.
struct ScanJob {
    const double *in;
    double *out;
    int64_t stride;
    int32_t K, C;
    int32_t chunk;            // first channel / 64
    int32_t pad;
};

struct MergeBatchParams {
    const MergeParams *jobs;
    const int32_t *job;       // [n_entries]
    const int32_t *map;       // [n_entries]
    int32_t n_entries;
    int32_t pad;
};

struct MapReduceParams {
    const float *twoF;        // [n_maps][n_cells]
    int64_t n_cells;
    int32_t n_maps;
    int32_t n_tiles;          // per map
    int64_t cells_per_tile;
    Partial *part;
};

// ---- launchers (kernels.hip) ------------------------------------------------
// Each returns hipSuccess or the launch error.
hipError_t launch_build_x32(const double *x64, float *x32, int64_t n, hipStream_t s);
hipError_t launch_weights(const WeightParams &p, int64_t total_max_per_block,
                          hipStream_t s);
// prec: 0 = FP64 sums, 1 = FP32 sums.  bins_per_group chosen by the caller
// from the supported set reported by exp_valu_config().
// n_groups bin groups of BG bins from p.bin_base.
hipError_t launch_exp_valu(const ExpValuParams &p, int prec, int R, int BG, int n_groups,
                           hipStream_t s);
// The same sums for grids whose t0 rows lie far apart: each row stages its
// own run of slots and the four waves of a workgroup take four consecutive
// blocks of blk_list (p.n_list blocks in groups of four).  Shapes: FP64
// R = 4 BG = 1, FP32 R = 8 BG = 1 and FP32 R = 4 BG = 2 (four-bin maps run
// their runs tiles as bin pairs).
hipError_t launch_exp_runs(const ExpValuParams &p, int prec, int R, int BG, int n_groups,
                           hipStream_t s);
// A/B/C only (FP64), R = 8 blocks, into p.abc_out.
// F_a, F_b only, R = 8 blocks, four bins per lane, n_groups bin groups from
// p.bin_base; A, B, C of every cell read from p.abc_out (short-band blocks
// of the matrix-core form).
hipError_t launch_exp_fonly(const ExpValuParams &p, int n_groups, hipStream_t s);
hipError_t launch_exp_abc(const ExpValuParams &p, hipStream_t s);
hipError_t launch_exp_mfma(const ExpMfmaParams &p, hipStream_t s);
hipError_t launch_exp_mfma_rows(const ExpMfmaRowsParams &p, hipStream_t s);
hipError_t launch_mfma_batch(const MfmaBatchParams &p, hipStream_t s);
hipError_t launch_exp_recur(const RecurParams &p, int BG, hipStream_t s);
hipError_t launch_shift_tables(const ShiftTableParams &p, int64_t max_entries, hipStream_t s);
// Entries per shifted table (one tau, part and shift) for a band of lblk.
// Matrix-core tile constants (compile-time tunables).
#ifndef TFS_MFMA_SK
#define TFS_MFMA_SK 256          // band slots per staged weight window
#endif
#ifndef TFS_MFMA_SHIFTS
#define TFS_MFMA_SHIFTS 4        // shifted weight copies: 4 (8-byte reads) or 8 (16-byte reads)
#endif
#ifndef TFS_MFMA_TWPAD
#define TFS_MFMA_TWPAD 96        // window width beyond SK (>= 72, multiple of 8; sets the LDS pitch:
                                 // SK + 96 = 352 entries spreads the 64 lanes' reads of the four
                                 // shifted copies over all 64 LDS banks)
#endif
constexpr int kMfmaSK = TFS_MFMA_SK;
constexpr int kMfmaShifts = TFS_MFMA_SHIFTS;
constexpr int kMfmaTW = TFS_MFMA_SK + TFS_MFMA_TWPAD;
constexpr int kMfmaPad = 128;    // zero entries in front of every shifted table
static_assert(TFS_MFMA_TWPAD >= 72 && TFS_MFMA_TWPAD % 8 == 0, "window padding");
static_assert(TFS_MFMA_SHIFTS == 4 || TFS_MFMA_SHIFTS == 8, "shifted copies");
// Entries per shifted table (one tau, part and shift) for a band of lblk:
// every staged window [d_lo + kPad, d_lo + kPad + kTW) with d_lo <= lblk - 1.
inline int32_t shift_table_len(int32_t lblk) { return (kMfmaPad + lblk + kMfmaTW + 8 + 7) / 8 * 8; }
hipError_t launch_build_planes(const float *x32, int32_t K, int32_t n_bins, int32_t bins16,
                               int32_t kp, int32_t *colexp, unsigned short *xhi, unsigned short *xlo,
                               hipStream_t s);
hipError_t launch_build_cplanes(const float *x32, int32_t K, int32_t n_bins, int32_t bins16, int32_t kpc,
                                const int32_t *colexp, unsigned short *chi, unsigned short *clo, hipStream_t s);
hipError_t launch_scan(const double *in, int64_t in_row_stride, double *out,
                       int32_t K, int32_t C, hipStream_t s);
hipError_t launch_rect(const RectParams &p, hipStream_t s);
hipError_t launch_merge(const MergeParams &p, hipStream_t s);
hipError_t launch_map_reduce(const MapReduceParams &p, hipStream_t s);
hipError_t launch_abc_recur(const AbcRecurParams &p, hipStream_t s);
hipError_t launch_abc_recur_batch(const AbcRecurBatchParams &p, hipStream_t s);
// Device address of this GPU's allocation-free workspace (noalloc.hip):
// looked up once per device with that device current, null before.
hipError_t noalloc_setup(int device);
void *noalloc_scratch(int device);
hipError_t launch_weights_batch(const WeightBatchParams &p, hipStream_t s);
hipError_t launch_abc_batch(const AbcBatchParams &p, hipStream_t s);
hipError_t launch_scan_batch(const ScanJob *jobs, int32_t n_jobs, hipStream_t s);
hipError_t launch_merge_batch(const MergeBatchParams &p, hipStream_t s);
hipError_t launch_fill_i32(int32_t *dst, int32_t n, int32_t value, hipStream_t s);
// variant = shape + (kShapeMixed + 1) * m: shape is an ExpShape (every exp
// job in the batch has that shape) or kShapeMixed; m = 0 builds for the
// stand-alone kernel's waves per SIMD, m = 1 for one fewer.  n_groups
// workgroups loop over the tile list.
constexpr int kFusedVariants = 2 * (kShapeMixed + 1);
inline int fused_shape(int variant) { return variant % (kShapeMixed + 1); }
hipError_t launch_fused(const FusedParams &p, int variant, int n_groups, hipStream_t s);
// Most workgroups of the fused kernel variant that fit on one CU at once.
int fused_groups_per_cu(int variant);

// Supported VALU tile shapes: tau columns per block R and bins per lane BG
// for a precision and bin count.
void exp_valu_config(int prec, int n_bins, int *R, int *BG);

}  // namespace tfs
