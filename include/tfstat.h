/*
 * tfstat — transient F-statistic maps on AMD MI355X (gfx950).
 *
 * C ABI of the library.  The method is the atoms-based transient
 * F-statistic of Keitel & Ashton (arXiv:1805.05652):
 *
 *   - Section 2 (eq. winrect, eq. winexp) defines the rectangular window
 *     (1 on [t0, t0 + tau]) and the exponential window
 *     (exp(-(t - t0)/tau) on [t0, t0 + 3 tau]);
 *   - section 2 (eq. F_FaFb) gives F from the windowed antenna sums A, B, C,
 *     their determinant D = A B - C^2 and the windowed data sums F_a, F_b;
 *   - section 2 (eq. Fmn) defines the transient map F_mn over a grid of start
 *     times t0_m and durations tau_n;
 *   - section 3 states the inputs: per-SFT vectors a^2, b^2, ab (real) and
 *     F_a, F_b (complex), a window type and a {t0, tau} grid;
 *   - the footnote of appendix A names the marginalised Bayes factor over
 *     the map, whose exponent is F (eq. F_OSG).
 *
 * Conventions (where the paper leaves the details open):
 *   - A window holds the SFTs whose START time t_j satisfies
 *     t0 <= t_j < t0 + tau (rect) or t0 <= t_j < t0 + 3 tau (exp); the
 *     decision is made in integer seconds.
 *   - A, B, C use weights w^2 and F_a, F_b use weights w.
 *   - Windows past the end of the data are truncated (appendix A), never
 *     renormalised; the full n_t0 x n_tau map is still produced.
 *   - A cell with D <= 1e-10 * A * B (empty, single-SFT or rank-one window)
 *     has 2F = 0.
 *   - logB = ln( (1/(n_t0 n_tau)) * sum_mn exp(F_mn) ), with F = 2F/2 and a
 *     flat prior over the grid cells; degenerate cells count with F = 0.
 *   - The argmax is the first maximum of 2F in row-major (m, n) order.
 *
 * Memory and threading:
 *   - Host pointers passed in are borrowed for the duration of the call.
 *   - Device memory for atoms and workspaces is sub-allocated from the arena
 *     the caller hands to tfstat_ctx_create; the library itself calls no
 *     device allocator.  The arena and the stream must outlive the context.
 *   - tfstat_fmap and tfstat_logB are synchronous on the context's stream.
 *   - tfstat_submit / tfstat_poll / tfstat_cancel are thread-safe; other
 *     calls on one context must not run concurrently with each other.
 *   - Results are deterministic for a given (atoms, window, precision).
 *
 * Errors: every function returns a tfstat_status; 0 is success.  On error no
 * output is written and tfstat_last_error() describes the failure (the
 * message is thread-local and valid until the next call on that thread).
 */
#ifndef TFSTAT_H
#define TFSTAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TFSTAT_OK = 0,
    TFSTAT_E_INVAL = -1,      /* bad argument (null pointer, bad enum, size) */
    TFSTAT_E_GRID = -2,       /* timestamps off the slot grid, bad t0/tau grid */
    TFSTAT_E_NOMEM = -3,      /* the arena cannot hold the request */
    TFSTAT_E_DEVICE = -4,     /* a HIP runtime call failed */
    TFSTAT_E_BUSY = -5,       /* serving queue full */
    TFSTAT_E_NOTFOUND = -6,   /* unknown atoms id or ticket */
    TFSTAT_E_CANCELLED = -7   /* the ticket was cancelled */
} tfstat_status;

typedef enum {
    TFSTAT_WIN_RECT = 0,      /* eq. winrect */
    TFSTAT_WIN_EXP = 1,       /* eq. winexp, cut off at 3 tau */
    TFSTAT_WIN_SHAPE = 2      /* any shape s((t - t0)/tau) given as samples (section 5:
                                 other window functions follow the exponential
                                 window's kernels); see tfstat_window */
} tfstat_window_type;

/*
 * Arithmetic of the windowed sums.  A, B, C, D and F are FP64 in every mode.
 *   FP64   : F_a, F_b sums in FP64.
 *   FP32   : F_a, F_b sums in FP32 (the paper's single precision).
 *   BF16X3 : F_a, F_b sums on bf16 matrix cores with split hi + lo operands
 *            (three products: hi*hi + hi*lo + lo*hi) and FP32 accumulation
 *            (section 3, exponential case: every cell is one banded
 *            contraction over the SFTs, shared by all bins), for
 *            exponential-window maps of 2 or more bins on any t0 grid, and
 *            for shape windows whose t0 rows fall on consecutive slots with
 *            one common offset.  Blocks of 8 taus whose shortest band is
 *            under 64 slots, one-bin exponential maps and other
 *            shape-window grids run the FP32 sums.  bf16 hi + lo keeps 16 significant
 *            bits per operand (relative residual up to 2^-17), so 2F can
 *            miss a 1e-4 relative bound on a few cells of badly conditioned
 *            windows; F16X3 meets it.  The first call on an atoms set builds
 *            its bf16 planes (16 bytes per slot and bin of arena; sets of
 *            2 to 48 bins 32 more, for the transposed form of their sums).
 *   F16X3  : as BF16X3 with IEEE half-precision hi + lo parts (22
 *            significant bits per operand, relative residual up to 2^-23),
 *            the data columns scaled by powers of two (one per bin and
 *            component, undone exactly in FP64) and the weights by 2^4, so
 *            that no part leaves the half-precision range.  Exponential
 *            windows only: shape windows run the FP32 sums.  In a map that
 *            has a block of 8 taus with every band at least 64 slots long,
 *            the blocks whose shortest band is at least 24 slots run on the
 *            matrix cores (shorter windows amplify the parts' rounding).
 *            Builds its own planes on first use (16 bytes per slot and bin;
 *            sets of 2 to 48 bins 32 more).
 *   RECUR64: exponential windows on a regular t0 grid whose step is a whole
 *            number of SFT slots (at most 64): every sum in FP64 by the exact
 *            recurrence of the window sums from one t0 to the next, O(1)
 *            per cell and channel instead of O(window length); windows
 *            holding fewer than two SFTs are summed directly.  Other grids
 *            run the FP64 direct sums.
 * Rectangular windows use FP64 prefix sums in every mode.
 */
typedef enum {
    TFSTAT_PREC_FP64 = 0,
    TFSTAT_PREC_FP32 = 1,
    TFSTAT_PREC_BF16X3 = 2,
    TFSTAT_PREC_RECUR64 = 3,
    TFSTAT_PREC_F16X3 = 4
} tfstat_precision;

/*
 * Search grid (eq. Fmn; section 3 allows gaps and resolutions other than
 * T_sft).  All times are integer seconds.  The start times are
 * t0_list[m] when t0_list is non-null, else t0_min + m * dt0 (dt0 >= 1);
 * likewise for tau.  Both sequences must be strictly increasing and every
 * tau must be >= 1; otherwise TFSTAT_E_GRID.
 *
 * Shape windows (type TFSTAT_WIN_SHAPE): the weight of an SFT starting at t
 * is s(x), x = (t - t0) / tau, for t in [t0, t0 + floor(tau * support_num /
 * support_den)) and 0 elsewhere; s is linear between the n_shape samples
 * shape[i] = s(i * S / (n_shape - 1)), S = support_num / support_den.  The
 * sums run through the exponential window's kernels with the samples in
 * place of the exponential.  Every t0 must sit at the same offset from the
 * SFT start grid (t0 - t_first = const mod t_sft; e.g. t0 on SFT starts),
 * else TFSTAT_E_GRID; 2 <= n_shape <= 65536; 1 <= support_num, support_den
 * <= 1024; tau <= 2^50; samples finite.  RECUR64 does not apply to shapes
 * (TFSTAT_E_INVAL).  For other types the shape fields are ignored.
 */
typedef struct {
    int32_t type;             /* tfstat_window_type */
    int32_t n_t0;             /* >= 1 */
    int32_t n_tau;            /* >= 1 */
    int32_t reserved;         /* must be 0 */
    int64_t t0_min, dt0;
    int64_t tau_min, dtau;
    const int64_t *t0_list;   /* optional, [n_t0] host memory */
    const int64_t *tau_list;  /* optional, [n_tau] host memory */
    const double *shape;      /* shape windows: [n_shape] samples, host memory */
    int32_t n_shape;
    int32_t support_num, support_den;
    int32_t reserved2;        /* must be 0 */
} tfstat_window;

/*
 * Atoms of one candidate (section 2: {a_j, b_j, F_aj, F_bj} per SFT j,
 * shipped as a^2, b^2, ab and complex F_a, F_b per section 3).  All host
 * memory.  Timestamps are SFT start times, strictly increasing, each equal
 * to timestamps[0] + k * t_sft for an integer k (SFTs on a common slot grid;
 * gaps allowed), else TFSTAT_E_GRID.  The antenna atoms are shared by all
 * frequency bins; fa and fb hold [n_bins][n_sft][2] interleaved (re, im).
 */
typedef struct {
    int32_t n_sft;            /* >= 1 */
    int32_t n_bins;           /* >= 1 */
    int64_t t_sft;            /* SFT length in seconds, >= 1 */
    const int64_t *timestamps;
    const double *a2, *b2, *ab;
    const double *fa, *fb;
} tfstat_atoms_desc;

/* Per-bin result of one map (appendix A footnote; eq. Fmn). */
typedef struct {
    double max2F;             /* largest 2F over the map */
    double logB;              /* marginalised log Bayes factor, see above */
    int64_t t0, tau;          /* grid values at the argmax */
    int32_t m, n;             /* argmax indices */
} tfstat_bin_result;

typedef struct tfstat_ctx tfstat_ctx;
typedef uint64_t tfstat_atoms_id;
typedef uint64_t tfstat_ticket;

/*
 * Creates a context on HIP device `device`.  `arena_dev` is device memory of
 * `arena_bytes` bytes (e.g. a torch tensor's storage), 256-byte aligned,
 * which the context sub-allocates; `hip_stream` is a hipStream_t (may be
 * null for the null stream) on which every synchronous call runs.
 * Errors: E_INVAL (null out, unaligned arena, arena under 1 MiB),
 * E_DEVICE (bad device).
 */
int tfstat_ctx_create(int device, void *arena_dev, size_t arena_bytes,
                      void *hip_stream, tfstat_ctx **out);

/* Waits for in-flight work, then releases host resources.  Atoms ids die. */
int tfstat_ctx_destroy(tfstat_ctx *ctx);

/*
 * Copies one candidate's atoms to the device and keeps them resident (as
 * zero-filled slots on the T_sft grid) until tfstat_atoms_free.
 * Errors: E_INVAL, E_GRID (see tfstat_atoms_desc), E_NOMEM, E_DEVICE.
 */
int tfstat_atoms_upload(tfstat_ctx *ctx, const tfstat_atoms_desc *desc,
                        tfstat_atoms_id *out);

/* Releases resident atoms.  E_NOTFOUND for an unknown id, E_BUSY while a
 * submitted request still uses them. */
int tfstat_atoms_free(tfstat_ctx *ctx, tfstat_atoms_id id);

/* Number of slots K and bins of resident atoms. */
int tfstat_atoms_info(tfstat_ctx *ctx, tfstat_atoms_id id, int32_t *n_slots,
                      int32_t *n_bins);

/*
 * Computes the transient F-statistic map of every bin of the atoms over the
 * window grid (eq. Fmn with eq. F_FaFb) and its per-bin results.
 *   twoF_dev  optional device pointer, float [n_bins][n_t0][n_tau]
 *             row-major, receives 2F; pass null to skip the map.
 *   res_host  host array of n_bins results.
 * Synchronous on the context stream.
 * Errors: E_INVAL, E_GRID, E_NOTFOUND, E_NOMEM (workspace), E_DEVICE.
 */
int tfstat_fmap(tfstat_ctx *ctx, tfstat_atoms_id id, const tfstat_window *win,
                int32_t precision, float *twoF_dev, tfstat_bin_result *res_host);

/*
 * Marginalised log Bayes factor of existing 2F maps (appendix A footnote):
 * logB = ln((1/(n_t0 n_tau)) sum exp(2F/2)), max-shifted, for each of
 * n_maps maps of twoF_dev (device, float [n_maps][n_t0][n_tau]).
 * Errors: E_INVAL, E_NOMEM, E_DEVICE.
 */
int tfstat_logB(tfstat_ctx *ctx, const float *twoF_dev, int32_t n_maps,
                int32_t n_t0, int32_t n_tau, double *logB_host);

/*
 * For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid device or pinned-host
 * allocation): tfstat_logB without any allocation.  Same kernels and the
 * same results, bit for bit, as tfstat_logB on the same maps.
 *   twoF_dev  device, float [n_maps][n_t0][n_tau] (read only);
 *   logB_dev  device, double [n_maps] (written).
 * The per-tile partials and per-map results live in one static device
 * array per GPU of TFSTAT_NOALLOC_SCRATCH_BYTES bytes, held until the
 * process ends; a call needs 24 * n_maps * ceil(n_t0 n_tau / 16384) bytes
 * (rounded up to 256) plus 24 * n_maps, and larger calls fail with E_INVAL.
 * The call is asynchronous on the context's stream (no host
 * synchronisation; the result is ready when the stream reaches it).  Every
 * call on one GPU shares that GPU's array: calls that may overlap on one
 * GPU (other streams, other contexts, other threads) race and must be
 * ordered by the caller.
 * Errors: E_INVAL (null pointer, sizes < 1, workspace above the limit),
 * E_DEVICE.
 */
#define TFSTAT_NOALLOC_SCRATCH_BYTES (4u << 20)
int tfstat_logB_noalloc(tfstat_ctx *ctx, const float *twoF_dev, int32_t n_maps,
                        int32_t n_t0, int32_t n_tau, double *logB_dev);

/*
 * A-posteriori comparison of two window models on the same atoms (section 5:
 * different window functions are compared through their Bayes factors).
 * Computes both maps like tfstat_fmap (no map is materialised) and writes,
 * per bin, the log odds of window model a against window model b with even
 * prior odds: log_odds_host[bin] = logB_a - logB_b, each logB marginalised
 * over its own grid with a flat prior.  The two windows may differ in type,
 * grid or both.  Synchronous on the context stream.
 * Errors: as tfstat_fmap for either window.
 */
int tfstat_window_odds(tfstat_ctx *ctx, tfstat_atoms_id id, const tfstat_window *win_a,
                       const tfstat_window *win_b, int32_t precision, double *log_odds_host);

/*
 * Serving: queues a map request over resident atoms and returns a ticket at
 * once.  Requests run concurrently on the device as workspace memory and
 * worker slots allow (admission by arena footprint); each result equals the
 * one tfstat_fmap gives for the same arguments.  No map is materialised.
 * Errors: E_INVAL, E_GRID, E_NOTFOUND, E_NOMEM (could never fit),
 * E_BUSY (queue full).
 */
int tfstat_submit(tfstat_ctx *ctx, tfstat_atoms_id id, const tfstat_window *win,
                  int32_t precision, tfstat_ticket *out);

/*
 * Non-blocking completion check.  *done is set to 1 and res_host (n_bins
 * results) is written when the request finished; the ticket is then
 * retired.  Returns the request's own error if it failed, E_CANCELLED for a
 * cancelled ticket, E_NOTFOUND for an unknown or retired ticket.
 */
int tfstat_poll(tfstat_ctx *ctx, tfstat_ticket t, tfstat_bin_result *res_host,
                int *done);

/* Cancels a queued request (a running one completes, its result dropped). */
int tfstat_cancel(tfstat_ctx *ctx, tfstat_ticket t);

/*
 * Serving admission.  Whenever one of the context's stream slots is free,
 * the requests at the head of the queue are admitted together: up to
 * max_batch of them (default 16), as many as the arena holds, run as one
 * batch with one persistent fused launch over all their tiles, plus the
 * matrix-core launches for BF16X3 / F16X3 requests (one for maps of 2 to 48
 * bins, one for wider maps; requests of one precision
 * each, of up to 2e9 window terms -- cells x slots x bins, or cells x bins
 * for rectangular windows; larger requests, matrix-core shape windows and
 * recurrence requests run alone with their own kernels).  max_batch = 1
 * admits one request per slot.  Results never depend on the batching.
 * Errors: E_INVAL (max_batch outside 1..1024).
 */
int tfstat_serve_config(tfstat_ctx *ctx, int32_t max_batch);

/*
 * Tiling of exponential-window maps (section 3: every cell sums its own
 * window).  The VALU sums take 64 t0 rows at a time.
 *
 * Runs form.  When the rows of a tile start far apart in slot space (a t0
 * step of many SFTs), the union of their windows does not fit one
 * shared-memory stage; such maps stage each row's own run of slots instead,
 * four tau blocks per workgroup.  A map takes the runs form when the median
 * over its 64-row tiles of the slot span between first and last row is at
 * least runs_min_spread (0 sends every map there).  A negative value
 * restores the default: the runs form when that span exceeds 448 slots,
 * what the band stage holds, for maps with two or more bins per lane or
 * FP64 sums (FP32 maps with one bin stay on the band-staged form, which
 * reads such rows through the caches).
 *
 * Split form.  An FP32 map with at least split_min_bins bins (default 8;
 * 0: never; a negative value restores the default) whose tiles fit the band
 * stage computes A, B, C of every cell once, in FP64, and then sums only
 * F_a, F_b, four bins per lane; otherwise every group of bins sums A, B, C
 * again.  An explicit runs_min_spread that the map reaches takes precedence.
 *
 * Every form sums the same terms with the same weights, so they agree
 * within rounding.  The choice is made when a map is planned (tfstat_fmap,
 * tfstat_submit, tfstat_batch_create), so a map gives the same results
 * alone, batched and served.  Errors: E_INVAL for a null ctx.
 */
int tfstat_tiling_config(tfstat_ctx *ctx, int32_t runs_min_spread, int32_t split_min_bins);

/*
 * Uneven batch: many maps -- different resident atoms, grids, numbers of
 * bins and window types -- computed together (the per-map work of section 3,
 * for the many candidates and frequency bins of section 5).  A batch is
 * planned once and can be run many times.  Each run is one captured HIP
 * graph: the weight tables and prefix sums of all maps, then ONE persistent
 * launch in which every workgroup draws tiles of all maps from a shared
 * list (largest expected cost first), then the per-bin merges.  Every
 * result equals what tfstat_fmap returns for the same map at the same
 * precision (same arithmetic per cell, same tile partials and merge order),
 * so a map's results do not depend on which other maps share its batch
 * (tune = 0 or 1; a forced variant, tune = -1 - v, may change tile shapes).
 * No maps are materialised.
 *   n_maps     number of maps; ids[i] and wins[i] describe map i.
 *   precision  TFSTAT_PREC_FP32, TFSTAT_PREC_FP64, TFSTAT_PREC_BF16X3 or
 *              TFSTAT_PREC_F16X3 (exponential sums; rectangular windows
 *              always use compensated FP64 prefixes).  In BF16X3 and F16X3
 *              the matrix-core work of all maps is one more launch after the
 *              persistent one; matrix-core shape windows are refused
 *              (E_INVAL; tfstat_fmap runs them).
 *   tune       0: each map's own tile shape, default launch width;
 *              1: time every candidate that keeps each map's own tile shape
 *              (the build for the stand-alone kernel's waves per SIMD or one
 *              fewer x persistent workgroups per CU) on this batch and keep
 *              the fastest; the choice is cached in the context under the
 *              batch's shape signature and reused by later batches of the
 *              same shape.  Results are those of tfstat_fmap either way.
 *              -1 - v: the fused-kernel variant v of tfstat_batch_stats
 *              (0 or 5 for FP64; 1..4 or 6..9 for FP32) at its widest
 *              launch, without the tuning cache; variants other than 0, 5
 *              (FP64) and 4, 9 (FP32) impose one tile shape on every map, so
 *              their results agree with tfstat_fmap within rounding only
 *              (which lets a caller compare the shapes).
 * The plan keeps its workspace in the arena, and its atoms busy, until
 * tfstat_batch_destroy.
 * Errors: E_INVAL, E_GRID, E_NOTFOUND, E_NOMEM, E_DEVICE.
 */
typedef struct tfstat_batch tfstat_batch;

typedef struct {
    int32_t variant;          /* fused-kernel build: tile shape (0 FP64 R4, 1 FP32 R8, 2 FP32 R4 x 2 bins,
                                 3 FP32 R4 x 4 bins, 4 per-map shape by its bin count), plus 5
                                 when built for one wave per SIMD fewer than the
                                 stand-alone kernel (more registers per wave) */
    int32_t groups;           /* persistent workgroups of the fused launch */
    int32_t n_tiles;          /* tiles in the shared list */
    int32_t n_results;        /* sum of n_bins over the maps */
    double tune_ms;           /* host time spent tuning (0 if not tuned here) */
    double last_ms;           /* device time of the last run (HIP events) */
    double last_fused_ms;     /* device time of the fused launch in the last timed run */
    double last_mfma_ms;      /* device time of the matrix-core launches of BF16X3 / F16X3
                                 maps in the last timed run (0 without such maps) */
} tfstat_batch_stats;

int tfstat_batch_create(tfstat_ctx *ctx, int32_t n_maps, const tfstat_atoms_id *ids,
                        const tfstat_window *wins, int32_t precision, int32_t tune,
                        tfstat_batch **out);

/* Runs the batch (synchronous).  res_host receives n_results entries: the
 * n_bins results of map 0, then those of map 1, and so on.  timed = 0
 * replays the captured graph; timed = 1 launches the same steps directly
 * with HIP events around the persistent fused launch (its time goes to
 * last_fused_ms; results are identical). */
int tfstat_batch_run(tfstat_ctx *ctx, tfstat_batch *b, int32_t timed,
                     tfstat_bin_result *res_host);

int tfstat_batch_stats_read(const tfstat_batch *b, tfstat_batch_stats *out);

int tfstat_batch_destroy(tfstat_ctx *ctx, tfstat_batch *b);

/*
 * Per-kernel timing.  When enabled, the context brackets each kernel launch
 * with HIP events on its stream; tfstat_profile_read returns, for kernel
 * class `kind` (see tfstat_kernel_kind), the number of launches and their
 * summed device time in milliseconds since the last reset.
 */
typedef enum {
    TFSTAT_K_UPLOAD = 0,      /* slot planes from uploaded atoms */
    TFSTAT_K_WEIGHTS = 1,     /* exponential weight tables */
    TFSTAT_K_EXP = 2,         /* exponential-window sums + finalize (VALU) */
    TFSTAT_K_SCAN = 3,        /* rectangular prefix sums */
    TFSTAT_K_RECT = 4,        /* rectangular cells + finalize */
    TFSTAT_K_MERGE = 5,       /* per-bin reduction merge */
    TFSTAT_K_MFMA = 6,        /* exponential F_a, F_b on matrix cores */
    TFSTAT_K_ABC = 7,         /* exponential A, B, C (FP64) */
    TFSTAT_K_RECUR = 8,       /* exponential sums by the t0 recurrence */
    TFSTAT_K_COUNT = 9
} tfstat_kernel_kind;

int tfstat_profile_enable(tfstat_ctx *ctx, int on);
int tfstat_profile_read(tfstat_ctx *ctx, int32_t kind, int64_t *launches,
                        double *total_ms);
int tfstat_profile_reset(tfstat_ctx *ctx);

/* Thread-local message for the last failing call on this thread. */
const char *tfstat_last_error(void);

/* Library version string. */
const char *tfstat_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TFSTAT_H */
