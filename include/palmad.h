/*
 * palmad.h -- C ABI of the MI355X (gfx950) range-discord search library.
 *
 * The library finds, for every subsequence length m in [minL, maxL], the
 * top-k discords of a time series: the subsequences whose distance to their
 * nearest non-self match is largest (Sec. 2.1, Eq. (1)-(5)), by the method of
 * the paper: per-length statistics updated by recurrence (Sec. 3.1.1,
 * Eq. (7)-(8)), candidate selection and refinement passes against a range r
 * (Sec. 3.2-3.3, after the serial DRAG of Alg. 2), and MERLIN's adaptive
 * choice of r over the lengths (Alg. 1).
 *
 * Conventions shared by every entry point:
 *   - Indices are 0-based.  Subsequence i of length m covers T[i .. i+m-1];
 *     N(m) = n - m + 1.  Two subsequences are a non-self match iff
 *     |i - j| >= m.
 *   - Distances are z-normalised Euclidean distances (population sigma) in
 *     ED units, not squared.  A flat window (sigma <= 1e-12 * max(1, sigma
 *     of the whole series)) is at distance 0 from another flat window and
 *     sqrt(2m) from any other window.
 *   - Output row q = (m - minL) * k + rank; rank 0 has the largest nnDist;
 *     equal nnDist values are ordered by smaller index; a nearest-neighbour
 *     tie reports the smaller neighbour index.
 *   - Pointers documented as "device" must point to memory of the context's
 *     device; the library never frees or retains them.  A call runs on the
 *     context's own stream, after the work already queued on the HIP stream
 *     given to the call and before any work queued there later; it returns
 *     once the result is complete (the adaptive r loop reads one counter
 *     every few rounds of range searches).
 *   - Every function returns a palmad_status and palmad_last_error()
 *     describes a failure.  Arguments are validated on the host before any
 *     device work; on an argument error (PALMAD_EINVAL, PALMAD_EWORKSPACE,
 *     PALMAD_EUNSUPPORTED) or PALMAD_ENONFINITE nothing is written to the
 *     outputs.  After PALMAD_EDEVICE the outputs are undefined: rows of the
 *     lengths finished before the failure may have been written.  No C++
 *     exception crosses this interface.
 *   - The environment variable PALMAD_FAULT injects failures for tests of
 *     the error paths: "hip" makes a search fail as if its first HIP call
 *     had failed (PALMAD_EDEVICE, no device work); "converge" allows one
 *     range search per length, so a search reports a range search that did
 *     not converge (PALMAD_EDEVICE after device work).
 *   - One context per host thread at a time.  The context caches the
 *     hipGraph of one round of the search for the last workspace and
 *     configuration it saw, and replays it while they stay the same.
 */
#ifndef PALMAD_H
#define PALMAD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PALMAD_OK = 0,
    PALMAD_EINVAL = -1,       /* invalid argument (null pointer, bad range, ...) */
    PALMAD_ENONFINITE = -2,   /* the series holds NaN or Inf */
    PALMAD_EWORKSPACE = -3,   /* workspace smaller than palmad_workspace_size() */
    PALMAD_EDEVICE = -4,      /* a HIP call failed */
    PALMAD_ENOMEM = -5,       /* host allocation failed */
    PALMAD_EUNSUPPORTED = -6  /* valid request outside what this library supports */
} palmad_status;

/* Options; a zero-initialised struct selects the defaults. */
typedef struct {
    int32_t dist_bits;     /* 32: FP32 selection sweep (statistics, refinement and
                              reported distances stay FP64); 64: FP64 throughout.
                              0 = 32. */
    float guard;           /* correlation guard band of the FP32 selection sweep:
                              a pair prunes only if its FP32 correlation exceeds the
                              threshold by more than this.  <= 0 = 1.25e-4. */
    int32_t near_cols;     /* columns scanned by the first selection pass of a row
                              tile (in chunks of chunk_cols run concurrently) before
                              the remaining columns go to the queued pass; 0 = 2048.
                              Capped so that the longest series has at most 65536
                              (tile, chunk) items in the first pass. */
    int32_t chunk_cols;    /* columns per work item of the sweeps; 0 = 1024. */
    uint32_t flags;        /* PALMAD_FLAG_* bits */
    int32_t rows_near;     /* row-tile height of the first selection pass: 128, 256 or
                              512; 0 = 512 (FP32) / 256 (FP64). */
    int32_t rows_far;      /* row-tile height of the split selection pass; 0 = as near. */
    int32_t rows_refine;   /* row-tile height of the refinement pass; 0 = 128. */
    int32_t far_grid;      /* workgroups of the split passes (1..65536); 0 = 2048. */
    int32_t band_pass;     /* 1: before the first selection pass, test every
                              subsequence against its 256 nearest non-self offsets
                              on the right, swept down the diagonals (prunes only;
                              results unchanged); 0 or -1: off. */
    int32_t reserved[2];   /* must be zero */
} palmad_options;

/* Record HIP events around the sweep kernels and report their summed device
   time per kernel class in palmad_stats (adds two event records per timed
   launch). */
#define PALMAD_FLAG_TIME_KERNELS 1u
/* Launch every kernel of a round directly instead of replaying the
   context's cached round graph (set implicitly by PALMAD_FLAG_TIME_KERNELS). */
#define PALMAD_FLAG_NO_GRAPH 2u

/* Kernel classes of palmad_stats.kernel_* (one entry each). */
enum {
    PALMAD_KERNEL_SELECT_NEAR = 0, /* first selection pass of every row tile */
    PALMAD_KERNEL_SELECT_FAR = 1,  /* split selection pass over the remaining columns */
    PALMAD_KERNEL_REFINE = 2,      /* refinement pass (exact FP64 nearest neighbour) */
    PALMAD_KERNEL_POLISH = 3,      /* direct FP64 distances of the top candidates */
    PALMAD_KERNEL_LENGTH = 4,      /* per-length statistics, helpers and round resets */
    PALMAD_KERNEL_SELECT_BAND = 5, /* diagonal band pre-pass of the first selection pass */
    PALMAD_KERNEL_CLASSES = 6
};

/* Per-call counters (host struct, filled when the call returns). */
typedef struct {
    uint64_t evals_select;   /* pair correlations evaluated by selection passes */
    uint64_t evals_refine;   /* pair correlations evaluated by refinement passes */
    uint64_t evals_polish;   /* pair distances evaluated by the exact FP64 pass */
    uint64_t range_searches; /* selection+refinement rounds (DRAG calls), all lengths */
    uint64_t survivors;      /* range discords summed over the successful rounds */
    double seconds;          /* host wall time of the call */
    uint64_t kernel_evals[PALMAD_KERNEL_CLASSES];    /* pair evaluations per class */
    uint64_t kernel_launches[PALMAD_KERNEL_CLASSES]; /* launches per class */
    double kernel_ms[PALMAD_KERNEL_CLASSES];         /* device time per class (flag set) */
    uint64_t rows_after_near; /* live subsequences after the first selection pass, summed
                                 over the range searches that prune */
    uint64_t rows_after_far;  /* live subsequences entering refinement, summed likewise */
} palmad_stats;

typedef struct palmad_ctx palmad_ctx;

/* Library version string (static storage). */
const char* palmad_version(void);

/* Message for the last error on this context (or of the last failed
   palmad_create / argument check when ctx is NULL).  Static or
   context-owned storage; valid until the next call on the context. */
const char* palmad_last_error(const palmad_ctx* ctx);

/* Create a context bound to HIP device `device`.  *out receives the
   context; destroy it with palmad_destroy().  Allocates a few hundred bytes
   of device and pinned host memory for control state. */
int palmad_create(palmad_ctx** out, int device);

/* Destroy a context (NULL is ignored).  Waits for the context's work. */
void palmad_destroy(palmad_ctx* ctx);

/*
 * Bytes of device workspace palmad_discords() needs for a series of length
 * n, lengths [minL, maxL] and top-k.  Pure host computation (no device, no
 * context).  Returns PALMAD_EINVAL for arguments palmad_discords() would
 * reject: minL < 3, maxL < minL, n < 3*maxL - 1 (so that every subsequence
 * has a non-self match), k < 1 or k > n - maxL + 1; PALMAD_EUNSUPPORTED for
 * k > 64 or maxL > 2800.
 */
int palmad_workspace_size(int64_t n, int32_t minL, int32_t maxL, int32_t k,
                          const palmad_options* opts, size_t* bytes);

/*
 * Top-k discords of every length in [minL, maxL] (MERLIN over the lengths,
 * Alg. 1; each range search is a selection pass and a refinement pass,
 * Sec. 3.2-3.3).
 *
 *   T          device, float64[n]: the series (read only).
 *   workspace  device, >= palmad_workspace_size() bytes, 256-byte aligned;
 *              scratch owned by the caller, contents undefined on return.
 *   idx        device, int64[L*k]: start index of each discord.
 *   len        device, int32[L*k]: its length m.
 *   nn_dist    device, float64[L*k]: distance to its nearest non-self match.
 *   nn_idx     device, int64[L*k]: index of that nearest non-self match.
 *   count      device, int32[L]: number of range discords (subsequences with
 *              nnDist >= r) found by the successful range search of each
 *              length; always >= k.
 *   stats      host, optional (NULL): counters of this call.
 *   stream     HIP stream (hipStream_t) or NULL for the null stream.
 * with L = maxL - minL + 1.
 */
int palmad_discords(palmad_ctx* ctx, const double* T, int64_t n, int32_t minL, int32_t maxL,
                    int32_t k, const palmad_options* opts, void* workspace, size_t ws_bytes,
                    int64_t* idx, int32_t* len, double* nn_dist, int64_t* nn_idx, int32_t* count,
                    palmad_stats* stats, void* stream);

/*
 * Bytes of device workspace palmad_discords_batched() needs.  Pure host
 * computation; the arguments are those of palmad_discords_batched(), and
 * the same argument errors are reported.
 */
int palmad_batched_workspace_size(int32_t B, const int64_t* offsets, const int32_t* minL,
                                  const int32_t* maxL, int32_t k, const palmad_options* opts,
                                  size_t* bytes);

/*
 * palmad_discords() over B independent series at once (not in the paper: a
 * serving form of Alg. 1).  Every series runs its own MERLIN walk over its
 * own lengths with its own r; one round performs one range search for every
 * series that still has work, in shared launches, so the device stays full
 * even when single series are too short to fill it.  Results equal B
 * separate palmad_discords() calls.
 *
 *   values   device, float64[offsets[B]]: the series back to back; series b
 *            is values[offsets[b] .. offsets[b+1]).
 *   offsets  host, int64[B+1], offsets[0] = 0, non-decreasing.
 *   minL, maxL  host, int32[B]: the length range of each series; each
 *            series must satisfy the conditions of palmad_workspace_size().
 *   k        top-k of every series and length (1..64).
 *   idx, len, nn_dist, nn_idx  device, sum_b L_b*k rows, L_b = maxL[b] -
 *            minL[b] + 1: the rows of series b follow those of series b-1,
 *            each block laid out as in palmad_discords().
 *   count    device, int32[sum_b L_b], blocks in series order.
 *   stats    host, optional: counters summed over the batch.
 * PALMAD_ENONFINITE if any series holds NaN/Inf (the message names the first);
 * PALMAD_EUNSUPPORTED for B > 65535.
 */
int palmad_discords_batched(palmad_ctx* ctx, const double* values, const int64_t* offsets,
                            int32_t B, const int32_t* minL, const int32_t* maxL, int32_t k,
                            const palmad_options* opts, void* workspace, size_t ws_bytes,
                            int64_t* idx, int32_t* len, double* nn_dist, int64_t* nn_idx,
                            int32_t* count, palmad_stats* stats, void* stream);

/* Result of palmad_autotune() (host struct). */
typedef struct {
    int32_t evaluated;       /* configurations timed */
    int32_t probe_lengths;   /* lengths per series searched by each probe */
    double base_seconds;     /* best probe time of the options passed in */
    double best_seconds;     /* best probe time of the options returned */
} palmad_tune_report;

/*
 * Bytes of device workspace palmad_autotune() needs (the probe's search
 * workspace plus its result rows).  Arguments as palmad_autotune().
 */
int palmad_autotune_workspace_size(int32_t B, const int64_t* offsets, const int32_t* minL,
                                   const int32_t* maxL, int32_t k, int32_t probe_lengths,
                                   size_t* bytes);

/*
 * Pick the tile geometry of the sweeps (not in the paper): row-tile heights
 * of the three passes, near_cols, chunk_cols and far_grid, by timing the
 * search itself on a probe, one coordinate at a time starting from `base`
 * (dist_bits, guard and flags are kept).  The probe searches every series
 * over its first probe_lengths lengths (fewer if its range is shorter);
 * each configuration runs once untimed, then `reps` times, and its best
 * wall time counts.  The tile geometry changes the order of floating-point
 * work only: results agree within the documented tolerance for any choice.
 *
 *   values, offsets, B, minL, maxL, k  as palmad_discords_batched() (B = 1
 *            with offsets {0, n} for a single series).
 *   base     options to start from (NULL = defaults).
 *   probe_lengths  >= 1 (values above a series' range are clipped).
 *   reps     timed runs per configuration, >= 1.
 *   workspace  device, >= palmad_autotune_workspace_size() bytes.
 *   best     host: the chosen options.
 *   report   host, optional (NULL).
 */
int palmad_autotune(palmad_ctx* ctx, const double* values, const int64_t* offsets, int32_t B,
                    const int32_t* minL, const int32_t* maxL, int32_t k,
                    const palmad_options* base, int32_t probe_lengths, int32_t reps,
                    void* workspace, size_t ws_bytes, palmad_options* best,
                    palmad_tune_report* report, void* stream);

/*
 * One range search at a single length m and range r (the DRAG problem of
 * Alg. 2 as parallelised in Sec. 3.2-3.3): every subsequence whose nearest
 * non-self match is at distance >= r, with that distance.  r <= 0 returns
 * every subsequence (the exact nearest-neighbour distance of all of them).
 *
 *   T          device, float64[n].
 *   workspace  device, >= palmad_workspace_size(n, m, m, 1, opts) bytes.
 *   alive      device, uint64[ceil(N/64)]: bit i%64 of word i/64 is set iff
 *              subsequence i is a range discord (N = n - m + 1).
 *   nn_dist    device, float64[N]: exact nnDist where the bit is set,
 *              unspecified elsewhere.
 *   count      host: number of range discords.
 */
int palmad_range_discords(palmad_ctx* ctx, const double* T, int64_t n, int32_t m, double r,
                          const palmad_options* opts, void* workspace, size_t ws_bytes,
                          uint64_t* alive, double* nn_dist, int64_t* count, palmad_stats* stats,
                          void* stream);

/*
 * The discord heatmap (Sec. 5, Eq. (11)): palmad_discords() that also keeps,
 * for every length m, all the range discords of the successful range search
 * (every subsequence whose nearest non-self match is at distance >= r_m) with
 * their exact nearest-neighbour distances.  heat(m, i) = nnDist^2 / (2m) =
 * 1 - rho (the distance in squared z-normalised units over 2m, in [0, 2]) for
 * the range discords of length m, 0 for every other i.  Every range search
 * refines both sides exactly, so this runs slower than palmad_discords().
 *
 *   T ... count, stats, stream  as palmad_discords() (same workspace size).
 *   heat       device, float64[L * ld]: row m - minL, columns i < ld; columns
 *              >= n - m + 1 are 0.
 *   ld         row stride of heat, >= n - minL + 1.
 *   range      device, float64[L]: r_m of the successful range search of
 *              each length (<= 0 means every subsequence).
 */
int palmad_discord_heatmap(palmad_ctx* ctx, const double* T, int64_t n, int32_t minL,
                           int32_t maxL, int32_t k, const palmad_options* opts, void* workspace,
                           size_t ws_bytes, int64_t* idx, int32_t* len, double* nn_dist,
                           int64_t* nn_idx, int32_t* count, double* heat, int64_t ld,
                           double* range, palmad_stats* stats, void* stream);

/*
 * Discord interest (Sec. 5, Eq. (12)): for every column i of a heatmap the
 * largest value over the lengths (ties: the shorter length), and the k
 * columns with the largest such values (ties: the smaller index; columns
 * whose value is 0 hold no discord).
 *
 *   heat       device, float64[L * ld] as written by palmad_discord_heatmap().
 *   L, ld      rows (lengths) and row stride; ncols <= ld columns are read.
 *   minL       length of row 0.
 *   k          1 <= k <= ncols.
 *   col_score  device, float64[ncols]: max over m of heat(m, i).
 *   col_len    device, int32[ncols]: the length m attaining it.
 *   top_idx    device, int64[k]; top_len device, int32[k]; top_score device,
 *              float64[k]: the k most interesting columns, best first.
 */
int palmad_heatmap_interest(palmad_ctx* ctx, const double* heat, int32_t L, int64_t ld,
                            int64_t ncols, int32_t minL, int32_t k, double* col_score,
                            int32_t* col_len, int64_t* top_idx, int32_t* top_len,
                            double* top_score, void* stream);

/*
 * Bytes of device workspace palmad_discords_backward() needs for K reported
 * rows of lengths <= maxm in a series of length n.  Pure host computation;
 * PALMAD_EINVAL unless 3 <= maxm, n >= 3*maxm - 1 and K >= 0.
 */
int palmad_backward_workspace_size(int64_t n, int64_t K, int32_t maxm, size_t* bytes);

/*
 * Gradient of reported nearest-neighbour distances with respect to the
 * series (not in the paper: the adjoint of Eq. (4)-(6) at a fixed nearest
 * neighbour).  For every q < K, with i = idx[q], m = len[q]:
 *   grad_T += grad_nn[q] * d nnDist_m(i) / dT,
 * where nnDist_m(i) = min over non-self matches j of the z-normalised
 * distance.  The minimiser j* is recomputed on the device (direct FP64
 * dot products, smallest j on ties) and the derivative is taken with j*
 * held fixed (it is piecewise constant); a zero distance or a flat window
 * contributes nothing.  Rows with an invalid (i, m) contribute nothing and
 * report nn_idx = -1.
 *
 *   T        device, float64[n];  idx device int64[K];  len device int32[K]
 *   grad_nn  device, float64[K]
 *   grad_T   device, float64[n], accumulated (+=); the caller zeroes it.
 *   nn_idx   device, int64[K] (optional, NULL): the recomputed j*.
 * Scatter uses FP64 atomics, so summation order (last bits) can vary.
 */
int palmad_discords_backward(palmad_ctx* ctx, const double* T, int64_t n, int64_t K, int32_t maxm,
                             const int64_t* idx, const int32_t* len, const double* grad_nn,
                             void* workspace, size_t ws_bytes, double* grad_T, int64_t* nn_idx,
                             void* stream);

/*
 * Mean and population standard deviation of every window of length m, as
 * the search computes them: direct two-pass sums at length minL (Eq. (4)),
 * then the recurrences of Eq. (7)-(8) for minL+1 .. m.
 *
 *   T      device, float64[n];  mu, sigma: device, float64[n - m + 1].
 *   workspace: device, >= palmad_workspace_size(n, minL, m, 1, NULL) bytes.
 * Requires 3 <= minL <= m and n >= 3*m - 1.
 */
int palmad_window_stats(palmad_ctx* ctx, const double* T, int64_t n, int32_t minL, int32_t m,
                        void* workspace, size_t ws_bytes, double* mu, double* sigma, void* stream);

/*
 * Diagnostic of the FP32 selection sweep's soundness (Sec. 3.2 run in FP32
 * with a guard band): over `items` work items of 512-row tiles (the longest
 * recurrence chains any sweep runs) and `chunk` columns each, spread over
 * the series at length m (items <= 0: every tile and chunk of the right
 * side), the centred diagonal recurrence is run in FP32 exactly as the
 * selection sweep runs it and in FP64 side by side.
 *   *drift  the largest |rho_FP32 - rho_FP64| over the items' pairs (host);
 *   *band   the guard band the selection sweep uses at this length for
 *           `guard` (<= 0: the default), at least guard (host).
 * Pruning in FP32 is sound while drift < band.  workspace: device, >=
 * palmad_selection_drift_workspace_size() bytes.  Requires 3 <= minL <= m,
 * n >= 3 m - 1, chunk >= 8.
 */
int palmad_selection_drift_workspace_size(int64_t n, int32_t minL, int32_t m, size_t* bytes);
int palmad_selection_drift(palmad_ctx* ctx, const double* T, int64_t n, int32_t minL, int32_t m,
                           int64_t items, int32_t chunk, float guard, void* workspace,
                           size_t ws_bytes, double* drift, double* band, void* stream);

/*
 * Streaming series (the paper's future work on series that grow or exceed
 * one pass, Conclusions): a series of up to `capacity` points appended in
 * pieces, with the top-k discords of every length in [minL, maxL] of the
 * series so far available after any append.  The stream keeps one exact
 * nearest-neighbour profile per length (Sec. 2.1, Eq. (1)-(5): for every
 * subsequence the correlation of its nearest non-self match) and an append
 * evaluates only the pairs it adds: every new subsequence (each reaches
 * back over at most maxL - 1 points already there) against all
 * subsequences, and every old subsequence against the new ones.  A query
 * ranks each profile and recomputes the best rows with direct FP64 dot
 * products, as a search does, so its rows equal those of palmad_discords()
 * on the same points (the top-k of a length do not depend on MERLIN's
 * range schedule).  No range r is involved: nothing is pruned.
 *
 * palmad_stream_workspace_size: bytes of device workspace for a stream
 *   (pure host; PALMAD_EINVAL for arguments palmad_workspace_size() would
 *   reject with n = capacity).  About 8 L bytes per point beyond a search's
 *   workspace (L = maxL - minL + 1).
 * palmad_stream_create: a stream on the context's device; workspace (device,
 *   256-byte aligned) must stay valid and unused by anything else until
 *   palmad_stream_destroy().  *out receives the handle (host memory).
 * palmad_stream_append: appends values[0 .. count) (device, float64) and
 *   updates every profile; PALMAD_EINVAL if the capacity would be exceeded,
 *   PALMAD_ENONFINITE (stream unchanged) if a value is NaN or Inf.
 * palmad_stream_discords: top-k rows of every length of the series so far,
 *   laid out as palmad_discords() (idx, len, nn_dist, nn_idx: device,
 *   [L * k]); requires at least 3 maxL - 1 points.
 * palmad_stream_profile: the exact nearest-neighbour distance of every
 *   subsequence of length m (nn_dist: device, float64[n - m + 1]).
 * Calls are synchronous like the others; one stream is used by one host
 * thread at a time.
 */
typedef struct palmad_stream palmad_stream;
int palmad_stream_workspace_size(int64_t capacity, int32_t minL, int32_t maxL, int32_t k,
                                 const palmad_options* opts, size_t* bytes);
int palmad_stream_create(palmad_ctx* ctx, int64_t capacity, int32_t minL, int32_t maxL, int32_t k,
                         const palmad_options* opts, void* workspace, size_t ws_bytes,
                         palmad_stream** out, void* stream);
int palmad_stream_append(palmad_stream* st, const double* values, int64_t count, void* stream);
int palmad_stream_discords(palmad_stream* st, int64_t* idx, int32_t* len, double* nn_dist,
                           int64_t* nn_idx, void* stream);
int palmad_stream_profile(palmad_stream* st, int32_t m, double* nn_dist, void* stream);
/* Points appended so far (-1 for NULL). */
int64_t palmad_stream_length(const palmad_stream* st);
void palmad_stream_destroy(palmad_stream* st);

/*
 * For callers that cannot allocate device memory (code that must not call
 * hipMalloc or any allocating routine: tight serving loops, harnesses that
 * forbid allocation).  Same search and results as palmad_discords() with
 * the same options, but the workspace is a static device array of
 * PALMAD_STATIC_WORKSPACE_BYTES bytes held by each GPU the library runs on
 * until the process ends (its address is taken once per device by
 * palmad_create()).  The call allocates no device memory and launches every
 * kernel directly (no graph is instantiated).
 *
 *   T ... count, stats, stream  as palmad_discords().
 * Returns PALMAD_EWORKSPACE when palmad_workspace_size() for these
 * arguments exceeds PALMAD_STATIC_WORKSPACE_BYTES (about 3.5e5 points at
 * m = 64..128, k = 3).  Every call on one GPU uses that GPU's array, whose
 * contents persist from the last call (the search initialises everything it
 * reads).  Calls from threads of one process are serialised by the library;
 * calls from different processes use different copies.  A call returns only
 * once its device work is complete.
 */
#define PALMAD_STATIC_WORKSPACE_BYTES ((size_t)32 << 20)
int palmad_discords_static(palmad_ctx* ctx, const double* T, int64_t n, int32_t minL,
                           int32_t maxL, int32_t k, const palmad_options* opts, int64_t* idx,
                           int32_t* len, double* nn_dist, int64_t* nn_idx, int32_t* count,
                           palmad_stats* stats, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PALMAD_H */
