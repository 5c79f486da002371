// Internal interface between the C ABI layer (capi.hip) and the kernels
// (kernels.hip, prep.hip, adjoint.hip).  Not installed; the public interface
// is include/palmad.h.
//
// The engine searches B series at once (B = 1 for a single series).  Every
// series carries its own MERLIN state (Alg. 1) in a device-resident control
// block; one "round" performs one range search (one DRAG call, Alg. 2) for
// every series that still has work, each at its own length and attempt.  All
// geometry and state are read from device descriptors, so a round is a fixed
// sequence of launches that can be captured once in a hipGraph.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace palmad {

constexpr int WAVE = 64;
constexpr int R_MAX = 512;   // tallest row tile (64 lanes x 8 rows)
constexpr int KP_EXTRA = 4;  // candidates polished beyond k
constexpr int K_MAX = 64;
constexpr int KP_MAX = K_MAX + KP_EXTRA;
constexpr int POLISH_COLS = 512;  // columns per exact-pass block (one partial each)
constexpr int TOPK_BLOCK = 1024;
constexpr int RED_BLOCKS = 256;   // series reductions: blocks of 256 threads
constexpr int MAX_ATTEMPTS = 5000;
// A round whose selection leaves at most this many live subsequences skips
// the refinement sweep: the exact pass evaluates all of them directly.
constexpr int DIRECT_MAX = KP_MAX;
// Row tiles that held survivors at the end of a round, or whose first-pass
// items swept at least 1/HOT_FRAC of the series' columns in all, lead the
// next round's first selection pass (at most HOT_MAX of them).
constexpr int HOT_MAX = 64;
constexpr int HOT_FRAC = 8;

// Pair-evaluation counters: EV_SLOTS slots per class, so that the many
// work items of a launch add to different addresses.
constexpr int EV_CLASSES = 5;  // first selection pass, split pass, refinement, exact pass, band pre-pass
constexpr int EV_SLOTS = 64;
enum { EV_NEAR = 0, EV_FAR = 1, EV_REF = 2, EV_POL = 3, EV_BAND = 4 };

// Device-resident control block of one series (the MERLIN state of Alg. 1
// plus the work counters of the current round).  Fields that work items
// update with atomics sit on cache lines of their own, away from the fields
// every item reads.
struct Ctrl {
    // controller (read by every work item)
    double r;          // current range (ED units)
    double step;       // decrement of the later-length rule
    double thr64;      // pruning threshold on the correlation: 1 - r^2/(2m); >= 1 disables
    double thr_sel;    // thr64 + guard: selection sweeps prune above this
    float thr32;       // thr_sel rounded up to float, for the FP32 selection sweep
    int32_t mode;      // 0: first length, 1: next four, 2: later lengths, 3: fixed r
    int32_t done;      // 1 once the current length succeeded
    int32_t prune;     // 1 if r > 0
    int32_t m;         // current length
    int32_t li;        // m - minL
    int32_t attempt;   // range searches so far at this length
    int32_t active;    // 1 if the series searches in this round
    int32_t finished;  // 1 once every length is done (or on error)
    int32_t started;
    int32_t new_len;   // 0: same length as last round, 1: update statistics, 2: initialise
    int32_t error;     // 1: did not converge within SweepCfg::max_attempts
    int32_t nonfinite; // set when the series holds NaN/Inf
    double flat_eps;   // sigma threshold of a flat window
    double sigmaT;     // population sigma of the whole series
    double gam2;       // squared local sigma contrast at the current length (FP32 guard)
    int64_t flat_min, flat_max;   // smallest/largest flat window index at m (or -1)
    uint32_t nhot;     // entries of SeriesDev::hot (set by k_round_end)
    int32_t hot_r;     // tile height the hot list was built for
    int32_t exact_ref; // 1: refinement sweeps both sides of every tile (set by k_round_end)
    int32_t band_over; // 1: more rows than KP_MAX may hold the k best exact values
    // work lists of the current round (built by k_tiles, read by the queued passes)
    alignas(128) uint32_t nlive_sel, maxc_sel;  // live selection tiles, most chunks of one tile
    uint32_t nlive_ref, maxc_ref;
    uint32_t live_ref;     // live subsequences entering refinement this round
    uint32_t nsurv;
    uint32_t ncand;
    // counters accumulated over the call
    alignas(128) unsigned long long rounds, survivors;
    unsigned long long rows_near, rows_far;  // live rows entering the split / refinement passes
};

// Static geometry and buffers of one series (host computes, device reads).
struct SeriesDev {
    // geometry
    int64_t n, Nmax, Npad, Tlen, nwords, npart;
    int32_t minL, maxL, k, kp, L, pad0;
    // input and workspace buffers
    const double* Tin;   // caller's series
    double* T;           // padded FP64 copy
    double* mu;          // [Npad+64], lengths with m - minL even
    double* var;         // [Npad+64]
    double* mu2;         // [Npad+64], lengths with m - minL odd
    double* var2;        // [Npad+64]
    float* df32;         // helpers, FP32 (SoA, Npad+64 each)
    float* dg32;
    float* inv32;
    double* df64;        // helpers, FP64
    double* dg64;
    double* inv64;
    unsigned long long* alive;   // bitmap [nwords]
    unsigned long long* rho;     // ordered-bits row max correlation [Npad]
    unsigned long long* rhs;     // ordered-bits row max of the selection sweep (right side) [Npad]
    unsigned long long* unc;     // bitmap [nwords]: rows whose rhs is above thr64 - guard
    int32_t* tsel;       // live selection tiles
    int32_t* tref;       // live refinement tiles
    int32_t* hot;        // hot tiles of the last round, ascending [HOT_MAX]
    uint32_t* twork;     // 64-column blocks swept by each first-pass tile this round [nwords]
    int64_t* cand;       // polished candidates [KP_MAX]
    double* part;        // polish partials [KP_MAX * npart * 2 + tail]
    double* xc;          // centred candidate windows [KP_MAX][maxL + 8], then their sums
    double* hist;        // nnDist history per length [L]
    unsigned long long* evc;  // pair evaluations [EV_CLASSES][EV_SLOTS]
    double* red;         // reduction scratch [2 * RED_BLOCKS]
    double* sgm;         // per block of 256 windows: largest, smallest sigma [2 * blocks]
    Ctrl* ctrl;
    // outputs (rows of this series; NULL for a bare range search)
    int64_t* idx;
    int32_t* len;
    double* nn;
    int64_t* nnidx;
    int32_t* count;
    // discord heatmap (NULL unless requested): heat[(m - minL) * heat_ld + i],
    // the final range r of every length in rlen[m - minL]
    double* heat;
    double* rlen;
    int64_t heat_ld;
};

// Per-series layout (host side; offsets relative to the series' base).
struct Layout {
    int64_t n, Nmax, Npad, Tlen, nwords, npart;
    int32_t minL, maxL, k, L, kp;
    size_t off_T, off_mu, off_var, off_mu2, off_var2, off_h32, off_h64, off_alive, off_rho, off_rhs, off_unc,
        off_tsel, off_tref, off_hot, off_twork, off_cand, off_part, off_xc, off_hist, off_evc, off_ctrl, off_red,
        off_sgm, total;
};
bool make_layout(int64_t n, int32_t minL, int32_t maxL, int32_t k, Layout* out);
SeriesDev carve(void* base, const Layout& lay);

// Prefix tables mapping a flat block index to (series, local block): entry b
// is the first flat block of series b; entry B the total.
enum PrefixKind {
    PFX_ELEM = 0,   // blocks of 256 over Npad+64 elements (statistics, resets)
    PFX_NEAR,       // first-pass selection items: tiles x chunks
    PFX_TSEL,       // blocks of 256 over selection tiles (compaction)
    PFX_TREF,       // blocks of 256 over refinement tiles (compaction)
    PFX_POLISH,     // blocks of POLISH_COLS columns (polish)
    PFX_BAND,       // row segments of the diagonal band pre-pass
    PFX_KINDS
};

struct Batch {
    SeriesDev* s;                    // device array [B]
    const int64_t* pfx[PFX_KINDS];   // device arrays [B+1]
    int32_t B;
    int32_t maxL_all;                // largest length over the batch (LDS sizing)
    int64_t Nmax_all;                // most subsequences of any series
    int32_t* remaining;              // device [2]: series with work left, series in error
    unsigned long long* sums;        // device [9]: counters summed over the batch
};

// Optional per-kernel event timing (host side).
constexpr int KCLASSES = 6;  // select near, select far, refine, polish, per-length statistics, band
struct KernelTimer {
    bool on;
    hipEvent_t ev[KCLASSES][2];
    double ms[KCLASSES];
    unsigned long long launches[KCLASSES];
    mutable bool used[KCLASSES];  // classes launched since the last accumulation
    void begin(int k, hipStream_t st) const
    {
        if (on) {
            (void)hipEventRecord(ev[k][0], st);
            used[k] = true;
        }
    }
    void end(int k, hipStream_t st) const
    {
        if (on) (void)hipEventRecord(ev[k][1], st);
    }
};

struct SweepCfg {
    int near_cols;
    int chunk_cols;
    float guard;
    int dist_bits;
    int far_grid;              // workgroups of the queued passes
    int q_near, q_far, q_ref;  // rows per lane of each pass's tiles (2, 4 or 8)
    int max_attempts;          // range searches allowed per length (MAX_ATTEMPTS)
    int band;                  // 1: diagonal band pre-pass before the first selection pass
    const KernelTimer* timer;
};

// Blocks of each prefix kind needed by one series under a configuration.
void series_blocks(const Layout& lay, const SweepCfg& cfg, int64_t out[PFX_KINDS]);

// ---- launchers (all asynchronous on `st`); `total[kind]` = pfx[kind][B] ----
hipError_t launch_prepare(const Batch& bt, const int64_t* total, hipStream_t st);
hipError_t launch_round(const Batch& bt, const SweepCfg& cfg, const int64_t* total, hipStream_t st);
hipError_t launch_set_fixed_r(const Batch& bt, double r, hipStream_t st);
hipError_t launch_range_out(const Batch& bt, int64_t N, unsigned long long* alive_out,
                            double* nn_out, hipStream_t st);
hipError_t launch_stats_to(const Batch& bt, int32_t minL, int32_t m, const int64_t* total,
                           hipStream_t st);
// Per-series counters summed over the batch: 9 values (see k_sum_stats).
hipError_t launch_sum_stats(const Batch& bt, unsigned long long* out, hipStream_t st);
// out[0] = series holding NaN/Inf, out[1] = the first of them (or -1).
hipError_t launch_nonfinite(const Batch& bt, int32_t* out, hipStream_t st);
hipError_t launch_set_len(const Batch& bt, int32_t m, hipStream_t st);
hipError_t launch_stats_out(const Batch& bt, int64_t N, double* mu, double* sigma, hipStream_t st);
// Interest of every heatmap column (largest value over the lengths, and that
// length) and the k most interesting columns.
hipError_t launch_interest(const double* heat, int32_t L, int64_t ld, int64_t ncols, int32_t minL,
                           int32_t k, double* col_score, int32_t* col_len, int64_t* top_idx,
                           int32_t* top_len, double* top_score, hipStream_t st);
hipError_t launch_adjoint(const double* Tpad, int64_t n, int64_t K, int32_t maxm,
                          const int64_t* idx, const int32_t* len, const double* gin,
                          const Ctrl* ctrl, double* part, int64_t nblk, double* grad,
                          int64_t* jstar, hipStream_t st);

// Streaming series (single series, bt.s[0].n = current length): profile
// updates after an append from n_old points, the top-k rows of every length
// from the profiles, one length's profile as distances, and a fill.
hipError_t launch_stream_update(const Batch& bt, const SweepCfg& cfg, const int64_t* total,
                                int32_t minL, int32_t maxL, unsigned long long* prof,
                                int64_t n_old, hipStream_t st);
hipError_t launch_stream_query(const Batch& bt, const int64_t* total, int32_t minL, int32_t maxL,
                               const unsigned long long* prof, int hot_rows, hipStream_t st);
hipError_t launch_stream_profile(const Batch& bt, const int64_t* total, int32_t minL, int32_t m,
                                 const unsigned long long* prof, double* nn, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, int64_t count, unsigned long long v,
                           hipStream_t st);
// Control blocks, histories, counters and bitmaps of every series to zero.
hipError_t launch_ctrl_init(const Batch& bt, hipStream_t st);
// Appended values: out[0] = 1 if any of src[0 .. count) is not finite.
hipError_t launch_check_finite(const double* src, int64_t count, int32_t* out, hipStream_t st);
// Copy src[0 .. count) into the padded series at n_old and recompute the
// series' population sigma (flat threshold) over its first s.n points.
hipError_t launch_stream_append(const Batch& bt, const double* src, int64_t n_old, int64_t count,
                                hipStream_t st);

// Diagnostic: statistics up to length m, the guard band, then out[0] =
// ordered bits of the largest |rho32 - rho64| of the FP32 selection
// recurrence over nitems sampled items, out[1] = the band (a double).
hipError_t launch_drift(const Batch& bt, const int64_t* total, int32_t minL, int32_t m,
                        int64_t nitems, int chunk, float guard, double* out, hipStream_t st);

// Device helper: series owning flat block `blk` (binary search over pfx).
__device__ __forceinline__ int series_of(const int64_t* pfx, int B, int64_t blk)
{
    int lo = 0, hi = B;  // pfx[lo] <= blk < pfx[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pfx[mid] <= blk) lo = mid;
        else hi = mid;
    }
    return lo;
}

}  // namespace palmad
