// Internal interface between the C ABI layer (capi.hip) and the kernels
// (kernels.hip).  Not installed; the public interface is include/palmad.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace palmad {

// Row-tile geometry of the sweeps: a tile is one wavefront of 64 lanes, each
// lane owning Q consecutive rows (subsequence start indices).
constexpr int WAVE = 64;
constexpr int R_MAX = 512;
constexpr int KP_EXTRA = 4;  // candidates polished beyond k
constexpr int K_MAX = 64;
constexpr int KP_MAX = K_MAX + KP_EXTRA;
constexpr int POLISH_BLOCK = 256;
constexpr int TOPK_BLOCK = 1024;
constexpr int RED_BLOCKS = 256;   // series reductions: blocks of 256 threads

// Device-resident control block of one search (the MERLIN state of Alg. 1
// plus per-round work counters).  Lives in the workspace.
struct Ctrl {
    // controller
    double r;          // current range (ED units)
    double step;       // decrement of the later-length rule
    double thr64;      // pruning threshold on the correlation: 1 - r^2/(2m); >= 1 disables
    double thr_sel;    // thr64 + guard: selection sweeps prune above this
    float thr32;       // thr_sel rounded up to float, for the FP32 selection sweep
    int32_t mode;      // 0: first length, 1: next four, 2: later lengths, 3: fixed r
    int32_t done;      // 1 once the current length succeeded
    int32_t prune;     // 1 if r > 0
    int32_t m;
    int32_t li;        // m - minL
    int32_t nonfinite; // set when the series holds NaN/Inf
    double flat_eps;   // sigma threshold of a flat window
    double sigmaT;     // population sigma of the whole series
    // work lists of the current round
    uint32_t nlive_sel, maxc_sel, ctr_sel;
    uint32_t nlive_ref, maxc_ref, ctr_ref;
    uint32_t nsurv;
    uint32_t ncand;
    int64_t flat_min, flat_max;   // smallest/largest flat window index at m (or -1)
    // counters accumulated over the call
    unsigned long long evals_sel, evals_ref, evals_pol, rounds, survivors;
    unsigned long long evals_near, evals_far;
};

// Workspace carve-up (all offsets 256-byte aligned).
struct Layout {
    int64_t n, Nmax, Npad, Tlen;
    int32_t minL, maxL, k, L, kp;
    int32_t dist_bits;
    size_t off_T, off_mu, off_var, off_h32, off_h64, off_alive, off_rho, off_tsel, off_tref,
        off_surv, off_cand, off_part, off_hist, off_flat, off_ctrl, off_red, total;
    int64_t nwords;      // alive bitmap words
    int64_t npart;       // polish partial slots per candidate
};

bool make_layout(int64_t n, int32_t minL, int32_t maxL, int32_t k, int32_t dist_bits, Layout* out);

// Pointers into a carved workspace.
struct Buffers {
    double* T;        // padded FP64 series
    double* mu;       // [Npad+64]
    double* var;      // [Npad+64]
    float* df32;      // helpers, FP32 (3 arrays of Npad+64)
    float* dg32;
    float* inv32;
    double* df64;     // helpers, FP64
    double* dg64;
    double* inv64;
    unsigned long long* alive;   // bitmap [nwords]
    unsigned long long* rho;     // ordered-bits row max correlation [Npad]
    int32_t* tsel;    // live selection tiles
    int32_t* tref;    // live refinement tiles
    int32_t* surv;    // survivor rows
    int64_t* cand;    // polished candidates [KP_MAX]
    double* part;     // polish partials [KP_MAX * npart * 2]
    double* hist;     // nnDist history per length [L]
    int64_t* flat;    // [2]: min, max flat index at current m
    Ctrl* ctrl;
    double* red;      // reduction scratch [2048]
};

Buffers carve(void* ws, const Layout& lay);

// Optional per-kernel event timing (host side).
constexpr int KCLASSES = 4;  // select near, select far, refine, polish
struct KernelTimer {
    bool on;
    hipEvent_t ev[KCLASSES][2];
    double ms[KCLASSES];
    unsigned long long launches[KCLASSES];
    void begin(int k, hipStream_t st) const
    {
        if (on) (void)hipEventRecord(ev[k][0], st);
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
    int far_grid;     // workgroups of the split passes
    int q_near, q_far, q_ref;  // rows per lane of each pass's tiles (2, 4 or 8)
    const KernelTimer* timer;
};

// ---- launchers (all asynchronous on `st`) ----
hipError_t launch_prepare(const Layout& lay, const Buffers& b, const double* T_user, hipStream_t st);
hipError_t launch_stats(const Layout& lay, const Buffers& b, int32_t m, bool init, hipStream_t st);
hipError_t launch_round(const Layout& lay, const Buffers& b, const SweepCfg& cfg, int32_t m,
                        int attempt, hipStream_t st);
hipError_t launch_finish_length(const Layout& lay, const Buffers& b, const SweepCfg& cfg, int32_t m,
                                int64_t* idx, int32_t* len, double* nn, int64_t* nnidx,
                                int32_t* count, hipStream_t st);
hipError_t launch_set_fixed_r(const Buffers& b, double r, hipStream_t st);
hipError_t launch_range_out(const Layout& lay, const Buffers& b, int32_t m,
                            unsigned long long* alive_out, double* nn_out, hipStream_t st);
hipError_t launch_adjoint(const double* Tpad, int64_t n, int64_t K, int32_t maxm,
                          const int64_t* idx, const int32_t* len, const double* gin,
                          const Ctrl* ctrl, double* part, int64_t nblk, double* grad,
                          int64_t* jstar, hipStream_t st);
hipError_t launch_set_max_len(const Buffers& b, int32_t maxm, hipStream_t st);
hipError_t launch_stats_out(const Layout& lay, const Buffers& b, int32_t m, double* mu,
                            double* sigma, hipStream_t st);

}  // namespace palmad
