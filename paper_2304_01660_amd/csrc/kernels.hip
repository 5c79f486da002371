// HIP kernels (gfx950) of the range-discord search.
//
// Method (paper): for each length m, per-subsequence mean/sigma by the
// recurrences of Eq. (7)-(8) (Sec. 3.1.1); a selection pass that drops every
// subsequence having a non-self match closer than r, scanning to the right of
// each row tile (Sec. 3.2, after phase 1 of Alg. 2); a refinement pass that
// computes the exact nearest-neighbour distance of the survivors and drops
// those closer than r (Sec. 3.3, phase 2 of Alg. 2); MERLIN's choice of r per
// length (Alg. 1).  Distances use the Pearson form of Eq. (6):
// ED^2 = 2m(1 - rho), rho = C_ij / (m sigma_i sigma_j) with C_ij the centred
// covariance of the two windows.
//
// MI355X mapping:
//   * A sweep work item is one wavefront owning a tile of R = 64*Q
//     consecutive rows (Q per lane) and a run of columns.  Along a column
//     step every row takes the value of its upper-left neighbour (Eq. (10)'s
//     diagonal update, here on the centred covariance:
//     C(i,j) = C(i-1,j-1) + df[i-1]*dg[j-1] + df[j-1]*dg[i-1]), so a lane's
//     Q rows shift inside registers and one DPP wave_shr moves the last row
//     into the next lane.  Lane 0's top row is taken from exact FP64 dot
//     products computed 64 columns at a time, so every value is at most R
//     recurrence steps from an exact one.
//   * Each block of 64 columns is staged in LDS with one burst of loads: the
//     T segment (for the boundary dot products) and, per step, the column
//     helpers df, dg, 1/(sqrt(m) sigma) and the boundary value, all read as
//     one broadcast record.
//   * Row and column prunes are lane masks; a column prune is one ballot per
//     step, flushed to the candidate bitmap every 64 columns with one atomic.
//   * Long scans are split into column chunks fed from a device work list in
//     nearest-first order, so the critical path is one chunk, not one row.
//   * Every kernel serves a batch of series: flat block indices map to
//     (series, block) through host-built prefix tables, the queued passes
//     drain each series' work list in turn, and all per-series geometry and
//     MERLIN state is read from device descriptors.
#include "engine.h"

#include <math.h>

#include <algorithm>

namespace palmad {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
constexpr int DPP_WAVE_SHR1 = 0x138;  // lane l <- lane l-1
constexpr int DPP_WAVE_ROL1 = 0x134;  // lane l <- lane l+1 (63 <- 0)

template <typename F>
__device__ __forceinline__ F f_inf();
template <>
__device__ __forceinline__ float f_inf<float>() { return __int_as_float(0x7f800000); }
template <>
__device__ __forceinline__ double f_inf<double>() { return __longlong_as_double(0x7ff0000000000000ll); }

__device__ __forceinline__ float f_fma(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double f_fma(double a, double b, double c) { return fma(a, b, c); }

// lane l <- src of lane l-1; lane 0 <- old of lane 0
__device__ __forceinline__ float dpp_shr1(float old, float src)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src),
                                                      DPP_WAVE_SHR1, 0xf, 0xf, false));
}
__device__ __forceinline__ double dpp_shr1(double old, double src)
{
    const long long o = __double_as_longlong(old), s = __double_as_longlong(src);
    const int lo = __builtin_amdgcn_update_dpp((int)o, (int)s, DPP_WAVE_SHR1, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(s >> 32), DPP_WAVE_SHR1, 0xf,
                                               0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// lane l <- lane l+1, lane 63 <- lane 0
__device__ __forceinline__ float dpp_rol1(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), DPP_WAVE_ROL1, 0xf, 0xf, false));
}
__device__ __forceinline__ double dpp_rol1(double v)
{
    const long long s = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)s, DPP_WAVE_ROL1, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(s >> 32), DPP_WAVE_ROL1, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ unsigned long long ord_of(double d)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(d);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double dbl_of(unsigned long long u)
{
    return (u >> 63) ? __longlong_as_double((long long)(u & 0x7fffffffffffffffull))
                     : __longlong_as_double((long long)~u);
}

// Values identical in every lane, made explicit so the compiler keeps them
// (and everything derived from them) in scalar registers.
__device__ __forceinline__ unsigned long long uniform64(unsigned long long v)
{
    const unsigned int lo = __builtin_amdgcn_readfirstlane((unsigned int)v);
    const unsigned int hi = __builtin_amdgcn_readfirstlane((unsigned int)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ int64_t uniform_i64(int64_t v) { return (int64_t)uniform64((unsigned long long)v); }

__device__ __forceinline__ unsigned long long load_word(const unsigned long long* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ double block_sum(double v, double* sh)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
    __syncthreads();
    return t;  // valid in thread 0
}

// Number of (row, column) pairs with rows in [ilo, ihi) and columns in
// [j0, j0+ns) that are non-self matches on the given side:
//   right side: j >= i + m;   left side: j <= i - m.
__device__ __forceinline__ unsigned long long pair_count(long long ilo, long long ihi, long long j0,
                                                         long long ns, long long m, bool left)
{
    if (ihi <= ilo || ns <= 0) return 0;
    unsigned long long tot = 0;
    if (!left) {
        // row i sees clamp(E - i, 0, ns) columns, E = j0 + ns - m
        const long long E = j0 + ns - m;
        const long long full_hi = min(ihi, E - ns + 1);  // i <= E - ns  -> ns columns
        if (full_hi > ilo) tot += (unsigned long long)(full_hi - ilo) * (unsigned long long)ns;
        const long long p = max(ilo, E - ns + 1), q = min(ihi, E);
        if (q > p) tot += (unsigned long long)((2 * E - p - q + 1) * (q - p) / 2);
    } else {
        // row i sees clamp(i - G, 0, ns) columns, G = j0 + m - 1
        const long long G = j0 + m - 1;
        const long long full_lo = max(ilo, G + ns);      // i >= G + ns -> ns columns
        if (ihi > full_lo) tot += (unsigned long long)(ihi - full_lo) * (unsigned long long)ns;
        const long long p = max(ilo, G + 1), q = min(ihi, G + ns);
        if (q > p) tot += (unsigned long long)((p + q - 1 - 2 * G) * (q - p) / 2);
    }
    return tot;
}

// ---------------------------------------------------------------------------
// round preparation: MERLIN's walk over the lengths and its choice of r
// (Alg. 1), for every series (one block)
// ---------------------------------------------------------------------------
// Advance every series: the first round starts at minL; after a successful
// round the next length starts; after a failed one the same length is
// searched again with the r that k_round_end lowered.  Then set the range of
// this round, its pruning threshold and reset the round's work counters.
// rem[0] (series with work left after the round, counted by k_round_end) and
// rem[1] (series that gave up, now or in an earlier round) start at zero here.
// Guard band of the FP32 selection sweep.  An FP32 correlation drifts from
// the exact one by rounding: the centred recurrence accumulates one rounding
// of the covariance per step over chains of at most R_MAX - 1 steps, and a
// pair's covariance is divided by m sigma_i sigma_j, so windows with a small
// spread next to windows with a large one (within the R_MAX windows a chain
// passes) amplify the covariance's absolute error.  With gamma the largest
// ratio of the nearby largest spread to a window's own spread, the drift
// measured on the device (k_drift, thousands of sampled 512-row tiles, and
// every tile of the smaller series) over the configured workloads stays
// below
//     2^-24 * sqrt(R_MAX) * gamma^2
// (random walks, ECG-like series; ECG-like beats between quiet baselines
// come closest); the band is four times that, and never below the caller's
// guard (default 1.25e-4).  A series with an extreme spread contrast thus
// gets a wide band (the selection sweep prunes less, the FP64 refinement
// decides), never an unsound one.
constexpr double GUARD_PER_CONTRAST2 = 4.0 * 0x1p-24 * 22.62741699796952;  // 4 u sqrt(512)

__device__ __forceinline__ double sel_guard(const Ctrl* c, float guard)
{
    if (guard <= 0.0f) return 0.0;  // FP64 selection sweep: no band
    const double gc = GUARD_PER_CONTRAST2 * c->gam2;
    return gc > (double)guard ? gc : (double)guard;
}

__device__ __forceinline__ void set_sel_thresholds(Ctrl* c, float guard)
{
    c->thr_sel = c->thr64 + sel_guard(c, guard);
    // round up: an FP32 threshold must never prune more than thr_sel
    c->thr32 = __double2float_ru(c->thr_sel);
}

__device__ void begin_range(const SeriesDev& s, Ctrl* c, float guard)
{
    const int li = c->li;
    const int32_t m = c->m;
    if (c->attempt == 0 && c->mode != 3) {
        if (li == 0) {
            c->mode = 0;
            c->r = 2.0 * sqrt((double)s.minL);
        } else if (li <= 4) {
            c->mode = 1;
            c->r = 0.99 * s.hist[li - 1];
        } else {
            double mean = 0.0;
            for (int q = 1; q <= 5; ++q) mean += s.hist[li - q];
            mean /= 5.0;
            double v = 0.0;
            for (int q = 1; q <= 5; ++q) {
                const double d = s.hist[li - q] - mean;
                v += d * d;
            }
            c->step = sqrt(v / 5.0);
            c->r = mean - 2.0 * c->step;
            c->mode = 2;
        }
    }
    const double r = c->r;
    c->prune = r > 0.0 ? 1 : 0;
    c->thr64 = r > 0.0 ? 1.0 - r * r / (2.0 * (double)m) : 2.0;
    // a new length's contrast is measured by k_length and k_guard, which
    // then resets the selection thresholds; a repeat keeps the current length's
    if (c->new_len) c->gam2 = 0.0;
    set_sel_thresholds(c, guard);
    c->nlive_sel = c->maxc_sel = 0;
    c->nlive_ref = c->maxc_ref = 0;
    c->nsurv = 0;
    c->ncand = 0;
    c->live_ref = 0;
    c->band_over = 0;
    if (c->new_len) {
        c->flat_min = 0x7fffffffffffffffll;
        c->flat_max = -1;
    }
}

__global__ void k_round_prep(SeriesDev* S, int B, float guard, int max_attempts, int32_t* rem)
{
    if (threadIdx.x == 0) {
        rem[0] = 0;
        rem[1] = 0;
    }
    __syncthreads();
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
        const SeriesDev& s = S[b];
        Ctrl* c = s.ctrl;
        if (c->finished) {
            c->active = 0;
            if (c->error) atomicAdd(&rem[1], 1);  // stays visible in later rounds
            continue;
        }
        if (!c->started) {
            c->started = 1;
            c->m = s.minL;
            c->li = 0;
            c->attempt = 0;
            c->new_len = 2;
        } else if (c->done) {
            if (c->m >= s.maxL) {
                c->finished = 1;
                c->active = 0;
                continue;
            }
            c->m += 1;
            c->li += 1;
            c->attempt = 0;
            c->new_len = 1;
        } else {
            c->attempt += 1;
            c->new_len = 0;
            if (c->attempt >= max_attempts) {
                c->error = 1;
                c->finished = 1;
                c->active = 0;
                atomicAdd(&rem[1], 1);
                continue;
            }
        }
        c->done = 0;
        c->active = 1;
        begin_range(s, c, guard);
    }
}

// ---------------------------------------------------------------------------
// per-length statistics (Eq. (4) at minL, Eq. (7)-(8) after), the column and
// row helpers, and the per-round reset of the bitmap and row maxima
// ---------------------------------------------------------------------------
// Statistics live in two buffers used alternately from one length to the
// next (mu/var for even m - minL, mu2/var2 for odd), so every thread can
// read the previous length's values of its own window and of the next one.
__device__ __forceinline__ const double* cur_mu(const SeriesDev& s, const Ctrl* c)
{
    return (c->li & 1) ? s.mu2 : s.mu;
}
__device__ __forceinline__ const double* cur_var(const SeriesDev& s, const Ctrl* c)
{
    return (c->li & 1) ? s.var2 : s.var;
}

// A round whose selection left at most DIRECT_MAX live subsequences: the
// refinement sweep is skipped and the exact pass evaluates every one of them.
__device__ __forceinline__ bool direct_round(const Ctrl* c) { return c->live_ref <= DIRECT_MAX; }

// Mean and variance of window p at length m: two passes (Eq. (4)).
__device__ __forceinline__ void direct_stats(const double* __restrict__ T, int64_t p, int32_t m,
                                             double& mean, double& var)
{
    double acc = 0.0;
    for (int k = 0; k < m; ++k) acc += T[p + k];
    mean = acc / (double)m;
    double q = 0.0;
    for (int k = 0; k < m; ++k) {
        const double d = T[p + k] - mean;
        q += d * d;
    }
    var = q / (double)m;
}

// Eq. (7)-(8): window p from length m-1 (mean mu0, variance v0) to m.
__device__ __forceinline__ void grow_stats(const double* __restrict__ T, int64_t p, int32_t m,
                                           double mu0, double v0, double& mean, double& var)
{
    const int32_t mo = m - 1;
    const double t = T[p + mo];
    const double dm = (double)mo;
    const double d = mu0 - t;
    mean = (dm * mu0 + t) / (dm + 1.0);
    var = dm / (dm + 1.0) * (v0 + d * d / (dm + 1.0));
}

// Block extremes of the window spreads (every block of k_length at a new
// length): the largest and smallest sigma of the block's non-flat windows.
__device__ void spread_extremes(const SeriesDev& s, int64_t lb, double smax, double smin)
{
    __shared__ double rmax[4], rmin[4];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        smax = fmax(smax, __shfl_xor(smax, o));
        smin = fmin(smin, __shfl_xor(smin, o));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        rmax[w] = smax;
        rmin[w] = smin;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = rmax[0], z = rmin[0];
        for (int q = 1; q < (int)(blockDim.x >> 6); ++q) {
            a = fmax(a, rmax[q]);
            z = fmin(z, rmin[q]);
        }
        s.sgm[2 * lb] = a;
        s.sgm[2 * lb + 1] = z;
    }
}

// The spread contrast of a new length and the round's selection thresholds
// (one block per series, after k_length): over every block of 256 windows,
// the largest spread of the two blocks on either side (a superset of the
// R_MAX - 1 windows a recurrence chain passes on each side) over the block's
// smallest spread, squared (see sel_guard).
constexpr int GUARD_BLOCK = 1024;
__global__ __launch_bounds__(GUARD_BLOCK) void k_guard(SeriesDev* S, float guard)
{
    const SeriesDev& s = S[blockIdx.x];
    Ctrl* c = s.ctrl;
    if (!c->active || !c->new_len || guard <= 0.0f) return;
    __shared__ double red[GUARD_BLOCK / 64];
    const int64_t nb = (s.n - c->m + 1 + 255) / 256;
    double g = 0.0;
    for (int64_t q = threadIdx.x; q < nb; q += blockDim.x) {
        const double lo = s.sgm[2 * q + 1];
        double hi = 0.0;
        for (int64_t e = (q >= 2 ? q - 2 : 0); e <= q + 2 && e < nb; ++e) hi = fmax(hi, s.sgm[2 * e]);
        if (lo < f_inf<double>()) {  // not a block of flat windows only
            const double rt = hi / lo;
            g = fmax(g, rt * rt);
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) g = fmax(g, __shfl_xor(g, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = g;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < GUARD_BLOCK / 64; ++q) g = fmax(g, red[q]);
        c->gam2 = g;
        set_sel_thresholds(c, guard);
    }
}

// df[i] = (t_{i+m} - t_i)/2, dg[i] = (t_{i+m} - mu_{i+1}) + (t_i - mu_i) for
// i < N-1 (zero beyond), inv[i] = 1/(sqrt(m) sigma_i) for non-flat i < N.
//
// At a new length every block also records the largest and smallest window
// sigma of its 256 windows, from which k_guard sets the FP32 guard band.
__global__ void k_length(SeriesDev* S, int B, const int64_t* __restrict__ pfx)
{
    const int b = series_of(pfx, B, blockIdx.x);
    const SeriesDev& s = S[b];
    Ctrl* c = s.ctrl;
    if (!c->active) return;
    const int64_t lb = blockIdx.x - pfx[b];
    const int64_t i = lb * (int64_t)blockDim.x + threadIdx.x;
    const int32_t m = c->m;
    const int64_t N = s.n - m + 1;
    double smax = 0.0, smin = f_inf<double>();  // spread extremes of this thread's window
    if (c->new_len && i < s.Npad + 64) {
        const double* __restrict__ T = s.T;
        const bool odd = (c->li & 1) != 0;
        double* mu_n = odd ? s.mu2 : s.mu;
        double* var_n = odd ? s.var2 : s.var;
        const double* mu_o = odd ? s.mu : s.mu2;
        const double* var_o = odd ? s.var : s.var2;
        double m0 = 0.0, v0 = 0.0, m1 = 0.0, v1 = 0.0;
        if (i < N) {
            if (c->new_len == 2) {
                direct_stats(T, i, m, m0, v0);
                if (i + 1 < N) direct_stats(T, i + 1, m, m1, v1);
            } else {
                grow_stats(T, i, m, mu_o[i], var_o[i], m0, v0);
                if (i + 1 < N) grow_stats(T, i + 1, m, mu_o[i + 1], var_o[i + 1], m1, v1);
            }
        }
        mu_n[i] = m0;
        var_n[i] = v0;
        double df = 0.0, dg = 0.0, inv = 0.0;
        if (i < N - 1) {
            const double a = T[i + m], e = T[i];
            df = (a - e) * 0.5;
            dg = (a - m1) + (e - m0);
        }
        if (i < N) {
            const double sg = sqrt(v0);
            if (sg <= c->flat_eps) {
                atomicMin((long long*)&c->flat_min, (long long)i);
                atomicMax((long long*)&c->flat_max, (long long)i);
            } else {
                inv = 1.0 / (sqrt((double)m) * sg);
                smax = smin = sg;
            }
        }
        s.df64[i] = df;
        s.dg64[i] = dg;
        s.inv64[i] = inv;
        s.df32[i] = (float)df;
        s.dg32[i] = (float)dg;
        s.inv32[i] = (float)inv;
    }
    if (c->new_len) spread_extremes(s, lb, smax, smin);
    // every round: all N subsequences start alive, row maxima at -inf
    if (i < s.nwords) {
        const int64_t lo = i * 64;
        unsigned long long bits = 0ull;
        if (lo + 64 <= N) bits = ~0ull;
        else if (lo < N) bits = (1ull << (N - lo)) - 1ull;
        s.alive[i] = bits;
        s.unc[i] = 0ull;
    }
    if (i < s.Npad) {
        s.rho[i] = 0x000fffffffffffffull;  // ordered bits of -inf
        s.rhs[i] = 0x000fffffffffffffull;
    }
}

// ---------------------------------------------------------------------------
// the sweeps
// ---------------------------------------------------------------------------
template <typename F>
struct SweepArgs {
    const double* __restrict__ T;
    const double* __restrict__ mu;
    const F* __restrict__ df;
    const F* __restrict__ dg;
    const F* __restrict__ inv;
    unsigned long long* alive;
    unsigned long long* rho;
    unsigned long long* rhs;
    unsigned long long* unc;
    uint32_t* twork;
    Ctrl* ctrl;
    int64_t N;
    int32_t m;
};

// Copy count doubles from global memory to LDS (the whole workgroup): groups
// of eight loads per thread are issued before their stores, so one memory
// latency covers 8 x blockDim values.
__device__ __forceinline__ void lds_fill(double* dst, const double* __restrict__ src, int count)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int base = 0; base < count; base += nt * 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int t = base + tid + nt * u;
            v[u] = t < count ? src[t] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int t = base + tid + nt * u;
            if (t < count) dst[t] = v[u];
        }
    }
}

// ----- exact values from the FP64 matrix cores -----
// A sweep needs exact FP64 centred dot products in two places: the first
// column of a work item (one per row of the tile) and the top row of the
// tile at every later column (the boundary that feeds the recurrence).
// Both are correlations of one short centred window v (m values) with a
// stretch of the series w:
//     D(p) = sum_k v[k] w[p + k],   p = 0 .. 255,
// which is one 16 x 16 tile of V_MFMA_F64_16X16X4F64 with the Toeplitz
// operand A[r][k] = v[k - r] and the Hankel operand B[k][c] = w[16 c + k]:
// D[r][c] = D(16 c + r).  Lane l supplies A[l % 16][k0 + l / 16] and
// B[k0 + l / 16][l % 16] and receives D[l / 16 + 4 q][l % 16], q < 4, i.e.
// D(p) for p = 16 (l % 16) + l / 16 + 4 q.  Two LDS reads per matrix
// instruction (1024 multiply-adds) replace the two reads per multiply-add of
// a vector loop, which left the sweeps bound by LDS bandwidth.
typedef double pm_acc_t __attribute__((ext_vector_type(4)));
constexpr int HK_PAD = 16;    // zeros before v (k - r >= -15)
constexpr int HK_TILE = 256;  // values D(p) per Hankel tile
// Columns per boundary batch: a whole tile for the FP32 sweeps; half a tile
// for FP64 records, whose smaller staging lets more refinement items stay
// resident (the FP32 sweeps measured slower at half a tile).
__host__ __device__ constexpr int bcols_of(int fbytes) { return fbytes == 8 ? HK_TILE / 2 : HK_TILE; }
template <typename F>
__host__ __device__ constexpr int batch_cols() { return bcols_of((int)sizeof(F)); }
// w is staged skewed (value p at p + p / 16), so that the 16 lanes reading
// w[16 c + k] for c = 0..15 hit distinct LDS banks.
__host__ __device__ constexpr int hk_skew(int p) { return p + (p >> 4); }
// k < 4 hk_steps(m) covers every k - r < m for r < 16
__host__ __device__ constexpr int hk_steps(int m) { return (m + 15 + 3) >> 2; }
// v with HK_PAD zeros before and zeros after: HK_PAD + 4 hk_steps(m) values
__host__ __device__ constexpr int hk_vp_doubles(int m) { return (HK_PAD + 4 * hk_steps(m) + 3) & ~3; }

__device__ __forceinline__ int hk_offset(int q)
{
    const int lane = threadIdx.x;
    return 16 * (lane & 15) + (lane >> 4) + 4 * q;
}

// D(p) for p < ncols (a multiple of 16, at most 256; see above): vp = v
// after HK_PAD zeros, zero beyond m; w = skewed LDS stretch starting at value
// wbase, at least wbase + ncols + m + 16 values.  Lanes of the columns
// c >= ncols / 16 read the stretch's first column instead: their D values
// are not meaningful.  One accumulator (the matrix core chains dependent
// accumulations), so the sweep keeps its registers.
__device__ __forceinline__ pm_acc_t hankel16(const double* vp, const double* w, int wbase, int m,
                                             int ncols = HK_TILE)
{
    const int lane = threadIdx.x;
    const int ca = lane & 15, ka = lane >> 4;
    const int K4 = hk_steps(m);
    const double* va = vp + HK_PAD + ka - ca;
    const int wb = wbase + 16 * (16 * ca < ncols ? ca : 0) + ka;
    pm_acc_t d = {0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < K4; ++s)
        d = __builtin_amdgcn_mfma_f64_16x16x4f64(va[4 * s], w[hk_skew(wb + 4 * s)], d, 0, 0, 0);
    return d;
}

// Copy count doubles from src into the skewed LDS stretch w (the whole
// wave: four loads in flight per lane before their stores).
__device__ __forceinline__ void stage_skewed(double* w, const double* __restrict__ src, int count)
{
    const int lane = threadIdx.x;
    for (int base = 0; base < count; base += 64 * 4) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = base + lane + 64 * u;
            v[u] = t < count ? src[t] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = base + lane + 64 * u;
            if (t < count) w[hk_skew(t)] = v[u];
        }
    }
}

// Column helpers of one step, staged in LDS per batch of columns.
template <typename F>
struct alignas(4 * sizeof(F)) H4 {
    F df, dg, inv;  // df[j-1], dg[j-1], 1/(sqrt(m) sigma_j)
    F B;            // C(i0, j): exact value of the tile's top row at column j
};

// LDS of a sweep work item with R-row tiles, in doubles:
//   xp   [hk_vp_doubles(m)]  the first column's centred window, then the
//                            tile's top-row centred window (padded for the
//                            Toeplitz operand)
//   ws   [sweep_ws_doubles]  skewed series stretch: the rows' windows while
//                            the first column is computed, then each batch's
//                            columns
//   hs   [batch records]     per-step helpers and boundary values of a batch
//                            (the first column's R row values before that)
//   rowv [R]                 refinement only: per-row 1/(sqrt(m) sigma_i)
// (fbytes: bytes of the sweep's float type; nc: columns per batch)
__host__ __device__ constexpr int sweep_ws_count(int m, int R, int nc) { return (R > nc ? R : nc) + m + 16; }
__host__ __device__ constexpr int sweep_ws_doubles(int m, int R, int nc)
{
    return (hk_skew(sweep_ws_count(m, R, nc) - 1) + 1 + 3) & ~3;
}
__host__ __device__ constexpr int sweep_hs_offset(int m, int R, int nc)
{
    return hk_vp_doubles(m) + sweep_ws_doubles(m, R, nc);
}
// (the region first holds the R first-column values of an item, as doubles)
__host__ __device__ constexpr int sweep_hs_doubles(int R, int fbytes, int nc)
{
    return nc * 4 * fbytes / 8 > R ? nc * 4 * fbytes / 8 : R;
}
__host__ __device__ constexpr int sweep_rowv_offset(int m, int R, int fbytes, int nc)
{
    return sweep_hs_offset(m, R, nc) + sweep_hs_doubles(R, fbytes, nc);
}
__host__ __device__ constexpr size_t sweep_lds_doubles(int m, int R, int fbytes, bool rowv, int nc)
{
    return (size_t)(sweep_rowv_offset(m, R, fbytes, nc) + (rowv ? R : 0));
}
__host__ __device__ constexpr size_t sweep_lds_doubles(int m, int R, int fbytes, bool rowv)
{
    return sweep_lds_doubles(m, R, fbytes, rowv, bcols_of(fbytes));
}

// Start of a sweep work item (one wavefront, row tile of R = 64 Q rows from
// i0, first column jbeg): acc[q] = C(rbase + q, jbeg), rbase = i0 + Q lane,
// the centred dot products sum_k t_{i+k} y_k - mu_i Sy with y the centred
// window of column jbeg, from R / 256 Hankel tiles (the rows' values pass
// through the hs region); then xp holds the tile's top-row centred window
// x with sum Sx (zero up to rounding) for the boundary values.
template <int Q>
__device__ void item_start(const double* __restrict__ T, const double* __restrict__ mu, int32_t m,
                           int64_t i0, int64_t jbeg, double* xp, double* ws, double* rowc,
                           double& Sx, double& Sy, double (&acc)[Q])
{
    constexpr int R = 64 * Q;
    const int lane = threadIdx.x;
    const int nvp = hk_vp_doubles(m);
    const double muj = mu[jbeg], mui0 = mu[i0];
    double mr[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) mr[q] = mu[i0 + Q * lane + q];
    // the column window (xp, zero padded) and the rows' stretch (ws)
    for (int t = lane; t < nvp; t += 64) {
        const int k = t - HK_PAD;
        xp[t] = (k >= 0 && k < m) ? T[jbeg + k] : 0.0;
    }
    stage_skewed(ws, T + i0, R + m + 16);
    __syncthreads();
    double sy = 0.0;
    for (int k = lane; k < m; k += 64) {
        const double v = xp[HK_PAD + k] - muj;
        xp[HK_PAD + k] = v;
        sy += v;
    }
    Sy = wave_sum(sy);
    __syncthreads();
#pragma unroll
    for (int h = 0; h < (R + 255) / 256; ++h) {
        const pm_acc_t D = hankel16(xp, ws, 256 * h, m, R - 256 * h < 256 ? R - 256 * h : 256);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int p = 256 * h + hk_offset(q);
            if (p < R) rowc[p] = D[q];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[q] = rowc[Q * lane + q] - mr[q] * Sy;
    // the top row's centred window
    double sx = 0.0;
    for (int k = lane; k < m; k += 64) {
        const double v = ws[hk_skew(k)] - mui0;
        xp[HK_PAD + k] = v;
        sx += v;
    }
    Sx = wave_sum(sx);
    __syncthreads();
}

// One batch of up to NC columns from j0: the series stretch t[j0 ..
// j0 + NC + m + 16) staged skewed, then hs[p] = {df[j0+p-1], dg[j0+p-1],
// inv[j0+p], B(j0+p)} with the exact top-row values B(j) = sum_k x_k t_{j+k}
// - mu_j Sx from one Hankel tile.  Reads stay inside the padded buffers
// (their padding exceeds one 512-row tile beyond the last subsequence).
template <typename F, int NC = batch_cols<F>()>
__device__ void stage_batch(const double* __restrict__ T, const double* __restrict__ mu,
                            const F* __restrict__ df, const F* __restrict__ dg,
                            const F* __restrict__ inv, int32_t m, int64_t j0, const double* xp,
                            double Sx, double* ws, H4<F>* hs)
{
    const int lane = threadIdx.x;
    __syncthreads();  // the previous batch is consumed
#pragma unroll
    for (int u = 0; u < NC / 64; ++u) {
        const int64_t j = j0 + lane + 64 * u;
        H4<F>& h = hs[lane + 64 * u];
        h.df = df[j - 1];
        h.dg = dg[j - 1];
        h.inv = inv[j];
    }
    stage_skewed(ws, T + j0, NC + m + 16);
    __syncthreads();
    const pm_acc_t D = hankel16(xp, ws, 0, m, NC);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int p = hk_offset(q);
        if (p < NC) hs[p].B = (F)(D[q] - mu[j0 + p] * Sx);
    }
    __syncthreads();
}

// ----- sweep machinery shared by selection and refinement -----

// Column helpers are read-only during a sweep and wave-uniform per step:
// reading them through the constant address space lets the compiler use
// scalar loads.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T* p)
{
    return (cptr<T>)p;
}

// Row state is kept as wave-uniform lane masks: bit l of dm[q] is set when
// the row of lane l, slot q is dead (pruned, invalid or past the end).
template <int Q>
__device__ __forceinline__ void rows_from_bitmap(const unsigned long long* alive, int64_t rbase,
                                                 unsigned long long (&dm)[Q])
{
    const unsigned int msk = (Q >= 32) ? 0xffffffffu : ((1u << Q) - 1u);
    const unsigned int live = (unsigned int)(load_word(&alive[rbase >> 6]) >> (rbase & 63)) & msk;
#pragma unroll
    for (int q = 0; q < Q; ++q) dm[q] = uniform64(__ballot(!((live >> q) & 1u)));
}

// Publish rows dead locally but still set in the bitmap; absorb rows the
// bitmap says are dead (`word`: the lane's bitmap word, loaded earlier so
// that its latency overlaps the sweep).  Returns true while some row of the
// tile is alive.
template <int Q>
__device__ __forceinline__ bool sync_rows_with(unsigned long long* alive, int64_t rbase,
                                               unsigned long long word,
                                               unsigned long long (&dm)[Q])
{
    const int lane = threadIdx.x;
    unsigned long long* wp = &alive[rbase >> 6];
    const int off = (int)(rbase & 63);
    const unsigned int msk = (Q >= 32) ? 0xffffffffu : ((1u << Q) - 1u);
    const unsigned int live = (unsigned int)(word >> off) & msk;
    unsigned int mine = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) mine |= (unsigned int)((dm[q] >> lane) & 1ull) << q;
    const unsigned int pub = live & mine;
    if (pub) atomicAnd(wp, ~((unsigned long long)pub << off));
    unsigned long long all = ~0ull;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        dm[q] = uniform64(dm[q] | __ballot(!((live >> q) & 1u)));
        all &= dm[q];
    }
    return __builtin_amdgcn_readfirstlane((int)(all != ~0ull)) != 0;
}

template <int Q>
__device__ __forceinline__ bool sync_rows(unsigned long long* alive, int64_t rbase,
                                          unsigned long long (&dm)[Q])
{
    return sync_rows_with<Q>(alive, rbase, load_word(&alive[rbase >> 6]), dm);
}

__device__ __forceinline__ void kill_columns(unsigned long long* alive, int64_t j0,
                                             unsigned long long bits)
{
    if (bits == 0ull) return;
    if (threadIdx.x == 0) {
        const int64_t w0 = j0 >> 6;
        const int off = (int)(j0 & 63);
        atomicAnd(&alive[w0], ~(bits << off));
        if (off) atomicAnd(&alive[w0 + 1], ~(bits >> (64 - off)));
    }
}

// One step of the diagonal recurrence for all Q slots of every lane.
// Registers rotate: before step u of a group of Q steps, slot q lives in
// C[(q - u) mod Q]; each register is updated in place, so the shift from
// slot q-1 to slot q costs nothing and only slot 0 needs the DPP move from
// the previous lane.  Lane 0 keeps the DPP's old operand instead: Bv, the
// exact boundary value of this step (identical in every lane).
template <typename F, int Q, int U>
__device__ __forceinline__ void advance(F (&C)[Q], const F (&a)[Q], const F (&b)[Q], F dfj, F dgj,
                                        F Bv)
{
#pragma unroll
    for (int q = 1; q < Q; ++q) {
        F& r = C[(q - 1 - U + 2 * Q) % Q];
        r = f_fma(a[q], dgj, f_fma(dfj, b[q], r));
    }
    F& r0 = C[(Q - 1 - U + 2 * Q) % Q];
    r0 = f_fma(a[0], dgj, f_fma(dfj, b[0], dpp_shr1(Bv, r0)));
}
template <int Q, int U>
__device__ __forceinline__ int slot_reg(int q)
{
    return (q - U - 1 + 2 * Q) % Q;  // register of slot q after step U
}

// ----- selection sweep -----
// One step U of a group: advance, then the pruning margin of every slot,
// C * inv_j - th = (rho - thr) / inv_i, which is > 0 exactly when the pair is
// closer than r.  The row keeps its largest margin (folded into the dead
// masks once per block); the column is hit when any slot's margin is > 0.
// MASK: only pairs with j >= i + m count (the triangle next to the band).
template <typename F, int Q, int U, bool MASK>
__device__ __forceinline__ void sel_step(F (&C)[Q], const F (&a)[Q], const F (&b)[Q],
                                         const F (&nth)[Q], F (&rm)[Q], const int32_t (&ri)[Q],
                                         F dfj, F dgj, F invj, F Bv, int32_t jm,
                                         unsigned long long& colbits, int s)
{
    advance<F, Q, U>(C, a, b, dfj, dgj, Bv);
    F mg[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        mg[q] = f_fma(C[slot_reg<Q, U>(q)], invj, nth[q]);
        if (MASK) mg[q] = (jm >= ri[q]) ? mg[q] : -f_inf<F>();
        rm[q] = fmax(rm[q], mg[q]);
    }
    F cm = mg[0];
#pragma unroll
    for (int q = 1; q < Q; ++q) cm = fmax(cm, mg[q]);
    if (uniform64(__ballot(cm > F(0))) != 0ull) colbits |= 1ull << s;
}

template <typename F, int Q, bool MASK>
__device__ __forceinline__ void sel_block(const SweepArgs<F>& A, int64_t j0, int nst, F (&C)[Q],
                                          const F (&a)[Q], const F (&b)[Q], const F (&nth)[Q],
                                          F (&rm)[Q], const int32_t (&ri)[Q], const H4<F>* hs,
                                          unsigned long long& colbits)
{
    for (int s0 = 0; s0 < nst; s0 += Q) {
        const int64_t jg = j0 + s0;
        H4<F> hv[Q];
#pragma unroll
        for (int u = 0; u < Q; ++u) hv[u] = hs[s0 + u];
        const int32_t jm = (int32_t)(jg - A.m);
        const int left = nst - s0;
#define SEL_STEP(U)                                                                            \
    if ((U) < left)                                                                            \
        sel_step<F, Q, ((U) < Q ? (U) : 0), MASK>(C, a, b, nth, rm, ri, hv[(U) % Q].df,       \
                                                  hv[(U) % Q].dg, hv[(U) % Q].inv,             \
                                                  hv[(U) % Q].B, jm + (U), colbits, s0 + (U));
        static_assert(Q == 2 || Q == 4 || Q == 8, "Q must be 2, 4 or 8");
        SEL_STEP(0)
        SEL_STEP(1)
        if (Q > 2) {
            SEL_STEP(2)
            SEL_STEP(3)
        }
        if (Q > 4) {
            SEL_STEP(4)
            SEL_STEP(5)
            SEL_STEP(6)
            SEL_STEP(7)
        }
#undef SEL_STEP
    }
}

// Margins of every slot after one step of a full block (no masks); returns
// the lane's largest margin (the column test).
template <typename F, int Q, int U>
__device__ __forceinline__ F sel_margins(F (&C)[Q], const F (&a)[Q], const F (&b)[Q],
                                         const F (&nth)[Q], const H4<F>& h, F (&mg)[Q])
{
    advance<F, Q, U>(C, a, b, h.df, h.dg, h.B);
#pragma unroll
    for (int q = 0; q < Q; ++q) mg[q] = f_fma(C[slot_reg<Q, U>(q)], h.inv, nth[q]);
    F cm = mg[0];
#pragma unroll
    for (int q = 1; q < Q; ++q) cm = fmax(cm, mg[q]);
    return cm;
}

template <typename F, int Q>
__device__ __forceinline__ void sel_group(F (&C)[Q], const F (&a)[Q], const F (&b)[Q],
                                          const F (&nth)[Q], F (&rm)[Q], const H4<F> (&hv)[Q],
                                          unsigned long long& colbits, int s0)
{
    unsigned long long bal[Q];
#define SEL_PAIR(U)                                                                    \
    {                                                                                  \
        F m0[Q], m1[Q];                                                                \
        const F c0 = sel_margins<F, Q, (U)>(C, a, b, nth, hv[(U)], m0);                \
        bal[(U)] = __ballot(c0 > F(0));                                                \
        const F c1 = sel_margins<F, Q, (U) + 1>(C, a, b, nth, hv[(U) + 1], m1);        \
        bal[(U) + 1] = __ballot(c1 > F(0));                                            \
        _Pragma("unroll") for (int q = 0; q < Q; ++q) rm[q] = fmax(rm[q], fmax(m0[q], m1[q])); \
    }
    static_assert(Q == 2 || Q == 4 || Q == 8, "Q must be 2, 4 or 8");
    SEL_PAIR(0)
    if (Q > 2) SEL_PAIR((Q > 2 ? 2 : 0))
    if (Q > 4) {
        SEL_PAIR((Q > 4 ? 4 : 0))
        SEL_PAIR((Q > 4 ? 6 : 0))
    }
#undef SEL_PAIR
    unsigned long long g = 0ull;
#pragma unroll
    for (int u = 0; u < Q; ++u)
        if (bal[u] != 0ull) g |= 1ull << u;
    colbits |= g << s0;
}

// A full block of 64 steps with every pair a non-self match, in groups of Q
// steps without per-step tests: row maxima fold two steps per max, column
// tests are kept as ballots and folded into colbits once per group.  (Reading
// the next group's helpers ahead costs registers, hence occupancy, and
// measured slower.)
template <typename F, int Q>
__device__ __forceinline__ void sel_block_full(F (&C)[Q], const F (&a)[Q], const F (&b)[Q],
                                               const F (&nth)[Q], F (&rm)[Q], const H4<F>* hs,
                                               unsigned long long& colbits)
{
    for (int s0 = 0; s0 < 64; s0 += Q) {
        H4<F> hv[Q];
#pragma unroll
        for (int u = 0; u < Q; ++u) hv[u] = hs[s0 + u];
        sel_group<F, Q>(C, a, b, nth, rm, hv, colbits, s0);
    }
}

template <typename F, int Q>
__device__ void sel_item(const SweepArgs<F>& A, int64_t i0, int64_t jbeg, int64_t jend, F thr,
                         double* lds, unsigned long long& evals, uint32_t* work)
{
    constexpr int R = 64 * Q;
    i0 = uniform_i64(i0);
    jbeg = uniform_i64(jbeg);
    jend = uniform_i64(jend);
    const int lane = threadIdx.x;
    const int32_t m = A.m;
    const int64_t N = A.N;
    const int64_t rbase = i0 + (int64_t)Q * lane;

    unsigned long long dm[Q];
    rows_from_bitmap<Q>(A.alive, rbase, dm);
    {
        unsigned long long all = ~0ull;
#pragma unroll
        for (int q = 0; q < Q; ++q) all &= dm[q];
        if (all == ~0ull) return;
    }
    double* xp = lds;
    double* ws = lds + hk_vp_doubles(m);
    H4<F>* hs = (H4<F>*)(lds + sweep_hs_offset(m, R, batch_cols<F>()));
    double Sx, Sy;
    F C[Q];
    {
        double acc[Q];
        item_start<Q>(A.T, A.mu, m, i0, jbeg, xp, ws, (double*)hs, Sx, Sy, acc);
#pragma unroll
        for (int q = 0; q < Q; ++q) C[q] = (F)acc[q];
    }
    F a[Q], b[Q], nth[Q], rm[Q];
    int32_t ri[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int64_t i = rbase + q;
        const bool top = (lane == 0) && (q == 0);
        const int64_t ip = top ? i : i - 1;
        a[q] = top ? F(0) : A.df[ip];
        b[q] = top ? F(0) : A.dg[ip];
        const F invi = A.inv[i];
        // margin offset: C * inv_j - thr / inv_i > 0  <=>  rho > thr
        nth[q] = (i < N && invi > F(0)) ? -(thr / invi) : -f_inf<F>();
        ri[q] = (int32_t)i;
        rm[q] = -f_inf<F>();
    }
    // column jbeg
    {
        const F invj = A.inv[jbeg];
        F cm = -f_inf<F>();
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            F mg = f_fma(C[q], invj, nth[q]);
            mg = ((int32_t)(jbeg - m) >= ri[q]) ? mg : -f_inf<F>();
            rm[q] = fmax(rm[q], mg);
            cm = fmax(cm, mg);
        }
        kill_columns(A.alive, jbeg, uniform64(__ballot(cm > F(0))) ? 1ull : 0ull);
#pragma unroll
        for (int q = 0; q < Q; ++q) dm[q] |= uniform64(__ballot(rm[q] > F(0)));
    }
    unsigned long long ev = pair_count(i0, std::min<int64_t>(i0 + R, N), jbeg, 1, m, false);
    bool go = sync_rows<Q>(A.alive, rbase, dm);
    uint32_t nblk = 0;
    int64_t j = jbeg + 1;
    while (go && j < jend) {
        // a batch of up to batch_cols columns (boundary values from one
        // Hankel tile), swept in blocks of 64 with the bitmap synchronised after
        // each
        stage_batch<F>(A.T, A.mu, A.df, A.dg, A.inv, m, j, xp, Sx, ws, hs);
        const int64_t jb_end = std::min<int64_t>(jend, j + batch_cols<F>());
        for (int sb = 0; go && j < jb_end; ++sb) {
            const int nst = (int)std::min<int64_t>(64, jb_end - j);
            const H4<F>* hb = hs + 64 * sb;
            const unsigned long long word = load_word(&A.alive[rbase >> 6]);
            unsigned long long colbits = 0ull;
            const bool full = (j - (i0 + R - 1)) >= m;
            if (Q <= 4 && full && nst == 64)  // taller tiles: the general path keeps fewer registers
                sel_block_full<F, Q>(C, a, b, nth, rm, hb, colbits);
            else if (full)
                sel_block<F, Q, false>(A, j, nst, C, a, b, nth, rm, ri, hb, colbits);
            else
                sel_block<F, Q, true>(A, j, nst, C, a, b, nth, rm, ri, hb, colbits);
            kill_columns(A.alive, j, colbits);
#pragma unroll
            for (int q = 0; q < Q; ++q) dm[q] |= uniform64(__ballot(rm[q] > F(0)));
            ev += pair_count(i0, std::min<int64_t>(i0 + R, N), j, nst, m, false);
            j += nst;
            go = sync_rows_with<Q>(A.alive, rbase, word, dm);
            ++nblk;
        }
    }
    if (work && lane == 0 && nblk) atomicAdd(work, nblk);
    // rows still alive: their largest correlation over this item's columns
    // (rho - thr = margin * inv_i), for the refinement that sweeps only the
    // left side of tiles whose rows are all clearly below the threshold;
    // rows above thr64 - guard are marked in unc
    const double ulim = 2.0 * A.ctrl->thr64 - A.ctrl->thr_sel;
    unsigned long long ub[Q];
    unsigned long long uany = 0ull;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int64_t i = rbase + q;
        bool u = false;
        if (!((dm[q] >> lane) & 1ull) && i < N && rm[q] > -f_inf<F>()) {
            const double rt = (double)rm[q] * (double)A.inv[i] + (double)thr;
            atomicMax(&A.rhs[i], ord_of(rt));
            u = rt > ulim;
        }
        ub[q] = uniform64(__ballot(u));
        uany |= ub[q];
    }
    // one atomic per bitmap word: lane l's slot q is row Q l + q of the tile
    if (uany != 0ull && lane == 0) {
        constexpr int LPW = 64 / Q;  // lanes per bitmap word
#pragma unroll
        for (int wd = 0; wd < Q; ++wd) {
            unsigned long long mask = 0ull;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                unsigned long long lb = (ub[q] >> (wd * LPW)) & ((LPW == 64) ? ~0ull : ((1ull << LPW) - 1ull));
                while (lb) {
                    const int l = __ffsll((long long)lb) - 1;
                    lb &= lb - 1ull;
                    mask |= 1ull << (Q * l + q);
                }
            }
            if (mask) atomicOr(&A.unc[(i0 >> 6) + wd], mask);
        }
    }
    evals += ev;
}

template <typename F>
__device__ __forceinline__ F sel_threshold(const Ctrl* c);
template <>
__device__ __forceinline__ float sel_threshold<float>(const Ctrl* c) { return c->thr32; }
template <>
__device__ __forceinline__ double sel_threshold<double>(const Ctrl* c) { return c->thr_sel; }

template <typename F>
__device__ __forceinline__ SweepArgs<F> args_of(const SeriesDev& s, Ctrl* c);
template <>
__device__ __forceinline__ SweepArgs<float> args_of<float>(const SeriesDev& s, Ctrl* c)
{
    SweepArgs<float> A;
    A.T = s.T;
    A.mu = cur_mu(s, c);
    A.df = s.df32;
    A.dg = s.dg32;
    A.inv = s.inv32;
    A.alive = s.alive;
    A.rho = s.rho;
    A.rhs = s.rhs;
    A.unc = s.unc;
    A.twork = s.twork;
    A.ctrl = c;
    A.m = c->m;
    A.N = s.n - A.m + 1;
    return A;
}
template <>
__device__ __forceinline__ SweepArgs<double> args_of<double>(const SeriesDev& s, Ctrl* c)
{
    SweepArgs<double> A;
    A.T = s.T;
    A.mu = cur_mu(s, c);
    A.df = s.df64;
    A.dg = s.dg64;
    A.inv = s.inv64;
    A.alive = s.alive;
    A.rho = s.rho;
    A.rhs = s.rhs;
    A.unc = s.unc;
    A.twork = s.twork;
    A.ctrl = c;
    A.m = c->m;
    A.N = s.n - A.m + 1;
    return A;
}

// ----- refinement sweep (FP64) -----
// MASK 0: all pairs valid; 1: right side (j >= i + m); 2: left side (j <= i - m).
template <int Q, int U, int MASK>
__device__ __forceinline__ void ref_step(double (&C)[Q], const double (&a)[Q], const double (&b)[Q],
                                         double (&mx)[Q], const int32_t (&ri)[Q], double dfj,
                                         double dgj, double invj, double Bv, int32_t jm,
                                         int32_t jp)
{
    advance<double, Q, U>(C, a, b, dfj, dgj, Bv);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        double v = C[slot_reg<Q, U>(q)] * invj;
        if (MASK == 1) v = (jm >= ri[q]) ? v : -f_inf<double>();
        if (MASK == 2) v = (jp <= ri[q]) ? v : -f_inf<double>();
        mx[q] = fmax(mx[q], v);
    }
}

template <int Q, int MASK>
__device__ __forceinline__ void ref_block(const SweepArgs<double>& A, int64_t j0, int nst,
                                          double (&C)[Q], const double (&a)[Q],
                                          const double (&b)[Q], double (&mx)[Q],
                                          const int32_t (&ri)[Q], const H4<double>* hs)
{
    for (int s0 = 0; s0 < nst; s0 += Q) {
        const int64_t jg = j0 + s0;
        H4<double> hv[Q];
#pragma unroll
        for (int u = 0; u < Q; ++u) hv[u] = hs[s0 + u];
        const int32_t jm = (int32_t)(jg - A.m), jp = (int32_t)(jg + A.m);
        const int left = nst - s0;
#define REF_STEP(U)                                                                             \
    if ((U) < left)                                                                             \
        ref_step<Q, ((U) < Q ? (U) : 0), MASK>(C, a, b, mx, ri, hv[(U) % Q].df, hv[(U) % Q].dg, \
                                               hv[(U) % Q].inv, hv[(U) % Q].B, jm + (U),        \
                                               jp + (U));
        static_assert(Q == 2 || Q == 4 || Q == 8, "Q must be 2, 4 or 8");
        REF_STEP(0)
        REF_STEP(1)
        if (Q > 2) {
            REF_STEP(2)
            REF_STEP(3)
        }
        if (Q > 4) {
            REF_STEP(4)
            REF_STEP(5)
            REF_STEP(6)
            REF_STEP(7)
        }
#undef REF_STEP
    }
}

// A full refinement block of 64 steps (every pair valid) in groups of Q
// steps without per-step tests; row maxima fold two steps per max.
template <int Q>
__device__ __forceinline__ void ref_block_full(double (&C)[Q], const double (&a)[Q],
                                               const double (&b)[Q], double (&mx)[Q],
                                               const H4<double>* hs)
{
    for (int s0 = 0; s0 < 64; s0 += Q) {
        H4<double> hv[Q];
#pragma unroll
        for (int u = 0; u < Q; ++u) hv[u] = hs[s0 + u];
#define REF_PAIR(U)                                                                        \
    {                                                                                      \
        double v0[Q], v1[Q];                                                               \
        advance<double, Q, (U)>(C, a, b, hv[(U)].df, hv[(U)].dg, hv[(U)].B);               \
        _Pragma("unroll") for (int q = 0; q < Q; ++q) v0[q] =                              \
            C[slot_reg<Q, (U)>(q)] * hv[(U)].inv;                                          \
        advance<double, Q, (U) + 1>(C, a, b, hv[(U) + 1].df, hv[(U) + 1].dg, hv[(U) + 1].B); \
        _Pragma("unroll") for (int q = 0; q < Q; ++q) v1[q] =                              \
            C[slot_reg<Q, (U) + 1>(q)] * hv[(U) + 1].inv;                                  \
        _Pragma("unroll") for (int q = 0; q < Q; ++q) mx[q] = fmax(mx[q], fmax(v0[q], v1[q])); \
    }
        static_assert(Q == 2 || Q == 4 || Q == 8, "Q must be 2, 4 or 8");
        REF_PAIR(0)
        if (Q > 2) REF_PAIR((Q > 2 ? 2 : 0))
        if (Q > 4) {
            REF_PAIR((Q > 4 ? 4 : 0))
            REF_PAIR((Q > 4 ? 6 : 0))
        }
#undef REF_PAIR
    }
}

template <int Q, int NC = batch_cols<double>()>
__device__ void ref_item(const SweepArgs<double>& A, int64_t i0, int64_t jbeg, int64_t jend,
                         bool left, double thr, int prune, double* lds, unsigned long long& evals)
{
    constexpr int R = 64 * Q;
    i0 = uniform_i64(i0);
    jbeg = uniform_i64(jbeg);
    jend = uniform_i64(jend);
    const int lane = threadIdx.x;
    const int32_t m = A.m;
    const int64_t N = A.N;
    const int64_t rbase = i0 + (int64_t)Q * lane;
    const Ctrl* c = A.ctrl;

    unsigned long long dm[Q];
    rows_from_bitmap<Q>(A.alive, rbase, dm);
    {
        unsigned long long all = ~0ull;
#pragma unroll
        for (int q = 0; q < Q; ++q) all &= dm[q];
        if (all == ~0ull) return;
    }
    double* xp = lds;
    double* ws = lds + hk_vp_doubles(m);
    H4<double>* hs = (H4<double>*)(lds + sweep_hs_offset(m, R, NC));
    double Sx, Sy;
    double C[Q];
    item_start<Q>(A.T, A.mu, m, i0, jbeg, xp, ws, (double*)hs, Sx, Sy, C);
    double a[Q], b[Q], mx[Q];
    int32_t ri[Q];
    // 1/(sqrt(m) sigma_i) of the lane's rows
    double* rowinv = lds + sweep_rowv_offset(m, R, 8, NC);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int64_t i = rbase + q;
        const bool top = (lane == 0) && (q == 0);
        const int64_t ip = top ? i : i - 1;
        a[q] = top ? 0.0 : A.df[ip];
        b[q] = top ? 0.0 : A.dg[ip];
        rowinv[Q * lane + q] = A.inv[i];
        mx[q] = -f_inf<double>();
        ri[q] = (int32_t)i;
    }
    {
        const double invj = A.inv[jbeg];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const bool ok = left ? ((int32_t)(jbeg + m) <= ri[q]) : ((int32_t)(jbeg - m) >= ri[q]);
            if (ok) mx[q] = fmax(mx[q], C[q] * invj);
        }
    }
    unsigned long long ev = pair_count(i0, std::min<int64_t>(i0 + R, N), jbeg, 1, m, left);
    int64_t j = jbeg + 1;
    bool go = true;
    while (go && j < jend) {
        stage_batch<double, NC>(A.T, A.mu, A.df, A.dg, A.inv, m, j, xp, Sx, ws, hs);
        const int64_t jb_end = std::min<int64_t>(jend, j + NC);
        for (int sb = 0; go && j < jb_end; ++sb) {
            const int nst = (int)std::min<int64_t>(64, jb_end - j);
            const H4<double>* hb = hs + 64 * sb;
            const unsigned long long word = load_word(&A.alive[rbase >> 6]);
            bool full;
            if (left) full = (i0 - (j + nst - 1)) >= m;
            else full = (j - (i0 + R - 1)) >= m;
            if (full && nst == 64) ref_block_full<Q>(C, a, b, mx, hb);
            else if (full) ref_block<Q, 0>(A, j, nst, C, a, b, mx, ri, hb);
            else if (left) ref_block<Q, 2>(A, j, nst, C, a, b, mx, ri, hb);
            else ref_block<Q, 1>(A, j, nst, C, a, b, mx, ri, hb);
            ev += pair_count(i0, std::min<int64_t>(i0 + R, N), j, nst, m, left);
            j += nst;
            if (prune) {
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const double iv = rowinv[Q * lane + q];
                    dm[q] |= uniform64(__ballot(iv > 0.0 && mx[q] * iv > thr));
                }
            }
            go = sync_rows_with<Q>(A.alive, rbase, word, dm);
        }
    }
    double invi[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) invi[q] = rowinv[Q * lane + q];
    // flat rows: correlation 1 with another flat window, 0 with any other
    const int64_t flo = c->flat_min, fhi = c->flat_max;
    bool flat[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int64_t i = rbase + q;
        flat[q] = (i < N) && !(invi[q] > 0.0);
        if (flat[q]) {
            const bool partner = (flo >= 0 && flo <= i - m) || (fhi >= 0 && fhi >= i + m);
            mx[q] = partner ? 1.0 : 0.0;
        }
        if (prune) dm[q] |= uniform64(__ballot(flat[q] && mx[q] > thr));
    }
    sync_rows<Q>(A.alive, rbase, dm);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int64_t i = rbase + q;
        const bool dead = (dm[q] >> lane) & 1ull;
        if (!dead && i < N && mx[q] > -f_inf<double>()) {
            const double rho = flat[q] ? mx[q] : mx[q] * invi[q];
            atomicMax(&A.rho[i], ord_of(rho));
        }
    }
    evals += ev;
}

// The first local item of this workgroup in a series whose items start at
// global number cum: the smallest it >= 0 with (cum + it) mod G = g.
__device__ __forceinline__ unsigned long long first_item(unsigned long long cum)
{
    const unsigned long long G = gridDim.x;
    return ((unsigned long long)blockIdx.x + G - cum % G) % G;
}

// ----- diagonal band pre-pass of the first selection pass -----
// The pairs (i, i + d), d in [m, m + BAND_D), of every subsequence — its
// nearest non-self matches on the right — swept down the diagonals.  A work
// item is one wavefront owning BAND_D consecutive diagonals (BAND_Q per
// lane, consecutive) over BAND_S consecutive rows.  Each lane carries its
// diagonals' values from row to row with the centred recurrence (R23) in
// the selection precision, started from exact FP64 values of the item's top
// row (one Hankel tile on the matrix cores), so every value is at most
// BAND_S steps from an exact one, as in the row-tile sweeps.  A pair that
// passes the selection test kills both subsequences: the row through the
// wave's ballot of the step, the column through per-lane bit histories
// (one add-with-carry per pair) merged in LDS and published once per item.
// No tile straddles the exclusion zone, so every pair evaluated counts.
// The pass only prunes: the row-tile passes after it still sweep each tile
// with a live row from its first non-self column, which keeps the recorded
// right-side maxima of the surviving rows complete.
constexpr int BAND_Q = 4;
constexpr int BAND_D = 64 * BAND_Q;      // diagonals per item
constexpr int BAND_S = 256;              // rows per item (a multiple of 64)
constexpr int BAND_C = BAND_S + BAND_D;  // column records per item (the last one is padding)
constexpr int BAND_W32 = (BAND_C + 64) / 32;  // column-kill words, aligned to the bitmap
static_assert(BAND_D == HK_TILE, "one Hankel tile gives the top row's values");

__host__ __device__ constexpr size_t band_lds_bytes(int m, int fbytes)
{
    // phase 1: top-row window + skewed series stretch for the Hankel tile
    // phase 2: column records, row records, column-kill bits
    return (size_t)8 * (hk_vp_doubles(m) + ((hk_skew(HK_TILE + m + 16 - 1) + 1 + 3) & ~3)) >
                   (size_t)4 * fbytes * (BAND_C + BAND_S) + 4 * BAND_W32
               ? (size_t)8 * (hk_vp_doubles(m) + ((hk_skew(HK_TILE + m + 16 - 1) + 1 + 3) & ~3))
               : (size_t)4 * fbytes * (BAND_C + BAND_S) + 4 * BAND_W32;
}

// One row step's kill tests, for the BAND_Q pairs of every lane: per slot
// km = 2 km + (mg > 0) (the lane's column history, newest step in bit 0) as
// one compare and one add-with-carry, and the row's history rh = 2 rh +
// (some pair of the wave has mg > 0) in scalar instructions.  (Written as C,
// the compiler reassociates the unrolled histories into sums of selected
// powers of two and keeps every step's masks alive until the end.)
#define BAND_CMP_F32 "v_cmp_lt_f32_e64"
#define BAND_CMP_F64 "v_cmp_lt_f64_e64"
#define BAND_HIT_ASM(CMP)                                                                   \
    CMP " %[m0], 0, %[g0]\n\t"                                                              \
        "v_addc_co_u32_e64 %[k0], %[co], %[k0], %[k0], %[m0]\n\t" CMP " %[m1], 0, %[g1]\n\t" \
        "v_addc_co_u32_e64 %[k1], %[co], %[k1], %[k1], %[m1]\n\t" CMP " %[m2], 0, %[g2]\n\t" \
        "v_addc_co_u32_e64 %[k2], %[co], %[k2], %[k2], %[m2]\n\t" CMP " %[m3], 0, %[g3]\n\t" \
        "v_addc_co_u32_e64 %[k3], %[co], %[k3], %[k3], %[m3]\n\t"                           \
        "s_or_b64 %[m0], %[m0], %[m1]\n\t"                                                   \
        "s_or_b64 %[m2], %[m2], %[m3]\n\t"                                                   \
        "s_or_b64 %[m0], %[m0], %[m2]\n\t"                                                   \
        "s_cmp_lg_u64 %[m0], 0\n\t"                                                          \
        "s_addc_u32 %[rh], %[rh], %[rh]"
template <typename F>
__device__ __forceinline__ void band_hits(const F (&mg)[BAND_Q], unsigned int (&km)[BAND_Q],
                                          unsigned int& rh)
{
    static_assert(BAND_Q == 4, "four slots per lane");
    unsigned long long m0, m1, m2, m3, co;
    if constexpr (sizeof(F) == 4) {
        asm(BAND_HIT_ASM(BAND_CMP_F32)
            : [k0] "+v"(km[0]), [k1] "+v"(km[1]), [k2] "+v"(km[2]), [k3] "+v"(km[3]),
              [rh] "+s"(rh), [m0] "=&s"(m0), [m1] "=&s"(m1), [m2] "=&s"(m2), [m3] "=&s"(m3),
              [co] "=&s"(co)
            : [g0] "v"(mg[0]), [g1] "v"(mg[1]), [g2] "v"(mg[2]), [g3] "v"(mg[3])
            : "scc");
    } else {
        asm(BAND_HIT_ASM(BAND_CMP_F64)
            : [k0] "+v"(km[0]), [k1] "+v"(km[1]), [k2] "+v"(km[2]), [k3] "+v"(km[3]),
              [rh] "+s"(rh), [m0] "=&s"(m0), [m1] "=&s"(m1), [m2] "=&s"(m2), [m3] "=&s"(m3),
              [co] "=&s"(co)
            : [g0] "v"(mg[0]), [g1] "v"(mg[1]), [g2] "v"(mg[2]), [g3] "v"(mg[3])
            : "scc");
    }
}

template <typename F>
__global__ __launch_bounds__(64) void k_select_band(SeriesDev* S, int B, const int64_t* __restrict__ pfx)
{
    extern __shared__ double lds[];
    const int b = series_of(pfx, B, blockIdx.x);
    const SeriesDev& s = S[b];
    Ctrl* c = s.ctrl;
    if (!c->active || !c->prune) return;
    const SweepArgs<F> A = args_of<F>(s, c);
    const int32_t m = A.m;
    const int64_t i0 = (int64_t)(blockIdx.x - pfx[b]) * BAND_S;
    const int64_t j0 = i0 + m;  // column of the top row on the first diagonal
    // every column of the item inside the series (the tail is left to the
    // row-tile passes)
    if (j0 + BAND_C - 1 > A.N) return;
    const int lane = threadIdx.x;
    const F thr = sel_threshold<F>(c);

    // exact top-row values C(i0, j0 + p), p < 256
    F C[BAND_Q];
    {
        double* xp = lds;
        double* ws = lds + hk_vp_doubles(m);
        const double mui0 = A.mu[i0];
        const int nvp = hk_vp_doubles(m);
        double sx = 0.0;
        for (int t = lane; t < nvp; t += 64) {
            const int k = t - HK_PAD;
            double v = 0.0;
            if (k >= 0 && k < m) {
                v = A.T[i0 + k] - mui0;
                sx += v;
            }
            xp[t] = v;
        }
        const double Sx = wave_sum(sx);
        stage_skewed(ws, A.T + j0, HK_TILE + m + 16);
        __syncthreads();
        const pm_acc_t D = hankel16(xp, ws, 0, m);
        __syncthreads();  // the stretch is consumed: its space takes the values
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int p = hk_offset(q);
            ws[p] = D[q] - A.mu[j0 + p] * Sx;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < BAND_Q; ++q) C[q] = (F)ws[BAND_Q * lane + q];
        __syncthreads();  // phase 1 is over
    }

    // column records (helpers of column j0 + e: df[j-1], dg[j-1], inv[j])
    // and row records (df[i-1], dg[i-1], -thr / inv_i: the margin offset)
    H4<F>* colh = (H4<F>*)lds;
    H4<F>* rowh = colh + BAND_C;
    uint32_t* kb = (uint32_t*)(rowh + BAND_S);
    {
        constexpr int NE = BAND_C / 64, NT = BAND_S / 64;
        F v[NE][3];
#pragma unroll
        for (int u = 0; u < NE; ++u) {
            const int64_t j = j0 + lane + 64 * u;
            v[u][0] = A.df[j - 1];
            v[u][1] = A.dg[j - 1];
            v[u][2] = A.inv[j];
        }
#pragma unroll
        for (int u = 0; u < NE; ++u) {
            H4<F> h;
            h.df = v[u][0];
            h.dg = v[u][1];
            h.inv = v[u][2];
            h.B = F(0);
            colh[lane + 64 * u] = h;
        }
        F r[NT][3];
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            const int t = lane + 64 * u;
            const int64_t ip = i0 + t - (t > 0 ? 1 : 0);  // row 0 takes no step
            r[u][0] = A.df[ip];
            r[u][1] = A.dg[ip];
            r[u][2] = A.inv[i0 + t];
        }
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            H4<F> h;
            h.df = r[u][0];
            h.dg = r[u][1];
            h.inv = r[u][2] > F(0) ? -(thr / r[u][2]) : -f_inf<F>();
            h.B = F(0);
            rowh[lane + 64 * u] = h;
        }
        if (lane < BAND_W32) kb[lane] = 0u;
    }
    __syncthreads();

    // row i0 + t, slot q of the lane: diagonal m + BAND_Q lane + q, column
    // record t + BAND_Q lane + q, held in hv[(q + t) % BAND_Q] (the records
    // shift down one slot per row; the top slot is read from LDS)
    const int off = (int)(j0 & 63);
    H4<F> hv[BAND_Q];
#pragma unroll
    for (int q = 0; q < BAND_Q; ++q) hv[q] = colh[BAND_Q * lane + q];
    unsigned int km[BAND_Q];
#pragma unroll
    for (int q = 0; q < BAND_Q; ++q) km[q] = 0u;
    unsigned long long rowbits = 0ull;
    unsigned int rhist = 0u;
    for (int t0 = 0; t0 < BAND_S; t0 += 32) {
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            const int t = t0 + u;
            const H4<F> rh = rowh[t];
            if (u != 0 || t0 != 0) {
                hv[(BAND_Q - 1 + u) % BAND_Q] = colh[t + BAND_Q * lane + BAND_Q - 1];
#pragma unroll
                for (int q = 0; q < BAND_Q; ++q) {
                    const H4<F>& h = hv[(q + u) % BAND_Q];
                    C[q] = f_fma(rh.df, h.dg, f_fma(h.df, rh.dg, C[q]));
                }
            }
            F mg[BAND_Q];
#pragma unroll
            for (int q = 0; q < BAND_Q; ++q) mg[q] = f_fma(C[q], hv[(q + u) % BAND_Q].inv, rh.inv);
            band_hits<F>(mg, km, rhist);
        }
        // bit 31 - u of rhist: row i0 + t0 + u; of km[q]: column record
        // t0 + u + BAND_Q lane + q
        rowbits |= (unsigned long long)__builtin_bitreverse32(rhist) << (t0 & 32);
        rhist = 0u;
#pragma unroll
        for (int q = 0; q < BAND_Q; ++q) {
            const unsigned int v = __builtin_bitreverse32(km[q]);
            if (v) {
                const int cb = off + t0 + BAND_Q * lane + q;
                atomicOr(&kb[cb >> 5], v << (cb & 31));
                if (cb & 31) atomicOr(&kb[(cb >> 5) + 1], v >> (32 - (cb & 31)));
            }
            km[q] = 0u;
        }
        if ((t0 & 63) == 32) {
            if (lane == 0 && rowbits) atomicAnd(&A.alive[(i0 + t0 - 32) >> 6], ~rowbits);
            rowbits = 0ull;
        }
    }
    __syncthreads();
    // the killed columns, one bitmap word per lane (kb bit off + e: column j0 + e)
    if (lane < BAND_W32 / 2) {
        const unsigned long long bits =
            (unsigned long long)kb[2 * lane] | ((unsigned long long)kb[2 * lane + 1] << 32);
        if (bits) atomicAnd(&A.alive[(j0 >> 6) + lane], ~bits);
    }
    if (lane == 0)
        atomicAdd(&s.evc[EV_BAND * EV_SLOTS + (blockIdx.x & (EV_SLOTS - 1))],
                  (unsigned long long)BAND_S * BAND_D);
}

// First selection pass: every row tile's nearest near_cols columns, split
// into chunks of `chunk` columns that run concurrently; each stops as soon
// as the whole tile is dead.
template <typename F, int Q>
__global__ __launch_bounds__(64) void k_select_near(SeriesDev* S, int B,
                                                    const int64_t* __restrict__ pfx, int near_cols,
                                                    int chunk)
{
    extern __shared__ double lds[];
    const int b = series_of(pfx, B, blockIdx.x);
    const SeriesDev& s = S[b];
    Ctrl* c = s.ctrl;
    if (!c->active || !c->prune) return;
    constexpr int R = 64 * Q;
    const int64_t lb = blockIdx.x - pfx[b];
    const SweepArgs<F> A = args_of<F>(s, c);
    // The series' blocks enumerate (tile, chunk) pairs: first every chunk of
    // the hot tiles (those that held survivors after the last round), then
    // the other tiles; both parts chunk-major, so that every tile's nearest
    // chunk is dispatched before its later ones, which then find the rows
    // their neighbours already pruned.
    const int64_t ntiles = (s.Nmax + R - 1) / R;
    const int64_t nsub = (pfx[b + 1] - pfx[b]) / ntiles;
    const unsigned int nhot = c->hot_r == R ? c->nhot : 0u;
    int64_t tile, cc;
    if (nhot == 0u) {
        tile = lb % ntiles;
        cc = lb / ntiles;
    } else {
        const int lane = threadIdx.x;
        const int hv = lane < (int)nhot ? s.hot[lane] : 0x7fffffff;
        const int64_t nh = (int64_t)nhot * nsub;
        if (lb < nh) {
            // rotated by the chunk so that one tile's chunks do not all fall
            // on the same XCD when nhot is a multiple of the XCD count
            cc = lb / nhot;
            tile = __builtin_amdgcn_readlane(hv, (int)((lb + cc) % nhot));
        } else {
            // the r-th tile that is not hot is r + #{i : hot[i] - i <= r}
            const int64_t x = lb - nh;
            const int64_t rest = ntiles - nhot;
            if (rest <= 0) return;
            const int64_t r = x % rest;
            cc = x / rest;
            tile = r + __popcll(__ballot(lane < (int)nhot && (int64_t)(hv - lane) <= r));
        }
    }
    const int64_t i0 = tile * R;
    if (i0 >= A.N) return;
    const int64_t j00 = i0 + A.m;
    const int64_t jbeg = j00 + cc * chunk;
    if (jbeg >= A.N || jbeg >= j00 + near_cols) return;
    const int64_t jend = std::min<int64_t>(std::min<int64_t>(A.N, jbeg + chunk), j00 + near_cols);
    const F thr = sel_threshold<F>(c);
    unsigned long long ev = 0;
    sel_item<F, Q>(A, i0, jbeg, jend, thr, lds, ev, &A.twork[tile]);
    if (threadIdx.x == 0 && ev) {
        atomicAdd(&s.evc[EV_NEAR * EV_SLOTS + (blockIdx.x & (EV_SLOTS - 1))], ev);
    }
}

// Remaining selection work: items (live tile, chunk) drawn nearest-first
// from each series' counter; a workgroup drains the series in rotated order.
// The FP32 two-row tile fits 128 registers, so four waves share a SIMD
// (three otherwise): the pass is bound by how many items are resident.
template <typename F, int Q>
__global__ __launch_bounds__(64, (sizeof(F) == 4 && Q <= 2) ? 4 : 1) void k_select_far(
    SeriesDev* S, int B, int near_cols, int chunk, int near_rows)
{
    extern __shared__ double lds[];
    constexpr int R = 64 * Q;
    // Items are dealt out statically: the items of series b get the global
    // numbers cum_b + it (cum_b = items of the series before it) and
    // workgroup g takes the global numbers g, g + G, ...  (a shared queue
    // counter would cost one serialised device-scope atomic per item).
    unsigned long long cum = 0;
    for (int b = 0; b < B; ++b) {
        const SeriesDev& s = S[b];
        Ctrl* c = s.ctrl;
        if (!c->active || !c->prune) continue;
        const unsigned int nlive = c->nlive_sel;
        const unsigned long long total = (unsigned long long)nlive * c->maxc_sel;
        if (total == 0) continue;
        const unsigned long long first = first_item(cum);
        cum += total;
        const SweepArgs<F> A = args_of<F>(s, c);
        const F thr = sel_threshold<F>(c);
        const int32_t* __restrict__ tiles = s.tsel;
        unsigned long long ev = 0;
        for (unsigned long long it = first; it < total; it += gridDim.x) {
            const unsigned long long cc = it / nlive;
            const unsigned int p = (unsigned int)(it % nlive);
            const int64_t i0 = (int64_t)tiles[p] * R;
            // continue where the first pass (tiles of near_rows rows) ended,
            // so that every row's right side is covered completely
            const int64_t jbeg = (i0 / near_rows) * near_rows + A.m + near_cols + (int64_t)cc * chunk;
            if (jbeg >= A.N) continue;
            const int64_t jend = std::min<int64_t>(A.N, jbeg + chunk);
            sel_item<F, Q>(A, i0, jbeg, jend, thr, lds, ev, nullptr);
        }
        if (threadIdx.x == 0 && ev) {
            atomicAdd(&s.evc[EV_FAR * EV_SLOTS + (blockIdx.x & (EV_SLOTS - 1))], ev);
        }
    }
}

// Live-tile lists.  mode 0: selection tiles (R rows), chunks to the right
// beyond the first pass; mode 1: refinement tiles, chunks on both sides.
// One thread per tile; the block's live tiles are compacted with wave
// ballots and a prefix over the block's waves, so each block makes one
// atomic per counter (device-scope atomics on one address serialise).
constexpr int TILES_BLOCK = 256;
__global__ __launch_bounds__(TILES_BLOCK) void k_tiles(SeriesDev* S, int B,
                                                       const int64_t* __restrict__ pfx, int R,
                                                       int mode, int near_cols, int chunk,
                                                       int near_rows)
{
    constexpr int NW = TILES_BLOCK / 64;
    __shared__ unsigned int wn[NW], wmax[NW];
    __shared__ unsigned long long wrows[NW];
    __shared__ unsigned int base_s;
    const int b = series_of(pfx, B, blockIdx.x);
    const SeriesDev& s = S[b];
    Ctrl* c = s.ctrl;
    if (!c->active) return;
    if (mode == 0 && !c->prune) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t t = (blockIdx.x - pfx[b]) * (int64_t)TILES_BLOCK + threadIdx.x;
    const int32_t m = c->m;
    const int64_t N = s.n - m + 1;
    const int64_t ntiles = (N + R - 1) / R;
    const int words = R / 64;
    unsigned int cnt = 0;
    int64_t nch = 0;
    bool both = true;
    if (t < ntiles) {
        unsigned long long any = 0ull;
        for (int q = 0; q < words; ++q) {
            const unsigned long long v = s.alive[t * words + q];
            any |= v;
            cnt += (unsigned int)__popcll(v);
        }
        const int64_t i0 = t * R;
        if (any == 0ull) {
            nch = 0;
        } else if (mode == 0) {
            // the first pass covered near_cols columns from its own tile's start
            const int64_t j0 = (i0 / near_rows) * near_rows + m + near_cols;
            nch = j0 >= N ? 0 : (N - j0 + chunk - 1) / chunk;
        } else {
            const int64_t lend = std::min<int64_t>(N, i0 + R - m);
            const int64_t nl = lend > 0 ? (lend + chunk - 1) / chunk : 0;
            const int64_t jr = i0 + m;
            const int64_t nr = jr < N ? (N - jr + chunk - 1) / chunk : 0;
            // The selection sweep covered the right side of every live row in
            // FP32; a row's exact maximum there is within the guard g of the
            // recorded one, so the right side needs the exact sweep only when
            // some live row's recorded maximum is above thr64 - g (or when
            // there was no selection sweep, or the round is an exact repeat,
            // or a bare range search or a heatmap, which report every
            // survivor's exact maximum).
            both = !c->prune || c->exact_ref || c->mode == 3 || s.heat != nullptr;
            if (!both) {
                unsigned long long u = 0ull;
                for (int q = 0; q < words; ++q) u |= s.alive[t * words + q] & s.unc[t * words + q];
                both = u != 0ull;
            }
            nch = nl + (both ? nr : 0);
        }
    }
    const bool entry = nch > 0;
    // live rows and entries of the wave, then of the block
    unsigned long long rows = cnt;
    unsigned int mx = (unsigned int)nch;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        rows += __shfl_xor(rows, o);
        mx = max(mx, (unsigned int)__shfl_xor((int)mx, o));
    }
    const unsigned long long bal = __ballot(entry);
    if (lane == 0) {
        wn[w] = (unsigned int)__popcll(bal);
        wrows[w] = rows;
        wmax[w] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int tot = 0, mxb = 0;
        unsigned long long rb = 0ull;
        for (int q = 0; q < NW; ++q) {
            tot += wn[q];
            rb += wrows[q];
            mxb = max(mxb, wmax[q]);
        }
        if (rb) {
            atomicAdd(mode == 0 ? &c->rows_near : &c->rows_far, rb);
            if (mode == 1) atomicAdd(&c->live_ref, (unsigned int)rb);
        }
        base_s = tot ? atomicAdd(mode == 0 ? &c->nlive_sel : &c->nlive_ref, tot) : 0u;
        if (tot) atomicMax(mode == 0 ? &c->maxc_sel : &c->maxc_ref, mxb);
    }
    __syncthreads();
    if (entry) {
        unsigned int before = 0;
        for (int q = 0; q < w; ++q) before += wn[q];
        const unsigned int slot =
            base_s + before + (unsigned int)__popcll(bal & ((1ull << lane) - 1ull));
        // refinement entries carry bit 31 when only the left side is swept
        (mode == 0 ? s.tsel : s.tref)[slot] =
            both ? (int32_t)t : (int32_t)((uint32_t)t | 0x80000000u);
    }
}

// Refinement: exact FP64 row maximum of rho over both sides for every tile
// holding survivors; items drawn nearest-first, alternating right and left.
template <int Q>
__global__ __launch_bounds__(64, (Q <= 4 ? 3 : 1)) void k_refine(SeriesDev* S, int B,
                                                                         int chunk)
{
    extern __shared__ double lds[];
    constexpr int R = 64 * Q;
    unsigned long long cum = 0;  // items dealt out as in k_select_far
    for (int b = 0; b < B; ++b) {
        const SeriesDev& s = S[b];
        Ctrl* c = s.ctrl;
        if (!c->active || direct_round(c)) continue;
        const unsigned int nlive = c->nlive_ref;
        const unsigned long long total = (unsigned long long)nlive * c->maxc_ref;
        if (total == 0) continue;
        const unsigned long long first = first_item(cum);
        cum += total;
        const SweepArgs<double> A = args_of<double>(s, c);
        const double thr = c->thr64;
        const int prune = c->prune;
        const int32_t* __restrict__ tiles = s.tref;
        unsigned long long ev = 0;
        for (unsigned long long it = first; it < total; it += gridDim.x) {
            const unsigned long long cc = it / nlive;
            const unsigned int p = (unsigned int)(it % nlive);
            const int32_t e = tiles[p];
            const int64_t i0 = (int64_t)(e & 0x7fffffff) * R;
            const int64_t lend = std::min<int64_t>(A.N, i0 + R - A.m);
            const int64_t nl = lend > 0 ? (lend + chunk - 1) / chunk : 0;
            const int64_t jr = i0 + A.m;
            const int64_t nr = (e >= 0 && jr < A.N) ? (A.N - jr + chunk - 1) / chunk : 0;
            if ((int64_t)cc >= nl + nr) continue;
            const int64_t mn = std::min(nl, nr);
            bool left;
            int64_t q;
            if ((int64_t)cc < 2 * mn) {
                left = (cc & 1u) != 0u;
                q = cc >> 1;
            } else {
                q = mn + ((int64_t)cc - 2 * mn);
                left = nl > nr;
            }
            int64_t jbeg, jend;
            if (left) {
                jend = lend - q * chunk;
                jbeg = std::max<int64_t>(0, jend - chunk);
            } else {
                jbeg = jr + q * chunk;
                jend = std::min<int64_t>(A.N, jbeg + chunk);
            }
            if (jbeg >= jend) continue;
            ref_item<Q>(A, i0, jbeg, jend, left, thr, prune, lds, ev);
        }
        if (threadIdx.x == 0 && ev)
            atomicAdd(&s.evc[EV_REF * EV_SLOTS + (blockIdx.x & (EV_SLOTS - 1))], ev);
    }
}

struct Key {
    unsigned long long u;  // ordered bits of rho (ascending rho = descending nnDist)
    long long i;
};
constexpr long long KEY_NONE = 0x7fffffffffffffffll;
__device__ __forceinline__ bool key_less(const Key& x, const Key& y)
{
    return x.u < y.u || (x.u == y.u && x.i < y.i);
}
__device__ __forceinline__ Key wave_min_key(Key k)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        Key y;
        y.u = __shfl_xor(k.u, o);
        y.i = __shfl_xor(k.i, o);
        if (key_less(y, k)) k = y;
    }
    return k;
}

// The round's range discords and the candidates to polish (one block per
// series).  After a refinement sweep: count the subsequences still alive
// (the range discords of this range search), pick the k + KP_EXTRA with the
// smallest refined correlation (largest distance; ties: smaller index).  Each
// wave first extracts the best of the bitmap words it owns by rounds of
// wave-wide minimum (no block barriers), then wave 0 extracts the best of
// the pooled per-wave lists.  In a direct round (no refinement sweep) every
// live subsequence becomes a candidate.  Finally write the candidates'
// centred windows x_k = t_{i+k} - mu_i and their sums for the exact pass.
// fn(q, word) for every nonzero word q of the bitmap taken by this thread
// (q = threadIdx.x + TOPK_BLOCK j): sixteen words are loaded before any is
// scanned, so one memory latency covers them.
template <typename Fn>
__device__ __forceinline__ void scan_words(const unsigned long long* __restrict__ alive, int64_t nw,
                                           Fn&& fn)
{
    constexpr int U = 16;
    for (int64_t q0 = threadIdx.x; q0 < nw; q0 += (int64_t)U * TOPK_BLOCK) {
        unsigned long long wv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = q0 + (int64_t)u * TOPK_BLOCK;
            wv[u] = q < nw ? alive[q] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (wv[u]) fn(q0 + (int64_t)u * TOPK_BLOCK, wv[u]);
    }
}

__global__ __launch_bounds__(TOPK_BLOCK) void k_select_top(SeriesDev* S)
{
    constexpr int NW = TOPK_BLOCK / 64;
    __shared__ unsigned long long pu[NW][KP_MAX];
    __shared__ long long pi[NW][KP_MAX];
    __shared__ unsigned int cnt_s[NW];
    __shared__ long long cand_s[KP_MAX];
    __shared__ unsigned int nc_s;
    __shared__ unsigned long long kth_s;
    __shared__ int kp_s;
    const SeriesDev& s = S[blockIdx.x];
    Ctrl* c = s.ctrl;
    if (!c->active) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int32_t m = c->m;
    const int64_t N = s.n - m + 1;
    const int64_t nw = (N + 63) / 64;
    const unsigned long long* __restrict__ alive = s.alive;
    const unsigned long long* __restrict__ rho = s.rho;
    const unsigned long long* __restrict__ rhs = s.rhs;
    const int k = s.k;
    // ranking key of a live row: its refined maximum, or, where refinement
    // swept only the left side, the larger of that and the selection sweep's
    // (within the guard of exact); an exact repeat ranks by exact values
    const bool exact = c->exact_ref || !c->prune || c->mode == 3 || s.heat != nullptr;
    auto key_of = [&](long long i) -> unsigned long long {
        return exact ? rho[i] : (rho[i] > rhs[i] ? rho[i] : rhs[i]);
    };
    int kp;
    if (direct_round(c)) {
        if (tid == 0) nc_s = 0;
        __syncthreads();
        scan_words(alive, nw, [&](int64_t q, unsigned long long bits) {
            while (bits) {
                const int t = __ffsll((long long)bits) - 1;
                bits &= bits - 1ull;
                const unsigned int slot = atomicAdd(&nc_s, 1u);
                if (slot < (unsigned int)KP_MAX) cand_s[slot] = q * 64 + t;
            }
        });
        __syncthreads();
        kp = (int)min(nc_s, (unsigned int)KP_MAX);
        if (kp < k) {
            if (tid == 0) {
                c->nsurv = (unsigned int)kp;
                c->ncand = 0;
            }
            return;
        }
        if (tid < kp) s.cand[tid] = cand_s[tid];
        if (tid == 0) {
            c->nsurv = (unsigned int)kp;  // refined by k_round_end
            c->ncand = (unsigned int)kp;
        }
    } else {
        unsigned int cnt = 0;
        scan_words(alive, nw, [&](int64_t, unsigned long long bits) { cnt += (unsigned int)__popcll(bits); });
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o);
        if (lane == 0) cnt_s[w] = cnt;
        __syncthreads();
        unsigned int ns = 0;
        for (int q = 0; q < NW; ++q) ns += cnt_s[q];
        if (ns < (unsigned int)k) {
            if (tid == 0) {
                c->nsurv = ns;
                c->ncand = 0;
            }
            return;
        }
        kp = (int)min(ns, (unsigned int)(k + KP_EXTRA));
        // per-wave best kp
        {
            Key last = {0ull, -1};
            for (int r = 0; r < kp; ++r) {
                Key best = {~0ull, KEY_NONE};
                scan_words(alive, nw, [&](int64_t q, unsigned long long bits) {
                    while (bits) {
                        const int t = __ffsll((long long)bits) - 1;
                        bits &= bits - 1ull;
                        const long long i = q * 64 + t;
                        const Key x = {key_of(i), i};
                        if ((r == 0 || key_less(last, x)) && key_less(x, best)) best = x;
                    }
                });
                best = wave_min_key(best);
                if (lane == 0) {
                    pu[w][r] = best.u;
                    pi[w][r] = best.i;
                }
                last = best;
                if (__builtin_amdgcn_readfirstlane((int)(best.i == KEY_NONE))) {
                    for (int q = r + 1 + lane; q < kp; q += 64) {
                        pu[w][q] = ~0ull;
                        pi[w][q] = KEY_NONE;
                    }
                    break;
                }
            }
        }
        __syncthreads();
        if (w == 0) {
            Key last = {0ull, -1};
            for (int r = 0; r < kp; ++r) {
                Key best = {~0ull, KEY_NONE};
                for (int e = lane; e < NW * kp; e += 64) {
                    const int ww = e / kp, rr = e - ww * kp;
                    const Key x = {pu[ww][rr], pi[ww][rr]};
                    if (x.i == KEY_NONE) continue;
                    if (r > 0 && !key_less(last, x)) continue;
                    if (key_less(x, best)) best = x;
                }
                best = wave_min_key(best);
                if (lane == 0) {
                    cand_s[r] = best.i;
                    s.cand[r] = best.i;
                    if (r == k - 1) kth_s = best.u;
                }
                last = best;
            }
        }
        if (tid == 0) kp_s = kp;
        __syncthreads();
        if (!exact) {
            // Every row whose key is within 2g of the k-th smallest may hold
            // one of the k smallest exact values (keys are within g of
            // exact): all of them are polished, up to KP_MAX; beyond that
            // the round is repeated with exact refinement.
            const double g = c->thr_sel - c->thr64;
            const unsigned long long ub = ord_of(dbl_of(kth_s) + 2.0 * g);
            if (tid == 0) nc_s = 0;
            __syncthreads();
            unsigned int nb = 0;
            scan_words(alive, nw, [&](int64_t q, unsigned long long bits) {
                while (bits) {
                    const int t = __ffsll((long long)bits) - 1;
                    bits &= bits - 1ull;
                    nb += key_of(q * 64 + t) <= ub ? 1u : 0u;
                }
            });
            if (nb) atomicAdd(&nc_s, nb);
            __syncthreads();
            const unsigned int nband = nc_s;
            __syncthreads();
            if (nband > (unsigned int)KP_MAX) {
                if (tid == 0) {
                    c->band_over = 1;
                    c->nsurv = ns;
                    c->ncand = 0;
                }
                return;
            }
            if (nband > (unsigned int)kp) {
                if (tid == 0) nc_s = 0;
                __syncthreads();
                scan_words(alive, nw, [&](int64_t q, unsigned long long bits) {
                    while (bits) {
                        const int t = __ffsll((long long)bits) - 1;
                        bits &= bits - 1ull;
                        const long long i = q * 64 + t;
                        if (key_of(i) <= ub) {
                            const unsigned int slot = atomicAdd(&nc_s, 1u);
                            cand_s[slot] = i;
                            s.cand[slot] = i;
                        }
                    }
                });
                if (tid == 0) kp_s = (int)nband;
                __syncthreads();
            }
        }
        kp = kp_s;
        if (tid == 0) {
            c->nsurv = ns;
            c->ncand = (unsigned int)kp;
        }
    }
    __syncthreads();
    const double* __restrict__ mu = cur_mu(s, c);
    const int64_t stride = (int64_t)s.maxL + 8;
    for (int r = w; r < kp; r += NW) {
        const int64_t i = cand_s[r];
        const double mui = mu[i];
        double* x = s.xc + r * stride;
        double sx = 0.0;
        for (int kk = lane; kk < m; kk += 64) {
            const double v = s.T[i + kk] - mui;
            x[kk] = v;
            sx += v;
        }
        sx = wave_sum(sx);
        if (lane == 0) s.xc[KP_MAX * stride + r] = sx;
    }
}

// Exact FP64 nearest-neighbour correlation of the candidate rows against
// every column: direct centred dot products (no recurrence), the reference
// the reported distances and neighbour indices come from.  It is a dense
// contraction X (candidates x m) . H (m x columns) with H[k][j] = t_{j+k},
// so it runs on the FP64 matrix cores: V_MFMA_F64_16X16X4F64 multiplies a
// 16 x 4 block of candidate values by a 4 x 16 block of the series, lane l
// supplying X[l % 16][l / 16] and H[l / 16][l % 16] and receiving
// D[l / 16 + 4 r][l % 16], r < 4.  A block is POLISH_COLS consecutive
// columns of one series (PM_CT tiles of 16 per wave) for one group of PM_G
// candidates (grid.y); the columns' values and chunks of PM_KC offsets of
// the candidates' centred windows are staged in LDS, so a lane reads one
// value per matrix instruction (1024 FMAs).  One (max rho, argmax j)
// partial per candidate and workgroup.
constexpr int PM_WAVES = POLISH_COLS / 128;   // waves per block
constexpr int PM_CT = 8;                      // 16-column tiles per wave
constexpr int PM_G = 16;                      // candidates per block
constexpr int PM_KC = 256;                    // window offsets per LDS chunk
constexpr int PM_XS = PM_KC + 1;              // LDS row stride of a candidate window (odd: no bank conflicts)
constexpr int PM_GRID = 512;                  // workgroups per candidate group (each sweeps blocks in turn)
// A workgroup sweeps the column blocks g, g + G, ... of the flat block space
// (all series, prefix table pfx); the candidates' windows stay in LDS while
// consecutive blocks belong to the same series and the window fits one chunk.
__global__ __launch_bounds__(64 * PM_WAVES) void k_polish(SeriesDev* S, int B,
                                                          const int64_t* __restrict__ pfx,
                                                          int64_t nblocks)
{
    static_assert(PM_WAVES * PM_CT * 16 == POLISH_COLS, "polish block geometry");
    extern __shared__ double lds[];
    __shared__ double red_v[PM_WAVES][PM_G];
    __shared__ long long red_j[PM_WAVES][PM_G];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int ca = lane & 15, ka = lane >> 4;
    const int colbase = w * 16 * PM_CT;
    const int g0 = (int)blockIdx.y * PM_G;
    double* xg = lds;                   // [PM_G][PM_XS] candidate window chunk
    double* ts = lds + PM_G * PM_XS;    // t[j0 .. j0 + POLISH_COLS + m + 4)
    int loaded = -1;                    // series whose single-chunk windows are in xg
    // running (max rho, smallest argmax j) of the lane's candidate rows over
    // the blocks of series `cur` this workgroup has swept; the blocks of one
    // series come in ascending order, so a strict > keeps the smaller j
    int cur = -1;
    int64_t cslot = 0;
    double best[4];
    long long bj[4];
    unsigned long long evb = 0;
    // one partial per (candidate, workgroup): slot = the workgroup's first
    // block of the series, which is below the grid size
    auto flush = [&]() {
        const SeriesDev& s = S[cur];
        const int ncand = (int)s.ctrl->ncand;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int o = 8; o >= 1; o >>= 1) {  // the 16 lanes of one candidate row
                const double v = __shfl_xor(best[r], o);
                const long long jj = __shfl_xor(bj[r], o);
                if (v > best[r] || (v == best[r] && jj < bj[r])) {
                    best[r] = v;
                    bj[r] = jj;
                }
            }
            if (ca == 0) {
                red_v[w][ka + 4 * r] = best[r];
                red_j[w][ka + 4 * r] = bj[r];
            }
        }
        __syncthreads();
        if (tid < PM_G && g0 + tid < ncand) {
            double bv = red_v[0][tid];
            long long bjj = red_j[0][tid];
            for (int q = 1; q < PM_WAVES; ++q)
                if (red_v[q][tid] > bv || (red_v[q][tid] == bv && red_j[q][tid] < bjj)) {
                    bv = red_v[q][tid];
                    bjj = red_j[q][tid];
                }
            const int64_t slot = ((int64_t)(g0 + tid) * s.npart + cslot) * 2;
            s.part[slot] = bv;
            s.part[slot + 1] = (double)bjj;
        }
        const unsigned long long e = (unsigned long long)wave_sum((double)evb);
        if (lane == 0 && e)
            atomicAdd(&s.evc[EV_POL * EV_SLOTS + ((blockIdx.x + blockIdx.y + w) & (EV_SLOTS - 1))], e);
        __syncthreads();  // red_v / red_j are free again
        cur = -1;
    };
    for (int64_t fb = blockIdx.x; fb < nblocks; fb += gridDim.x) {
        const int b = series_of(pfx, B, fb);
        if (cur >= 0 && b != cur) flush();
        const SeriesDev& s = S[b];
        Ctrl* c = s.ctrl;
        if (!c->active) continue;
        const int ncand = (int)c->ncand;
        if (g0 >= ncand) continue;
        const int32_t m = c->m;
        const int64_t N = s.n - m + 1;
        const double* __restrict__ mu = cur_mu(s, c);
        const double* __restrict__ inv = s.inv64;  // 1/(sqrt(m) sigma), 0 for a flat window
        const int64_t blk = fb - pfx[b];
        if (cur < 0) {
            cur = b;
            cslot = blk;
            evb = 0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                best[r] = -f_inf<double>();
                bj[r] = 0x7fffffffffffffffll;
            }
        }
        const int64_t j0 = blk * POLISH_COLS;
        const int64_t stride = (int64_t)s.maxL + 8;
        const double* __restrict__ xc = s.xc;
        pm_acc_t acc[PM_CT];
#pragma unroll
        for (int ct = 0; ct < PM_CT; ++ct) acc[ct] = (pm_acc_t){0.0, 0.0, 0.0, 0.0};
        const bool single = m <= PM_KC;
        for (int kb = 0; kb < m; kb += PM_KC) {
            const int kn = min(PM_KC, m - kb);
            __syncthreads();  // the previous chunk and block are consumed
            if (kb == 0) lds_fill(ts, s.T + j0, POLISH_COLS + m + 4);
            if (!single || loaded != b) {
                // eight loads in flight per thread before their stores
                for (int e0 = 0; e0 < PM_G * PM_KC; e0 += 8 * 64 * PM_WAVES) {
                    double v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int e = e0 + tid + 64 * PM_WAVES * u;
                        const int g = e / PM_KC, k = e - g * PM_KC;
                        const int cid = min(g0 + g, ncand - 1);
                        v[u] = k < kn ? xc[cid * stride + kb + k] : 0.0;  // zero past m
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int e = e0 + tid + 64 * PM_WAVES * u;
                        const int g = e / PM_KC, k = e - g * PM_KC;
                        xg[g * PM_XS + k] = v[u];
                    }
                }
                loaded = single ? b : -1;
            }
            __syncthreads();
            const double* xa = xg + ca * PM_XS + ka;
            const double* tb = ts + colbase + kb + ka + ca;
            for (int k4 = 0; k4 < kn; k4 += 4) {
                const double av = xa[k4];
#pragma unroll
                for (int ct = 0; ct < PM_CT; ++ct)
                    acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, tb[k4 + 16 * ct], acc[ct], 0, 0, 0);
            }
        }
        // epilogue: lane holds D[ka + 4 r][16 ct + ca]; rho = C inv_i inv_j
        const double* __restrict__ sxs = xc + KP_MAX * stride;
        int64_t ci[4];
        double sxv[4], ivi[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int cid = min(g0 + ka + 4 * r, ncand - 1);
            ci[r] = s.cand[cid];
            sxv[r] = sxs[cid];
            ivi[r] = inv[ci[r]];
        }
#pragma unroll
        for (int ct = 0; ct < PM_CT; ++ct) {
            const int64_t j = j0 + colbase + 16 * ct + ca;
            if (j >= N) continue;
            const double ivj = inv[j], muj = mu[j];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (j <= ci[r] - m || j >= ci[r] + m) {
                    double rh;
                    if (ivi[r] == 0.0 || ivj == 0.0) {  // a flat window (R11)
                        rh = (ivi[r] == 0.0 && ivj == 0.0) ? 1.0 : 0.0;
                    } else {
                        const double Cv = acc[ct][r] - muj * sxv[r];
                        rh = fmin(1.0, fmax(-1.0, Cv * ivi[r] * ivj));
                    }
                    if (rh > best[r]) {  // a lane's columns ascend with ct and with the block
                        best[r] = rh;
                        bj[r] = j;
                    }
                    if (g0 + ka + 4 * r < ncand) ++evb;
                }
            }
        }
    }
    if (cur >= 0) flush();
}

// Close the round of every series (one block each): reduce the polish
// partials to each candidate's exact (rho, j), rank the candidates, write the
// length's top-k rows when the round found at least k range discords, and
// lower MERLIN's r otherwise; count the series with work left in rem[0].
constexpr int END_BLOCK = 1024;
__global__ __launch_bounds__(END_BLOCK) void k_round_end(SeriesDev* S, int32_t* rem, int hot_rows,
                                                          int npol)
{
    __shared__ double nn_s[KP_MAX];
    __shared__ long long id_s[KP_MAX];
    __shared__ long long jj_s[KP_MAX];
    const SeriesDev& s = S[blockIdx.x];
    Ctrl* c = s.ctrl;
    if (!c->active) return;
    __shared__ int valid_s[KP_MAX];
    __shared__ unsigned int nvalid_s;
    const int k = s.k;
    const int32_t m = c->m;
    const int li = c->li;
    const int kp = (int)c->ncand;
    const bool direct = direct_round(c);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (kp >= k) {
        // tpc threads per candidate (all candidates at once, tpc as large as
        // the block allows, at most a wave): strided partials loaded eight at
        // a time before they are compared (they come from other XCDs' caches,
        // so each batch costs a full memory latency), then a reduction over
        // the tpc threads.  k_polish's npol workgroups left one partial each
        // in the slots below min(blocks of this length, npol).
        const int64_t npart = s.npart;
        const int64_t nblk = std::min<int64_t>((s.n - m + 1 + POLISH_COLS - 1) / POLISH_COLS, npol);
        int tpc = 64;
        while (tpc > 1 && tpc * kp > END_BLOCK) tpc >>= 1;
        const int sub = tid & (tpc - 1);
        for (int cid = tid / tpc; cid < kp; cid += END_BLOCK / tpc) {
            double best = -f_inf<double>(), bj = 1e300;
            const double* pc = s.part + (int64_t)cid * npart * 2;
            for (int64_t p0 = sub; p0 < nblk; p0 += 8 * (int64_t)tpc) {
                double v[8], jj[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int64_t p = p0 + (int64_t)u * tpc;
                    v[u] = p < nblk ? pc[p * 2] : -f_inf<double>();
                    jj[u] = p < nblk ? pc[p * 2 + 1] : 1e300;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (v[u] > best || (v[u] == best && jj[u] < bj)) {
                        best = v[u];
                        bj = jj[u];
                    }
            }
            for (int o = tpc >> 1; o >= 1; o >>= 1) {
                const double v = __shfl_xor(best, o);
                const double jj = __shfl_xor(bj, o);
                if (v > best || (v == best && jj < bj)) {
                    best = v;
                    bj = jj;
                }
            }
            if (sub == 0) {
                const double d2 = 2.0 * (double)m * (1.0 - best);
                const long long i = s.cand[cid];
                nn_s[cid] = sqrt(fmin(4.0 * (double)m, fmax(0.0, d2)));
                id_s[cid] = i;
                jj_s[cid] = (long long)bj;
                // a direct round decides here which live subsequences are range
                // discords (distance >= r, i.e. rho <= thr64), as refinement would
                int ok_i = 1;
                if (direct) {
                    ok_i = !(c->prune && best > c->thr64);
                    if (ok_i) s.rho[i] = ord_of(best);
                    else atomicAnd(&s.alive[i >> 6], ~(1ull << (i & 63)));
                }
                valid_s[cid] = ok_i;
            }
        }
    }
    if (s.heat) __threadfence();  // the direct round's bitmap and rho updates, read below
    __syncthreads();
    if (tid == 0) {
        unsigned int nv = 0;
        for (int q = 0; q < kp; ++q) nv += (unsigned int)valid_s[q];
        nvalid_s = nv;
    }
    __syncthreads();
    const unsigned int ns = direct ? (kp >= k ? nvalid_s : (unsigned int)kp) : c->nsurv;
    // the candidates could not be narrowed to KP_MAX: same r again, with both
    // sides of every tile refined exactly
    const bool redo = c->band_over != 0;
    const bool ok = ns >= (unsigned int)k && kp >= k && !redo;
    if (ok && tid < kp && valid_s[tid]) {
        int rank = 0;
        for (int q = 0; q < kp; ++q)
            if (valid_s[q] &&
                (nn_s[q] > nn_s[tid] || (nn_s[q] == nn_s[tid] && id_s[q] < id_s[tid])))
                ++rank;
        if (rank < k) {
            const int64_t row = (int64_t)li * k + rank;
            if (s.idx) {
                s.idx[row] = id_s[tid];
                s.len[row] = m;
                s.nn[row] = nn_s[tid];
                s.nnidx[row] = jj_s[tid];
            }
            if (rank == k - 1) s.hist[li] = nn_s[tid];
        }
    }
    __syncthreads();
    if (ok && s.heat) {
        // the discord heatmap row of this length (Eq. (11)): every range
        // discord (the alive bits) with its exact nearest-neighbour
        // correlation, as ED^2 / (2m) = 1 - rho; 0 elsewhere
        const int64_t N = s.n - m + 1;
        double* hrow = s.heat + (int64_t)li * s.heat_ld;
        for (int64_t i = tid; i < s.heat_ld; i += END_BLOCK) {
            double v = 0.0;
            if (i < N && ((load_word(&s.alive[i >> 6]) >> (i & 63)) & 1ull)) {
                const double rh =
                    dbl_of(__hip_atomic_load(&s.rho[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                v = fmin(2.0, fmax(0.0, 1.0 - rh));
            }
            hrow[i] = v;
        }
        if (tid == 0) s.rlen[li] = c->r;
    }
    if (tid == 0) {
        c->rounds += 1;
        c->nsurv = ns;
        c->exact_ref = redo ? 1 : 0;
        if (ok) {
            c->done = 1;
            c->survivors += ns;
            if (s.count) s.count[li] = (int32_t)ns;
        } else if (!redo) {
            c->done = 0;
            if (c->mode == 0) c->r *= 0.5;
            else if (c->mode == 1) c->r *= 0.99;
            else if (c->mode == 2) c->r = (c->step > 0.0) ? c->r - c->step : 0.99 * c->r;
        } else {
            c->done = 0;
        }
        if (!(c->done && c->m >= s.maxL)) atomicAdd(&rem[0], 1);
    }
    // Hot tiles of hot_rows rows, in ascending order (the first HOT_MAX of
    // them): those that still hold survivors or whose first-pass items swept
    // at least N / HOT_FRAC columns this round.  The next round's first
    // selection pass dispatches all their chunks before any other tile's, so
    // that the longest work items of the pass start first.  The per-tile
    // work counters restart.
    __shared__ unsigned int wcnt_s[END_BLOCK / 64];
    __shared__ unsigned int base_s;
    // (the bitmap atomics of this block completed before the barrier; the
    // scan reads the bitmap with agent-scope loads)
    __syncthreads();
    if (tid == 0) base_s = 0;
    const int64_t ntl = (s.n - m + 1 + hot_rows - 1) / hot_rows;
    const int wpt = hot_rows / 64;
    const uint32_t hot_work = (uint32_t)((s.n - m + 1 + 64 * HOT_FRAC - 1) / (64 * HOT_FRAC));
    for (int64_t t0 = 0; t0 < ntl; t0 += END_BLOCK) {
        __syncthreads();
        const unsigned int base = base_s;
        const int64_t t = t0 + tid;
        bool hot = false;
        if (t < ntl) {
            unsigned long long any = 0ull;
            for (int w2 = 0; w2 < wpt; ++w2) any |= load_word(&s.alive[t * wpt + w2]);
            hot = any != 0ull || s.twork[t] >= hot_work;
            s.twork[t] = 0u;
        }
        const unsigned long long bal = __ballot(hot);
        if (lane == 0) wcnt_s[w] = (unsigned int)__popcll(bal);
        __syncthreads();
        unsigned int before = 0, total = 0;
        for (int q = 0; q < END_BLOCK / 64; ++q) {
            before += (q < w) ? wcnt_s[q] : 0u;
            total += wcnt_s[q];
        }
        const unsigned int pos =
            base + before + (unsigned int)__popcll(bal & ((1ull << lane) - 1ull));
        if (hot && pos < (unsigned int)HOT_MAX) s.hot[pos] = (int32_t)t;
        __syncthreads();
        if (tid == 0) base_s = base + total;
    }
    __syncthreads();
    if (tid == 0) {
        c->nhot = base_s < (unsigned int)HOT_MAX ? base_s : (unsigned int)HOT_MAX;
        c->hot_r = hot_rows;
    }
}

// ---------------------------------------------------------------------------
// diagnostic: drift of the FP32 selection recurrence from FP64
// ---------------------------------------------------------------------------
// Items of 512-row tiles (the longest recurrence chains any sweep runs) and
// `chunk` columns to their right, spread over the series (tiles evenly,
// columns at varying distance): the centred diagonal recurrence is run in
// FP32 exactly as the selection sweep runs it (FP32 helpers, exact
// boundary values rounded to FP32) and in FP64 (the refinement sweep's
// arithmetic), side by side from the same exact first column.  The largest
// |rho32 - rho64| over the items' non-self pairs (rho = C inv_i inv_j) goes
// to out[0] (ordered bits, atomicMax).
template <int U>
__device__ __forceinline__ void drift_step(float (&C32)[8], double (&C64)[8], const float (&a32)[8],
                                           const float (&b32)[8], const double (&a64)[8],
                                           const double (&b64)[8], const H4<float>& h32,
                                           const H4<double>& h64, const float (&iv32)[8],
                                           const double (&iv64)[8], const int64_t (&ri)[8],
                                           int64_t j, int32_t m, int64_t N, double& mx)
{
    advance<float, 8, U>(C32, a32, b32, h32.df, h32.dg, h32.B);
    advance<double, 8, U>(C64, a64, b64, h64.df, h64.dg, h64.B);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        if (j - m >= ri[q] && ri[q] < N && j < N) {
            const float r32 = C32[slot_reg<8, U>(q)] * h32.inv * iv32[q];
            const double r64 = C64[slot_reg<8, U>(q)] * h64.inv * iv64[q];
            mx = fmax(mx, fabs((double)r32 - r64));
        }
    }
}

__global__ __launch_bounds__(64) void k_drift(SeriesDev* S, int64_t nitems, int chunk,
                                              unsigned long long* out)
{
    constexpr int Q = 8, R = 64 * Q;
    extern __shared__ double lds[];
    const SeriesDev& s = S[0];
    Ctrl* c = s.ctrl;
    const SweepArgs<float> A32 = args_of<float>(s, c);
    const SweepArgs<double> A64 = args_of<double>(s, c);
    const int32_t m = A64.m;
    const int64_t N = A64.N;
    const int lane = threadIdx.x;
    double* xp = lds;
    double* ws = lds + hk_vp_doubles(m);
    constexpr int NC = batch_cols<double>();  // both precisions in batches of the FP64 width
    H4<double>* hs64 = (H4<double>*)(lds + sweep_hs_offset(m, R, NC));
    H4<float>* hs32 = (H4<float>*)(lds + sweep_hs_offset(m, R, NC) + sweep_hs_doubles(R, 8, NC));
    const int64_t ntiles = (N + R - 1) / R;
    // nitems <= 0: every (tile, chunk) of the right side, chunk-major
    const int64_t nchall = (N + chunk - 1) / chunk;
    const bool all = nitems <= 0;
    const int64_t total = all ? ntiles * nchall : nitems;
    double mx = 0.0;
    for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
        const int64_t i0 = uniform_i64(all ? (it % ntiles) * R : ((it * ntiles) / nitems) * R);
        const int64_t span = N - (i0 + m);
        if (span <= 0) continue;
        const int64_t nch = std::max<int64_t>(1, span / chunk);
        const int64_t cc = all ? it / ntiles : (it * 37) % nch;
        if (all && cc * chunk >= span) continue;
        const int64_t jbeg = uniform_i64(i0 + m + cc * chunk);
        const int64_t jend = std::min<int64_t>(N, jbeg + 1 + chunk);
        double Sx, Sy, acc[Q];
        item_start<Q>(A64.T, A64.mu, m, i0, jbeg, xp, ws, (double*)hs64, Sx, Sy, acc);
        float C32[Q], a32[Q], b32[Q], iv32[Q];
        double C64[Q], a64[Q], b64[Q], iv64[Q];
        int64_t ri[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int64_t i = i0 + Q * lane + q;
            const bool top = (lane == 0) && (q == 0);
            const int64_t ip = top ? i : i - 1;
            C64[q] = acc[q];
            C32[q] = (float)acc[q];
            a32[q] = top ? 0.0f : A32.df[ip];
            b32[q] = top ? 0.0f : A32.dg[ip];
            a64[q] = top ? 0.0 : A64.df[ip];
            b64[q] = top ? 0.0 : A64.dg[ip];
            iv32[q] = A32.inv[i];
            iv64[q] = A64.inv[i];
            ri[q] = i;
        }
        for (int64_t j = jbeg + 1; j + Q <= jend; ) {
            stage_batch<double, NC>(A64.T, A64.mu, A64.df, A64.dg, A64.inv, m, j, xp, Sx, ws, hs64);
            stage_batch<float, NC>(A32.T, A32.mu, A32.df, A32.dg, A32.inv, m, j, xp, Sx, ws, hs32);
            const int64_t jb_end = std::min<int64_t>(jend, j + NC);
            for (int s0 = 0; j + Q <= jb_end; s0 += Q, j += Q) {
#define DRIFT_STEP(U)                                                                          \
    drift_step<U>(C32, C64, a32, b32, a64, b64, hs32[s0 + (U)], hs64[s0 + (U)], iv32, iv64, ri, \
                  j + (U), m, N, mx);
                DRIFT_STEP(0) DRIFT_STEP(1) DRIFT_STEP(2) DRIFT_STEP(3)
                DRIFT_STEP(4) DRIFT_STEP(5) DRIFT_STEP(6) DRIFT_STEP(7)
#undef DRIFT_STEP
            }
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    if (lane == 0) atomicMax(out, ord_of(mx));
}

// The guard band the selection sweep uses at the current length (after
// k_guard), as a double in out[1].
__global__ void k_drift_band(SeriesDev* S, float guard, double* out)
{
    out[1] = sel_guard(S[0].ctrl, guard);
}

// ---------------------------------------------------------------------------
// streaming series: exact nearest-neighbour profiles per length, updated by
// the pairs each append adds (the discord definition, Sec. 2.1, applied to a
// series that grows; the top-k of a length are then those of its profile)
// ---------------------------------------------------------------------------
// After an append from n_old to n points, the subsequences of length m that
// start at i >= N_old = n_old - m + 1 are new; each reaches back over at most
// m - 1 points that were already there (the halo).  The pairs the append
// adds are (new row, any column) and (old row, new column):
//   part A  the row tiles from the one holding N_old sweep every column,
//           both sides (left-side and right-side chunks alternate, nearest
//           first);
//   part B  the row tiles holding old rows sweep the new columns (right
//           side only: every new column is to the right of every old row).
// Rows of part A's first tile below N_old are swept again in full, which
// only re-derives their maxima.  The refinement sweep does the work with
// pruning off; every row's running maximum of rho stays in its length's
// profile (ordered bits, prof[(m - minL) Npad + i]).
template <int Q>
__global__ __launch_bounds__(64, (Q <= 4 ? 3 : 1)) void k_stream_band(SeriesDev* S,
                                                                      unsigned long long* prof,
                                                                      int64_t n_old, int chunk)
{
    extern __shared__ double lds[];
    constexpr int R = 64 * Q;
    const SeriesDev& s = S[0];
    Ctrl* c = s.ctrl;
    SweepArgs<double> A = args_of<double>(s, c);
    A.rho = prof + (int64_t)c->li * s.Npad;
    const int32_t m = A.m;
    const int64_t N = A.N;
    const int64_t Nold = std::max<int64_t>(0, n_old - m + 1);
    if (Nold >= N) return;
    const int64_t a0 = (Nold / R) * R;
    const int64_t tA = (N - a0 + R - 1) / R;
    const int64_t cA = (N + chunk - 1) / chunk;
    const int64_t itemsA = tA * 2 * cA;
    const int64_t tB = (Nold + R - 1) / R;
    const int64_t cB = (N - Nold + chunk - 1) / chunk;
    const int64_t total = itemsA + tB * cB;
    unsigned long long ev = 0;
    for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
        int64_t i0, jbeg, jend;
        bool left;
        if (it < itemsA) {
            const int64_t t = it % tA, r = it / tA;
            const int64_t cc = r >> 1;
            left = (r & 1) != 0;
            i0 = a0 + t * R;
            if (left) {
                jend = std::min<int64_t>(N, i0 + R - m) - cc * chunk;
                jbeg = std::max<int64_t>(0, jend - chunk);
            } else {
                jbeg = i0 + m + cc * chunk;
                jend = std::min<int64_t>(N, jbeg + chunk);
            }
        } else {
            const int64_t x = it - itemsA;
            const int64_t t = x % tB, cc = x / tB;
            i0 = t * R;
            left = false;
            jbeg = std::max<int64_t>(Nold, i0 + m) + cc * chunk;
            jend = std::min<int64_t>(N, jbeg + chunk);
        }
        if (jbeg >= jend) continue;
        ref_item<Q, HK_TILE>(A, i0, jbeg, jend, left, 2.0, 0, lds, ev);
    }
    if (threadIdx.x == 0 && ev)
        atomicAdd(&s.evc[EV_REF * EV_SLOTS + (blockIdx.x & (EV_SLOTS - 1))], ev);
}

// A query at the current length: the profile becomes the round's row
// maxima and every subsequence a live candidate (no pruning), so that
// k_select_top, k_polish and k_round_end rank the profile, recompute the
// best candidates exactly and write the length's top-k rows, as in a search
// round without pruning.
__global__ void k_stream_query(SeriesDev* S, const unsigned long long* __restrict__ prof)
{
    const SeriesDev& s = S[0];
    Ctrl* c = s.ctrl;
    const int64_t N = s.n - c->m + 1;
    const unsigned long long* p = prof + (int64_t)c->li * s.Npad;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < s.Npad;
         i += (int64_t)gridDim.x * blockDim.x)
        s.rho[i] = i < N ? p[i] : 0x000fffffffffffffull;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c->mode = 3;
        c->r = 0.0;
        c->prune = 0;
        c->thr64 = c->thr_sel = 2.0;
        c->thr32 = 2.0f;
        c->exact_ref = 0;
        c->band_over = 0;
        c->live_ref = 0xffffffffu;  // not a direct round
        c->nsurv = c->ncand = 0;
        c->done = 0;
    }
}

// The exact profile of the current length as distances (Eq. (6)):
// nn[i] = sqrt(2m (1 - rho_i)) for i < N.
__global__ void k_stream_profile(SeriesDev* S, const unsigned long long* __restrict__ prof,
                                 double* nn)
{
    const SeriesDev& s = S[0];
    const Ctrl* c = s.ctrl;
    const int32_t m = c->m;
    const int64_t N = s.n - m + 1;
    const unsigned long long* p = prof + (int64_t)c->li * s.Npad;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double rh = dbl_of(p[i]);
        nn[i] = sqrt(fmin(4.0 * (double)m, fmax(0.0, 2.0 * (double)m * (1.0 - rh))));
    }
}

__global__ void k_fill_u64(unsigned long long* p, int64_t count, unsigned long long v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename F, int Q>
static void launch_near(const Batch& bt, const SweepCfg& cfg, const int64_t* total, hipStream_t st)
{
    const size_t lds = sizeof(double) * sweep_lds_doubles(bt.maxL_all, 64 * Q, (int)sizeof(F), false);
    if (total[PFX_NEAR] == 0) return;
    cfg.timer->begin(0, st);
    hipLaunchKernelGGL((k_select_near<F, Q>), dim3((unsigned int)total[PFX_NEAR]), dim3(64), lds,
                       st, bt.s, bt.B, bt.pfx[PFX_NEAR], cfg.near_cols, cfg.chunk_cols);
    cfg.timer->end(0, st);
}

template <typename F, int Q>
static void launch_far(const Batch& bt, const SweepCfg& cfg, const int64_t* total, hipStream_t st)
{
    const size_t lds = sizeof(double) * sweep_lds_doubles(bt.maxL_all, 64 * Q, (int)sizeof(F), false);
    hipLaunchKernelGGL(k_tiles, dim3((unsigned int)total[PFX_TSEL]), dim3(TILES_BLOCK), 0, st, bt.s, bt.B,
                       bt.pfx[PFX_TSEL], 64 * Q, 0, cfg.near_cols, cfg.chunk_cols, 64 * cfg.q_near);
    cfg.timer->begin(1, st);
    hipLaunchKernelGGL((k_select_far<F, Q>), dim3(cfg.far_grid), dim3(64), lds, st, bt.s, bt.B,
                       cfg.near_cols, cfg.chunk_cols, 64 * cfg.q_near);
    cfg.timer->end(1, st);
}

template <int Q>
static void launch_refine(const Batch& bt, const SweepCfg& cfg, const int64_t* total, hipStream_t st)
{
    hipLaunchKernelGGL(k_tiles, dim3((unsigned int)total[PFX_TREF]), dim3(TILES_BLOCK), 0, st, bt.s, bt.B,
                       bt.pfx[PFX_TREF], 64 * Q, 1, 0, cfg.chunk_cols, 64 * cfg.q_near);
    const size_t lds = sizeof(double) * sweep_lds_doubles(bt.maxL_all, 64 * Q, (int)sizeof(double), true);
    cfg.timer->begin(2, st);
    hipLaunchKernelGGL((k_refine<Q>), dim3(cfg.far_grid), dim3(64), lds, st, bt.s, bt.B,
                       cfg.chunk_cols);
    cfg.timer->end(2, st);
}

template <typename F>
static void launch_select(const Batch& bt, const SweepCfg& cfg, const int64_t* total,
                          hipStream_t st)
{
    if (cfg.band && total[PFX_BAND] > 0) {
        cfg.timer->begin(5, st);
        hipLaunchKernelGGL((k_select_band<F>), dim3((unsigned int)total[PFX_BAND]), dim3(64),
                           band_lds_bytes(bt.maxL_all, (int)sizeof(F)), st, bt.s, bt.B, bt.pfx[PFX_BAND]);
        cfg.timer->end(5, st);
    }
    switch (cfg.q_near) {
    case 2: launch_near<F, 2>(bt, cfg, total, st); break;
    case 4: launch_near<F, 4>(bt, cfg, total, st); break;
    default: launch_near<F, 8>(bt, cfg, total, st); break;
    }
    if ((int64_t)cfg.near_cols >= bt.Nmax_all) {
        // the first pass already covers every column of every series
        return;
    }
    switch (cfg.q_far) {
    case 2: launch_far<F, 2>(bt, cfg, total, st); break;
    case 4: launch_far<F, 4>(bt, cfg, total, st); break;
    default: launch_far<F, 8>(bt, cfg, total, st); break;
    }
}

// One round: every series with work does one range search at its current
// length (a fixed launch sequence; all parameters come from the device).
hipError_t launch_round(const Batch& bt, const SweepCfg& cfg, const int64_t* total, hipStream_t st)
{
    const unsigned int elem = (unsigned int)total[PFX_ELEM];
    hipLaunchKernelGGL(k_round_prep, dim3(1), dim3(256), 0, st, bt.s, bt.B, cfg.guard,
                       cfg.max_attempts, bt.remaining);
    cfg.timer->begin(4, st);
    hipLaunchKernelGGL(k_length, dim3(elem), dim3(256), 0, st, bt.s, bt.B, bt.pfx[PFX_ELEM]);
    cfg.timer->end(4, st);
    hipLaunchKernelGGL(k_guard, dim3(bt.B), dim3(GUARD_BLOCK), 0, st, bt.s, cfg.guard);
    if (cfg.dist_bits == 64) launch_select<double>(bt, cfg, total, st);
    else launch_select<float>(bt, cfg, total, st);
    switch (cfg.q_ref) {
    case 4: launch_refine<4>(bt, cfg, total, st); break;
    case 8: launch_refine<8>(bt, cfg, total, st); break;
    default: launch_refine<2>(bt, cfg, total, st); break;
    }
    hipLaunchKernelGGL(k_select_top, dim3(bt.B), dim3(TOPK_BLOCK), 0, st, bt.s);
    const size_t lds = sizeof(double) * (size_t)(PM_G * PM_XS + POLISH_COLS + bt.maxL_all + 4);
    cfg.timer->begin(3, st);
    const int npol = (int)std::min<int64_t>(total[PFX_POLISH], PM_GRID);
    hipLaunchKernelGGL(k_polish, dim3((unsigned int)npol, (KP_MAX + PM_G - 1) / PM_G),
                       dim3(64 * PM_WAVES), lds, st, bt.s, bt.B, bt.pfx[PFX_POLISH],
                       total[PFX_POLISH]);
    cfg.timer->end(3, st);
    hipLaunchKernelGGL(k_round_end, dim3(bt.B), dim3(END_BLOCK), 0, st, bt.s, bt.remaining,
                       64 * cfg.q_near, npol);
    return hipGetLastError();
}

__global__ void k_set_len(SeriesDev* S, int32_t m, int32_t new_len);

hipError_t launch_drift(const Batch& bt, const int64_t* total, int32_t minL, int32_t m,
                        int64_t nitems, int chunk, float guard, double* out, hipStream_t st)
{
    const hipError_t e = launch_stats_to(bt, minL, m, total, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_guard, dim3(1), dim3(GUARD_BLOCK), 0, st, bt.s, guard);
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, (unsigned long long*)out, (int64_t)1,
                       0ull);
    constexpr int NC = batch_cols<double>();
    const size_t lds = sizeof(double) * (sweep_hs_offset(bt.maxL_all, 512, NC) + sweep_hs_doubles(512, 8, NC) +
                                         sweep_hs_doubles(0, 4, NC));
    hipLaunchKernelGGL(k_drift, dim3(1024), dim3(64), lds, st, bt.s, nitems, chunk,
                       (unsigned long long*)out);
    hipLaunchKernelGGL(k_drift_band, dim3(1), dim3(1), 0, st, bt.s, guard, out);
    return hipGetLastError();
}

// Streaming: one append's profile updates at every length (statistics,
// helpers, band sweeps), a query's top-k rows at every length, the profile
// of one length, and the reset of every profile.
template <int Q>
static void launch_band(const Batch& bt, const SweepCfg& cfg, unsigned long long* prof,
                        int64_t n_old, hipStream_t st)
{
    const size_t lds = sizeof(double) * sweep_lds_doubles(bt.maxL_all, 64 * Q, (int)sizeof(double), true, HK_TILE);
    hipLaunchKernelGGL((k_stream_band<Q>), dim3(cfg.far_grid), dim3(64), lds, st, bt.s, prof, n_old,
                       cfg.chunk_cols);
}

hipError_t launch_stream_update(const Batch& bt, const SweepCfg& cfg, const int64_t* total,
                                int32_t minL, int32_t maxL, unsigned long long* prof,
                                int64_t n_old, hipStream_t st)
{
    for (int32_t m = minL; m <= maxL; ++m) {
        hipLaunchKernelGGL(k_set_len, dim3(1), dim3(1), 0, st, bt.s, m, m == minL ? 2 : 1);
        hipLaunchKernelGGL(k_length, dim3((unsigned int)total[PFX_ELEM]), dim3(256), 0, st, bt.s, 1,
                           bt.pfx[PFX_ELEM]);
        switch (cfg.q_ref) {
        case 4: launch_band<4>(bt, cfg, prof, n_old, st); break;
        case 8: launch_band<8>(bt, cfg, prof, n_old, st); break;
        default: launch_band<2>(bt, cfg, prof, n_old, st); break;
        }
    }
    return hipGetLastError();
}

hipError_t launch_stream_query(const Batch& bt, const int64_t* total, int32_t minL, int32_t maxL,
                               const unsigned long long* prof, int hot_rows, hipStream_t st)
{
    const size_t lds = sizeof(double) * (size_t)(PM_G * PM_XS + POLISH_COLS + bt.maxL_all + 4);
    const int npol = (int)std::min<int64_t>(total[PFX_POLISH], PM_GRID);
    for (int32_t m = minL; m <= maxL; ++m) {
        hipLaunchKernelGGL(k_set_len, dim3(1), dim3(1), 0, st, bt.s, m, m == minL ? 2 : 1);
        hipLaunchKernelGGL(k_length, dim3((unsigned int)total[PFX_ELEM]), dim3(256), 0, st, bt.s, 1,
                           bt.pfx[PFX_ELEM]);
        hipLaunchKernelGGL(k_stream_query, dim3(256), dim3(256), 0, st, bt.s, prof);
        hipLaunchKernelGGL(k_select_top, dim3(1), dim3(TOPK_BLOCK), 0, st, bt.s);
        hipLaunchKernelGGL(k_polish, dim3((unsigned int)npol, (KP_MAX + PM_G - 1) / PM_G),
                           dim3(64 * PM_WAVES), lds, st, bt.s, 1, bt.pfx[PFX_POLISH],
                           total[PFX_POLISH]);
        hipLaunchKernelGGL(k_round_end, dim3(1), dim3(END_BLOCK), 0, st, bt.s, bt.remaining, hot_rows,
                           npol);
    }
    return hipGetLastError();
}

hipError_t launch_stream_profile(const Batch& bt, const int64_t* total, int32_t minL, int32_t m,
                                 const unsigned long long* prof, double* nn, hipStream_t st)
{
    const hipError_t e = launch_stats_to(bt, minL, m, total, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_stream_profile, dim3(256), dim3(256), 0, st, bt.s, prof, nn);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t count, unsigned long long v, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_u64, dim3(1024), dim3(256), 0, st, p, count, v);
    return hipGetLastError();
}

__global__ void k_set_fixed_r(SeriesDev* S, double r)
{
    Ctrl* c = S[0].ctrl;
    c->mode = 3;
    c->r = r;
}

hipError_t launch_set_fixed_r(const Batch& bt, double r, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_fixed_r, dim3(1), dim3(1), 0, st, bt.s, r);
    return hipGetLastError();
}

__global__ void k_set_len(SeriesDev* S, int32_t m, int32_t new_len)
{
    const SeriesDev& s = S[0];
    Ctrl* c = s.ctrl;
    c->m = m;
    c->li = m - s.minL;
    c->new_len = new_len;
    c->active = 1;
    if (new_len) {
        c->flat_min = 0x7fffffffffffffffll;
        c->flat_max = -1;
    }
}

hipError_t launch_set_len(const Batch& bt, int32_t m, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_len, dim3(1), dim3(1), 0, st, bt.s, m, 0);
    return hipGetLastError();
}

// Statistics of S[0] at lengths minL..m only (no search).
hipError_t launch_stats_to(const Batch& bt, int32_t minL, int32_t m, const int64_t* total,
                           hipStream_t st)
{
    for (int32_t mm = minL; mm <= m; ++mm) {
        hipLaunchKernelGGL(k_set_len, dim3(1), dim3(1), 0, st, bt.s, mm, mm == minL ? 2 : 1);
        hipLaunchKernelGGL(k_length, dim3((unsigned int)total[PFX_ELEM]), dim3(256), 0, st, bt.s, 1,
                           bt.pfx[PFX_ELEM]);
    }
    return hipGetLastError();
}

// Sum of the per-series counters of a call (one block):
// out = {evals_sel, evals_ref, evals_pol, rounds, survivors, evals_near, evals_far,
//        rows_near, rows_far, evals_band}.
__global__ void k_sum_stats(SeriesDev* S, int B, unsigned long long* out)
{
    __shared__ unsigned long long acc[10];
    if (threadIdx.x < 10) acc[threadIdx.x] = 0ull;
    __syncthreads();
    for (int b = 0; b < B; ++b) {
        const SeriesDev& s = S[b];
        for (int e = threadIdx.x; e < EV_CLASSES * EV_SLOTS; e += blockDim.x) {
            const unsigned long long v = s.evc[e];
            const int cls = e / EV_SLOTS;
            if (v) {
                if (cls == EV_NEAR || cls == EV_FAR || cls == EV_BAND) atomicAdd(&acc[0], v);
                atomicAdd(&acc[cls == EV_NEAR  ? 5
                               : cls == EV_FAR ? 6
                               : cls == EV_REF ? 1
                               : cls == EV_POL ? 2
                                               : 9],
                          v);
            }
        }
        if (threadIdx.x == 0) {
            const Ctrl* c = s.ctrl;
            acc[3] += c->rounds;
            acc[4] += c->survivors;
            acc[7] += c->rows_near;
            acc[8] += c->rows_far;
        }
        __syncthreads();
    }
    if (threadIdx.x < 10) out[threadIdx.x] = acc[threadIdx.x];
}

hipError_t launch_sum_stats(const Batch& bt, unsigned long long* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum_stats, dim3(1), dim3(256), 0, st, bt.s, bt.B, out);
    return hipGetLastError();
}

__global__ void k_range_out(SeriesDev* S, int64_t N, unsigned long long* alive_out, double* nn_out)
{
    const SeriesDev& s = S[0];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int32_t m = s.ctrl->m;
    const bool on = (s.alive[i >> 6] >> (i & 63)) & 1ull;
    if ((i & 63) == 0) alive_out[i >> 6] = s.alive[i >> 6];
    double d = 0.0;
    if (on) {
        const double r = dbl_of(s.rho[i]);
        d = sqrt(fmin(4.0 * (double)m, fmax(0.0, 2.0 * (double)m * (1.0 - r))));
    }
    nn_out[i] = d;
}

hipError_t launch_range_out(const Batch& bt, int64_t N, unsigned long long* alive_out,
                            double* nn_out, hipStream_t st)
{
    hipLaunchKernelGGL(k_range_out, dim3((unsigned int)((N + 255) / 256)), dim3(256), 0, st, bt.s,
                       N, alive_out, nn_out);
    return hipGetLastError();
}

__global__ void k_stats_out(SeriesDev* S, int64_t N, double* mo, double* so)
{
    const SeriesDev& s = S[0];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    mo[i] = cur_mu(s, s.ctrl)[i];
    so[i] = sqrt(cur_var(s, s.ctrl)[i]);
}

hipError_t launch_stats_out(const Batch& bt, int64_t N, double* mu, double* sigma, hipStream_t st)
{
    hipLaunchKernelGGL(k_stats_out, dim3((unsigned int)((N + 255) / 256)), dim3(256), 0, st, bt.s,
                       N, mu, sigma);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per-series workspace layout and work geometry
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// discord interest (Eq. (12)): per heatmap column the largest value over the
// lengths (ties: the shorter length), then the k columns with the largest
// values (ties: the smaller index)
// ---------------------------------------------------------------------------
__global__ void k_interest_cols(const double* __restrict__ heat, int32_t L, int64_t ld,
                                int64_t ncols, int32_t minL, double* score, int32_t* blen)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncols) return;
    // eight rows' loads are issued before they are compared
    double best = -1.0;
    int32_t bm = 0;
    for (int32_t l0 = 0; l0 < L; l0 += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = l0 + u < L ? heat[(int64_t)(l0 + u) * ld + i] : -1.0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (v[u] > best) {
                best = v[u];
                bm = l0 + u;
            }
    }
    score[i] = best;
    blen[i] = minL + bm;
}

constexpr int INTEREST_BLOCK = 1024;
__global__ __launch_bounds__(INTEREST_BLOCK) void k_interest_top(const double* __restrict__ score,
                                                                const int32_t* __restrict__ blen,
                                                                int64_t ncols, int32_t k,
                                                                int64_t* top_idx, int32_t* top_len,
                                                                double* top_score)
{
    __shared__ double bv_s[INTEREST_BLOCK / 64];
    __shared__ long long bi_s[INTEREST_BLOCK / 64];
    __shared__ double lastv_s;
    __shared__ long long lasti_s;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // order: larger score first, then smaller index; round r takes the best
    // column strictly after round r - 1's in that order
    for (int r = 0; r < k; ++r) {
        const double lv = r ? lastv_s : 0.0;
        const long long li = r ? lasti_s : -1;
        double bv = -1.0;
        long long bi = -1;
        for (int64_t i0 = tid; i0 < ncols; i0 += 16 * INTEREST_BLOCK) {
            double vs[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int64_t i = i0 + (int64_t)u * INTEREST_BLOCK;
                vs[u] = i < ncols ? score[i] : -1.0;
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int64_t i = i0 + (int64_t)u * INTEREST_BLOCK;
                const double v = vs[u];
                const bool after = r == 0 || v < lv || (v == lv && i > li);
                if (i < ncols && after && (v > bv || (v == bv && (bi < 0 || i < bi)))) {
                    bv = v;
                    bi = i;
                }
            }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const double v = __shfl_xor(bv, o);
            const long long j = __shfl_xor(bi, o);
            if (j >= 0 && (bi < 0 || v > bv || (v == bv && j < bi))) {
                bv = v;
                bi = j;
            }
        }
        if (lane == 0) {
            bv_s[w] = bv;
            bi_s[w] = bi;
        }
        __syncthreads();
        if (tid == 0) {
            double v = bv_s[0];
            long long j = bi_s[0];
            for (int q = 1; q < INTEREST_BLOCK / 64; ++q)
                if (bi_s[q] >= 0 && (j < 0 || bv_s[q] > v || (bv_s[q] == v && bi_s[q] < j))) {
                    v = bv_s[q];
                    j = bi_s[q];
                }
            top_idx[r] = j;
            top_len[r] = j >= 0 ? blen[j] : 0;
            top_score[r] = j >= 0 ? v : 0.0;
            lastv_s = v;
            lasti_s = j;
        }
        __syncthreads();
    }
}

hipError_t launch_interest(const double* heat, int32_t L, int64_t ld, int64_t ncols, int32_t minL,
                           int32_t k, double* col_score, int32_t* col_len, int64_t* top_idx,
                           int32_t* top_len, double* top_score, hipStream_t st)
{
    hipLaunchKernelGGL(k_interest_cols, dim3((unsigned int)((ncols + 255) / 256)), dim3(256), 0, st,
                       heat, L, ld, ncols, minL, col_score, col_len);
    hipLaunchKernelGGL(k_interest_top, dim3(1), dim3(INTEREST_BLOCK), 0, st, col_score, col_len,
                       ncols, k, top_idx, top_len, top_score);
    return hipGetLastError();
}

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

bool make_layout(int64_t n, int32_t minL, int32_t maxL, int32_t k, Layout* out)
{
    Layout l = {};
    l.n = n;
    l.minL = minL;
    l.maxL = maxL;
    l.k = k;
    l.L = maxL - minL + 1;
    l.kp = k + KP_EXTRA;
    l.Nmax = n - minL + 1;
    l.Npad = ((l.Nmax + 1 + R_MAX - 1) / R_MAX) * R_MAX + R_MAX;
    l.Tlen = l.Npad + maxL + 256;
    l.nwords = l.Npad / 64 + 1;
    l.npart = (l.Nmax + POLISH_COLS - 1) / POLISH_COLS;
    const size_t hl = (size_t)(l.Npad + 64);
    size_t o = 0;
    l.off_T = o;     o = al256(o + sizeof(double) * (size_t)l.Tlen);
    l.off_mu = o;    o = al256(o + sizeof(double) * hl);
    l.off_var = o;   o = al256(o + sizeof(double) * hl);
    l.off_mu2 = o;   o = al256(o + sizeof(double) * hl);
    l.off_var2 = o;  o = al256(o + sizeof(double) * hl);
    l.off_h32 = o;   o = al256(o + 3 * al256(sizeof(float) * hl));
    l.off_h64 = o;   o = al256(o + 3 * al256(sizeof(double) * hl));
    l.off_alive = o; o = al256(o + sizeof(unsigned long long) * (size_t)l.nwords);
    l.off_rho = o;   o = al256(o + sizeof(unsigned long long) * (size_t)l.Npad);
    l.off_rhs = o;   o = al256(o + sizeof(unsigned long long) * (size_t)l.Npad);
    l.off_unc = o;   o = al256(o + sizeof(unsigned long long) * (size_t)l.nwords);
    l.off_tsel = o;  o = al256(o + sizeof(int32_t) * (size_t)(l.Npad / 64 + 1));
    l.off_tref = o;  o = al256(o + sizeof(int32_t) * (size_t)(l.Npad / 64 + 1));
    l.off_hot = o;   o = al256(o + sizeof(int32_t) * (size_t)HOT_MAX);
    l.off_twork = o; o = al256(o + sizeof(uint32_t) * (size_t)l.nwords);
    l.off_cand = o;  o = al256(o + sizeof(int64_t) * (size_t)KP_MAX);
    l.off_part = o;  o = al256(o + sizeof(double) * (size_t)(2 * KP_MAX * (l.npart + 1)));
    l.off_xc = o;    o = al256(o + sizeof(double) * (size_t)KP_MAX * (size_t)(maxL + 9));
    l.off_hist = o;  o = al256(o + sizeof(double) * (size_t)(l.L > 0 ? l.L : 1));
    l.off_evc = o;   o = al256(o + sizeof(unsigned long long) * EV_CLASSES * EV_SLOTS);
    l.off_ctrl = o;  o = al256(o + sizeof(Ctrl));
    l.off_red = o;   o = al256(o + sizeof(double) * 2 * RED_BLOCKS);
    l.off_sgm = o;   o = al256(o + sizeof(double) * 2 * (size_t)((l.Npad + 64 + 255) / 256));
    l.total = o;
    *out = l;
    return true;
}

SeriesDev carve(void* base, const Layout& l)
{
    char* p = (char*)base;
    const size_t hl = (size_t)(l.Npad + 64);
    SeriesDev s = {};
    s.n = l.n;
    s.Nmax = l.Nmax;
    s.Npad = l.Npad;
    s.Tlen = l.Tlen;
    s.nwords = l.nwords;
    s.npart = l.npart;
    s.minL = l.minL;
    s.maxL = l.maxL;
    s.k = l.k;
    s.kp = l.kp;
    s.L = l.L;
    s.T = (double*)(p + l.off_T);
    s.mu = (double*)(p + l.off_mu);
    s.var = (double*)(p + l.off_var);
    s.mu2 = (double*)(p + l.off_mu2);
    s.var2 = (double*)(p + l.off_var2);
    s.df32 = (float*)(p + l.off_h32);
    s.dg32 = (float*)(p + l.off_h32 + al256(sizeof(float) * hl));
    s.inv32 = (float*)(p + l.off_h32 + 2 * al256(sizeof(float) * hl));
    s.df64 = (double*)(p + l.off_h64);
    s.dg64 = (double*)(p + l.off_h64 + al256(sizeof(double) * hl));
    s.inv64 = (double*)(p + l.off_h64 + 2 * al256(sizeof(double) * hl));
    s.alive = (unsigned long long*)(p + l.off_alive);
    s.rho = (unsigned long long*)(p + l.off_rho);
    s.rhs = (unsigned long long*)(p + l.off_rhs);
    s.unc = (unsigned long long*)(p + l.off_unc);
    s.tsel = (int32_t*)(p + l.off_tsel);
    s.tref = (int32_t*)(p + l.off_tref);
    s.hot = (int32_t*)(p + l.off_hot);
    s.twork = (uint32_t*)(p + l.off_twork);
    s.cand = (int64_t*)(p + l.off_cand);
    s.part = (double*)(p + l.off_part);
    s.xc = (double*)(p + l.off_xc);
    s.hist = (double*)(p + l.off_hist);
    s.evc = (unsigned long long*)(p + l.off_evc);
    s.ctrl = (Ctrl*)(p + l.off_ctrl);
    s.red = (double*)(p + l.off_red);
    s.sgm = (double*)(p + l.off_sgm);
    return s;
}

void series_blocks(const Layout& l, const SweepCfg& cfg, int64_t out[PFX_KINDS])
{
    const int rn = 64 * cfg.q_near, rf = 64 * cfg.q_far, rr = 64 * cfg.q_ref;
    // chunks of the first pass: near_cols, at most every column
    const int64_t span = std::min<int64_t>((int64_t)cfg.near_cols, l.Nmax);
    const int64_t nsub = (span + cfg.chunk_cols - 1) / cfg.chunk_cols;
    out[PFX_ELEM] = (l.Npad + 64 + 255) / 256;
    out[PFX_NEAR] = ((l.Nmax + rn - 1) / rn) * nsub;
    out[PFX_TSEL] = ((l.Nmax + rf - 1) / rf + 255) / 256;
    out[PFX_TREF] = ((l.Nmax + rr - 1) / rr + 255) / 256;
    out[PFX_POLISH] = l.npart;
    out[PFX_BAND] = (l.Nmax + BAND_S - 1) / BAND_S;
}

}  // namespace palmad
