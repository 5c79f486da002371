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
// round preparation: MERLIN's walk over the lengths (Alg. 1)
// ---------------------------------------------------------------------------
// Advance every series: the first round starts at minL; after a successful
// round the next length starts; after a failed one the same length is
// searched again with the r that k_round_end lowered.
__global__ void k_round_prep(SeriesDev* S, int B)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const SeriesDev& s = S[b];
    Ctrl* c = s.ctrl;
    if (c->finished) {
        c->active = 0;
        return;
    }
    if (!c->started) {
        c->started = 1;
        c->m = s.minL;
        c->li = 0;
        c->attempt = 0;
        c->new_len = 2;
        c->done = 0;
        c->active = 1;
        return;
    }
    if (c->done) {
        if (c->m >= s.maxL) {
            c->finished = 1;
            c->active = 0;
            return;
        }
        c->m += 1;
        c->li += 1;
        c->attempt = 0;
        c->new_len = 1;
        c->done = 0;
    } else {
        c->attempt += 1;
        c->new_len = 0;
        if (c->attempt >= MAX_ATTEMPTS) {
            c->error = 1;
            c->finished = 1;
            c->active = 0;
            return;
        }
    }
    c->active = 1;
}

// ---------------------------------------------------------------------------
// per-length statistics (Eq. (4) at minL, Eq. (7)-(8) after) and helpers
// ---------------------------------------------------------------------------
__global__ void k_stats(SeriesDev* S, int B, const int64_t* __restrict__ pfx)
{
    const int b = series_of(pfx, B, blockIdx.x);
    const SeriesDev& s = S[b];
    Ctrl* c = s.ctrl;
    if (!c->active || c->new_len == 0) return;
    const int64_t i = (blockIdx.x - pfx[b]) * (int64_t)blockDim.x + threadIdx.x;
    if (i == 0) {
        c->flat_min = 0x7fffffffffffffffll;
        c->flat_max = -1;
    }
    if (i >= s.Npad + 64) return;
    const double* __restrict__ T = s.T;
    const int32_t m = c->m;
    if (c->new_len == 2) {
        // Eq. (4): direct two-pass statistics at the first length
        const int64_t N = s.n - m + 1;
        if (i >= N) {
            s.mu[i] = 0.0;
            s.var[i] = 0.0;
            return;
        }
        double acc = 0.0;
        for (int k = 0; k < m; ++k) acc += T[i + k];
        const double mean = acc / (double)m;
        double q = 0.0;
        for (int k = 0; k < m; ++k) {
            const double d = T[i + k] - mean;
            q += d * d;
        }
        s.mu[i] = mean;
        s.var[i] = q / (double)m;
    } else {
        // Eq. (7)-(8): length m from length m-1, in place
        const int32_t mo = m - 1;
        const int64_t N1 = s.n - mo;  // windows of length m
        if (i >= N1) {
            s.mu[i] = 0.0;
            s.var[i] = 0.0;
            return;
        }
        const double t = T[i + mo];
        const double mu0 = s.mu[i];
        const double dm = (double)mo;
        const double d = mu0 - t;
        s.mu[i] = (dm * mu0 + t) / (dm + 1.0);
        s.var[i] = dm / (dm + 1.0) * (s.var[i] + d * d / (dm + 1.0));
    }
}

// df[i] = (t_{i+m} - t_i)/2, dg[i] = (t_{i+m} - mu_{i+1}) + (t_i - mu_i) for
// i < N-1 (zero beyond), inv[i] = 1/(sqrt(m) sigma_i) for non-flat i < N.
__global__ void k_helpers(SeriesDev* S, int B, const int64_t* __restrict__ pfx)
{
    const int b = series_of(pfx, B, blockIdx.x);
    const SeriesDev& s = S[b];
    Ctrl* c = s.ctrl;
    if (!c->active || c->new_len == 0) return;
    const int64_t i = (blockIdx.x - pfx[b]) * (int64_t)blockDim.x + threadIdx.x;
    if (i >= s.Npad + 64) return;
    const int32_t m = c->m;
    const int64_t N = s.n - m + 1;
    const double* __restrict__ T = s.T;
    double df = 0.0, dg = 0.0, inv = 0.0;
    if (i < N - 1) {
        const double a = T[i + m], e = T[i];
        df = (a - e) * 0.5;
        dg = (a - s.mu[i + 1]) + (e - s.mu[i]);
    }
    if (i < N) {
        const double sg = sqrt(s.var[i]);
        if (sg <= c->flat_eps) {
            atomicMin((long long*)&c->flat_min, (long long)i);
            atomicMax((long long*)&c->flat_max, (long long)i);
        } else {
            inv = 1.0 / (sqrt((double)m) * sg);
        }
    }
    s.df64[i] = df;
    s.dg64[i] = dg;
    s.inv64[i] = inv;
    s.df32[i] = (float)df;
    s.dg32[i] = (float)dg;
    s.inv32[i] = (float)inv;
}

// ---------------------------------------------------------------------------
// round control (MERLIN's r, Alg. 1) and per-round reset
// ---------------------------------------------------------------------------
__global__ void k_round_begin(SeriesDev* S, int B, const int64_t* __restrict__ pfx, float guard)
{
    const int b = series_of(pfx, B, blockIdx.x);
    const SeriesDev& s = S[b];
    Ctrl* c = s.ctrl;
    if (!c->active) return;
    const int64_t g = (blockIdx.x - pfx[b]) * (int64_t)blockDim.x + threadIdx.x;
    const int32_t m = c->m;
    if (g == 0) {
        const int li = c->li;
        if (c->attempt == 0) {
            c->done = 0;
            if (c->mode != 3) {
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
        }
        const double r = c->r;
        c->prune = r > 0.0 ? 1 : 0;
        c->thr64 = r > 0.0 ? 1.0 - r * r / (2.0 * (double)m) : 2.0;
        c->thr_sel = c->thr64 + (double)guard;
        // round up: an FP32 threshold must never prune more than thr_sel
        c->thr32 = __double2float_ru(c->thr_sel);
        c->nlive_sel = c->maxc_sel = 0;
        c->nlive_ref = c->maxc_ref = 0;
        c->ctr_sel = c->ctr_ref = 0ull;
        c->nsurv = 0;
        c->ncand = 0;
    }
    const int64_t N = s.n - m + 1;
    if (g < s.nwords) {
        const int64_t lo = g * 64;
        unsigned long long bits = 0ull;
        if (lo + 64 <= N) bits = ~0ull;
        else if (lo < N) bits = (1ull << (N - lo)) - 1ull;
        s.alive[g] = bits;
    }
    if (g < s.Npad) s.rho[g] = 0x000fffffffffffffull;  // ordered bits of -inf
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
    Ctrl* ctrl;
    int64_t N;
    int32_t m;
};

// Stage the centred windows of the tile's first row (xs, for the top
// boundary) and of the first column (ys, for the initial column) in LDS,
// zero padded by 64, and return their sums (zero up to rounding).
__device__ __forceinline__ void stage_windows(const double* __restrict__ T,
                                              const double* __restrict__ mu, int32_t m, int64_t i0,
                                              int64_t jbeg, double* xs, double* ys, double& Sx,
                                              double& Sy)
{
    const int lane = threadIdx.x;
    const double mui = mu[i0], muj = mu[jbeg];
    double sx = 0.0, sy = 0.0;
    for (int k = lane; k < m + 64; k += 64) {
        double x = 0.0, y = 0.0;
        if (k < m) {
            x = T[i0 + k] - mui;
            y = T[jbeg + k] - muj;
        }
        xs[k] = x;
        ys[k] = y;
        sx += x;
        sy += y;
    }
    Sx = wave_sum(sx);
    Sy = wave_sum(sy);
    __syncthreads();
}

// C(rbase+q, jbeg) for the lane's Q rows: sum_k t_{i+k} y_k - mu_i * Sy.
template <int Q>
__device__ __forceinline__ void initial_column(const double* __restrict__ T,
                                               const double* __restrict__ mu, int32_t m,
                                               int64_t rbase, const double* ys, double Sy,
                                               double (&acc)[Q])
{
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[q] = 0.0;
    for (int k0 = 0; k0 < m; k0 += Q) {
        double z[2 * Q - 1];
#pragma unroll
        for (int e = 0; e < 2 * Q - 1; ++e) z[e] = T[rbase + k0 + e];
#pragma unroll
        for (int kk = 0; kk < Q; ++kk) {
            const double yk = ys[k0 + kk];
#pragma unroll
            for (int q = 0; q < Q; ++q) acc[q] = fma(z[q + kk], yk, acc[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[q] -= mu[rbase + q] * Sy;
}

// Column helpers of one step, staged in LDS per block of 64 columns.
template <typename F>
struct alignas(4 * sizeof(F)) H4 {
    F df, dg, inv;  // df[j-1], dg[j-1], 1/(sqrt(m) sigma_j)
    F B;            // C(i0, j): exact value of the tile's top row at column j
};

// LDS of a sweep work item, in doubles: xs[m+64] | win[m+128] | hs[256].
// win holds the first column's centred window while the initial column is
// computed, then the T segment of the current block.
__host__ __device__ constexpr int sweep_hs_offset(int m) { return (2 * m + 192 + 3) & ~3; }
__host__ __device__ constexpr size_t sweep_lds_doubles(int m) { return (size_t)(sweep_hs_offset(m) + 256); }

// Stage the block starting at column j0 in LDS: one burst of independent
// loads brings the T segment and the column helpers, then lane l computes
// the exact top-boundary value B(j0 + l) = C(i0, j0 + l) from LDS.  hs[s]
// then holds everything step s needs.
template <typename F>
__device__ __forceinline__ void stage_block(const double* __restrict__ T, const double* __restrict__ mu,
                                            const F* __restrict__ df, const F* __restrict__ dg,
                                            const F* __restrict__ inv, int32_t m, int64_t j0,
                                            const double* xs, double Sx, double* win, H4<F>* hs)
{
    const int lane = threadIdx.x;
    __syncthreads();  // the previous block is done with win and hs
    const double muj = mu[j0 + lane];
    H4<F> h;
    h.df = df[j0 + lane - 1];
    h.dg = dg[j0 + lane - 1];
    h.inv = inv[j0 + lane];
    for (int t = lane; t < m + 68; t += 64) win[t] = T[j0 + t];
    __syncthreads();
    const double* tw = win + lane;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int k = 0; k < m; k += 4) {
        a0 = fma(xs[k], tw[k], a0);
        a1 = fma(xs[k + 1], tw[k + 1], a1);
        a2 = fma(xs[k + 2], tw[k + 2], a2);
        a3 = fma(xs[k + 3], tw[k + 3], a3);
    }
    h.B = (F)((a0 + a1) + (a2 + a3) - muj * Sx);
    hs[lane] = h;
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
// bitmap says are dead.  Returns true while some row of the tile is alive.
template <int Q>
__device__ __forceinline__ bool sync_rows(unsigned long long* alive, int64_t rbase,
                                          unsigned long long (&dm)[Q])
{
    const int lane = threadIdx.x;
    unsigned long long* wp = &alive[rbase >> 6];
    const int off = (int)(rbase & 63);
    const unsigned int msk = (Q >= 32) ? 0xffffffffu : ((1u << Q) - 1u);
    const unsigned int live = (unsigned int)(load_word(wp) >> off) & msk;
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

template <typename F, int Q>
__device__ void sel_item(const SweepArgs<F>& A, int64_t i0, int64_t jbeg, int64_t jend, F thr,
                         double* lds, unsigned long long& evals)
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
    double* xs = lds;
    double* ys = lds + (m + 64);
    H4<F>* hs = (H4<F>*)(lds + sweep_hs_offset(m));
    double Sx, Sy;
    stage_windows(A.T, A.mu, m, i0, jbeg, xs, ys, Sx, Sy);
    F C[Q];
    {
        double acc[Q];
        initial_column<Q>(A.T, A.mu, m, rbase, ys, Sy, acc);
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
    int64_t j = jbeg + 1;
    while (go && j < jend) {
        const int nst = (int)std::min<int64_t>(64, jend - j);
        stage_block<F>(A.T, A.mu, A.df, A.dg, A.inv, m, j, xs, Sx, ys, hs);
        unsigned long long colbits = 0ull;
        const bool full = (j - (i0 + R - 1)) >= m;
        if (full)
            sel_block<F, Q, false>(A, j, nst, C, a, b, nth, rm, ri, hs, colbits);
        else
            sel_block<F, Q, true>(A, j, nst, C, a, b, nth, rm, ri, hs, colbits);
        kill_columns(A.alive, j, colbits);
#pragma unroll
        for (int q = 0; q < Q; ++q) dm[q] |= uniform64(__ballot(rm[q] > F(0)));
        ev += pair_count(i0, std::min<int64_t>(i0 + R, N), j, nst, m, false);
        j += nst;
        go = sync_rows<Q>(A.alive, rbase, dm);
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
    A.mu = s.mu;
    A.df = s.df32;
    A.dg = s.dg32;
    A.inv = s.inv32;
    A.alive = s.alive;
    A.rho = s.rho;
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
    A.mu = s.mu;
    A.df = s.df64;
    A.dg = s.dg64;
    A.inv = s.inv64;
    A.alive = s.alive;
    A.rho = s.rho;
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

template <int Q>
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
    double* xs = lds;
    double* ys = lds + (m + 64);
    H4<double>* hs = (H4<double>*)(lds + sweep_hs_offset(m));
    double Sx, Sy;
    stage_windows(A.T, A.mu, m, i0, jbeg, xs, ys, Sx, Sy);
    double C[Q];
    initial_column<Q>(A.T, A.mu, m, rbase, ys, Sy, C);
    double a[Q], b[Q], invi[Q], mx[Q];
    int32_t ri[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int64_t i = rbase + q;
        const bool top = (lane == 0) && (q == 0);
        const int64_t ip = top ? i : i - 1;
        a[q] = top ? 0.0 : A.df[ip];
        b[q] = top ? 0.0 : A.dg[ip];
        invi[q] = A.inv[i];
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
        const int nst = (int)std::min<int64_t>(64, jend - j);
        stage_block<double>(A.T, A.mu, A.df, A.dg, A.inv, m, j, xs, Sx, ys, hs);
        bool full;
        if (left) full = (i0 - (j + nst - 1)) >= m;
        else full = (j - (i0 + R - 1)) >= m;
        if (full) ref_block<Q, 0>(A, j, nst, C, a, b, mx, ri, hs);
        else if (left) ref_block<Q, 2>(A, j, nst, C, a, b, mx, ri, hs);
        else ref_block<Q, 1>(A, j, nst, C, a, b, mx, ri, hs);
        ev += pair_count(i0, std::min<int64_t>(i0 + R, N), j, nst, m, left);
        j += nst;
        if (prune) {
#pragma unroll
            for (int q = 0; q < Q; ++q) dm[q] |= uniform64(__ballot(invi[q] > 0.0 && mx[q] * invi[q] > thr));
        }
        go = sync_rows<Q>(A.alive, rbase, dm);
    }
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

// First selection pass: every row tile's nearest near_cols columns, split
// into nsub chunks of `chunk` columns that run concurrently; each stops as
// soon as the whole tile is dead.
template <typename F, int Q>
__global__ __launch_bounds__(64) void k_select_near(SeriesDev* S, int B,
                                                    const int64_t* __restrict__ pfx, int near_cols,
                                                    int chunk, int nsub)
{
    extern __shared__ double lds[];
    const int b = series_of(pfx, B, blockIdx.x);
    const SeriesDev& s = S[b];
    Ctrl* c = s.ctrl;
    if (!c->active || !c->prune) return;
    constexpr int R = 64 * Q;
    const int64_t lb = blockIdx.x - pfx[b];
    const SweepArgs<F> A = args_of<F>(s, c);
    const int64_t i0 = (lb / nsub) * R;
    if (i0 >= A.N) return;
    const int64_t j00 = i0 + A.m;
    const int64_t jbeg = j00 + (lb % nsub) * chunk;
    if (jbeg >= A.N || jbeg >= j00 + near_cols) return;
    const int64_t jend = std::min<int64_t>(std::min<int64_t>(A.N, jbeg + chunk), j00 + near_cols);
    const F thr = sel_threshold<F>(c);
    unsigned long long ev = 0;
    sel_item<F, Q>(A, i0, jbeg, jend, thr, lds, ev);
    if (threadIdx.x == 0 && ev) {
        atomicAdd(&c->evals_sel, ev);
        atomicAdd(&c->evals_near, ev);
    }
}

// Remaining selection work: items (live tile, chunk) drawn nearest-first
// from each series' counter; a workgroup drains the series in rotated order.
template <typename F, int Q>
__global__ __launch_bounds__(64) void k_select_far(SeriesDev* S, int B, int near_cols, int chunk)
{
    extern __shared__ double lds[];
    constexpr int R = 64 * Q;
    for (int t = 0; t < B; ++t) {
        const int b = (int)((blockIdx.x + (unsigned int)t) % (unsigned int)B);
        const SeriesDev& s = S[b];
        Ctrl* c = s.ctrl;
        if (!c->active || !c->prune) continue;
        const unsigned int nlive = c->nlive_sel;
        const unsigned long long total = (unsigned long long)nlive * c->maxc_sel;
        if (total == 0) continue;
        const SweepArgs<F> A = args_of<F>(s, c);
        const F thr = sel_threshold<F>(c);
        const int32_t* __restrict__ tiles = s.tsel;
        unsigned long long ev = 0;
        for (;;) {
            unsigned long long it = 0;
            if (threadIdx.x == 0) it = atomicAdd(&c->ctr_sel, 1ull);
            it = uniform64(it);
            if (it >= total) break;
            const unsigned long long cc = it / nlive;
            const unsigned int p = (unsigned int)(it % nlive);
            const int64_t i0 = (int64_t)tiles[p] * R;
            const int64_t jbeg = i0 + A.m + near_cols + (int64_t)cc * chunk;
            if (jbeg >= A.N) continue;
            const int64_t jend = std::min<int64_t>(A.N, jbeg + chunk);
            sel_item<F, Q>(A, i0, jbeg, jend, thr, lds, ev);
        }
        if (threadIdx.x == 0 && ev) {
            atomicAdd(&c->evals_sel, ev);
            atomicAdd(&c->evals_far, ev);
        }
    }
}

// Live-tile lists.  mode 0: selection tiles (R rows), chunks to the right
// beyond the first pass; mode 1: refinement tiles, chunks on both sides.
__global__ void k_tiles(SeriesDev* S, int B, const int64_t* __restrict__ pfx, int R, int mode,
                        int near_cols, int chunk)
{
    const int b = series_of(pfx, B, blockIdx.x);
    const SeriesDev& s = S[b];
    Ctrl* c = s.ctrl;
    if (!c->active) return;
    if (mode == 0 && !c->prune) return;
    const int64_t t = (blockIdx.x - pfx[b]) * (int64_t)blockDim.x + threadIdx.x;
    const int32_t m = c->m;
    const int64_t N = s.n - m + 1;
    const int64_t ntiles = (N + R - 1) / R;
    if (t >= ntiles) return;
    const int words = R / 64;
    unsigned long long any = 0ull;
    for (int w = 0; w < words; ++w) any |= s.alive[t * words + w];
    if (!any) return;
    const int64_t i0 = t * R;
    int64_t nch;
    if (mode == 0) {
        const int64_t j0 = i0 + m + near_cols;
        nch = j0 >= N ? 0 : (N - j0 + chunk - 1) / chunk;
    } else {
        const int64_t lend = std::min<int64_t>(N, i0 + R - m);
        const int64_t nl = lend > 0 ? (lend + chunk - 1) / chunk : 0;
        const int64_t jr = i0 + m;
        const int64_t nr = jr < N ? (N - jr + chunk - 1) / chunk : 0;
        nch = nl + nr;
    }
    if (nch <= 0) return;
    const unsigned int slot = atomicAdd(mode == 0 ? &c->nlive_sel : &c->nlive_ref, 1u);
    (mode == 0 ? s.tsel : s.tref)[slot] = (int32_t)t;
    atomicMax(mode == 0 ? &c->maxc_sel : &c->maxc_ref, (unsigned int)nch);
}

// Refinement: exact FP64 row maximum of rho over both sides for every tile
// holding survivors; items drawn nearest-first, alternating right and left.
template <int Q>
__global__ __launch_bounds__(64) void k_refine(SeriesDev* S, int B, int chunk)
{
    extern __shared__ double lds[];
    constexpr int R = 64 * Q;
    for (int t = 0; t < B; ++t) {
        const int b = (int)((blockIdx.x + (unsigned int)t) % (unsigned int)B);
        const SeriesDev& s = S[b];
        Ctrl* c = s.ctrl;
        if (!c->active) continue;
        const unsigned int nlive = c->nlive_ref;
        const unsigned long long total = (unsigned long long)nlive * c->maxc_ref;
        if (total == 0) continue;
        const SweepArgs<double> A = args_of<double>(s, c);
        const double thr = c->thr64;
        const int prune = c->prune;
        const int32_t* __restrict__ tiles = s.tref;
        unsigned long long ev = 0;
        for (;;) {
            unsigned long long it = 0;
            if (threadIdx.x == 0) it = atomicAdd(&c->ctr_ref, 1ull);
            it = uniform64(it);
            if (it >= total) break;
            const unsigned long long cc = it / nlive;
            const unsigned int p = (unsigned int)(it % nlive);
            const int64_t i0 = (int64_t)tiles[p] * R;
            const int64_t lend = std::min<int64_t>(A.N, i0 + R - A.m);
            const int64_t nl = lend > 0 ? (lend + chunk - 1) / chunk : 0;
            const int64_t jr = i0 + A.m;
            const int64_t nr = jr < A.N ? (A.N - jr + chunk - 1) / chunk : 0;
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
        if (threadIdx.x == 0 && ev) atomicAdd(&c->evals_ref, ev);
    }
}

// Survivor list: every row whose bit is still set.
__global__ void k_survivors(SeriesDev* S, int B, const int64_t* __restrict__ pfx)
{
    const int b = series_of(pfx, B, blockIdx.x);
    const SeriesDev& s = S[b];
    Ctrl* c = s.ctrl;
    if (!c->active) return;
    const int64_t w = (blockIdx.x - pfx[b]) * (int64_t)blockDim.x + threadIdx.x;
    const int64_t N = s.n - c->m + 1;
    if (w >= (N + 63) / 64) return;
    unsigned long long bits = s.alive[w];
    const int cnt = __popcll(bits);
    if (!cnt) return;
    unsigned int base = atomicAdd(&c->nsurv, (unsigned int)cnt);
    while (bits) {
        const int t = __ffsll((long long)bits) - 1;
        s.surv[base++] = (int32_t)(w * 64 + t);
        bits &= bits - 1ull;
    }
}

struct Key {
    unsigned long long u;  // ordered bits of rho (ascending rho = descending nnDist)
    long long i;
};
__device__ __forceinline__ bool key_less(const Key& x, const Key& y)
{
    return x.u < y.u || (x.u == y.u && x.i < y.i);
}

__global__ __launch_bounds__(TOPK_BLOCK) void k_topk(SeriesDev* S)
{
    __shared__ unsigned long long su[TOPK_BLOCK / 64];
    __shared__ long long si[TOPK_BLOCK / 64];
    const SeriesDev& s = S[blockIdx.x];
    Ctrl* c = s.ctrl;
    if (!c->active) return;
    const int k = s.k;
    const unsigned int ns = c->nsurv;
    if (ns < (unsigned int)k) {
        if (threadIdx.x == 0) c->ncand = 0;
        return;
    }
    const int32_t* __restrict__ surv = s.surv;
    const unsigned long long* __restrict__ rho = s.rho;
    const int kp = (int)min(ns, (unsigned int)(k + KP_EXTRA));
    Key last = {0ull, -1};
    bool have_last = false;
    for (int r = 0; r < kp; ++r) {
        Key best = {~0ull, 0x7fffffffffffffffll};
        for (unsigned int q = threadIdx.x; q < ns; q += TOPK_BLOCK) {
            const long long i = surv[q];
            const Key x = {rho[i], i};
            if (have_last && !key_less(last, x)) continue;
            if (key_less(x, best)) best = x;
        }
        for (int o = 32; o >= 1; o >>= 1) {
            Key y;
            y.u = __shfl_xor(best.u, o);
            y.i = __shfl_xor(best.i, o);
            if (key_less(y, best)) best = y;
        }
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            su[w] = best.u;
            si[w] = best.i;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            Key bb = {su[0], si[0]};
            for (int q = 1; q < TOPK_BLOCK / 64; ++q) {
                const Key y = {su[q], si[q]};
                if (key_less(y, bb)) bb = y;
            }
            su[0] = bb.u;
            si[0] = bb.i;
            s.cand[r] = bb.i;
        }
        __syncthreads();
        last.u = su[0];
        last.i = si[0];
        have_last = true;
        __syncthreads();
    }
    if (threadIdx.x == 0) c->ncand = (unsigned int)kp;
}

// Exact FP64 nearest-neighbour correlation of the candidate rows against
// every column: direct centred dot products (no recurrence), the reference
// the reported distances and neighbour indices come from.  A block owns 256
// consecutive columns of one series, stages their windows in LDS once and
// evaluates every candidate against them; it writes one (max rho, argmax j)
// partial per candidate.
__global__ __launch_bounds__(POLISH_BLOCK) void k_polish(SeriesDev* S, int B,
                                                         const int64_t* __restrict__ pfx)
{
    extern __shared__ double lds[];
    __shared__ double sh[16];
    __shared__ double red_v[POLISH_BLOCK / 64];
    __shared__ long long red_j[POLISH_BLOCK / 64];
    const int b = series_of(pfx, B, blockIdx.x);
    const SeriesDev& s = S[b];
    Ctrl* c = s.ctrl;
    if (!c->active) return;
    const int ncand = (int)c->ncand;
    if (ncand == 0) return;
    const int32_t m = c->m;
    const int64_t N = s.n - m + 1;
    const double* __restrict__ T = s.T;
    const double* __restrict__ mu = s.mu;
    const double* __restrict__ var = s.var;
    double* ts = lds;                          // T[j0 .. j0 + 256 + m + 64)
    double* xs = lds + POLISH_BLOCK + m + 64;  // centred candidate window, zero padded
    const int tid = threadIdx.x;
    const int64_t blk = blockIdx.x - pfx[b];
    const int64_t j0 = blk * POLISH_BLOCK;
    for (int t = tid; t < POLISH_BLOCK + m + 64; t += POLISH_BLOCK) ts[t] = T[j0 + t];
    const int64_t j = j0 + tid;
    const double feps = c->flat_eps;
    const bool colok = j < N;
    const double sgj = colok ? sqrt(var[j]) : 1.0;
    const double muj = colok ? mu[j] : 0.0;
    const bool flat_j = colok && sgj <= feps;
    unsigned long long ev = 0;
    for (int cid = 0; cid < ncand; ++cid) {
        const int64_t i = s.cand[cid];
        const double mui = mu[i];
        double sx = 0.0;
        __syncthreads();  // previous candidate's xs fully consumed
        for (int k = tid; k < m + 64; k += POLISH_BLOCK) {
            const double x = k < m ? T[i + k] - mui : 0.0;
            xs[k] = x;
            sx += x;
        }
        const double s0 = block_sum(sx, sh);
        if (tid == 0) sh[15] = s0;
        __syncthreads();
        const double Sx = sh[15];
        const double sgi = sqrt(var[i]);
        const bool flat_i = sgi <= feps;
        double best = -f_inf<double>();
        long long bj = 0x7fffffffffffffffll;
        if (colok && (j <= i - m || j >= i + m)) {
            double rh;
            if (flat_i || flat_j) {
                rh = (flat_i && flat_j) ? 1.0 : 0.0;
            } else {
                const double* t = ts + tid;
                double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
                for (int k = 0; k < m; k += 4) {
                    a0 = fma(xs[k], t[k], a0);
                    a1 = fma(xs[k + 1], t[k + 1], a1);
                    a2 = fma(xs[k + 2], t[k + 2], a2);
                    a3 = fma(xs[k + 3], t[k + 3], a3);
                }
                const double Cv = (a0 + a1) + (a2 + a3) - muj * Sx;
                rh = Cv / ((double)m * sgi * sgj);
                rh = fmin(1.0, fmax(-1.0, rh));
            }
            best = rh;
            bj = j;
            ++ev;
        }
        for (int o = 32; o >= 1; o >>= 1) {
            const double v = __shfl_xor(best, o);
            const long long jj = __shfl_xor(bj, o);
            if (v > best || (v == best && jj < bj)) {
                best = v;
                bj = jj;
            }
        }
        const int w = tid >> 6;
        if ((tid & 63) == 0) {
            red_v[w] = best;
            red_j[w] = bj;
        }
        __syncthreads();
        if (tid == 0) {
            for (int q = 1; q < POLISH_BLOCK / 64; ++q)
                if (red_v[q] > best || (red_v[q] == best && red_j[q] < bj)) {
                    best = red_v[q];
                    bj = red_j[q];
                }
            const int64_t slot = ((int64_t)cid * s.npart + blk) * 2;
            s.part[slot] = best;
            s.part[slot + 1] = (double)bj;
        }
    }
    ev = (unsigned long long)wave_sum((double)ev);
    if ((tid & 63) == 0 && ev) atomicAdd(&c->evals_pol, ev);
}

// Reduce the polish partials of each candidate to (rho, j) in part's tail.
// grid: (KP_MAX, B).
__global__ void k_polish_reduce(SeriesDev* S)
{
    __shared__ double rv[4];
    __shared__ double rj[4];
    const SeriesDev& s = S[blockIdx.y];
    Ctrl* c = s.ctrl;
    if (!c->active) return;
    const int cid = blockIdx.x;
    if ((unsigned int)cid >= c->ncand) return;
    const int64_t npart = s.npart;
    const int32_t m = c->m;
    const int64_t nblk = (s.n - m + 1 + POLISH_BLOCK - 1) / POLISH_BLOCK;
    double best = -f_inf<double>(), bj = 1e300;
    for (int64_t p = threadIdx.x; p < nblk; p += blockDim.x) {
        const double v = s.part[((int64_t)cid * npart + p) * 2];
        const double jj = s.part[((int64_t)cid * npart + p) * 2 + 1];
        if (v > best || (v == best && jj < bj)) {
            best = v;
            bj = jj;
        }
    }
    for (int o = 32; o >= 1; o >>= 1) {
        const double v = __shfl_xor(best, o);
        const double jj = __shfl_xor(bj, o);
        if (v > best || (v == best && jj < bj)) {
            best = v;
            bj = jj;
        }
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        rv[w] = best;
        rj[w] = bj;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q)
            if (rv[q] > best || (rv[q] == best && rj[q] < bj)) {
                best = rv[q];
                bj = rj[q];
            }
        const int64_t tail = (int64_t)KP_MAX * npart * 2;
        s.part[tail + cid * 2] = best;
        s.part[tail + cid * 2 + 1] = bj;
    }
}

// Rank the polished candidates, write the length's top-k rows when the round
// found at least k range discords, and advance MERLIN's r otherwise.
// grid: B blocks of 128 threads.
__global__ void k_round_end(SeriesDev* S)
{
    __shared__ double nn_s[KP_MAX];
    __shared__ long long id_s[KP_MAX];
    __shared__ long long jj_s[KP_MAX];
    const SeriesDev& s = S[blockIdx.x];
    Ctrl* c = s.ctrl;
    if (!c->active) return;
    const int k = s.k;
    const int32_t m = c->m;
    const int li = c->li;
    const unsigned int ns = c->nsurv;
    const int kp = (int)c->ncand;
    const bool ok = ns >= (unsigned int)k && kp >= k;
    const int64_t tail = (int64_t)KP_MAX * s.npart * 2;
    const int t = threadIdx.x;
    if (ok && t < kp) {
        const double rho = s.part[tail + t * 2];
        const double d2 = 2.0 * (double)m * (1.0 - rho);
        nn_s[t] = sqrt(fmin(4.0 * (double)m, fmax(0.0, d2)));
        id_s[t] = s.cand[t];
        jj_s[t] = (long long)s.part[tail + t * 2 + 1];
    }
    __syncthreads();
    if (ok && t < kp) {
        int rank = 0;
        for (int q = 0; q < kp; ++q)
            if (nn_s[q] > nn_s[t] || (nn_s[q] == nn_s[t] && id_s[q] < id_s[t])) ++rank;
        if (rank < k) {
            const int64_t row = (int64_t)li * k + rank;
            if (s.idx) {
                s.idx[row] = id_s[t];
                s.len[row] = m;
                s.nn[row] = nn_s[t];
                s.nnidx[row] = jj_s[t];
            }
            if (rank == k - 1) s.hist[li] = nn_s[t];
        }
    }
    __syncthreads();
    if (t == 0) {
        c->rounds += 1;
        if (ok) {
            c->done = 1;
            c->survivors += ns;
            if (s.count) s.count[li] = (int32_t)ns;
        } else {
            c->done = 0;
            if (c->mode == 0) c->r *= 0.5;
            else if (c->mode == 1) c->r *= 0.99;
            else if (c->mode == 2) c->r = (c->step > 0.0) ? c->r - c->step : 0.99 * c->r;
        }
    }
}

// Series with work left after this round (one block).
__global__ void k_remaining(SeriesDev* S, int B, int32_t* out)
{
    __shared__ int cnt[2];
    if (threadIdx.x == 0) {
        cnt[0] = 0;
        cnt[1] = 0;
    }
    __syncthreads();
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
        const Ctrl* c = S[b].ctrl;
        const bool left = !c->finished && !(c->started && c->done && c->m >= S[b].maxL);
        if (left) atomicAdd(&cnt[0], 1);
        if (c->error) atomicAdd(&cnt[1], 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = cnt[0];
        out[1] = cnt[1];
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename F, int Q>
static void launch_near(const Batch& bt, const SweepCfg& cfg, const int64_t* total, hipStream_t st)
{
    const size_t lds = sizeof(double) * sweep_lds_doubles(bt.maxL_all);
    const int nsub = (cfg.near_cols + cfg.chunk_cols - 1) / cfg.chunk_cols;
    if (total[PFX_NEAR] == 0) return;
    cfg.timer->begin(0, st);
    hipLaunchKernelGGL((k_select_near<F, Q>), dim3((unsigned int)total[PFX_NEAR]), dim3(64), lds,
                       st, bt.s, bt.B, bt.pfx[PFX_NEAR], cfg.near_cols, cfg.chunk_cols, nsub);
    cfg.timer->end(0, st);
}

template <typename F, int Q>
static void launch_far(const Batch& bt, const SweepCfg& cfg, const int64_t* total, hipStream_t st)
{
    const size_t lds = sizeof(double) * sweep_lds_doubles(bt.maxL_all);
    hipLaunchKernelGGL(k_tiles, dim3((unsigned int)total[PFX_TSEL]), dim3(256), 0, st, bt.s, bt.B,
                       bt.pfx[PFX_TSEL], 64 * Q, 0, cfg.near_cols, cfg.chunk_cols);
    cfg.timer->begin(1, st);
    hipLaunchKernelGGL((k_select_far<F, Q>), dim3(cfg.far_grid), dim3(64), lds, st, bt.s, bt.B,
                       cfg.near_cols, cfg.chunk_cols);
    cfg.timer->end(1, st);
}

template <int Q>
static void launch_refine(const Batch& bt, const SweepCfg& cfg, const int64_t* total, hipStream_t st)
{
    hipLaunchKernelGGL(k_tiles, dim3((unsigned int)total[PFX_TREF]), dim3(256), 0, st, bt.s, bt.B,
                       bt.pfx[PFX_TREF], 64 * Q, 1, 0, cfg.chunk_cols);
    const size_t lds = sizeof(double) * sweep_lds_doubles(bt.maxL_all);
    cfg.timer->begin(2, st);
    hipLaunchKernelGGL((k_refine<Q>), dim3(cfg.far_grid), dim3(64), lds, st, bt.s, bt.B,
                       cfg.chunk_cols);
    cfg.timer->end(2, st);
}

template <typename F>
static void launch_select(const Batch& bt, const SweepCfg& cfg, const int64_t* total,
                          hipStream_t st)
{
    switch (cfg.q_near) {
    case 2: launch_near<F, 2>(bt, cfg, total, st); break;
    case 4: launch_near<F, 4>(bt, cfg, total, st); break;
    default: launch_near<F, 8>(bt, cfg, total, st); break;
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
    hipLaunchKernelGGL(k_round_prep, dim3((bt.B + 63) / 64), dim3(64), 0, st, bt.s, bt.B);
    hipLaunchKernelGGL(k_stats, dim3(elem), dim3(256), 0, st, bt.s, bt.B, bt.pfx[PFX_ELEM]);
    hipLaunchKernelGGL(k_helpers, dim3(elem), dim3(256), 0, st, bt.s, bt.B, bt.pfx[PFX_ELEM]);
    hipLaunchKernelGGL(k_round_begin, dim3(elem), dim3(256), 0, st, bt.s, bt.B, bt.pfx[PFX_ELEM],
                       cfg.guard);
    if (cfg.dist_bits == 64) launch_select<double>(bt, cfg, total, st);
    else launch_select<float>(bt, cfg, total, st);
    switch (cfg.q_ref) {
    case 4: launch_refine<4>(bt, cfg, total, st); break;
    case 8: launch_refine<8>(bt, cfg, total, st); break;
    default: launch_refine<2>(bt, cfg, total, st); break;
    }
    hipLaunchKernelGGL(k_survivors, dim3((unsigned int)total[PFX_WORDS]), dim3(256), 0, st, bt.s,
                       bt.B, bt.pfx[PFX_WORDS]);
    hipLaunchKernelGGL(k_topk, dim3(bt.B), dim3(TOPK_BLOCK), 0, st, bt.s);
    const size_t lds = sizeof(double) * (size_t)(POLISH_BLOCK + 2 * (bt.maxL_all + 64));
    cfg.timer->begin(3, st);
    hipLaunchKernelGGL(k_polish, dim3((unsigned int)total[PFX_POLISH]), dim3(POLISH_BLOCK), lds, st,
                       bt.s, bt.B, bt.pfx[PFX_POLISH]);
    cfg.timer->end(3, st);
    hipLaunchKernelGGL(k_polish_reduce, dim3(KP_MAX, bt.B), dim3(256), 0, st, bt.s);
    hipLaunchKernelGGL(k_round_end, dim3(bt.B), dim3(128), 0, st, bt.s);
    hipLaunchKernelGGL(k_remaining, dim3(1), dim3(256), 0, st, bt.s, bt.B, bt.remaining);
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
    Ctrl* c = S[0].ctrl;
    c->m = m;
    c->new_len = new_len;
    c->active = 1;
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
        hipLaunchKernelGGL(k_stats, dim3((unsigned int)total[PFX_ELEM]), dim3(256), 0, st, bt.s, 1,
                           bt.pfx[PFX_ELEM]);
    }
    return hipGetLastError();
}

// Sum of the per-series counters of a call (one block):
// out = {evals_sel, evals_ref, evals_pol, rounds, survivors, evals_near, evals_far}.
__global__ void k_sum_stats(SeriesDev* S, int B, unsigned long long* out)
{
    __shared__ unsigned long long acc[7];
    if (threadIdx.x < 7) acc[threadIdx.x] = 0ull;
    __syncthreads();
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
        const Ctrl* c = S[b].ctrl;
        atomicAdd(&acc[0], c->evals_sel);
        atomicAdd(&acc[1], c->evals_ref);
        atomicAdd(&acc[2], c->evals_pol);
        atomicAdd(&acc[3], c->rounds);
        atomicAdd(&acc[4], c->survivors);
        atomicAdd(&acc[5], c->evals_near);
        atomicAdd(&acc[6], c->evals_far);
    }
    __syncthreads();
    if (threadIdx.x < 7) out[threadIdx.x] = acc[threadIdx.x];
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
    mo[i] = s.mu[i];
    so[i] = sqrt(s.var[i]);
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
    l.npart = (l.Nmax + POLISH_BLOCK - 1) / POLISH_BLOCK;
    const size_t hl = (size_t)(l.Npad + 64);
    size_t o = 0;
    l.off_T = o;     o = al256(o + sizeof(double) * (size_t)l.Tlen);
    l.off_mu = o;    o = al256(o + sizeof(double) * hl);
    l.off_var = o;   o = al256(o + sizeof(double) * hl);
    l.off_h32 = o;   o = al256(o + 3 * al256(sizeof(float) * hl));
    l.off_h64 = o;   o = al256(o + 3 * al256(sizeof(double) * hl));
    l.off_alive = o; o = al256(o + sizeof(unsigned long long) * (size_t)l.nwords);
    l.off_rho = o;   o = al256(o + sizeof(unsigned long long) * (size_t)l.Npad);
    l.off_tsel = o;  o = al256(o + sizeof(int32_t) * (size_t)(l.Npad / 64 + 1));
    l.off_tref = o;  o = al256(o + sizeof(int32_t) * (size_t)(l.Npad / 64 + 1));
    l.off_surv = o;  o = al256(o + sizeof(int32_t) * (size_t)l.Npad);
    l.off_cand = o;  o = al256(o + sizeof(int64_t) * (size_t)KP_MAX);
    l.off_part = o;  o = al256(o + sizeof(double) * (size_t)(2 * KP_MAX * (l.npart + 1)));
    l.off_hist = o;  o = al256(o + sizeof(double) * (size_t)(l.L > 0 ? l.L : 1));
    l.off_ctrl = o;  o = al256(o + sizeof(Ctrl));
    l.off_red = o;   o = al256(o + sizeof(double) * 2 * RED_BLOCKS);
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
    s.df32 = (float*)(p + l.off_h32);
    s.dg32 = (float*)(p + l.off_h32 + al256(sizeof(float) * hl));
    s.inv32 = (float*)(p + l.off_h32 + 2 * al256(sizeof(float) * hl));
    s.df64 = (double*)(p + l.off_h64);
    s.dg64 = (double*)(p + l.off_h64 + al256(sizeof(double) * hl));
    s.inv64 = (double*)(p + l.off_h64 + 2 * al256(sizeof(double) * hl));
    s.alive = (unsigned long long*)(p + l.off_alive);
    s.rho = (unsigned long long*)(p + l.off_rho);
    s.tsel = (int32_t*)(p + l.off_tsel);
    s.tref = (int32_t*)(p + l.off_tref);
    s.surv = (int32_t*)(p + l.off_surv);
    s.cand = (int64_t*)(p + l.off_cand);
    s.part = (double*)(p + l.off_part);
    s.hist = (double*)(p + l.off_hist);
    s.ctrl = (Ctrl*)(p + l.off_ctrl);
    s.red = (double*)(p + l.off_red);
    return s;
}

void series_blocks(const Layout& l, const SweepCfg& cfg, int64_t out[PFX_KINDS])
{
    const int rn = 64 * cfg.q_near, rf = 64 * cfg.q_far, rr = 64 * cfg.q_ref;
    const int nsub = (cfg.near_cols + cfg.chunk_cols - 1) / cfg.chunk_cols;
    out[PFX_ELEM] = (l.Npad + 64 + 255) / 256;
    out[PFX_NEAR] = ((l.Nmax + rn - 1) / rn) * nsub;
    out[PFX_TSEL] = ((l.Nmax + rf - 1) / rf + 255) / 256;
    out[PFX_TREF] = ((l.Nmax + rr - 1) / rr + 255) / 256;
    out[PFX_WORDS] = (l.nwords + 255) / 256;
    out[PFX_POLISH] = l.npart;
}

}  // namespace palmad
