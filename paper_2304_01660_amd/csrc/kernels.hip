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
//   * Column helpers (df, dg, 1/(sqrt(m) sigma)) are wave-uniform per step
//     and come through scalar loads.
//   * Row and column prunes are lane masks; a column prune is one ballot per
//     step, flushed to the candidate bitmap every 64 columns with one atomic.
//   * Long scans are split into column chunks fed from a device work list in
//     nearest-first order, so the critical path is one chunk, not one row.
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
// per-length statistics (Eq. (4) at minL, Eq. (7)-(8) after) and helpers
// ---------------------------------------------------------------------------
__global__ void k_stats_init(const double* __restrict__ T, int64_t n, int32_t m, int64_t len,
                             double* __restrict__ mu, double* __restrict__ var, Ctrl* ctrl)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        ctrl->flat_min = 0x7fffffffffffffffll;
        ctrl->flat_max = -1;
    }
    if (i >= len) return;
    const int64_t N = n - m + 1;
    if (i >= N) {
        mu[i] = 0.0;
        var[i] = 0.0;
        return;
    }
    double s = 0.0;
    for (int k = 0; k < m; ++k) s += T[i + k];
    const double mean = s / (double)m;
    double q = 0.0;
    for (int k = 0; k < m; ++k) {
        const double d = T[i + k] - mean;
        q += d * d;
    }
    mu[i] = mean;
    var[i] = q / (double)m;
}

// Statistics of length m+1 from length m, in place (Eq. (7)-(8)).
__global__ void k_stats_update(const double* __restrict__ T, int64_t n, int32_t m, int64_t len,
                               double* __restrict__ mu, double* __restrict__ var, Ctrl* ctrl)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        ctrl->flat_min = 0x7fffffffffffffffll;
        ctrl->flat_max = -1;
    }
    if (i >= len) return;
    const int64_t N1 = n - m;  // windows of length m+1
    if (i >= N1) {
        mu[i] = 0.0;
        var[i] = 0.0;
        return;
    }
    const double t = T[i + m];
    const double mo = mu[i];
    const double dm = (double)m;
    const double d = mo - t;
    mu[i] = (dm * mo + t) / (dm + 1.0);
    var[i] = dm / (dm + 1.0) * (var[i] + d * d / (dm + 1.0));
}

// df[i] = (t_{i+m} - t_i)/2, dg[i] = (t_{i+m} - mu_{i+1}) + (t_i - mu_i) for
// i < N-1 (zero beyond), inv[i] = 1/(sqrt(m) sigma_i) for non-flat i < N.
__global__ void k_helpers(const double* __restrict__ T, int64_t n, int32_t m, int64_t len,
                          const double* __restrict__ mu, const double* __restrict__ var,
                          float* __restrict__ df32, float* __restrict__ dg32,
                          float* __restrict__ inv32, double* __restrict__ df64,
                          double* __restrict__ dg64, double* __restrict__ inv64, Ctrl* ctrl)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    const int64_t N = n - m + 1;
    double df = 0.0, dg = 0.0, inv = 0.0;
    if (i < N - 1) {
        const double a = T[i + m], c = T[i];
        df = (a - c) * 0.5;
        dg = (a - mu[i + 1]) + (c - mu[i]);
    }
    if (i < N) {
        const double sg = sqrt(var[i]);
        if (sg <= ctrl->flat_eps) {
            atomicMin((long long*)&ctrl->flat_min, (long long)i);
            atomicMax((long long*)&ctrl->flat_max, (long long)i);
        } else {
            inv = 1.0 / (sqrt((double)m) * sg);
        }
    }
    df64[i] = df;
    dg64[i] = dg;
    inv64[i] = inv;
    df32[i] = (float)df;
    dg32[i] = (float)dg;
    inv32[i] = (float)inv;
}

hipError_t launch_stats(const Layout& lay, const Buffers& b, int32_t m, bool init, hipStream_t st)
{
    const int64_t len = lay.Npad + 64;
    const int blocks = (int)((len + 255) / 256);
    if (init)
        hipLaunchKernelGGL(k_stats_init, dim3(blocks), dim3(256), 0, st, b.T, lay.n, m, len, b.mu,
                           b.var, b.ctrl);
    else
        hipLaunchKernelGGL(k_stats_update, dim3(blocks), dim3(256), 0, st, b.T, lay.n, m - 1, len,
                           b.mu, b.var, b.ctrl);
    hipLaunchKernelGGL(k_helpers, dim3(blocks), dim3(256), 0, st, b.T, lay.n, m, len, b.mu, b.var,
                       b.df32, b.dg32, b.inv32, b.df64, b.dg64, b.inv64, b.ctrl);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// round control (MERLIN's r, Alg. 1) and per-round reset
// ---------------------------------------------------------------------------
__global__ void k_round_begin(Ctrl* c, const double* hist, int32_t m, int32_t li, int32_t minL,
                              int attempt, float guard, int64_t N, int64_t Npad,
                              unsigned long long* alive, unsigned long long* rho, int64_t nwords)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g == 0) {
        if (attempt == 0) {
            c->done = 0;
            if (c->mode != 3) {
                if (li == 0) {
                    c->mode = 0;
                    c->r = 2.0 * sqrt((double)minL);
                } else if (li <= 4) {
                    c->mode = 1;
                    c->r = 0.99 * hist[li - 1];
                } else {
                    double mean = 0.0;
                    for (int q = 1; q <= 5; ++q) mean += hist[li - q];
                    mean /= 5.0;
                    double v = 0.0;
                    for (int q = 1; q <= 5; ++q) {
                        const double d = hist[li - q] - mean;
                        v += d * d;
                    }
                    c->step = sqrt(v / 5.0);
                    c->r = mean - 2.0 * c->step;
                    c->mode = 2;
                }
            }
        }
        const double r = c->r;
        c->m = m;
        c->li = li;
        c->prune = r > 0.0 ? 1 : 0;
        c->thr64 = r > 0.0 ? 1.0 - r * r / (2.0 * (double)m) : 2.0;
        c->thr_sel = c->thr64 + (double)guard;
        // round up: an FP32 threshold must never prune more than thr_sel
        c->thr32 = __double2float_ru(c->thr_sel);
        c->nlive_sel = c->maxc_sel = c->ctr_sel = 0;
        c->nlive_ref = c->maxc_ref = c->ctr_ref = 0;
        c->nsurv = 0;
        c->ncand = 0;
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t w = g; w < nwords; w += stride) {
        const int64_t lo = w * 64;
        unsigned long long bits = 0ull;
        if (lo + 64 <= N) bits = ~0ull;
        else if (lo < N) bits = (1ull << (N - lo)) - 1ull;
        alive[w] = bits;
    }
    const unsigned long long neg = 0x000fffffffffffffull;  // ordered bits of -inf
    for (int64_t i = g; i < Npad; i += stride) rho[i] = neg;
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

// First selection pass: every row tile's nearest near_cols columns, split
// into chunks of `chunk` columns that run concurrently (blockIdx.y); each
// stops as soon as the whole tile is dead.
template <typename F, int Q>
__global__ __launch_bounds__(64) void k_select_near(SweepArgs<F> A, int near_cols, int chunk)
{
    extern __shared__ double lds[];
    const Ctrl* c = A.ctrl;
    if (!c->prune) return;
    constexpr int R = 64 * Q;
    const int64_t i0 = (int64_t)blockIdx.x * R;
    if (i0 >= A.N) return;
    const int64_t j00 = i0 + A.m;
    const int64_t jbeg = j00 + (int64_t)blockIdx.y * chunk;
    if (jbeg >= A.N || jbeg >= j00 + near_cols) return;
    const int64_t jend = std::min<int64_t>(std::min<int64_t>(A.N, jbeg + chunk), j00 + near_cols);
    const F thr = sel_threshold<F>(c);
    unsigned long long ev = 0;
    sel_item<F, Q>(A, i0, jbeg, jend, thr, lds, ev);
    if (threadIdx.x == 0 && ev) {
        atomicAdd(&A.ctrl->evals_sel, ev);
        atomicAdd(&A.ctrl->evals_near, ev);
    }
}

template <typename F, int Q>
__global__ __launch_bounds__(64) void k_select_far(SweepArgs<F> A, const int32_t* __restrict__ tiles,
                                                   int near_cols, int chunk)
{
    extern __shared__ double lds[];
    Ctrl* c = A.ctrl;
    if (!c->prune) return;
    constexpr int R = 64 * Q;
    const unsigned int nlive = c->nlive_sel;
    const unsigned long long total = (unsigned long long)nlive * c->maxc_sel;
    const F thr = sel_threshold<F>(c);
    unsigned long long ev = 0;
    for (;;) {
        unsigned int it = 0;
        if (threadIdx.x == 0) it = atomicAdd(&c->ctr_sel, 1u);
        it = __builtin_amdgcn_readfirstlane(it);
        if ((unsigned long long)it >= total) break;
        const unsigned int cc = it / nlive, p = it % nlive;
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

// Live-tile lists.  mode 0: selection tiles (R rows), chunks to the right
// beyond the first pass; mode 1: refinement tiles, chunks on both sides.
__global__ void k_tiles(const unsigned long long* __restrict__ alive, int64_t N, int32_t m, int R,
                        int mode, int near_cols, int chunk, int32_t* list, Ctrl* c)
{
    if (mode == 0 && !c->prune) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ntiles = (N + R - 1) / R;
    if (t >= ntiles) return;
    const int words = R / 64;
    unsigned long long any = 0ull;
    for (int w = 0; w < words; ++w) any |= alive[t * words + w];
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
    list[slot] = (int32_t)t;
    atomicMax(mode == 0 ? &c->maxc_sel : &c->maxc_ref, (unsigned int)nch);
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

template <int Q>
__global__ __launch_bounds__(64) void k_refine(SweepArgs<double> A, const int32_t* __restrict__ tiles,
                                               int chunk)
{
    extern __shared__ double lds[];
    Ctrl* c = A.ctrl;
    constexpr int R = 64 * Q;
    const unsigned int nlive = c->nlive_ref;
    const unsigned long long total = (unsigned long long)nlive * c->maxc_ref;
    const double thr = c->thr64;
    const int prune = c->prune;
    unsigned long long ev = 0;
    for (;;) {
        unsigned int it = 0;
        if (threadIdx.x == 0) it = atomicAdd(&c->ctr_ref, 1u);
        it = __builtin_amdgcn_readfirstlane(it);
        if ((unsigned long long)it >= total) break;
        const unsigned int cc = it / nlive, p = it % nlive;
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


// Survivor list: every row whose bit is still set.
__global__ void k_survivors(const unsigned long long* __restrict__ alive, int64_t nwords,
                            int32_t* surv, Ctrl* c)
{
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nwords) return;
    unsigned long long bits = alive[w];
    const int cnt = __popcll(bits);
    if (!cnt) return;
    unsigned int base = atomicAdd(&c->nsurv, (unsigned int)cnt);
    while (bits) {
        const int t = __ffsll((long long)bits) - 1;
        surv[base++] = (int32_t)(w * 64 + t);
        bits &= bits - 1ull;
    }
}

template <typename F>
static SweepArgs<F> sweep_args(const Layout& lay, const Buffers& b, int32_t m);
template <>
SweepArgs<float> sweep_args<float>(const Layout& lay, const Buffers& b, int32_t m)
{
    SweepArgs<float> A;
    A.T = b.T;
    A.mu = b.mu;
    A.df = b.df32;
    A.dg = b.dg32;
    A.inv = b.inv32;
    A.alive = b.alive;
    A.rho = b.rho;
    A.ctrl = b.ctrl;
    A.N = lay.n - m + 1;
    A.m = m;
    return A;
}
template <>
SweepArgs<double> sweep_args<double>(const Layout& lay, const Buffers& b, int32_t m)
{
    SweepArgs<double> A;
    A.T = b.T;
    A.mu = b.mu;
    A.df = b.df64;
    A.dg = b.dg64;
    A.inv = b.inv64;
    A.alive = b.alive;
    A.rho = b.rho;
    A.ctrl = b.ctrl;
    A.N = lay.n - m + 1;
    A.m = m;
    return A;
}

template <typename F, int Q>
static void launch_near(const Layout& lay, const Buffers& b, const SweepCfg& cfg, int32_t m,
                        hipStream_t st)
{
    constexpr int R = 64 * Q;
    const SweepArgs<F> A = sweep_args<F>(lay, b, m);
    const size_t lds = sizeof(double) * sweep_lds_doubles(m);
    const int ntiles = (int)((A.N + R - 1) / R);
    const int nsub = (cfg.near_cols + cfg.chunk_cols - 1) / cfg.chunk_cols;
    cfg.timer->begin(0, st);
    hipLaunchKernelGGL((k_select_near<F, Q>), dim3(ntiles, nsub), dim3(64), lds, st, A,
                       cfg.near_cols, cfg.chunk_cols);
    cfg.timer->end(0, st);
}

template <typename F, int Q>
static void launch_far(const Layout& lay, const Buffers& b, const SweepCfg& cfg, int32_t m,
                       hipStream_t st)
{
    constexpr int R = 64 * Q;
    const SweepArgs<F> A = sweep_args<F>(lay, b, m);
    const size_t lds = sizeof(double) * sweep_lds_doubles(m);
    const int ntiles = (int)((A.N + R - 1) / R);
    hipLaunchKernelGGL(k_tiles, dim3((ntiles + 255) / 256), dim3(256), 0, st, b.alive, A.N, m, R, 0,
                       cfg.near_cols, cfg.chunk_cols, b.tsel, b.ctrl);
    cfg.timer->begin(1, st);
    hipLaunchKernelGGL((k_select_far<F, Q>), dim3(cfg.far_grid), dim3(64), lds, st, A, b.tsel,
                       cfg.near_cols, cfg.chunk_cols);
    cfg.timer->end(1, st);
}

template <int Q>
static void launch_refine(const Layout& lay, const Buffers& b, const SweepCfg& cfg, int32_t m,
                          hipStream_t st)
{
    constexpr int R = 64 * Q;
    const SweepArgs<double> A = sweep_args<double>(lay, b, m);
    const int ntiles = (int)((A.N + R - 1) / R);
    hipLaunchKernelGGL(k_tiles, dim3((ntiles + 255) / 256), dim3(256), 0, st, b.alive, A.N, m, R, 1,
                       0, cfg.chunk_cols, b.tref, b.ctrl);
    const size_t lds = sizeof(double) * sweep_lds_doubles(m);
    cfg.timer->begin(2, st);
    hipLaunchKernelGGL((k_refine<Q>), dim3(cfg.far_grid), dim3(64), lds, st, A, b.tref,
                       cfg.chunk_cols);
    cfg.timer->end(2, st);
}

// Row tiles of 128, 256 or 512 subsequences (Q = 2, 4, 8 rows per lane).
template <typename F>
static void launch_select(const Layout& lay, const Buffers& b, const SweepCfg& cfg, int32_t m,
                          hipStream_t st)
{
    switch (cfg.q_near) {
    case 2: launch_near<F, 2>(lay, b, cfg, m, st); break;
    case 4: launch_near<F, 4>(lay, b, cfg, m, st); break;
    default: launch_near<F, 8>(lay, b, cfg, m, st); break;
    }
    switch (cfg.q_far) {
    case 2: launch_far<F, 2>(lay, b, cfg, m, st); break;
    case 4: launch_far<F, 4>(lay, b, cfg, m, st); break;
    default: launch_far<F, 8>(lay, b, cfg, m, st); break;
    }
}

hipError_t launch_round(const Layout& lay, const Buffers& b, const SweepCfg& cfg, int32_t m,
                        int attempt, hipStream_t st)
{
    const int64_t N = lay.n - m + 1;
    {
        const int64_t work = std::max<int64_t>(lay.nwords, lay.Npad);
        const int blocks = (int)std::min<int64_t>(2048, (work + 255) / 256);
        hipLaunchKernelGGL(k_round_begin, dim3(blocks), dim3(256), 0, st, b.ctrl, b.hist, m,
                           m - lay.minL, lay.minL, attempt, cfg.guard, N, lay.Npad, b.alive, b.rho,
                           lay.nwords);
    }
    if (cfg.dist_bits == 64)
        launch_select<double>(lay, b, cfg, m, st);
    else
        launch_select<float>(lay, b, cfg, m, st);
    switch (cfg.q_ref) {
    case 4: launch_refine<4>(lay, b, cfg, m, st); break;
    case 8: launch_refine<8>(lay, b, cfg, m, st); break;
    default: launch_refine<2>(lay, b, cfg, m, st); break;
    }
    {
        const int64_t nw = (N + 63) / 64;
        hipLaunchKernelGGL(k_survivors, dim3((int)((nw + 255) / 256)), dim3(256), 0, st, b.alive,
                           nw, b.surv, b.ctrl);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// top-k candidates, exact FP64 polish, MERLIN bookkeeping
// ---------------------------------------------------------------------------
struct Key {
    unsigned long long u;  // ordered bits of rho (ascending rho = descending nnDist)
    long long i;
};
__device__ __forceinline__ bool key_less(const Key& x, const Key& y)
{
    return x.u < y.u || (x.u == y.u && x.i < y.i);
}

__global__ __launch_bounds__(TOPK_BLOCK) void k_topk(const int32_t* __restrict__ surv,
                                                     const unsigned long long* __restrict__ rho,
                                                     Ctrl* c, int k, int64_t* cand)
{
    __shared__ unsigned long long su[TOPK_BLOCK / 64];
    __shared__ long long si[TOPK_BLOCK / 64];
    const unsigned int ns = c->nsurv;
    if (ns < (unsigned int)k) {
        if (threadIdx.x == 0) c->ncand = 0;
        return;
    }
    const int kp = (int)min<unsigned int>(ns, (unsigned int)(k + KP_EXTRA));
    Key last = {0ull, -1};
    bool have_last = false;
    for (int r = 0; r < kp; ++r) {
        Key best = {~0ull, 0x7fffffffffffffffll};
        for (unsigned int s = threadIdx.x; s < ns; s += TOPK_BLOCK) {
            const long long i = surv[s];
            const Key x = {rho[i], i};
            if (have_last && !key_less(last, x)) continue;
            if (key_less(x, best)) best = x;
        }
        // wave reduce
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
            cand[r] = bb.i;
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
// consecutive columns, stages their windows in LDS once and evaluates every
// candidate against them; it writes one (max rho, argmax j) partial per
// candidate.
__global__ __launch_bounds__(POLISH_BLOCK) void k_polish(const double* __restrict__ T,
                                                         const double* __restrict__ mu,
                                                         const double* __restrict__ var, int64_t N,
                                                         int32_t m, const int64_t* __restrict__ cand,
                                                         Ctrl* c, double* part, int64_t npart)
{
    extern __shared__ double lds[];
    double* ts = lds;                        // T[j0 .. j0 + 256 + m + 64)
    double* xs = lds + POLISH_BLOCK + m + 64; // centred candidate window, zero padded
    __shared__ double sh[16];
    __shared__ double red_v[POLISH_BLOCK / 64];
    __shared__ long long red_j[POLISH_BLOCK / 64];
    const int ncand = (int)c->ncand;
    if (ncand == 0) return;
    const int tid = threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.x * POLISH_BLOCK;
    for (int t = tid; t < POLISH_BLOCK + m + 64; t += POLISH_BLOCK) ts[t] = T[j0 + t];
    const int64_t j = j0 + tid;
    const double feps = c->flat_eps;
    const bool colok = j < N;
    const double sgj = colok ? sqrt(var[j]) : 1.0;
    const double muj = colok ? mu[j] : 0.0;
    const bool flat_j = colok && sgj <= feps;
    unsigned long long ev = 0;
    for (int cid = 0; cid < ncand; ++cid) {
        const int64_t i = cand[cid];
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
            double rho;
            if (flat_i || flat_j) {
                rho = (flat_i && flat_j) ? 1.0 : 0.0;
            } else {
                const double* t = ts + tid;
                double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
                for (int k = 0; k < m; k += 4) {
                    a0 = fma(xs[k], t[k], a0);
                    a1 = fma(xs[k + 1], t[k + 1], a1);
                    a2 = fma(xs[k + 2], t[k + 2], a2);
                    a3 = fma(xs[k + 3], t[k + 3], a3);
                }
                const double C = (a0 + a1) + (a2 + a3) - muj * Sx;
                rho = C / ((double)m * sgi * sgj);
                rho = fmin(1.0, fmax(-1.0, rho));
            }
            best = rho;
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
            const int64_t slot = ((int64_t)cid * npart + blockIdx.x) * 2;
            part[slot] = best;
            part[slot + 1] = (double)bj;
        }
    }
    ev = (unsigned long long)wave_sum((double)ev);
    if ((tid & 63) == 0 && ev) atomicAdd(&c->evals_pol, ev);
}

// Reduce the polish partials of each candidate to (rho, j) in part's tail.
__global__ void k_polish_reduce(double* part, int64_t npart, Ctrl* c)
{
    __shared__ double rv[4];
    __shared__ double rj[4];
    const int cid = blockIdx.x;
    if ((unsigned int)cid >= c->ncand) return;
    double best = -f_inf<double>(), bj = 1e300;
    for (int64_t p = threadIdx.x; p < npart; p += blockDim.x) {
        const double v = part[((int64_t)cid * npart + p) * 2];
        const double jj = part[((int64_t)cid * npart + p) * 2 + 1];
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
        part[tail + cid * 2] = best;
        part[tail + cid * 2 + 1] = bj;
    }
}

// Rank the polished candidates, write the length's top-k rows when the round
// found at least k range discords, and advance MERLIN's r otherwise.
__global__ void k_round_end(const int64_t* __restrict__ cand, const double* __restrict__ part,
                            int64_t npart, Ctrl* c, double* hist, int32_t m, int32_t li, int k,
                            int64_t* idx, int32_t* len, double* nn, int64_t* nnidx, int32_t* count)
{
    __shared__ double nn_s[KP_MAX];
    __shared__ long long id_s[KP_MAX];
    __shared__ long long jj_s[KP_MAX];
    const unsigned int ns = c->nsurv;
    const int kp = (int)c->ncand;
    const bool ok = ns >= (unsigned int)k && kp >= k;
    const int64_t tail = (int64_t)KP_MAX * npart * 2;
    const int t = threadIdx.x;
    if (ok && t < kp) {
        const double rho = part[tail + t * 2];
        const double d2 = 2.0 * (double)m * (1.0 - rho);
        nn_s[t] = sqrt(fmin(4.0 * (double)m, fmax(0.0, d2)));
        id_s[t] = cand[t];
        jj_s[t] = (long long)part[tail + t * 2 + 1];
    }
    __syncthreads();
    if (ok && t < kp) {
        int rank = 0;
        for (int q = 0; q < kp; ++q)
            if (nn_s[q] > nn_s[t] || (nn_s[q] == nn_s[t] && id_s[q] < id_s[t])) ++rank;
        if (rank < k) {
            const int64_t row = (int64_t)li * k + rank;
            idx[row] = id_s[t];
            len[row] = m;
            nn[row] = nn_s[t];
            nnidx[row] = jj_s[t];
            if (rank == k - 1) hist[li] = nn_s[t];
        }
    }
    __syncthreads();
    if (t == 0) {
        c->rounds += 1;
        if (ok) {
            c->done = 1;
            c->survivors += ns;
            if (count) count[li] = (int32_t)ns;
        } else {
            c->done = 0;
            if (c->mode == 0) c->r *= 0.5;
            else if (c->mode == 1) c->r *= 0.99;
            else if (c->mode == 2) c->r = (c->step > 0.0) ? c->r - c->step : 0.99 * c->r;
        }
    }
}

hipError_t launch_finish_length(const Layout& lay, const Buffers& b, const SweepCfg& cfg, int32_t m,
                                int64_t* idx, int32_t* len, double* nn, int64_t* nnidx,
                                int32_t* count, hipStream_t st)
{
    const int64_t N = lay.n - m + 1;
    hipLaunchKernelGGL(k_topk, dim3(1), dim3(TOPK_BLOCK), 0, st, b.surv, b.rho, b.ctrl, lay.k,
                       b.cand);
    const size_t lds = sizeof(double) * (size_t)(POLISH_BLOCK + 2 * (m + 64));
    cfg.timer->begin(3, st);
    hipLaunchKernelGGL(k_polish, dim3((unsigned int)lay.npart), dim3(POLISH_BLOCK), lds, st, b.T,
                       b.mu, b.var, N, m, b.cand, b.ctrl, b.part, lay.npart);
    cfg.timer->end(3, st);
    hipLaunchKernelGGL(k_polish_reduce, dim3(lay.kp), dim3(256), 0, st, b.part, lay.npart, b.ctrl);
    hipLaunchKernelGGL(k_round_end, dim3(1), dim3(KP_MAX < 64 ? 64 : 128), 0, st, b.cand, b.part,
                       lay.npart, b.ctrl, b.hist, m, m - lay.minL, lay.k, idx, len, nn, nnidx,
                       count);
    return hipGetLastError();
}

__global__ void k_set_fixed_r(Ctrl* c, double r)
{
    c->mode = 3;
    c->r = r;
}

__global__ void k_set_max_len(Ctrl* c, int32_t maxm) { c->m = maxm; }

hipError_t launch_set_max_len(const Buffers& b, int32_t maxm, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_max_len, dim3(1), dim3(1), 0, st, b.ctrl, maxm);
    return hipGetLastError();
}

hipError_t launch_set_fixed_r(const Buffers& b, double r, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_fixed_r, dim3(1), dim3(1), 0, st, b.ctrl, r);
    return hipGetLastError();
}

__global__ void k_range_out(const unsigned long long* __restrict__ alive,
                            const unsigned long long* __restrict__ rho, int64_t N, int32_t m,
                            unsigned long long* alive_out, double* nn_out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const bool on = (alive[i >> 6] >> (i & 63)) & 1ull;
    if ((i & 63) == 0) alive_out[i >> 6] = alive[i >> 6];
    double d = 0.0;
    if (on) {
        const double r = dbl_of(rho[i]);
        d = sqrt(fmin(4.0 * (double)m, fmax(0.0, 2.0 * (double)m * (1.0 - r))));
    }
    nn_out[i] = d;
}

hipError_t launch_range_out(const Layout& lay, const Buffers& b, int32_t m,
                            unsigned long long* alive_out, double* nn_out, hipStream_t st)
{
    const int64_t N = lay.n - m + 1;
    hipLaunchKernelGGL(k_range_out, dim3((int)((N + 255) / 256)), dim3(256), 0, st, b.alive, b.rho,
                       N, m, alive_out, nn_out);
    return hipGetLastError();
}

__global__ void k_stats_out(const double* __restrict__ mu, const double* __restrict__ var, int64_t N,
                            double* mo, double* so)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    mo[i] = mu[i];
    so[i] = sqrt(var[i]);
}

hipError_t launch_stats_out(const Layout& lay, const Buffers& b, int32_t m, double* mu,
                            double* sigma, hipStream_t st)
{
    const int64_t N = lay.n - m + 1;
    hipLaunchKernelGGL(k_stats_out, dim3((int)((N + 255) / 256)), dim3(256), 0, st, b.mu, b.var, N,
                       mu, sigma);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

bool make_layout(int64_t n, int32_t minL, int32_t maxL, int32_t k, int32_t dist_bits, Layout* out)
{
    Layout l = {};
    l.n = n;
    l.minL = minL;
    l.maxL = maxL;
    l.k = k;
    l.L = maxL - minL + 1;
    l.kp = k + KP_EXTRA;
    l.dist_bits = dist_bits;
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
    l.off_hist = o;  o = al256(o + sizeof(double) * (size_t)l.L);
    l.off_flat = o;  o = al256(o + sizeof(int64_t) * 2);
    l.off_ctrl = o;  o = al256(o + sizeof(Ctrl));
    l.off_red = o;   o = al256(o + sizeof(double) * 2 * RED_BLOCKS);
    l.total = o;
    *out = l;
    return true;
}

Buffers carve(void* ws, const Layout& l)
{
    char* p = (char*)ws;
    const size_t hl = (size_t)(l.Npad + 64);
    Buffers b;
    b.T = (double*)(p + l.off_T);
    b.mu = (double*)(p + l.off_mu);
    b.var = (double*)(p + l.off_var);
    b.df32 = (float*)(p + l.off_h32);
    b.dg32 = (float*)(p + l.off_h32 + al256(sizeof(float) * hl));
    b.inv32 = (float*)(p + l.off_h32 + 2 * al256(sizeof(float) * hl));
    b.df64 = (double*)(p + l.off_h64);
    b.dg64 = (double*)(p + l.off_h64 + al256(sizeof(double) * hl));
    b.inv64 = (double*)(p + l.off_h64 + 2 * al256(sizeof(double) * hl));
    b.alive = (unsigned long long*)(p + l.off_alive);
    b.rho = (unsigned long long*)(p + l.off_rho);
    b.tsel = (int32_t*)(p + l.off_tsel);
    b.tref = (int32_t*)(p + l.off_tref);
    b.surv = (int32_t*)(p + l.off_surv);
    b.cand = (int64_t*)(p + l.off_cand);
    b.part = (double*)(p + l.off_part);
    b.hist = (double*)(p + l.off_hist);
    b.flat = (int64_t*)(p + l.off_flat);
    b.ctrl = (Ctrl*)(p + l.off_ctrl);
    b.red = (double*)(p + l.off_red);
    return b;
}

}  // namespace palmad
