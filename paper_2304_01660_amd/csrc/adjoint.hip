// Adjoint of the reported nearest-neighbour distances (backward pass).
//
// For a reported discord i of length m, nnDist = min over non-self matches j
// of ED(x^, y^), the z-normalised distance of Eq. (4)-(5).  Almost
// everywhere the minimiser j* is locally constant, so
//   d nnDist / d t_{i+k} = (rho * x^_k - y^_k) / (sigma_i * d)
//   d nnDist / d t_{j*+k} = (rho * y^_k - x^_k) / (sigma_j* * d)
// with d = nnDist and rho the Pearson correlation of the two windows
// (d^2 = 2m(1 - rho), Eq. (6)).  The minimiser is not stored by the forward
// pass: each row is recomputed here with direct FP64 dot products against
// every column (ties -> smallest j), then the gradient is scattered into
// grad_T with FP64 atomics.  A zero distance or a flat window contributes
// nothing (the distance is not differentiable there).
#include "engine.h"

#include <math.h>

#include <algorithm>

namespace palmad {

constexpr int ADJ_BLOCK = 256;

__device__ __forceinline__ double adj_wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Block-wide sum, result broadcast to every thread.
__device__ double adj_block_sum(double v, double* sh)
{
    v = adj_wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
    return t;
}

// Mean and population sigma of window [p, p+m) (two passes, block-wide).
__device__ void adj_window_stats(const double* T, int64_t p, int32_t m, double* sh, double& mu,
                                 double& sg)
{
    double s = 0.0;
    for (int k = threadIdx.x; k < m; k += blockDim.x) s += T[p + k];
    mu = adj_block_sum(s, sh) / (double)m;
    double q = 0.0;
    for (int k = threadIdx.x; k < m; k += blockDim.x) {
        const double d = T[p + k] - mu;
        q += d * d;
    }
    sg = sqrt(adj_block_sum(q, sh) / (double)m);
}

// Partial nearest neighbour of reported row q against the 256 columns of
// block x: (max rho, smallest argmax j).
__global__ __launch_bounds__(ADJ_BLOCK) void k_adj_rows(const double* __restrict__ T, int64_t n,
                                                        const int64_t* __restrict__ idx,
                                                        const int32_t* __restrict__ len,
                                                        const Ctrl* ctrl, double* part,
                                                        int64_t nblk)
{
    extern __shared__ double lds[];
    __shared__ double sh[8];
    __shared__ double rv[ADJ_BLOCK / 64];
    __shared__ long long rj[ADJ_BLOCK / 64];
    const int q = blockIdx.y;
    const int64_t i = idx[q];
    const int32_t m = len[q];
    const int64_t N = n - m + 1;
    const int64_t j0 = (int64_t)blockIdx.x * ADJ_BLOCK;
    const int tid = threadIdx.x;
    double best = -1e300;
    long long bj = 0x7fffffffffffffffll;
    const bool row_ok = m >= 3 && m <= ctrl->m && i >= 0 && i < N;  // ctrl->m holds max length
    if (row_ok && j0 < N) {
        double* xs = lds;              // centred window of row i, padded
        double* ts = lds + (m + 64);   // T[j0 .. j0 + 256 + m + 64)
        double mui, sgi;
        adj_window_stats(T, i, m, sh, mui, sgi);
        for (int k = tid; k < m + 64; k += ADJ_BLOCK) xs[k] = k < m ? T[i + k] - mui : 0.0;
        for (int t = tid; t < ADJ_BLOCK + m + 64; t += ADJ_BLOCK) ts[t] = T[j0 + t];
        __syncthreads();
        const double feps = ctrl->flat_eps;
        const bool flat_i = sgi <= feps;
        const int64_t j = j0 + tid;
        if (j < N && (j <= i - m || j >= i + m)) {
            const double* t = ts + tid;
            double s = 0.0;
            for (int k = 0; k < m; ++k) s += t[k];
            const double muj = s / (double)m;
            double v = 0.0, c0 = 0.0, c1 = 0.0;
            for (int k = 0; k < m; ++k) {
                const double dk = t[k] - muj;
                v = fma(dk, dk, v);
                if (k & 1) c1 = fma(xs[k], dk, c1);
                else c0 = fma(xs[k], dk, c0);
            }
            const double sgj = sqrt(v / (double)m);
            const bool flat_j = sgj <= feps;
            double rho;
            if (flat_i || flat_j) rho = (flat_i && flat_j) ? 1.0 : 0.0;
            else rho = fmin(1.0, fmax(-1.0, (c0 + c1) / ((double)m * sgi * sgj)));
            best = rho;
            bj = j;
        }
    }
    for (int o = 32; o >= 1; o >>= 1) {
        const double v = __shfl_xor(best, o);
        const long long jj = __shfl_xor(bj, o);
        if (v > best || (v == best && jj < bj)) {
            best = v;
            bj = jj;
        }
    }
    if ((tid & 63) == 0) {
        rv[tid >> 6] = best;
        rj[tid >> 6] = bj;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < ADJ_BLOCK / 64; ++w)
            if (rv[w] > best || (rv[w] == best && rj[w] < bj)) {
                best = rv[w];
                bj = rj[w];
            }
        const int64_t slot = ((int64_t)q * nblk + blockIdx.x) * 2;
        part[slot] = best;
        part[slot + 1] = bj == 0x7fffffffffffffffll ? 1e300 : (double)bj;  // 1e300: none
    }
}

// Per reported row: reduce the partials to j*, then scatter
// g * d nnDist / dT over both windows.
__global__ __launch_bounds__(ADJ_BLOCK) void k_adj_scatter(const double* __restrict__ T,
                                                           const int64_t* __restrict__ idx,
                                                           const int32_t* __restrict__ len,
                                                           const double* __restrict__ gin,
                                                           const Ctrl* ctrl, const double* part,
                                                           int64_t nblk, double* grad,
                                                           int64_t* jstar_out)
{
    __shared__ double sh[8];
    __shared__ double rv[ADJ_BLOCK / 64];
    __shared__ double rj[ADJ_BLOCK / 64];
    __shared__ double bcast[2];
    const int q = blockIdx.x;
    const int tid = threadIdx.x;
    double best = -1e300, bj = 1e300;
    for (int64_t p = tid; p < nblk; p += ADJ_BLOCK) {
        const double v = part[((int64_t)q * nblk + p) * 2];
        const double jj = part[((int64_t)q * nblk + p) * 2 + 1];
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
    if ((tid & 63) == 0) {
        rv[tid >> 6] = best;
        rj[tid >> 6] = bj;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < ADJ_BLOCK / 64; ++w)
            if (rv[w] > best || (rv[w] == best && rj[w] < bj)) {
                best = rv[w];
                bj = rj[w];
            }
        bcast[0] = best;
        bcast[1] = bj;
    }
    __syncthreads();
    const double rho = bcast[0];
    const bool found = bcast[1] < 1e299;
    const int64_t js = found ? (int64_t)bcast[1] : -1;
    const int64_t i = idx[q];
    const int32_t m = len[q];
    if (tid == 0 && jstar_out) jstar_out[q] = js;
    if (!found) return;
    const double g = gin[q];
    double mui, sgi, muj, sgj;
    adj_window_stats(T, i, m, sh, mui, sgi);
    adj_window_stats(T, js, m, sh, muj, sgj);
    const double feps = ctrl->flat_eps;
    const double d = sqrt(fmax(0.0, 2.0 * (double)m * (1.0 - rho)));
    if (!(d > 0.0) || sgi <= feps || sgj <= feps || g == 0.0) return;
    for (int k = tid; k < m; k += ADJ_BLOCK) {
        const double xh = (T[i + k] - mui) / sgi;
        const double yh = (T[js + k] - muj) / sgj;
        atomicAdd(&grad[i + k], g * (rho * xh - yh) / (sgi * d));
        atomicAdd(&grad[js + k], g * (rho * yh - xh) / (sgj * d));
    }
}

hipError_t launch_adjoint(const double* Tpad, int64_t n, int64_t K, int32_t maxm,
                          const int64_t* idx, const int32_t* len, const double* gin,
                          const Ctrl* ctrl, double* part, int64_t nblk, double* grad,
                          int64_t* jstar, hipStream_t st)
{
    if (K <= 0) return hipSuccess;
    const size_t lds = sizeof(double) * (size_t)(2 * (maxm + 64) + ADJ_BLOCK);
    hipLaunchKernelGGL(k_adj_rows, dim3((unsigned int)nblk, (unsigned int)K), dim3(ADJ_BLOCK), lds,
                       st, Tpad, n, idx, len, ctrl, part, nblk);
    hipLaunchKernelGGL(k_adj_scatter, dim3((unsigned int)K), dim3(ADJ_BLOCK), 0, st, Tpad, idx, len,
                       gin, ctrl, part, nblk, grad, jstar);
    return hipGetLastError();
}

}  // namespace palmad
