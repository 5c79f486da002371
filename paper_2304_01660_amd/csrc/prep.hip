// Series preparation kernels: padded FP64 copy, finiteness check and the
// population sigma of the whole series (which sets the flat-window
// threshold).  Built with full IEEE semantics, unlike the sweep kernels, so
// that NaN/Inf detection cannot be optimised away.
#include "engine.h"

#include <math.h>

#include <algorithm>

namespace palmad {

__device__ __forceinline__ double wave_sum_p(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// ---------------------------------------------------------------------------
// preparation: padded FP64 copy, finiteness, sigma of the series
// ---------------------------------------------------------------------------
constexpr int RED_THREADS = 256;

__device__ double block_sum_p(double v, double* sh)
{
    v = wave_sum_p(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
    __syncthreads();
    return t;  // valid in thread 0
}

__global__ void k_ctrl_init(Ctrl* c, double* hist, int L, unsigned long long* alive, int64_t nwords)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g == 0) {
        Ctrl z = {};
        z.flat_min = -1;
        z.flat_max = -1;
        *c = z;
    }
    if (g < L) hist[g] = 0.0;
    for (int64_t w = g; w < nwords; w += (int64_t)gridDim.x * blockDim.x) alive[w] = 0ull;
}

__global__ void k_copy_sum(const double* __restrict__ Tu, int64_t n, double* __restrict__ T,
                           int64_t Tlen, double* red, Ctrl* ctrl)
{
    __shared__ double sh[16];
    double s = 0.0;
    int bad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < Tlen; i += stride) {
        double v = 0.0;
        if (i < n) {
            v = Tu[i];
            if (!isfinite(v)) {
                bad = 1;
                v = 0.0;
            }
            s += v;
        }
        T[i] = v;
    }
    const double t = block_sum_p(s, sh);
    if (threadIdx.x == 0) red[blockIdx.x] = t;
    if (bad) atomicOr(&ctrl->nonfinite, 1);
}

__global__ void k_sqdev(const double* __restrict__ T, int64_t n, double* red)
{
    __shared__ double sh[16];
    __shared__ double mean_s;
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < RED_BLOCKS; ++i) t += red[i];
        mean_s = t / (double)n;
    }
    __syncthreads();
    const double mean = mean_s;
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double d = T[i] - mean;
        s += d * d;
    }
    const double t = block_sum_p(s, sh);
    if (threadIdx.x == 0) red[RED_BLOCKS + blockIdx.x] = t;
}

__global__ void k_sigma_final(const double* red, int64_t n, Ctrl* ctrl)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < RED_BLOCKS; ++i) t += red[RED_BLOCKS + i];
        const double sg = sqrt(t / (double)n);
        ctrl->sigmaT = sg;
        ctrl->flat_eps = 1e-12 * (sg > 1.0 ? sg : 1.0);
    }
}

hipError_t launch_prepare(const Layout& lay, const Buffers& b, const double* T_user, hipStream_t st)
{
    const int64_t g = std::max<int64_t>(lay.L, 1);
    const int blocks = (int)std::min<int64_t>(1024, (std::max<int64_t>(g, lay.nwords) + 255) / 256);
    hipLaunchKernelGGL(k_ctrl_init, dim3(max(blocks, 1)), dim3(256), 0, st, b.ctrl, b.hist, lay.L,
                       b.alive, lay.nwords);
    hipLaunchKernelGGL(k_copy_sum, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st, T_user, lay.n, b.T,
                       lay.Tlen, b.red, b.ctrl);
    hipLaunchKernelGGL(k_sqdev, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st, b.T, lay.n, b.red);
    hipLaunchKernelGGL(k_sigma_final, dim3(1), dim3(64), 0, st, b.red, lay.n, b.ctrl);
    return hipGetLastError();
}

}  // namespace palmad
