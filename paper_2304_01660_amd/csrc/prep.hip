// Series preparation kernels: padded FP64 copy, finiteness check and the
// population sigma of the whole series (which sets the flat-window
// threshold).  Built with full IEEE semantics, unlike the search kernels, so
// that NaN/Inf detection cannot be optimised away.  grid.y indexes the
// series of a batch.
#include "engine.h"

#include <math.h>

#include <algorithm>

namespace palmad {

constexpr int RED_THREADS = 256;

__device__ __forceinline__ double wave_sum_p(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

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

__global__ void k_ctrl_init(SeriesDev* S)
{
    const SeriesDev& s = S[blockIdx.y];
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g == 0) {
        Ctrl z = {};
        z.flat_min = -1;
        z.flat_max = -1;
        *s.ctrl = z;
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = g; i < s.L; i += stride) s.hist[i] = 0.0;
    for (int64_t i = g; i < EV_CLASSES * EV_SLOTS; i += stride) s.evc[i] = 0ull;
    for (int64_t w = g; w < s.nwords; w += stride) {
        s.alive[w] = 0ull;
        s.twork[w] = 0u;
    }
}

__global__ void k_copy_sum(SeriesDev* S)
{
    const SeriesDev& s = S[blockIdx.y];
    __shared__ double sh[16];
    double acc = 0.0;
    int bad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < s.Tlen; i += stride) {
        double v = 0.0;
        if (i < s.n) {
            v = s.Tin[i];
            if (!isfinite(v)) {
                bad = 1;
                v = 0.0;
            }
            acc += v;
        }
        s.T[i] = v;
    }
    const double t = block_sum_p(acc, sh);
    if (threadIdx.x == 0) s.red[blockIdx.x] = t;
    if (bad) atomicOr(&s.ctrl->nonfinite, 1);
}

__global__ void k_sqdev(SeriesDev* S)
{
    const SeriesDev& s = S[blockIdx.y];
    __shared__ double sh[16];
    __shared__ double mean_s;
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < RED_BLOCKS; ++i) t += s.red[i];
        mean_s = t / (double)s.n;
    }
    __syncthreads();
    const double mean = mean_s;
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < s.n; i += stride) {
        const double d = s.T[i] - mean;
        acc += d * d;
    }
    const double t = block_sum_p(acc, sh);
    if (threadIdx.x == 0) s.red[RED_BLOCKS + blockIdx.x] = t;
}

__global__ void k_sigma_final(SeriesDev* S)
{
    const SeriesDev& s = S[blockIdx.x];
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < RED_BLOCKS; ++i) t += s.red[RED_BLOCKS + i];
        const double sg = sqrt(t / (double)s.n);
        s.ctrl->sigmaT = sg;
        s.ctrl->flat_eps = 1e-12 * (sg > 1.0 ? sg : 1.0);
    }
}

hipError_t launch_ctrl_init(const Batch& bt, hipStream_t st)
{
    hipLaunchKernelGGL(k_ctrl_init, dim3(64, bt.B), dim3(256), 0, st, bt.s);
    return hipGetLastError();
}

hipError_t launch_prepare(const Batch& bt, const int64_t* total, hipStream_t st)
{
    (void)total;
    hipLaunchKernelGGL(k_ctrl_init, dim3(64, bt.B), dim3(256), 0, st, bt.s);
    hipLaunchKernelGGL(k_copy_sum, dim3(RED_BLOCKS, bt.B), dim3(RED_THREADS), 0, st, bt.s);
    hipLaunchKernelGGL(k_sqdev, dim3(RED_BLOCKS, bt.B), dim3(RED_THREADS), 0, st, bt.s);
    hipLaunchKernelGGL(k_sigma_final, dim3(bt.B), dim3(64), 0, st, bt.s);
    return hipGetLastError();
}

// Streaming appends (one series): the appended values' finiteness, their
// copy into the padded series at n_old, and the sum of the first s.n values
// in the same order as k_copy_sum, so that sigma of the series (hence the
// flat threshold) equals that of a search over the same values.
__global__ void k_check_finite(const double* __restrict__ src, int64_t count, int32_t* out)
{
    __shared__ int bad_s;
    if (threadIdx.x == 0) bad_s = 0;
    __syncthreads();
    int bad = 0;
    for (int64_t i = threadIdx.x; i < count; i += blockDim.x) bad |= !isfinite(src[i]);
    if (bad) atomicOr(&bad_s, 1);
    __syncthreads();
    if (threadIdx.x == 0) out[0] = bad_s;
}

__global__ void k_stream_copy(SeriesDev* S, const double* __restrict__ src, int64_t n_old,
                              int64_t count)
{
    const SeriesDev& s = S[0];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        s.T[n_old + i] = src[i];
}

__global__ void k_stream_sum(SeriesDev* S)
{
    const SeriesDev& s = S[0];
    __shared__ double sh[16];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < s.n; i += stride)
        acc += s.T[i];
    const double t = block_sum_p(acc, sh);
    if (threadIdx.x == 0) s.red[blockIdx.x] = t;
}

hipError_t launch_check_finite(const double* src, int64_t count, int32_t* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_check_finite, dim3(1), dim3(1024), 0, st, src, count, out);
    return hipGetLastError();
}

hipError_t launch_stream_append(const Batch& bt, const double* src, int64_t n_old, int64_t count,
                                hipStream_t st)
{
    hipLaunchKernelGGL(k_stream_copy, dim3(256), dim3(256), 0, st, bt.s, src, n_old, count);
    hipLaunchKernelGGL(k_stream_sum, dim3(RED_BLOCKS, 1), dim3(RED_THREADS), 0, st, bt.s);
    hipLaunchKernelGGL(k_sqdev, dim3(RED_BLOCKS, 1), dim3(RED_THREADS), 0, st, bt.s);
    hipLaunchKernelGGL(k_sigma_final, dim3(1), dim3(64), 0, st, bt.s);
    return hipGetLastError();
}

__global__ void k_nonfinite(SeriesDev* S, int B, int32_t* out)
{
    __shared__ int cnt, first;
    if (threadIdx.x == 0) {
        cnt = 0;
        first = 0x7fffffff;
    }
    __syncthreads();
    for (int b = threadIdx.x; b < B; b += blockDim.x)
        if (S[b].ctrl->nonfinite) {
            atomicAdd(&cnt, 1);
            atomicMin(&first, b);
        }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = cnt;
        out[1] = cnt ? first : -1;
    }
}

hipError_t launch_nonfinite(const Batch& bt, int32_t* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_nonfinite, dim3(1), dim3(256), 0, st, bt.s, bt.B, out);
    return hipGetLastError();
}

}  // namespace palmad
