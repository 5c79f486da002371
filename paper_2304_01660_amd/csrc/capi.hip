// C ABI of the range-discord library (declared in include/palmad.h).
//
// Host side only: argument validation, workspace carving and the MERLIN
// driver loop (Alg. 1) over the lengths.  Each range search (one DRAG call of
// Alg. 2, parallelised as in Sec. 3.2-3.3) is a fixed sequence of kernel
// launches on the caller's stream; the driver reads one device flag per
// search to learn whether the length produced k discords.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/palmad.h"
#include "engine.h"

using namespace palmad;

struct palmad_ctx {
    int device;
    std::string err;
    int32_t* pinned;  // host-pinned flag mirror
    hipEvent_t ev[KCLASSES][2];
    bool have_events;
};

namespace {

thread_local std::string g_err;

int fail(palmad_ctx* ctx, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(palmad_ctx* ctx, int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(ctx, PALMAD_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

struct Opts {
    int dist_bits;
    float guard;
    int near_cols;
    int chunk_cols;
    unsigned int flags;
    int rows_near, rows_far, rows_refine;
    int far_grid;
};

int read_opts(palmad_ctx* ctx, const palmad_options* o, Opts* out)
{
    Opts r = {32, 1e-4f, 2048, 1024, 0u, 0, 0, 0, 2048};
    if (o) {
        if (o->flags & ~PALMAD_FLAG_TIME_KERNELS)
            return fail(ctx, PALMAD_EINVAL, "unknown option flags 0x%x", o->flags);
        r.flags = o->flags;
        const int32_t rows[3] = {o->rows_near, o->rows_far, o->rows_refine};
        for (int i = 0; i < 3; ++i)
            if (rows[i] != 0 && rows[i] != 128 && rows[i] != 256 && rows[i] != 512)
                return fail(ctx, PALMAD_EINVAL, "tile rows must be 0, 128, 256 or 512 (got %d)",
                            rows[i]);
        r.rows_near = o->rows_near;
        r.rows_far = o->rows_far;
        r.rows_refine = o->rows_refine;
        if (o->far_grid < 0 || o->far_grid > 65536)
            return fail(ctx, PALMAD_EINVAL, "far_grid must be in [0, 65536] (got %d)", o->far_grid);
        if (o->far_grid > 0) r.far_grid = o->far_grid;
        for (int i = 0; i < 3; ++i)
            if (o->reserved[i] != 0) return fail(ctx, PALMAD_EINVAL, "options.reserved must be zero");
        if (o->dist_bits != 0) {
            if (o->dist_bits != 32 && o->dist_bits != 64)
                return fail(ctx, PALMAD_EINVAL, "dist_bits must be 0, 32 or 64 (got %d)",
                            o->dist_bits);
            r.dist_bits = o->dist_bits;
        }
        if (o->guard > 0.0f) r.guard = o->guard;
        if (o->near_cols < 0 || o->chunk_cols < 0)
            return fail(ctx, PALMAD_EINVAL, "near_cols and chunk_cols must be >= 0");
        if (o->near_cols > 0) r.near_cols = o->near_cols;
        if (o->chunk_cols > 0) r.chunk_cols = o->chunk_cols;
    }
    if (r.near_cols < 64 || r.chunk_cols < 64)
        return fail(ctx, PALMAD_EINVAL, "near_cols and chunk_cols must be >= 64");
    *out = r;
    return PALMAD_OK;
}

// Largest length whose LDS staging (two centred windows + padding, FP64)
// fits a 64 KiB workgroup allocation.
constexpr int32_t MAXL_LIMIT = 3000;

int validate(palmad_ctx* ctx, int64_t n, int32_t minL, int32_t maxL, int32_t k)
{
    if (minL < 3) return fail(ctx, PALMAD_EINVAL, "minL must be >= 3 (got %d)", minL);
    if (maxL < minL) return fail(ctx, PALMAD_EINVAL, "maxL (%d) < minL (%d)", maxL, minL);
    if (n < 3 * (int64_t)maxL - 1)
        return fail(ctx, PALMAD_EINVAL,
                    "n (%lld) must be >= 3*maxL - 1 (%lld) so every subsequence has a non-self "
                    "match",
                    (long long)n, 3 * (long long)maxL - 1);
    if (n >= (int64_t)0x7fff0000)
        return fail(ctx, PALMAD_EUNSUPPORTED, "n (%lld) must be < 2^31 - 2^16", (long long)n);
    if (maxL > MAXL_LIMIT)
        return fail(ctx, PALMAD_EUNSUPPORTED, "maxL (%d) above the supported %d", maxL, MAXL_LIMIT);
    if (k < 1) return fail(ctx, PALMAD_EINVAL, "k must be >= 1 (got %d)", k);
    if (k > K_MAX) return fail(ctx, PALMAD_EUNSUPPORTED, "k (%d) above the supported %d", k, K_MAX);
    if ((int64_t)k > n - maxL + 1)
        return fail(ctx, PALMAD_EINVAL, "k (%d) exceeds the number of subsequences", k);
    return PALMAD_OK;
}

SweepCfg cfg_of(const Opts& o, const KernelTimer* timer)
{
    SweepCfg c;
    c.near_cols = o.near_cols;
    c.chunk_cols = o.chunk_cols;
    c.guard = o.dist_bits == 64 ? 0.0f : o.guard;
    c.dist_bits = o.dist_bits;
    c.far_grid = o.far_grid;
    const int near_rows = o.rows_near ? o.rows_near : (o.dist_bits == 64 ? 256 : 512);
    const int far_rows = o.rows_far ? o.rows_far : near_rows;
    const int ref_rows = o.rows_refine ? o.rows_refine : 128;
    c.q_near = near_rows / 64;
    c.q_far = far_rows / 64;
    c.q_ref = ref_rows / 64;
    c.timer = timer;
    return c;
}

KernelTimer make_timer(palmad_ctx* ctx, const Opts& o)
{
    KernelTimer t = {};
    t.on = (o.flags & PALMAD_FLAG_TIME_KERNELS) && ctx->have_events;
    for (int k = 0; k < KCLASSES; ++k) {
        t.ev[k][0] = ctx->ev[k][0];
        t.ev[k][1] = ctx->ev[k][1];
    }
    return t;
}

// After a synchronised round: add the device time of every class launched.
int accumulate(palmad_ctx* ctx, KernelTimer& t, int nclasses)
{
    if (!t.on) return PALMAD_OK;
    for (int k = 0; k < nclasses; ++k) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, t.ev[k][0], t.ev[k][1]));
        t.ms[k] += ms;
        t.launches[k] += 1;
    }
    return PALMAD_OK;
}

int check_ws(palmad_ctx* ctx, void* ws, size_t ws_bytes, const Layout& lay)
{
    if (!ws) return fail(ctx, PALMAD_EINVAL, "workspace is NULL");
    if (((uintptr_t)ws & 255u) != 0) return fail(ctx, PALMAD_EINVAL, "workspace not 256-byte aligned");
    if (ws_bytes < lay.total)
        return fail(ctx, PALMAD_EWORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes,
                    lay.total);
    return PALMAD_OK;
}

// Copy the series, check finiteness and compute the flat-window threshold.
int prepare(palmad_ctx* ctx, const Layout& lay, const Buffers& b, const double* T, hipStream_t st)
{
    HIP_TRY(launch_prepare(lay, b, T, st));
    HIP_TRY(hipMemcpyAsync(ctx->pinned, &b.ctrl->nonfinite, sizeof(int32_t), hipMemcpyDeviceToHost,
                           st));
    HIP_TRY(hipStreamSynchronize(st));
    if (*ctx->pinned) return fail(ctx, PALMAD_ENONFINITE, "the series holds NaN or Inf values");
    return PALMAD_OK;
}

int read_stats(palmad_ctx* ctx, const Buffers& b, palmad_stats* stats, double secs,
               const KernelTimer& t, hipStream_t st)
{
    if (!stats) return PALMAD_OK;
    Ctrl h;
    HIP_TRY(hipMemcpyAsync(&h, b.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    std::memset(stats, 0, sizeof *stats);
    stats->evals_select = h.evals_sel;
    stats->evals_refine = h.evals_ref;
    stats->evals_polish = h.evals_pol;
    stats->range_searches = h.rounds;
    stats->survivors = h.survivors;
    stats->seconds = secs;
    stats->kernel_evals[PALMAD_KERNEL_SELECT_NEAR] = h.evals_near;
    stats->kernel_evals[PALMAD_KERNEL_SELECT_FAR] = h.evals_far;
    stats->kernel_evals[PALMAD_KERNEL_REFINE] = h.evals_ref;
    stats->kernel_evals[PALMAD_KERNEL_POLISH] = h.evals_pol;
    for (int k = 0; k < KCLASSES; ++k) {
        stats->kernel_launches[k] = t.launches[k];
        stats->kernel_ms[k] = t.ms[k];
    }
    return PALMAD_OK;
}

}  // namespace

extern "C" {

const char* palmad_version(void) { return "palmad-mi355x 0.1 (gfx950)"; }

const char* palmad_last_error(const palmad_ctx* ctx)
{
    if (ctx) return ctx->err.c_str();
    return g_err.c_str();
}

int palmad_create(palmad_ctx** out, int device)
{
    palmad_ctx* ctx = nullptr;
    if (!out) return fail(nullptr, PALMAD_EINVAL, "out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0)
        return fail(nullptr, PALMAD_EDEVICE, "no HIP device available (%s)",
                    e != hipSuccess ? hipGetErrorString(e) : "count 0");
    if (device < 0 || device >= count)
        return fail(nullptr, PALMAD_EINVAL, "device %d out of range [0, %d)", device, count);
    HIP_TRY(hipSetDevice(device));
    ctx = new (std::nothrow) palmad_ctx();
    if (!ctx) return fail(nullptr, PALMAD_ENOMEM, "context allocation failed");
    ctx->device = device;
    ctx->pinned = nullptr;
    e = hipHostMalloc((void**)&ctx->pinned, 64, hipHostMallocDefault);
    if (e != hipSuccess) {
        delete ctx;
        return fail(nullptr, PALMAD_EDEVICE, "hipHostMalloc failed: %s", hipGetErrorString(e));
    }
    ctx->have_events = true;
    for (int k = 0; k < KCLASSES; ++k)
        for (int q = 0; q < 2; ++q)
            if (hipEventCreate(&ctx->ev[k][q]) != hipSuccess) ctx->have_events = false;
    *out = ctx;
    return PALMAD_OK;
}

void palmad_destroy(palmad_ctx* ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->have_events)
        for (int k = 0; k < KCLASSES; ++k)
            for (int q = 0; q < 2; ++q) (void)hipEventDestroy(ctx->ev[k][q]);
    delete ctx;
}

int palmad_workspace_size(int64_t n, int32_t minL, int32_t maxL, int32_t k,
                          const palmad_options* opts, size_t* bytes)
{
    palmad_ctx* ctx = nullptr;
    if (!bytes) return fail(nullptr, PALMAD_EINVAL, "bytes is NULL");
    int rc = validate(nullptr, n, minL, maxL, k);
    if (rc) return rc;
    Opts o;
    rc = read_opts(nullptr, opts, &o);
    if (rc) return rc;
    Layout lay;
    if (!make_layout(n, minL, maxL, k, o.dist_bits, &lay))
        return fail(ctx, PALMAD_EINVAL, "layout failed");
    *bytes = lay.total;
    return PALMAD_OK;
}

int palmad_discords(palmad_ctx* ctx, const double* T, int64_t n, int32_t minL, int32_t maxL,
                    int32_t k, const palmad_options* opts, void* workspace, size_t ws_bytes,
                    int64_t* idx, int32_t* len, double* nn_dist, int64_t* nn_idx, int32_t* count,
                    palmad_stats* stats, void* stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!ctx) return fail(nullptr, PALMAD_EINVAL, "ctx is NULL");
    if (!T || !idx || !len || !nn_dist || !nn_idx || !count)
        return fail(ctx, PALMAD_EINVAL, "null input or output pointer");
    int rc = validate(ctx, n, minL, maxL, k);
    if (rc) return rc;
    Opts o;
    rc = read_opts(ctx, opts, &o);
    if (rc) return rc;
    Layout lay;
    make_layout(n, minL, maxL, k, o.dist_bits, &lay);
    rc = check_ws(ctx, workspace, ws_bytes, lay);
    if (rc) return rc;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    const Buffers b = carve(workspace, lay);
    KernelTimer timer = make_timer(ctx, o);
    const SweepCfg cfg = cfg_of(o, &timer);
    rc = prepare(ctx, lay, b, T, st);
    if (rc) return rc;
    for (int32_t m = minL; m <= maxL; ++m) {
        HIP_TRY(launch_stats(lay, b, m, m == minL, st));
        for (int attempt = 0;; ++attempt) {
            if (attempt > 5000)
                return fail(ctx, PALMAD_EDEVICE, "length %d: range search did not converge", m);
            HIP_TRY(launch_round(lay, b, cfg, m, attempt, st));
            HIP_TRY(launch_finish_length(lay, b, cfg, m, idx, len, nn_dist, nn_idx, count, st));
            HIP_TRY(hipMemcpyAsync(ctx->pinned, &b.ctrl->done, sizeof(int32_t),
                                   hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            rc = accumulate(ctx, timer, KCLASSES);
            if (rc) return rc;
            if (*ctx->pinned) break;
        }
    }
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return read_stats(ctx, b, stats, secs, timer, st);
}

int palmad_range_discords(palmad_ctx* ctx, const double* T, int64_t n, int32_t m, double r,
                          const palmad_options* opts, void* workspace, size_t ws_bytes,
                          uint64_t* alive, double* nn_dist, int64_t* count, palmad_stats* stats,
                          void* stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!ctx) return fail(nullptr, PALMAD_EINVAL, "ctx is NULL");
    if (!T || !alive || !nn_dist || !count)
        return fail(ctx, PALMAD_EINVAL, "null input or output pointer");
    if (!(r == r)) return fail(ctx, PALMAD_EINVAL, "r is NaN");
    int rc = validate(ctx, n, m, m, 1);
    if (rc) return rc;
    Opts o;
    rc = read_opts(ctx, opts, &o);
    if (rc) return rc;
    Layout lay;
    make_layout(n, m, m, 1, o.dist_bits, &lay);
    rc = check_ws(ctx, workspace, ws_bytes, lay);
    if (rc) return rc;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    const Buffers b = carve(workspace, lay);
    KernelTimer timer = make_timer(ctx, o);
    const SweepCfg cfg = cfg_of(o, &timer);
    rc = prepare(ctx, lay, b, T, st);
    if (rc) return rc;
    HIP_TRY(launch_stats(lay, b, m, true, st));
    HIP_TRY(launch_set_fixed_r(b, r, st));
    HIP_TRY(launch_round(lay, b, cfg, m, 0, st));
    HIP_TRY(launch_range_out(lay, b, m, (unsigned long long*)alive, nn_dist, st));
    HIP_TRY(hipMemcpyAsync(ctx->pinned, &b.ctrl->nsurv, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *count = (int64_t)(uint32_t)*ctx->pinned;
    rc = accumulate(ctx, timer, 3);  // no polish in a single range search
    if (rc) return rc;
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return read_stats(ctx, b, stats, secs, timer, st);
}

namespace {
struct BwdLayout {
    Layout lay;
    int64_t nblk;
    size_t off_part, total;
};
bool bwd_layout(int64_t n, int64_t K, int32_t maxm, BwdLayout* out)
{
    BwdLayout b = {};
    make_layout(n, maxm, maxm, 1, 64, &b.lay);
    b.lay.L = 0;  // no length history
    b.nblk = (n + 255) / 256;
    b.off_part = b.lay.total;
    b.total = b.off_part + (((size_t)std::max<int64_t>(K, 1) * (size_t)b.nblk * 2 * sizeof(double) +
                             255) & ~(size_t)255);
    *out = b;
    return true;
}
}  // namespace

int palmad_backward_workspace_size(int64_t n, int64_t K, int32_t maxm, size_t* bytes)
{
    palmad_ctx* ctx = nullptr;
    if (!bytes) return fail(nullptr, PALMAD_EINVAL, "bytes is NULL");
    if (K < 0) return fail(nullptr, PALMAD_EINVAL, "K must be >= 0");
    int rc = validate(nullptr, n, maxm, maxm, 1);
    if (rc) return rc;
    BwdLayout b;
    bwd_layout(n, K, maxm, &b);
    *bytes = b.total;
    (void)ctx;
    return PALMAD_OK;
}

int palmad_discords_backward(palmad_ctx* ctx, const double* T, int64_t n, int64_t K, int32_t maxm,
                             const int64_t* idx, const int32_t* len, const double* grad_nn,
                             void* workspace, size_t ws_bytes, double* grad_T, int64_t* nn_idx,
                             void* stream)
{
    if (!ctx) return fail(nullptr, PALMAD_EINVAL, "ctx is NULL");
    if (K < 0) return fail(ctx, PALMAD_EINVAL, "K must be >= 0");
    if (!T || !grad_T || (K > 0 && (!idx || !len || !grad_nn)))
        return fail(ctx, PALMAD_EINVAL, "null input or output pointer");
    int rc = validate(ctx, n, maxm, maxm, 1);
    if (rc) return rc;
    if (K > 65535) return fail(ctx, PALMAD_EUNSUPPORTED, "K (%lld) above 65535", (long long)K);
    BwdLayout bl;
    bwd_layout(n, K, maxm, &bl);
    if (!workspace) return fail(ctx, PALMAD_EINVAL, "workspace is NULL");
    if (((uintptr_t)workspace & 255u) != 0)
        return fail(ctx, PALMAD_EINVAL, "workspace not 256-byte aligned");
    if (ws_bytes < bl.total)
        return fail(ctx, PALMAD_EWORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes,
                    bl.total);
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    const Buffers b = carve(workspace, bl.lay);
    rc = prepare(ctx, bl.lay, b, T, st);
    if (rc) return rc;
    if (K == 0) return PALMAD_OK;
    HIP_TRY(launch_set_max_len(b, maxm, st));
    double* part = (double*)((char*)workspace + bl.off_part);
    HIP_TRY(launch_adjoint(b.T, n, K, maxm, idx, len, grad_nn, b.ctrl, part, bl.nblk, grad_T,
                           nn_idx, st));
    HIP_TRY(hipStreamSynchronize(st));
    return PALMAD_OK;
}

int palmad_window_stats(palmad_ctx* ctx, const double* T, int64_t n, int32_t minL, int32_t m,
                        void* workspace, size_t ws_bytes, double* mu, double* sigma, void* stream)
{
    if (!ctx) return fail(nullptr, PALMAD_EINVAL, "ctx is NULL");
    if (!T || !mu || !sigma) return fail(ctx, PALMAD_EINVAL, "null input or output pointer");
    int rc = validate(ctx, n, minL, m, 1);
    if (rc) return rc;
    Layout lay;
    make_layout(n, minL, m, 1, 32, &lay);
    rc = check_ws(ctx, workspace, ws_bytes, lay);
    if (rc) return rc;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    const Buffers b = carve(workspace, lay);
    rc = prepare(ctx, lay, b, T, st);
    if (rc) return rc;
    for (int32_t mm = minL; mm <= m; ++mm) HIP_TRY(launch_stats(lay, b, mm, mm == minL, st));
    HIP_TRY(launch_stats_out(lay, b, m, mu, sigma, st));
    HIP_TRY(hipStreamSynchronize(st));
    return PALMAD_OK;
}

}  // extern "C"
