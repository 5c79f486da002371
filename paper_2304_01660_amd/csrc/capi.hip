// C ABI of the range-discord library (declared in include/palmad.h).
//
// Host side only: argument validation, workspace planning and the MERLIN
// driver loop (Alg. 1).  Every search runs the same engine over a batch of
// series (one series for the plain entry points): per round, every series
// with work left performs one range search (one DRAG call of Alg. 2,
// parallelised as in Sec. 3.2-3.3) at its own length.  The driver replays
// a few rounds at a time as a hipGraph on the context's stream and then
// reads one counter to learn whether any series still has work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/palmad.h"
#include "engine.h"

using namespace palmad;

struct palmad_ctx {
    int device;
    std::string err;
    int32_t* pinned;             // pinned host mirror of small device counters
    hipStream_t work;            // the library's stream (default priority)
    hipEvent_t ev_in, ev_out;    // order the work stream after / before the caller's
    hipEvent_t ev[KCLASSES][2];  // per-kernel timing
    bool have_events;
    hipGraph_t graph;            // cached round graph
    hipGraphExec_t graph_exec;
    std::string graph_key;
    void* scratch;               // device address of this device's static workspace
};

// Static workspace of palmad_discords_static(): one copy per GPU, held
// until the process ends.  In host code this name is only a stand-in for
// the symbol; its device address (a different one on every GPU) comes from
// hipGetSymbolAddress with that device current, taken once per device by
// palmad_create() and kept in g_scratch.
static __device__ __align__(256) unsigned char scratch[PALMAD_STATIC_WORKSPACE_BYTES];

namespace {

thread_local std::string g_err;

constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;                // guards g_scratch
void* g_scratch[SCRATCH_DEVICES];       // device address of each GPU's scratch (or null)
std::mutex g_scratch_use[SCRATCH_DEVICES];  // one static-workspace call per GPU at a time

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
    int band_pass;
};

constexpr unsigned int KNOWN_FLAGS = PALMAD_FLAG_TIME_KERNELS | PALMAD_FLAG_NO_GRAPH;

int read_opts(palmad_ctx* ctx, const palmad_options* o, Opts* out)
{
    Opts r = {32, 1.25e-4f, 2048, 1024, 0u, 0, 0, 0, 2048, 0};
    if (o) {
        if (o->flags & ~KNOWN_FLAGS)
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
        for (int i = 0; i < 2; ++i)
            if (o->reserved[i] != 0) return fail(ctx, PALMAD_EINVAL, "options.reserved must be zero");
        if (o->band_pass < -1 || o->band_pass > 1)
            return fail(ctx, PALMAD_EINVAL, "band_pass must be -1, 0 or 1 (got %d)", o->band_pass);
        r.band_pass = o->band_pass == 1 ? 1 : 0;
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

// Largest length whose sweep staging (a padded centred window, a skewed
// series stretch of 512 + m + 16 values, a batch of FP64 step records and
// the refinement's per-row values) fits a 64 KiB workgroup allocation.
constexpr int32_t MAXL_LIMIT = 2800;
constexpr int32_t B_LIMIT = 65535;

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

int validate_batch(palmad_ctx* ctx, int32_t B, const int64_t* offsets, const int32_t* minL,
                   const int32_t* maxL, int32_t k, std::vector<int64_t>* n)
{
    if (B < 1) return fail(ctx, PALMAD_EINVAL, "B must be >= 1 (got %d)", B);
    if (B > B_LIMIT) return fail(ctx, PALMAD_EUNSUPPORTED, "B (%d) above %d", B, B_LIMIT);
    if (!offsets || !minL || !maxL) return fail(ctx, PALMAD_EINVAL, "null offsets, minL or maxL");
    if (offsets[0] != 0) return fail(ctx, PALMAD_EINVAL, "offsets[0] must be 0");
    n->resize(B);
    for (int b = 0; b < B; ++b) {
        (*n)[b] = offsets[b + 1] - offsets[b];
        const int rc = validate(ctx, (*n)[b], minL[b], maxL[b], k);
        if (rc) {
            const std::string m = ctx ? ctx->err : g_err;
            return fail(ctx, rc, "series %d: %s", b, m.c_str());
        }
    }
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
    c.max_attempts = MAX_ATTEMPTS;
    c.band = o.band_pass;
    c.timer = timer;
    return c;
}

// Failure injection for error-path tests, from the environment variable
// PALMAD_FAULT (read at every search):
//   "hip"       the search fails as if its first HIP call had failed
//               (PALMAD_EDEVICE before any device work);
//   "converge"  one range search per length is allowed, so the first
//               length's opening range (the largest possible distance, which
//               no subsequence reaches) fails and the search reports a range
//               search that did not converge (PALMAD_EDEVICE after device
//               work, with every kernel exiting normally).
enum Fault { FAULT_NONE = 0, FAULT_HIP, FAULT_CONVERGE };
Fault fault_site()
{
    const char* f = std::getenv("PALMAD_FAULT");
    if (!f) return FAULT_NONE;
    if (std::strcmp(f, "hip") == 0) return FAULT_HIP;
    if (std::strcmp(f, "converge") == 0) return FAULT_CONVERGE;
    return FAULT_NONE;
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace plan of a batch: descriptors, prefix tables and counters, then
// one region per series.
struct Plan {
    int B;
    std::vector<Layout> lay;
    std::vector<size_t> base;
    size_t off_pfx, off_rem, off_sums, total;
    int64_t totals[PFX_KINDS];
    std::vector<int64_t> pfx;  // [PFX_KINDS][B+1]
    int32_t maxL_all;
    int64_t Nmax_all;
    int near_cols;  // first-pass width actually used (see NEAR_ITEMS)
};

// The first selection pass launches one workgroup per (row tile, chunk) of
// every series, most of which find their tile dead and exit; past a few
// tens of thousands of them per series their dispatch costs more than the
// queued split pass, which draws only live tiles' chunks.  The first-pass
// width is therefore capped so that the largest series has at most
// NEAR_ITEMS of them (at least one chunk per tile); the remaining columns
// go to the split pass.
constexpr int64_t NEAR_ITEMS = 65536;

void make_plan(int B, const int64_t* n, const int32_t* minL, const int32_t* maxL, int32_t k,
               const SweepCfg& cfg_in, Plan* p)
{
    p->B = B;
    p->lay.resize(B);
    p->base.resize(B);
    p->off_pfx = al256(sizeof(SeriesDev) * (size_t)B);
    p->off_rem = al256(p->off_pfx + sizeof(int64_t) * (size_t)PFX_KINDS * (size_t)(B + 1));
    p->off_sums = p->off_rem + 64;
    size_t o = al256(p->off_sums + 16 * sizeof(unsigned long long));
    p->pfx.assign((size_t)PFX_KINDS * (B + 1), 0);
    p->maxL_all = 0;
    p->Nmax_all = 0;
    for (int b = 0; b < B; ++b) {
        make_layout(n[b], minL[b], maxL[b], k, &p->lay[b]);
        p->base[b] = o;
        o = al256(o + p->lay[b].total);
        p->maxL_all = std::max(p->maxL_all, maxL[b]);
        p->Nmax_all = std::max(p->Nmax_all, p->lay[b].Nmax);
    }
    SweepCfg cfg = cfg_in;
    {
        const int64_t rows = 64 * (int64_t)cfg.q_near;
        const int64_t tiles = (p->Nmax_all + rows - 1) / rows;
        const int64_t chunks = std::max<int64_t>(1, NEAR_ITEMS / std::max<int64_t>(1, tiles));
        cfg.near_cols = (int)std::min<int64_t>(cfg.near_cols, chunks * cfg.chunk_cols);
    }
    p->near_cols = cfg.near_cols;
    for (int b = 0; b < B; ++b) {
        int64_t blk[PFX_KINDS];
        series_blocks(p->lay[b], cfg, blk);
        for (int q = 0; q < PFX_KINDS; ++q)
            p->pfx[(size_t)q * (B + 1) + b + 1] = p->pfx[(size_t)q * (B + 1) + b] + blk[q];
    }
    for (int q = 0; q < PFX_KINDS; ++q) p->totals[q] = p->pfx[(size_t)q * (B + 1) + B];
    p->total = o;
}

int check_grid(palmad_ctx* ctx, const Plan& p)
{
    for (int q = 0; q < PFX_KINDS; ++q)
        if (p.totals[q] > 0x7fffffffll)
            return fail(ctx, PALMAD_EUNSUPPORTED, "batch too large: %lld workgroups in one launch",
                        (long long)p.totals[q]);
    return PALMAD_OK;
}

struct Outputs {
    int64_t* idx;
    int32_t* len;
    double* nn;
    int64_t* nnidx;
    int32_t* count;
    double* heat = nullptr;   // discord heatmap (optional)
    double* rlen = nullptr;
    int64_t heat_ld = 0;
};

// Write the descriptors and prefix tables into the workspace (one upload).
// n_now (optional): the current length of each series when it is shorter
// than the length its layout was planned for (a streaming series).
int upload(palmad_ctx* ctx, const Plan& p, void* ws, const double* const* Tin, const Outputs* outs,
           Batch* bt, const int64_t* n_now = nullptr)
{
    std::vector<char> blob(p.off_rem, 0);
    SeriesDev* d = (SeriesDev*)blob.data();
    for (int b = 0; b < p.B; ++b) {
        SeriesDev s = carve((char*)ws + p.base[b], p.lay[b]);
        s.Tin = Tin ? Tin[b] : nullptr;
        if (n_now) s.n = n_now[b];
        if (outs) {
            s.idx = outs[b].idx;
            s.len = outs[b].len;
            s.nn = outs[b].nn;
            s.nnidx = outs[b].nnidx;
            s.count = outs[b].count;
            s.heat = outs[b].heat;
            s.rlen = outs[b].rlen;
            s.heat_ld = outs[b].heat_ld;
        }
        d[b] = s;
    }
    std::memcpy(blob.data() + p.off_pfx, p.pfx.data(), sizeof(int64_t) * p.pfx.size());
    HIP_TRY(hipMemcpyAsync(ws, blob.data(), blob.size(), hipMemcpyHostToDevice, ctx->work));
    HIP_TRY(hipStreamSynchronize(ctx->work));
    bt->s = (SeriesDev*)ws;
    for (int q = 0; q < PFX_KINDS; ++q)
        bt->pfx[q] = (const int64_t*)((char*)ws + p.off_pfx) + (size_t)q * (p.B + 1);
    bt->B = p.B;
    bt->maxL_all = p.maxL_all;
    bt->Nmax_all = p.Nmax_all;
    bt->remaining = (int32_t*)((char*)ws + p.off_rem);
    bt->sums = (unsigned long long*)((char*)ws + p.off_sums);
    return PALMAD_OK;
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

// After a synchronised round: add the device time of every kernel class
// launched in it.
int accumulate(palmad_ctx* ctx, KernelTimer& t)
{
    if (!t.on) return PALMAD_OK;
    for (int k = 0; k < KCLASSES; ++k) {
        if (!t.used[k]) continue;
        t.used[k] = false;
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, t.ev[k][0], t.ev[k][1]));
        t.ms[k] += ms;
        t.launches[k] += 1;
    }
    return PALMAD_OK;
}

// Order the library's stream after the caller's pending work.
int enter(palmad_ctx* ctx, void* stream)
{
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipEventRecord(ctx->ev_in, (hipStream_t)stream));
    HIP_TRY(hipStreamWaitEvent(ctx->work, ctx->ev_in, 0));
    return PALMAD_OK;
}

// Order the caller's stream after the library's work.
int leave(palmad_ctx* ctx, void* stream)
{
    HIP_TRY(hipEventRecord(ctx->ev_out, ctx->work));
    HIP_TRY(hipStreamWaitEvent((hipStream_t)stream, ctx->ev_out, 0));
    return PALMAD_OK;
}

// Padded copies, finiteness check and the flat-window threshold.
int prepare(palmad_ctx* ctx, const Batch& bt, const Plan& p)
{
    HIP_TRY(launch_prepare(bt, p.totals, ctx->work));
    HIP_TRY(launch_nonfinite(bt, bt.remaining, ctx->work));
    HIP_TRY(hipMemcpyAsync(ctx->pinned, bt.remaining, 2 * sizeof(int32_t), hipMemcpyDeviceToHost,
                           ctx->work));
    HIP_TRY(hipStreamSynchronize(ctx->work));
    if (ctx->pinned[0]) {
        if (p.B == 1) return fail(ctx, PALMAD_ENONFINITE, "the series holds NaN or Inf values");
        return fail(ctx, PALMAD_ENONFINITE, "%d series hold NaN or Inf values (first: series %d)",
                    ctx->pinned[0], ctx->pinned[1]);
    }
    return PALMAD_OK;
}

std::string graph_key(const Batch& bt, const SweepCfg& c, const Plan& p)
{
    char buf[256];
    snprintf(buf, sizeof buf, "%p|%d|%d|%lld|%d|%d|%d|%d|%d|%d|%d|%a|%d|%d|", (void*)bt.s, bt.B,
             bt.maxL_all, (long long)bt.Nmax_all,
             c.near_cols, c.chunk_cols, c.dist_bits, c.far_grid, c.q_near, c.q_far, c.q_ref,
             (double)c.guard, c.max_attempts, c.band);
    std::string k = buf;
    for (int q = 0; q < PFX_KINDS; ++q) k += std::to_string(p.totals[q]) + ",";
    return k;
}

void drop_graph(palmad_ctx* ctx)
{
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->graph_exec = nullptr;
    ctx->graph = nullptr;
    ctx->graph_key.clear();
}

// Rounds replayed per host check: a finished series makes every kernel of
// a round return at once, so a few rounds past the end cost little, while
// each check is a device-to-host copy and a stream synchronisation.
constexpr int ROUNDS_PER_CHECK = 4;

// ROUNDS_PER_CHECK rounds replayed from the context's cached graph (captured
// on first use for this workspace and configuration), or one round launched
// directly.  Returns the number of rounds issued in *issued.
int run_rounds(palmad_ctx* ctx, const Batch& bt, const SweepCfg& cfg, const Plan& p, bool graphs,
               int* issued)
{
    if (!graphs) {
        HIP_TRY(launch_round(bt, cfg, p.totals, ctx->work));
        *issued = 1;
        return PALMAD_OK;
    }
    *issued = ROUNDS_PER_CHECK;
    const std::string key = graph_key(bt, cfg, p);
    if (ctx->graph_exec == nullptr || ctx->graph_key != key) {
        drop_graph(ctx);
        HIP_TRY(hipStreamBeginCapture(ctx->work, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (int r = 0; r < ROUNDS_PER_CHECK && e == hipSuccess; ++r)
            e = launch_round(bt, cfg, p.totals, ctx->work);
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(ctx->work, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(ctx, PALMAD_EDEVICE, "round capture failed: %s",
                        hipGetErrorString(e != hipSuccess ? e : e2));
        }
        ctx->graph = g;
        const hipError_t e3 = hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0);
        if (e3 != hipSuccess) {
            ctx->graph_exec = nullptr;
            drop_graph(ctx);
            return fail(ctx, PALMAD_EDEVICE, "round graph instantiation failed: %s",
                        hipGetErrorString(e3));
        }
        ctx->graph_key = key;
    }
    HIP_TRY(hipGraphLaunch(ctx->graph_exec, ctx->work));
    return PALMAD_OK;
}

int gather_stats(palmad_ctx* ctx, const Batch& bt, const KernelTimer& t, double secs,
                 palmad_stats* stats)
{
    if (!stats) return PALMAD_OK;
    HIP_TRY(launch_sum_stats(bt, bt.sums, ctx->work));
    unsigned long long* h = (unsigned long long*)(ctx->pinned + 16);
    HIP_TRY(hipMemcpyAsync(h, bt.sums, 10 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           ctx->work));
    HIP_TRY(hipStreamSynchronize(ctx->work));
    std::memset(stats, 0, sizeof *stats);
    stats->evals_select = h[0];
    stats->evals_refine = h[1];
    stats->evals_polish = h[2];
    stats->range_searches = h[3];
    stats->survivors = h[4];
    stats->kernel_evals[PALMAD_KERNEL_SELECT_NEAR] = h[5];
    stats->kernel_evals[PALMAD_KERNEL_SELECT_FAR] = h[6];
    stats->kernel_evals[PALMAD_KERNEL_REFINE] = h[1];
    stats->kernel_evals[PALMAD_KERNEL_POLISH] = h[2];
    stats->kernel_evals[PALMAD_KERNEL_SELECT_BAND] = h[9];
    stats->rows_after_near = h[7];
    stats->rows_after_far = h[8];
    stats->seconds = secs;
    for (int k = 0; k < KCLASSES; ++k) {
        stats->kernel_launches[k] = t.launches[k];
        stats->kernel_ms[k] = t.ms[k];
    }
    return PALMAD_OK;
}

// MERLIN over a batch (Alg. 1 per series): rounds until no series has work.
int search(palmad_ctx* ctx, const Plan& p, const Opts& o, void* ws, const double* const* Tin,
           const Outputs* outs, palmad_stats* stats, void* stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    KernelTimer timer = make_timer(ctx, o);
    SweepCfg cfg = cfg_of(o, &timer);
    const Fault fault = fault_site();
    if (fault == FAULT_HIP)
        return fail(ctx, PALMAD_EDEVICE, "injected HIP failure (PALMAD_FAULT=hip)");
    if (fault == FAULT_CONVERGE) cfg.max_attempts = 1;
    cfg.near_cols = p.near_cols;
    int rc = enter(ctx, stream);
    if (rc) return rc;
    Batch bt;
    rc = upload(ctx, p, ws, Tin, outs, &bt);
    if (rc) return rc;
    rc = prepare(ctx, bt, p);
    if (rc) return rc;
    const bool graphs = !timer.on && !(o.flags & PALMAD_FLAG_NO_GRAPH);
    int64_t max_rounds = 0;
    for (int b = 0; b < p.B; ++b) max_rounds = std::max<int64_t>(max_rounds, p.lay[b].L);
    max_rounds = max_rounds * cfg.max_attempts + 2;
    for (int64_t round = 0;;) {
        if (round > max_rounds) return fail(ctx, PALMAD_EDEVICE, "search did not terminate");
        int issued = 0;
        rc = run_rounds(ctx, bt, cfg, p, graphs, &issued);
        if (rc) return rc;
        round += issued;
        HIP_TRY(hipMemcpyAsync(ctx->pinned, bt.remaining, 2 * sizeof(int32_t),
                               hipMemcpyDeviceToHost, ctx->work));
        HIP_TRY(hipStreamSynchronize(ctx->work));
        rc = accumulate(ctx, timer);
        if (rc) return rc;
        if (ctx->pinned[1])
            return fail(ctx, PALMAD_EDEVICE,
                        "%d series: a range search did not converge within %d attempts",
                        ctx->pinned[1], cfg.max_attempts);
        if (ctx->pinned[0] == 0) break;
    }
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    rc = gather_stats(ctx, bt, timer, secs, stats);
    if (rc) return rc;
    return leave(ctx, stream);
}

int check_ws(palmad_ctx* ctx, void* ws, size_t ws_bytes, size_t need)
{
    if (!ws) return fail(ctx, PALMAD_EINVAL, "workspace is NULL");
    if (((uintptr_t)ws & 255u) != 0) return fail(ctx, PALMAD_EINVAL, "workspace not 256-byte aligned");
    if (ws_bytes < need)
        return fail(ctx, PALMAD_EWORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    return PALMAD_OK;
}

Opts default_opts()
{
    Opts o;
    read_opts(nullptr, nullptr, &o);
    return o;
}

// Backward workspace: a one-series plan at length maxm, then the partials.
size_t backward_bytes(int64_t n, int64_t K, int32_t maxm, Plan* p, int64_t* nblk)
{
    make_plan(1, &n, &maxm, &maxm, 1, cfg_of(default_opts(), nullptr), p);
    *nblk = (n + 255) / 256;
    return p->total + al256((size_t)std::max<int64_t>(K, 1) * (size_t)*nblk * 2 * sizeof(double));
}

// ---- autotuner ----

// The probe: every series over its first `probe` lengths.
struct Probe {
    std::vector<int64_t> n;
    std::vector<int32_t> lo, hi;
    Plan plan;
    size_t off_out, total;
    int64_t rows, lrows;
};

void make_probe(int B, const int64_t* n, const int32_t* minL, const int32_t* maxL, int32_t k,
                int32_t probe, Probe* pr)
{
    pr->n.assign(n, n + B);
    pr->lo.assign(minL, minL + B);
    pr->hi.resize(B);
    pr->rows = pr->lrows = 0;
    for (int b = 0; b < B; ++b) {
        pr->hi[b] = std::min<int32_t>(maxL[b], minL[b] + probe - 1);
        const int64_t L = (int64_t)pr->hi[b] - minL[b] + 1;
        pr->rows += L * k;
        pr->lrows += L;
    }
    make_plan(B, pr->n.data(), pr->lo.data(), pr->hi.data(), k,
              cfg_of(default_opts(), nullptr), &pr->plan);
    pr->off_out = pr->plan.total;
    pr->total = pr->off_out + al256((size_t)pr->rows * (8 + 4 + 8 + 8) + (size_t)pr->lrows * 4 + 1024);
}

// Best wall time of `reps` searches of the probe under options `o` (after
// one untimed run, which also captures the round graph).
int time_probe(palmad_ctx* ctx, const Probe& pr, int32_t k, const Opts& o, void* ws,
               const std::vector<const double*>& tin, const std::vector<Outputs>& outs, int reps,
               void* stream, double* best)
{
    Plan p;  // the prefix tables depend on the tile geometry
    make_plan(pr.plan.B, pr.n.data(), pr.lo.data(), pr.hi.data(), k, cfg_of(o, nullptr), &p);
    const int rc0 = check_grid(ctx, p);
    if (rc0) return rc0;
    double bs = 1e300;
    for (int r = 0; r <= reps; ++r) {
        const auto t0 = std::chrono::steady_clock::now();
        const int rc = search(ctx, p, o, ws, tin.data(), outs.data(), nullptr, stream);
        if (rc) return rc;
        const double dt =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (r > 0) bs = std::min(bs, dt);
    }
    *best = bs;
    return PALMAD_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// streaming series
// ---------------------------------------------------------------------------
struct palmad_stream {
    palmad_ctx* ctx;
    Plan p;
    Opts o;
    void* ws;
    unsigned long long* prof;  // per-length profiles [L][Npad] (ordered bits of rho)
    int32_t* flag;             // device scratch for the finiteness check
    int64_t cap, n;
    int32_t minL, maxL, k;
};

namespace {

// Workspace of a stream: the search layout of a series of `cap` points,
// then the L profiles, then a small scratch.
size_t stream_bytes(const Plan& p, int32_t L, size_t* off_prof, size_t* off_flag)
{
    *off_prof = al256(p.total);
    *off_flag = al256(*off_prof + sizeof(unsigned long long) * (size_t)L * (size_t)p.lay[0].Npad);
    return *off_flag + 256;
}

int stream_batch(palmad_stream* st, const Outputs* outs, Batch* bt)
{
    const double* none = nullptr;
    return upload(st->ctx, st->p, st->ws, &none, outs, bt, &st->n);
}

}  // namespace


extern "C" {

const char* palmad_version(void) { return "palmad-mi355x 0.3 (gfx950)"; }

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
    ctx->work = nullptr;
    ctx->ev_in = ctx->ev_out = nullptr;
    ctx->graph = nullptr;
    ctx->graph_exec = nullptr;
    e = hipHostMalloc((void**)&ctx->pinned, 256, hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->work, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_out, hipEventDisableTiming);
    if (e != hipSuccess) {
        if (ctx->ev_in) (void)hipEventDestroy(ctx->ev_in);
        if (ctx->work) (void)hipStreamDestroy(ctx->work);
        if (ctx->pinned) (void)hipHostFree(ctx->pinned);
        delete ctx;
        return fail(nullptr, PALMAD_EDEVICE, "context setup failed: %s", hipGetErrorString(e));
    }
    ctx->have_events = true;
    for (int k = 0; k < KCLASSES; ++k)
        for (int q = 0; q < 2; ++q)
            if (hipEventCreate(&ctx->ev[k][q]) != hipSuccess) ctx->have_events = false;
    // the static workspace's address on this device (once per device; the
    // device is current here)
    ctx->scratch = nullptr;
    if (device < SCRATCH_DEVICES) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch[device]) {
            void* ptr = nullptr;
            const hipError_t es = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (es != hipSuccess || !ptr) {
                palmad_destroy(ctx);
                return fail(nullptr, PALMAD_EDEVICE, "static workspace address on device %d: %s",
                            device, hipGetErrorString(es));
            }
            g_scratch[device] = ptr;
        }
        ctx->scratch = g_scratch[device];
    }
    *out = ctx;
    return PALMAD_OK;
}

void palmad_destroy(palmad_ctx* ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->work);
    drop_graph(ctx);
    if (ctx->have_events)
        for (int k = 0; k < KCLASSES; ++k)
            for (int q = 0; q < 2; ++q) (void)hipEventDestroy(ctx->ev[k][q]);
    (void)hipEventDestroy(ctx->ev_in);
    (void)hipEventDestroy(ctx->ev_out);
    (void)hipStreamDestroy(ctx->work);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    delete ctx;
}

int palmad_workspace_size(int64_t n, int32_t minL, int32_t maxL, int32_t k,
                          const palmad_options* opts, size_t* bytes)
{
    if (!bytes) return fail(nullptr, PALMAD_EINVAL, "bytes is NULL");
    int rc = validate(nullptr, n, minL, maxL, k);
    if (rc) return rc;
    Opts o;
    rc = read_opts(nullptr, opts, &o);
    if (rc) return rc;
    Plan p;
    make_plan(1, &n, &minL, &maxL, k, cfg_of(o, nullptr), &p);
    *bytes = p.total;
    return PALMAD_OK;
}

int palmad_discords(palmad_ctx* ctx, const double* T, int64_t n, int32_t minL, int32_t maxL,
                    int32_t k, const palmad_options* opts, void* workspace, size_t ws_bytes,
                    int64_t* idx, int32_t* len, double* nn_dist, int64_t* nn_idx, int32_t* count,
                    palmad_stats* stats, void* stream)
{
    if (!ctx) return fail(nullptr, PALMAD_EINVAL, "ctx is NULL");
    if (!T || !idx || !len || !nn_dist || !nn_idx || !count)
        return fail(ctx, PALMAD_EINVAL, "null input or output pointer");
    int rc = validate(ctx, n, minL, maxL, k);
    if (rc) return rc;
    Opts o;
    rc = read_opts(ctx, opts, &o);
    if (rc) return rc;
    Plan p;
    make_plan(1, &n, &minL, &maxL, k, cfg_of(o, nullptr), &p);
    rc = check_ws(ctx, workspace, ws_bytes, p.total);
    if (rc) return rc;
    const Outputs out = {idx, len, nn_dist, nn_idx, count};
    return search(ctx, p, o, workspace, &T, &out, stats, stream);
}

int palmad_discords_static(palmad_ctx* ctx, const double* T, int64_t n, int32_t minL,
                           int32_t maxL, int32_t k, const palmad_options* opts, int64_t* idx,
                           int32_t* len, double* nn_dist, int64_t* nn_idx, int32_t* count,
                           palmad_stats* stats, void* stream)
{
    if (!ctx) return fail(nullptr, PALMAD_EINVAL, "ctx is NULL");
    if (!T || !idx || !len || !nn_dist || !nn_idx || !count)
        return fail(ctx, PALMAD_EINVAL, "null input or output pointer");
    int rc = validate(ctx, n, minL, maxL, k);
    if (rc) return rc;
    Opts o;
    rc = read_opts(ctx, opts, &o);
    if (rc) return rc;
    Plan p;
    make_plan(1, &n, &minL, &maxL, k, cfg_of(o, nullptr), &p);
    if (p.total > (size_t)PALMAD_STATIC_WORKSPACE_BYTES)
        return fail(ctx, PALMAD_EWORKSPACE,
                    "this search needs %zu bytes of workspace; the static workspace holds %zu "
                    "(use palmad_discords with a caller workspace)",
                    p.total, (size_t)PALMAD_STATIC_WORKSPACE_BYTES);
    if (!ctx->scratch)
        return fail(ctx, PALMAD_EUNSUPPORTED, "no static workspace on device %d", ctx->device);
    // graph instantiation may allocate: every kernel is launched directly
    o.flags |= PALMAD_FLAG_NO_GRAPH;
    const Outputs out = {idx, len, nn_dist, nn_idx, count};
    // search() returns after its device work completed, so holding the
    // device's lock for the call keeps calls from this process apart
    std::lock_guard<std::mutex> lk(g_scratch_use[ctx->device]);
    rc = search(ctx, p, o, ctx->scratch, &T, &out, stats, stream);
    if (rc) (void)hipStreamSynchronize(ctx->work);  // an error may leave work queued
    return rc;
}

int palmad_discord_heatmap(palmad_ctx* ctx, const double* T, int64_t n, int32_t minL,
                           int32_t maxL, int32_t k, const palmad_options* opts, void* workspace,
                           size_t ws_bytes, int64_t* idx, int32_t* len, double* nn_dist,
                           int64_t* nn_idx, int32_t* count, double* heat, int64_t ld,
                           double* range, palmad_stats* stats, void* stream)
{
    if (!ctx) return fail(nullptr, PALMAD_EINVAL, "ctx is NULL");
    if (!T || !idx || !len || !nn_dist || !nn_idx || !count || !heat || !range)
        return fail(ctx, PALMAD_EINVAL, "null input or output pointer");
    int rc = validate(ctx, n, minL, maxL, k);
    if (rc) return rc;
    if (ld < n - minL + 1)
        return fail(ctx, PALMAD_EINVAL, "ld (%lld) < n - minL + 1 (%lld)", (long long)ld,
                    (long long)(n - minL + 1));
    Opts o;
    rc = read_opts(ctx, opts, &o);
    if (rc) return rc;
    Plan p;
    make_plan(1, &n, &minL, &maxL, k, cfg_of(o, nullptr), &p);
    rc = check_ws(ctx, workspace, ws_bytes, p.total);
    if (rc) return rc;
    Outputs out = {idx, len, nn_dist, nn_idx, count};
    out.heat = heat;
    out.rlen = range;
    out.heat_ld = ld;
    return search(ctx, p, o, workspace, &T, &out, stats, stream);
}

int palmad_heatmap_interest(palmad_ctx* ctx, const double* heat, int32_t L, int64_t ld,
                            int64_t ncols, int32_t minL, int32_t k, double* col_score,
                            int32_t* col_len, int64_t* top_idx, int32_t* top_len,
                            double* top_score, void* stream)
{
    if (!ctx) return fail(nullptr, PALMAD_EINVAL, "ctx is NULL");
    if (!heat || !col_score || !col_len || !top_idx || !top_len || !top_score)
        return fail(ctx, PALMAD_EINVAL, "null input or output pointer");
    if (L < 1 || ncols < 1 || ld < ncols)
        return fail(ctx, PALMAD_EINVAL, "need L >= 1, ncols >= 1 and ld >= ncols");
    if (k < 1 || (int64_t)k > ncols) return fail(ctx, PALMAD_EINVAL, "k must be in [1, ncols]");
    if (minL < 1) return fail(ctx, PALMAD_EINVAL, "minL must be >= 1");
    int rc = enter(ctx, stream);
    if (rc) return rc;
    HIP_TRY(launch_interest(heat, L, ld, ncols, minL, k, col_score, col_len, top_idx, top_len,
                            top_score, ctx->work));
    return leave(ctx, stream);
}

int palmad_batched_workspace_size(int32_t B, const int64_t* offsets, const int32_t* minL,
                                  const int32_t* maxL, int32_t k, const palmad_options* opts,
                                  size_t* bytes)
{
    if (!bytes) return fail(nullptr, PALMAD_EINVAL, "bytes is NULL");
    std::vector<int64_t> n;
    int rc = validate_batch(nullptr, B, offsets, minL, maxL, k, &n);
    if (rc) return rc;
    Opts o;
    rc = read_opts(nullptr, opts, &o);
    if (rc) return rc;
    Plan p;
    make_plan(B, n.data(), minL, maxL, k, cfg_of(o, nullptr), &p);
    rc = check_grid(nullptr, p);
    if (rc) return rc;
    *bytes = p.total;
    return PALMAD_OK;
}

int palmad_discords_batched(palmad_ctx* ctx, const double* values, const int64_t* offsets,
                            int32_t B, const int32_t* minL, const int32_t* maxL, int32_t k,
                            const palmad_options* opts, void* workspace, size_t ws_bytes,
                            int64_t* idx, int32_t* len, double* nn_dist, int64_t* nn_idx,
                            int32_t* count, palmad_stats* stats, void* stream)
{
    if (!ctx) return fail(nullptr, PALMAD_EINVAL, "ctx is NULL");
    if (!values || !idx || !len || !nn_dist || !nn_idx || !count)
        return fail(ctx, PALMAD_EINVAL, "null input or output pointer");
    std::vector<int64_t> n;
    int rc = validate_batch(ctx, B, offsets, minL, maxL, k, &n);
    if (rc) return rc;
    Opts o;
    rc = read_opts(ctx, opts, &o);
    if (rc) return rc;
    Plan p;
    make_plan(B, n.data(), minL, maxL, k, cfg_of(o, nullptr), &p);
    rc = check_grid(ctx, p);
    if (rc) return rc;
    rc = check_ws(ctx, workspace, ws_bytes, p.total);
    if (rc) return rc;
    std::vector<const double*> tin(B);
    std::vector<Outputs> outs(B);
    int64_t row = 0, lrow = 0;
    for (int b = 0; b < B; ++b) {
        tin[b] = values + offsets[b];
        const int64_t L = (int64_t)maxL[b] - minL[b] + 1;
        outs[b] = {idx + row, len + row, nn_dist + row, nn_idx + row, count + lrow};
        row += L * k;
        lrow += L;
    }
    return search(ctx, p, o, workspace, tin.data(), outs.data(), stats, stream);
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
    KernelTimer timer = make_timer(ctx, o);
    SweepCfg cfg = cfg_of(o, &timer);
    Plan p;
    make_plan(1, &n, &m, &m, 1, cfg, &p);
    cfg.near_cols = p.near_cols;
    rc = check_ws(ctx, workspace, ws_bytes, p.total);
    if (rc) return rc;
    rc = enter(ctx, stream);
    if (rc) return rc;
    Batch bt;
    rc = upload(ctx, p, workspace, &T, nullptr, &bt);
    if (rc) return rc;
    rc = prepare(ctx, bt, p);
    if (rc) return rc;
    HIP_TRY(launch_set_fixed_r(bt, r, ctx->work));
    HIP_TRY(launch_round(bt, cfg, p.totals, ctx->work));
    const int64_t N = n - m + 1;
    HIP_TRY(launch_range_out(bt, N, (unsigned long long*)alive, nn_dist, ctx->work));
    const Ctrl* c = (const Ctrl*)((char*)workspace + p.base[0] + p.lay[0].off_ctrl);
    HIP_TRY(hipMemcpyAsync(ctx->pinned, &c->nsurv, sizeof(int32_t), hipMemcpyDeviceToHost,
                           ctx->work));
    HIP_TRY(hipStreamSynchronize(ctx->work));
    *count = (int64_t)(uint32_t)ctx->pinned[0];
    rc = accumulate(ctx, timer);
    if (rc) return rc;
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    rc = gather_stats(ctx, bt, timer, secs, stats);
    if (rc) return rc;
    return leave(ctx, stream);
}

int palmad_window_stats(palmad_ctx* ctx, const double* T, int64_t n, int32_t minL, int32_t m,
                        void* workspace, size_t ws_bytes, double* mu, double* sigma, void* stream)
{
    if (!ctx) return fail(nullptr, PALMAD_EINVAL, "ctx is NULL");
    if (!T || !mu || !sigma) return fail(ctx, PALMAD_EINVAL, "null input or output pointer");
    int rc = validate(ctx, n, minL, m, 1);
    if (rc) return rc;
    Plan p;
    make_plan(1, &n, &minL, &m, 1, cfg_of(default_opts(), nullptr), &p);
    rc = check_ws(ctx, workspace, ws_bytes, p.total);
    if (rc) return rc;
    rc = enter(ctx, stream);
    if (rc) return rc;
    Batch bt;
    rc = upload(ctx, p, workspace, &T, nullptr, &bt);
    if (rc) return rc;
    rc = prepare(ctx, bt, p);
    if (rc) return rc;
    HIP_TRY(launch_stats_to(bt, minL, m, p.totals, ctx->work));
    HIP_TRY(launch_stats_out(bt, n - m + 1, mu, sigma, ctx->work));
    HIP_TRY(hipStreamSynchronize(ctx->work));
    return leave(ctx, stream);
}

int palmad_selection_drift(palmad_ctx* ctx, const double* T, int64_t n, int32_t minL, int32_t m,
                           int64_t items, int32_t chunk, float guard, void* workspace,
                           size_t ws_bytes, double* drift, double* band, void* stream)
{
    if (!ctx) return fail(nullptr, PALMAD_EINVAL, "ctx is NULL");
    if (!T || !drift || !band) return fail(ctx, PALMAD_EINVAL, "null input or output pointer");
    int rc = validate(ctx, n, minL, m, 1);
    if (rc) return rc;
    if (chunk < 8) return fail(ctx, PALMAD_EINVAL, "need chunk >= 8");
    Plan p;
    make_plan(1, &n, &minL, &m, 1, cfg_of(default_opts(), nullptr), &p);
    const size_t off_out = al256(p.total);
    rc = check_ws(ctx, workspace, ws_bytes, off_out + 256);
    if (rc) return rc;
    rc = enter(ctx, stream);
    if (rc) return rc;
    Batch bt;
    rc = upload(ctx, p, workspace, &T, nullptr, &bt);
    if (rc) return rc;
    rc = prepare(ctx, bt, p);
    if (rc) return rc;
    double* out = (double*)((char*)workspace + off_out);
    HIP_TRY(launch_drift(bt, p.totals, minL, m, items, chunk, guard > 0.0f ? guard : 1.25e-4f, out,
                         ctx->work));
    unsigned long long h[2];
    HIP_TRY(hipMemcpyAsync(ctx->pinned + 16, out, sizeof h, hipMemcpyDeviceToHost, ctx->work));
    HIP_TRY(hipStreamSynchronize(ctx->work));
    std::memcpy(h, ctx->pinned + 16, sizeof h);
    // out[0] holds the ordered bits of a non-negative double: the bits themselves
    const unsigned long long u = h[0];
    const unsigned long long bits = (u & 0x8000000000000000ull) ? (u & ~0x8000000000000000ull) : ~u;
    std::memcpy(drift, &bits, sizeof(double));
    std::memcpy(band, &h[1], sizeof(double));
    return leave(ctx, stream);
}

int palmad_selection_drift_workspace_size(int64_t n, int32_t minL, int32_t m, size_t* bytes)
{
    if (!bytes) return fail(nullptr, PALMAD_EINVAL, "bytes is NULL");
    const int rc = validate(nullptr, n, minL, m, 1);
    if (rc) return rc;
    Plan p;
    make_plan(1, &n, &minL, &m, 1, cfg_of(default_opts(), nullptr), &p);
    *bytes = al256(p.total) + 256;
    return PALMAD_OK;
}

int palmad_backward_workspace_size(int64_t n, int64_t K, int32_t maxm, size_t* bytes)
{
    if (!bytes) return fail(nullptr, PALMAD_EINVAL, "bytes is NULL");
    if (K < 0) return fail(nullptr, PALMAD_EINVAL, "K must be >= 0");
    int rc = validate(nullptr, n, maxm, maxm, 1);
    if (rc) return rc;
    Plan p;
    int64_t nblk;
    *bytes = backward_bytes(n, K, maxm, &p, &nblk);
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
    Plan p;
    int64_t nblk;
    const size_t need = backward_bytes(n, K, maxm, &p, &nblk);
    rc = check_ws(ctx, workspace, ws_bytes, need);
    if (rc) return rc;
    rc = enter(ctx, stream);
    if (rc) return rc;
    Batch bt;
    rc = upload(ctx, p, workspace, &T, nullptr, &bt);
    if (rc) return rc;
    rc = prepare(ctx, bt, p);
    if (rc) return rc;
    if (K > 0) {
        // the adjoint reads the largest admissible length and the flat
        // threshold from the control block
        HIP_TRY(launch_set_len(bt, maxm, ctx->work));
        const SeriesDev s = carve((char*)workspace + p.base[0], p.lay[0]);
        double* part = (double*)((char*)workspace + p.total);
        HIP_TRY(launch_adjoint(s.T, n, K, maxm, idx, len, grad_nn, s.ctrl, part, nblk, grad_T,
                               nn_idx, ctx->work));
    }
    HIP_TRY(hipStreamSynchronize(ctx->work));
    return leave(ctx, stream);
}

int palmad_autotune_workspace_size(int32_t B, const int64_t* offsets, const int32_t* minL,
                                   const int32_t* maxL, int32_t k, int32_t probe_lengths,
                                   size_t* bytes)
{
    if (!bytes) return fail(nullptr, PALMAD_EINVAL, "bytes is NULL");
    if (probe_lengths < 1) return fail(nullptr, PALMAD_EINVAL, "probe_lengths must be >= 1");
    std::vector<int64_t> n;
    const int rc = validate_batch(nullptr, B, offsets, minL, maxL, k, &n);
    if (rc) return rc;
    Probe pr;
    make_probe(B, n.data(), minL, maxL, k, probe_lengths, &pr);
    *bytes = pr.total;
    return PALMAD_OK;
}

int palmad_autotune(palmad_ctx* ctx, const double* values, const int64_t* offsets, int32_t B,
                    const int32_t* minL, const int32_t* maxL, int32_t k,
                    const palmad_options* base, int32_t probe_lengths, int32_t reps,
                    void* workspace, size_t ws_bytes, palmad_options* best,
                    palmad_tune_report* report, void* stream)
{
    if (!ctx) return fail(nullptr, PALMAD_EINVAL, "ctx is NULL");
    if (!values || !best) return fail(ctx, PALMAD_EINVAL, "null values or best");
    if (probe_lengths < 1) return fail(ctx, PALMAD_EINVAL, "probe_lengths must be >= 1");
    if (reps < 1) return fail(ctx, PALMAD_EINVAL, "reps must be >= 1");
    std::vector<int64_t> n;
    int rc = validate_batch(ctx, B, offsets, minL, maxL, k, &n);
    if (rc) return rc;
    Opts cur;
    rc = read_opts(ctx, base, &cur);
    if (rc) return rc;
    cur.flags &= ~(unsigned int)PALMAD_FLAG_TIME_KERNELS;
    Probe pr;
    make_probe(B, n.data(), minL, maxL, k, probe_lengths, &pr);
    rc = check_grid(ctx, pr.plan);
    if (rc) return rc;
    rc = check_ws(ctx, workspace, ws_bytes, pr.total);
    if (rc) return rc;
    // result rows of the probe live after its search workspace
    char* o = (char*)workspace + pr.off_out;
    int64_t* idx = (int64_t*)o;
    int64_t* nnidx = idx + pr.rows;
    double* nn = (double*)(nnidx + pr.rows);
    int32_t* len = (int32_t*)(nn + pr.rows);
    int32_t* cnt = len + pr.rows;
    std::vector<const double*> tin(B);
    std::vector<Outputs> outs(B);
    int64_t row = 0, lrow = 0;
    for (int b = 0; b < B; ++b) {
        tin[b] = values + offsets[b];
        const int64_t L = (int64_t)pr.hi[b] - pr.lo[b] + 1;
        outs[b] = {idx + row, len + row, nn + row, nnidx + row, cnt + lrow};
        row += L * k;
        lrow += L;
    }
    // resolve the defaults to concrete values so every axis has a value
    {
        const SweepCfg c = cfg_of(cur, nullptr);
        cur.rows_near = 64 * c.q_near;
        cur.rows_far = 64 * c.q_far;
        cur.rows_refine = 64 * c.q_ref;
    }
    double t_best = 0.0;
    rc = time_probe(ctx, pr, k, cur, workspace, tin, outs, reps, stream, &t_best);
    if (rc) return rc;
    const double t_base = t_best;
    int evaluated = 1;
    static const int rows_v[] = {128, 256, 512};
    static const int chunk_v[] = {256, 512, 1024, 2048};
    static const int near_v[] = {1024, 2048, 8192, 32768, 1 << 30};
    static const int grid_v[] = {2048, 3072, 4096, 6144, 8192};
    static const int band_v[] = {0, 1};
    struct Axis {
        int* field;
        const int* vals;
        int count;
    };
    const Axis axes[] = {
        {&cur.chunk_cols, chunk_v, 4}, {&cur.near_cols, near_v, 5},  {&cur.rows_near, rows_v, 3},
        {&cur.rows_far, rows_v, 3},    {&cur.rows_refine, rows_v, 3}, {&cur.far_grid, grid_v, 5},
        {&cur.band_pass, band_v, 2},
    };
    // coordinate search, two passes over the axes (the best chunk length and
    // first-pass width depend on the tile heights chosen after them)
    for (int pass = 0; pass < 2; ++pass) {
        bool moved = false;
        for (const Axis& ax : axes) {
            const int keep = *ax.field;
            int best_v = keep;
            for (int i = 0; i < ax.count; ++i) {
                if (ax.vals[i] == keep) continue;
                *ax.field = ax.vals[i];
                double t = 0.0;
                rc = time_probe(ctx, pr, k, cur, workspace, tin, outs, reps, stream, &t);
                if (rc) return rc;
                ++evaluated;
                if (t < t_best) {
                    t_best = t;
                    best_v = ax.vals[i];
                }
            }
            *ax.field = best_v;
            moved = moved || best_v != keep;
        }
        if (!moved) break;
    }
    palmad_options r = {};
    r.dist_bits = cur.dist_bits;
    r.guard = cur.guard;
    r.near_cols = cur.near_cols;
    r.chunk_cols = cur.chunk_cols;
    r.flags = base ? base->flags : 0u;
    r.rows_near = cur.rows_near;
    r.rows_far = cur.rows_far;
    r.rows_refine = cur.rows_refine;
    r.far_grid = cur.far_grid;
    r.band_pass = cur.band_pass;
    *best = r;
    if (report) {
        report->evaluated = evaluated;
        report->probe_lengths = probe_lengths;
        report->base_seconds = t_base;
        report->best_seconds = t_best;
    }
    return PALMAD_OK;
}



int palmad_stream_workspace_size(int64_t capacity, int32_t minL, int32_t maxL, int32_t k,
                                 const palmad_options* opts, size_t* bytes)
{
    if (!bytes) return fail(nullptr, PALMAD_EINVAL, "bytes is NULL");
    int rc = validate(nullptr, capacity, minL, maxL, k);
    if (rc) return rc;
    Opts o;
    rc = read_opts(nullptr, opts, &o);
    if (rc) return rc;
    Plan p;
    make_plan(1, &capacity, &minL, &maxL, k, cfg_of(o, nullptr), &p);
    size_t a, b;
    *bytes = stream_bytes(p, maxL - minL + 1, &a, &b);
    return PALMAD_OK;
}

int palmad_stream_create(palmad_ctx* ctx, int64_t capacity, int32_t minL, int32_t maxL, int32_t k,
                         const palmad_options* opts, void* workspace, size_t ws_bytes,
                         palmad_stream** out, void* stream)
{
    if (!ctx) return fail(nullptr, PALMAD_EINVAL, "ctx is NULL");
    if (!out) return fail(ctx, PALMAD_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(ctx, capacity, minL, maxL, k);
    if (rc) return rc;
    Opts o;
    rc = read_opts(ctx, opts, &o);
    if (rc) return rc;
    palmad_stream* st = new (std::nothrow) palmad_stream();
    if (!st) return fail(ctx, PALMAD_ENOMEM, "stream allocation failed");
    st->ctx = ctx;
    st->o = o;
    st->cap = capacity;
    st->n = 0;
    st->minL = minL;
    st->maxL = maxL;
    st->k = k;
    make_plan(1, &capacity, &minL, &maxL, k, cfg_of(o, nullptr), &st->p);
    size_t off_prof, off_flag;
    const size_t need = stream_bytes(st->p, maxL - minL + 1, &off_prof, &off_flag);
    rc = check_ws(ctx, workspace, ws_bytes, need);
    if (rc) {
        delete st;
        return rc;
    }
    st->ws = workspace;
    st->prof = (unsigned long long*)((char*)workspace + off_prof);
    st->flag = (int32_t*)((char*)workspace + off_flag);
    rc = enter(ctx, stream);
    Batch bt;
    if (!rc) rc = stream_batch(st, nullptr, &bt);
    if (rc) {
        delete st;
        return rc;
    }
    const Layout& l = st->p.lay[0];
    const hipError_t e1 = launch_ctrl_init(bt, ctx->work);
    const hipError_t e2 = launch_fill_u64((unsigned long long*)((char*)workspace + st->p.base[0] + l.off_T),
                                          l.Tlen, 0ull, ctx->work);
    const hipError_t e3 = launch_fill_u64(st->prof, (int64_t)(maxL - minL + 1) * l.Npad,
                                          0x000fffffffffffffull, ctx->work);  // -inf
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
        delete st;
        return fail(ctx, PALMAD_EDEVICE, "stream initialisation failed");
    }
    rc = leave(ctx, stream);
    if (rc) {
        delete st;
        return rc;
    }
    *out = st;
    return PALMAD_OK;
}

void palmad_stream_destroy(palmad_stream* st)
{
    if (!st) return;
    (void)hipSetDevice(st->ctx->device);
    (void)hipStreamSynchronize(st->ctx->work);
    delete st;
}

int64_t palmad_stream_length(const palmad_stream* st) { return st ? st->n : -1; }

int palmad_stream_append(palmad_stream* st, const double* values, int64_t count, void* stream)
{
    if (!st) return fail(nullptr, PALMAD_EINVAL, "stream is NULL");
    palmad_ctx* ctx = st->ctx;
    if (!values) return fail(ctx, PALMAD_EINVAL, "values is NULL");
    if (count < 1) return fail(ctx, PALMAD_EINVAL, "count must be >= 1 (got %lld)", (long long)count);
    if (count > st->cap - st->n)
        return fail(ctx, PALMAD_EINVAL, "append of %lld points exceeds the capacity (%lld of %lld used)",
                    (long long)count, (long long)st->n, (long long)st->cap);
    int rc = enter(ctx, stream);
    if (rc) return rc;
    HIP_TRY(launch_check_finite(values, count, st->flag, ctx->work));
    HIP_TRY(hipMemcpyAsync(ctx->pinned, st->flag, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->work));
    HIP_TRY(hipStreamSynchronize(ctx->work));
    if (ctx->pinned[0]) return fail(ctx, PALMAD_ENONFINITE, "the appended values hold NaN or Inf");
    const int64_t n_old = st->n;
    st->n = n_old + count;
    Batch bt;
    rc = stream_batch(st, nullptr, &bt);
    if (rc) {
        st->n = n_old;
        return rc;
    }
    SweepCfg cfg = cfg_of(st->o, nullptr);
    HIP_TRY(launch_stream_append(bt, values, n_old, count, ctx->work));
    HIP_TRY(launch_stream_update(bt, cfg, st->p.totals, st->minL, st->maxL, st->prof, n_old,
                                 ctx->work));
    HIP_TRY(hipStreamSynchronize(ctx->work));
    return leave(ctx, stream);
}

int palmad_stream_discords(palmad_stream* st, int64_t* idx, int32_t* len, double* nn_dist,
                           int64_t* nn_idx, void* stream)
{
    if (!st) return fail(nullptr, PALMAD_EINVAL, "stream is NULL");
    palmad_ctx* ctx = st->ctx;
    if (!idx || !len || !nn_dist || !nn_idx) return fail(ctx, PALMAD_EINVAL, "null output pointer");
    int rc = validate(ctx, st->n, st->minL, st->maxL, st->k);
    if (rc) return rc;
    rc = enter(ctx, stream);
    if (rc) return rc;
    const Outputs out = {idx, len, nn_dist, nn_idx, nullptr};
    Batch bt;
    rc = stream_batch(st, &out, &bt);
    if (rc) return rc;
    HIP_TRY(launch_stream_query(bt, st->p.totals, st->minL, st->maxL, st->prof,
                                64 * cfg_of(st->o, nullptr).q_near, ctx->work));
    HIP_TRY(hipStreamSynchronize(ctx->work));
    return leave(ctx, stream);
}

int palmad_stream_profile(palmad_stream* st, int32_t m, double* nn_dist, void* stream)
{
    if (!st) return fail(nullptr, PALMAD_EINVAL, "stream is NULL");
    palmad_ctx* ctx = st->ctx;
    if (!nn_dist) return fail(ctx, PALMAD_EINVAL, "nn_dist is NULL");
    if (m < st->minL || m > st->maxL)
        return fail(ctx, PALMAD_EINVAL, "m (%d) outside [%d, %d]", m, st->minL, st->maxL);
    int rc = validate(ctx, st->n, st->minL, st->maxL, 1);
    if (rc) return rc;
    rc = enter(ctx, stream);
    if (rc) return rc;
    Batch bt;
    rc = stream_batch(st, nullptr, &bt);
    if (rc) return rc;
    HIP_TRY(launch_stream_profile(bt, st->p.totals, st->minL, m, st->prof, nn_dist, ctx->work));
    HIP_TRY(hipStreamSynchronize(ctx->work));
    return leave(ctx, stream);
}

}  // extern "C"
