/*
 * oracle/merlin.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, serial, FP64 reference implementation of range-discord search over
 * a range of subsequence lengths (MERLIN driving DRAG), written from the
 * paper's definitions (Sec. 2.1) and its serial algorithms (Sec. 2.2,
 * Alg. 1 and Alg. 2).  It exists so that tests, the smoke check and the
 * benchmark's CPU baseline have something slow and obviously correct to
 * compare the GPU path against.  The product library never links, loads or
 * calls this file, and this file shares no code, header or table with it.
 *
 * Deliberate choices, each a reading of a point the paper leaves open:
 *   - Indices are 0-based; subsequence i covers T[i .. i+m-1].
 *   - Two subsequences are a non-self match iff |i - j| >= m (Sec. 2.1).
 *   - Statistics are computed directly per window with two passes in FP64
 *     (mean first, then the mean squared deviation): the definition of
 *     Eq. (4) with the population 1/m normalisation.  The recurrences of
 *     Eq. (7)-(8) are NOT used here, so they are checked, not assumed.
 *   - Distances are computed on explicitly z-normalised windows, Eq. (4)
 *     followed by Eq. (5).  The dot-product form of Eq. (6) is not used.
 *   - r and every reported nnDist are in Euclidean-distance units.  When
 *     r <= 0 nothing can be closer than r, so nothing is pruned.
 *   - A window is flat when its sigma <= 1e-12 * max(1, sigma of the whole
 *     series).  A flat window is at distance 0 from another flat window and
 *     at distance sqrt(2m) from any other window.
 *   - MERLIN repeats DRAG at one length while fewer than k discords are
 *     found; after a failure r is lowered before the retry; the nnDist of a
 *     length that feeds the next r is the smallest of its reported top-k;
 *     the spread of the last five is a population standard deviation; when
 *     that spread is zero, r is lowered by 1% instead.
 *   - Ties: larger nnDist first, then smaller index; a nearest neighbour
 *     tie keeps the smaller neighbour index.
 *
 * Built plainly this file is serial.  Built with -fopenmp (the second
 * library the Python wrapper offers, for the largest workloads), phase 1's
 * inner loop over the current candidates of each scanned subsequence is
 * split over threads once the candidate list is long, and phase 2 scans
 * each candidate on a thread of its own.  Every decision in either loop
 * depends only on the pair (scanned subsequence, candidate) and on the
 * candidate's own running nearest-neighbour state, so every candidate sees
 * the subsequences in the order of Alg. 2 and every result (indices,
 * distances, neighbour indices, evaluation counts) is the same as the
 * serial build's.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL -1
#define OR_ENOMEM -5

/* Threads the OpenMP build uses after this call (want > 0 sets it); the
   serial build always reports 1. */
int oracle_threads(int want)
{
#ifdef _OPENMP
    if (want > 0) omp_set_num_threads(want);
    return omp_get_max_threads();
#else
    (void)want;
    return 1;
#endif
}

/* Flat-window threshold factor (see header). */
static const double FLAT_REL = 1e-12;

/* Population standard deviation of the whole series, two passes. */
static double series_sigma(const double* T, int64_t n)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += T[i];
    double mu = s / (double)n;
    double q = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double d = T[i] - mu;
        q += d * d;
    }
    return sqrt(q / (double)n);
}

/*
 * Eq. (4): mean and population standard deviation of every window of length
 * m, each computed from scratch in two passes.
 */
void oracle_window_stats(const double* T, int64_t n, int32_t m, double* mu, double* sigma)
{
    int64_t N = n - m + 1;
    for (int64_t i = 0; i < N; ++i) {
        double s = 0.0;
        for (int32_t k = 0; k < m; ++k) s += T[i + k];
        double mean = s / (double)m;
        double q = 0.0;
        for (int32_t k = 0; k < m; ++k) {
            double d = T[i + k] - mean;
            q += d * d;
        }
        mu[i] = mean;
        sigma[i] = sqrt(q / (double)m);
    }
}

typedef struct {
    const double* T;
    int64_t n;
    int32_t m;
    int64_t N;
    double* mu;
    double* sigma;
    unsigned char* flat;
} series_m;

static int series_m_init(series_m* s, const double* T, int64_t n, int32_t m, double flat_eps)
{
    s->T = T;
    s->n = n;
    s->m = m;
    s->N = n - m + 1;
    s->mu = (double*)malloc(sizeof(double) * (size_t)s->N);
    s->sigma = (double*)malloc(sizeof(double) * (size_t)s->N);
    s->flat = (unsigned char*)malloc((size_t)s->N);
    if (!s->mu || !s->sigma || !s->flat) {
        free(s->mu);
        free(s->sigma);
        free(s->flat);
        return OR_ENOMEM;
    }
    oracle_window_stats(T, n, m, s->mu, s->sigma);
    for (int64_t i = 0; i < s->N; ++i) s->flat[i] = (s->sigma[i] <= flat_eps) ? 1 : 0;
    return OR_OK;
}

static void series_m_free(series_m* s)
{
    free(s->mu);
    free(s->sigma);
    free(s->flat);
}

/*
 * Squared Euclidean distance between the z-normalised windows i and j,
 * Eq. (4) then Eq. (5).  Summation stops early once the partial sum reaches
 * `bound2` (the EarlyAbandonED procedure of Sec. 2.2); the partial sum is
 * returned then, which is >= bound2.
 */
static double zdist2(const series_m* s, int64_t i, int64_t j, double bound2)
{
    if (s->flat[i] || s->flat[j]) {
        if (s->flat[i] && s->flat[j]) return 0.0;
        return 2.0 * (double)s->m;
    }
    const double* x = s->T + i;
    const double* y = s->T + j;
    double mx = s->mu[i], my = s->mu[j];
    double sx = s->sigma[i], sy = s->sigma[j];
    double acc = 0.0;
    for (int32_t k = 0; k < s->m; ++k) {
        double d = (x[k] - mx) / sx - (y[k] - my) / sy;
        acc += d * d;
        if (acc >= bound2) return acc;
    }
    return acc;
}

static int64_t iabs64(int64_t a) { return a < 0 ? -a : a; }

/*
 * DRAG (Alg. 2) at length m with range r.
 *
 * Phase 1 (candidate selection): scan the subsequences in order; every
 * candidate that is a non-self match of the scanned subsequence and closer
 * than r is dropped, and the scanned subsequence becomes a candidate only if
 * it was closer than r to none of them.
 *
 * Phase 2 (refinement): scan all subsequences again; a candidate with a
 * non-self match closer than r is dropped, otherwise its nearest-neighbour
 * distance is the minimum over all of its non-self matches, found with
 * early abandoning at the current best.
 *
 * On return out_idx/out_nn/out_nnidx hold the surviving candidates (the
 * range discords) in increasing index order; the count is returned via
 * *out_count.  Buffers must hold N = n - m + 1 entries.
 */
/* Candidate lists at least this long have their inner loop split over
   threads in the OpenMP build; shorter ones stay serial (thread start-up
   would cost more than the loop). */
#define PAR_MIN_CANDIDATES 256

/*
 * Phase 1 inner step for the candidates cand[a0 .. a1): hit[a] = 1 when
 * candidate cand[a] is a non-self match of subsequence sidx closer than r.
 * Returns the number of distance evaluations made.
 */
static uint64_t phase1_hits(const series_m* s, int64_t sidx, const int64_t* cand, int64_t a0,
                            int64_t a1, double r2, unsigned char* hit)
{
    uint64_t ev = 0;
    for (int64_t a = a0; a < a1; ++a) {
        int64_t c = cand[a];
        hit[a] = 0;
        if (iabs64(sidx - c) >= s->m) {
            ++ev;
            if (zdist2(s, sidx, c, r2) < r2) hit[a] = 1;
        }
    }
    return ev;
}

/*
 * Phase 2 inner step for the candidates cand[a0 .. a1) against subsequence
 * sidx: a non-self match closer than r marks the candidate dead (hit = 1);
 * otherwise a closer match updates the candidate's nearest neighbour (strict
 * <, so the first, i.e. smallest, index wins ties).  Returns the number of
 * distance evaluations made.
 */
static uint64_t phase2_step(const series_m* s, int64_t sidx, const int64_t* cand, int64_t a0,
                            int64_t a1, int prune, double r2, double* nn2, int64_t* nnj,
                            unsigned char* hit)
{
    uint64_t ev = 0;
    for (int64_t a = a0; a < a1; ++a) {
        int64_t c = cand[a];
        hit[a] = 0;
        if (iabs64(sidx - c) >= s->m) {
            ++ev;
            double d2 = zdist2(s, sidx, c, nn2[c]);
            if (prune && d2 < r2) {
                hit[a] = 1;
            } else if (d2 < nn2[c]) {
                nn2[c] = d2;
                nnj[c] = sidx;
            }
        }
    }
    return ev;
}

#ifdef _OPENMP
static uint64_t phase1_hits_par(const series_m* s, int64_t sidx, const int64_t* cand, int64_t nc,
                                double r2, unsigned char* hit)
{
    uint64_t ev = 0;
    int64_t chunk = 64;
#pragma omp parallel for schedule(dynamic) reduction(+ : ev)
    for (int64_t a0 = 0; a0 < nc; a0 += chunk) {
        int64_t a1 = a0 + chunk < nc ? a0 + chunk : nc;
        ev += phase1_hits(s, sidx, cand, a0, a1, r2, hit);
    }
    return ev;
}

/*
 * The whole of phase 2 with the candidates split over threads.  A
 * candidate's fate in phase 2 depends only on its own scan: it is compared
 * with the subsequences in increasing order until one of them is closer
 * than r, and its running nearest neighbour is its own.  Scanning each
 * candidate to the end (or to its first hit) on its own thread therefore
 * evaluates exactly the pairs the interleaved scan evaluates, in the same
 * order per candidate, with the same results.  hit[a] = 1 marks a
 * candidate dropped by a hit.
 */
static uint64_t phase2_par(const series_m* s, const int64_t* cand, int64_t nc, int prune,
                           double r2, double* nn2, int64_t* nnj, unsigned char* hit)
{
    uint64_t ev = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : ev)
    for (int64_t a = 0; a < nc; ++a) {
        hit[a] = 0;
        for (int64_t sidx = 0; sidx < s->N; ++sidx) {
            ev += phase2_step(s, sidx, cand, a, a + 1, prune, r2, nn2, nnj, hit);
            if (hit[a]) break;
        }
    }
    return ev;
}
#endif

/*
 * DRAG (Alg. 2) at length m with range r.
 *
 * Phase 1 (candidate selection): scan the subsequences in order; every
 * candidate that is a non-self match of the scanned subsequence and closer
 * than r is dropped, and the scanned subsequence becomes a candidate only if
 * it was closer than r to none of them.
 *
 * Phase 2 (refinement): scan all subsequences again; a candidate with a
 * non-self match closer than r is dropped, otherwise its nearest-neighbour
 * distance is the minimum over all of its non-self matches, found with
 * early abandoning at the current best.
 *
 * On return out_idx/out_nn/out_nnidx hold the surviving candidates (the
 * range discords) in increasing index order; the count is returned via
 * *out_count and the number of distance evaluations is added to *evals.
 * Buffers must hold N = n - m + 1 entries.
 */
static int drag_core(const series_m* s, double r, int64_t* out_idx, double* out_nn,
                     int64_t* out_nnidx, int64_t* out_count, uint64_t* evals)
{
    const int64_t N = s->N;
    const int prune = r > 0.0;
    const double r2 = prune ? r * r : 0.0;
    uint64_t ev = 0;

    int64_t* cand = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
    unsigned char* hit = (unsigned char*)malloc((size_t)N);
    double* nn2 = (double*)malloc(sizeof(double) * (size_t)N);
    int64_t* nnj = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
    if (!cand || !hit || !nn2 || !nnj) {
        free(cand);
        free(hit);
        free(nn2);
        free(nnj);
        return OR_ENOMEM;
    }

    /* ---- phase 1 ---- */
    int64_t nc = 0;
    cand[nc++] = 0;
    for (int64_t sidx = 1; sidx < N; ++sidx) {
        int is_cand = 1;
        if (prune) {
#ifdef _OPENMP
            if (nc >= PAR_MIN_CANDIDATES)
                ev += phase1_hits_par(s, sidx, cand, nc, r2, hit);
            else
#endif
                ev += phase1_hits(s, sidx, cand, 0, nc, r2, hit);
            /* drop every hit candidate, keeping the list in index order */
            int64_t w = 0;
            for (int64_t a = 0; a < nc; ++a) {
                if (hit[a]) is_cand = 0;
                else cand[w++] = cand[a];
            }
            nc = w;
        }
        if (is_cand) cand[nc++] = sidx;
    }

    /* ---- phase 2 ---- */
    for (int64_t a = 0; a < nc; ++a) {
        nn2[cand[a]] = INFINITY;
        nnj[cand[a]] = -1;
    }
    /* The candidate list stays sorted by index (phase 1 appends in scan
       order and removal keeps relative order), so dead entries can be
       compacted out as the scan proceeds. */
#ifdef _OPENMP
    if (nc >= 2) {
        ev += phase2_par(s, cand, nc, prune, r2, nn2, nnj, hit);
        int64_t w = 0;
        for (int64_t a = 0; a < nc; ++a)
            if (!hit[a]) cand[w++] = cand[a];
        nc = w;
    } else
#endif
    for (int64_t sidx = 0; sidx < N; ++sidx) {
        ev += phase2_step(s, sidx, cand, 0, nc, prune, r2, nn2, nnj, hit);
        int64_t w = 0;
        for (int64_t a = 0; a < nc; ++a)
            if (!hit[a]) cand[w++] = cand[a];
        nc = w;
    }
    for (int64_t a = 0; a < nc; ++a) {
        int64_t c = cand[a];
        out_idx[a] = c;
        out_nn[a] = sqrt(nn2[c]);
        out_nnidx[a] = nnj[c];
    }
    *out_count = nc;
    *evals += ev;
    free(cand);
    free(hit);
    free(nn2);
    free(nnj);
    return OR_OK;
}

static double flat_eps_of(const double* T, int64_t n)
{
    double sg = series_sigma(T, n);
    return FLAT_REL * (sg > 1.0 ? sg : 1.0);
}

/* Public DRAG entry: one range-discord search at length m and range r. */
int oracle_drag(const double* T, int64_t n, int32_t m, double r, int64_t* out_idx, double* out_nn,
                int64_t* out_nnidx, int64_t* out_count, uint64_t* out_evals)
{
    if (!T || !out_idx || !out_nn || !out_nnidx || !out_count) return OR_EINVAL;
    if (m < 3 || n < 2 * (int64_t)m) return OR_EINVAL;
    series_m s;
    if (series_m_init(&s, T, n, m, flat_eps_of(T, n)) != OR_OK) return OR_ENOMEM;
    uint64_t ev = 0;
    int rc = drag_core(&s, r, out_idx, out_nn, out_nnidx, out_count, &ev);
    if (out_evals) *out_evals = ev;
    series_m_free(&s);
    return rc;
}

/*
 * Exact nearest-non-self-match distance of one subsequence: the minimum over
 * every j with |i - j| >= m of the z-normalised distance (the quantity whose
 * maximum defines a discord, Eq. (3)).  Ties keep the smaller j.
 */
int oracle_nn_row(const double* T, int64_t n, int32_t m, int64_t i, double* out_nn, int64_t* out_j)
{
    if (!T || !out_nn || !out_j || m < 3 || i < 0 || i > n - m) return OR_EINVAL;
    series_m s;
    if (series_m_init(&s, T, n, m, flat_eps_of(T, n)) != OR_OK) return OR_ENOMEM;
    double best = INFINITY;
    int64_t bj = -1;
    for (int64_t j = 0; j < s.N; ++j) {
        if (iabs64(i - j) < m) continue;
        double d2 = zdist2(&s, i, j, best);
        if (d2 < best) {
            best = d2;
            bj = j;
        }
    }
    *out_nn = sqrt(best);
    *out_j = bj;
    series_m_free(&s);
    return OR_OK;
}

/* Order for reporting: larger nnDist first, then smaller index. */
typedef struct {
    int64_t idx;
    double nn;
    int64_t nnidx;
} disc;

static int disc_cmp(const void* a, const void* b)
{
    const disc* x = (const disc*)a;
    const disc* y = (const disc*)b;
    if (x->nn > y->nn) return -1;
    if (x->nn < y->nn) return 1;
    if (x->idx < y->idx) return -1;
    if (x->idx > y->idx) return 1;
    return 0;
}

/*
 * MERLIN (Alg. 1): for every length m in [minL, maxL], call DRAG with an
 * adaptively chosen r until at least k discords of that length are found,
 * then report the k with the largest nnDist.
 *
 *   m = minL:              r = 2*sqrt(minL), halved after each failure.
 *   minL < m <= minL + 4:  r = 0.99 * nnDist(m-1), times 0.99 after each failure.
 *   m >= minL + 5:         r = mean - 2*std of nnDist(m-5..m-1), lowered by
 *                          that std after each failure (by 1% when std = 0).
 *
 * Output row q = (m - minL) * k + rank.  calls[m - minL] receives the number
 * of DRAG invocations at that length and r_final[m - minL] the r of the
 * successful one; evals (optional) the total number of distance evaluations.
 */
int oracle_merlin(const double* T, int64_t n, int32_t minL, int32_t maxL, int32_t k, int64_t* idx,
                  int32_t* len, double* nn, int64_t* nnidx, int32_t* calls, double* r_final,
                  uint64_t* evals)
{
    if (!T || !idx || !len || !nn || !nnidx) return OR_EINVAL;
    if (minL < 3 || maxL < minL || k < 1) return OR_EINVAL;
    if (n < 3 * (int64_t)maxL - 1) return OR_EINVAL;
    if ((int64_t)k > n - maxL + 1) return OR_EINVAL;

    const double feps = flat_eps_of(T, n);
    const int32_t L = maxL - minL + 1;
    double* hist = (double*)malloc(sizeof(double) * (size_t)L);
    int64_t Nmax = n - minL + 1;
    int64_t* d_idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)Nmax);
    double* d_nn = (double*)malloc(sizeof(double) * (size_t)Nmax);
    int64_t* d_nnidx = (int64_t*)malloc(sizeof(int64_t) * (size_t)Nmax);
    disc* order = (disc*)malloc(sizeof(disc) * (size_t)Nmax);
    if (!hist || !d_idx || !d_nn || !d_nnidx || !order) {
        free(hist);
        free(d_idx);
        free(d_nn);
        free(d_nnidx);
        free(order);
        return OR_ENOMEM;
    }
    uint64_t total_evals = 0;
    int rc = OR_OK;
    for (int32_t m = minL; m <= maxL && rc == OR_OK; ++m) {
        const int32_t li = m - minL;
        series_m s;
        if (series_m_init(&s, T, n, m, feps) != OR_OK) {
            rc = OR_ENOMEM;
            break;
        }
        double r, step = 0.0;
        int mode;
        if (li == 0) {
            r = 2.0 * sqrt((double)minL);
            mode = 0;
        } else if (li <= 4) {
            r = 0.99 * hist[li - 1];
            mode = 1;
        } else {
            double mean = 0.0;
            for (int q = 1; q <= 5; ++q) mean += hist[li - q];
            mean /= 5.0;
            double var = 0.0;
            for (int q = 1; q <= 5; ++q) {
                double d = hist[li - q] - mean;
                var += d * d;
            }
            step = sqrt(var / 5.0);
            r = mean - 2.0 * step;
            mode = 2;
        }
        int32_t ncall = 0;
        int64_t cnt = 0;
        for (;;) {
            ++ncall;
            rc = drag_core(&s, r, d_idx, d_nn, d_nnidx, &cnt, &total_evals);
            if (rc != OR_OK) break;
            if (cnt >= k) break;
            if (mode == 0) r *= 0.5;
            else if (mode == 1) r *= 0.99;
            else r = (step > 0.0) ? r - step : 0.99 * r;
        }
        series_m_free(&s);
        if (rc != OR_OK) break;
        for (int64_t a = 0; a < cnt; ++a) {
            order[a].idx = d_idx[a];
            order[a].nn = d_nn[a];
            order[a].nnidx = d_nnidx[a];
        }
        qsort(order, (size_t)cnt, sizeof(disc), disc_cmp);
        for (int32_t q = 0; q < k; ++q) {
            int64_t row = (int64_t)li * k + q;
            idx[row] = order[q].idx;
            len[row] = m;
            nn[row] = order[q].nn;
            nnidx[row] = order[q].nnidx;
        }
        hist[li] = order[k - 1].nn;
        if (calls) calls[li] = ncall;
        if (r_final) r_final[li] = r;
    }
    if (evals) *evals = total_evals;
    free(hist);
    free(d_idx);
    free(d_nn);
    free(d_nnidx);
    free(order);
    return rc;
}

/*
 * Gradient of one reported nnDist with respect to the series values, at a
 * fixed discord i, its nearest neighbour j and length m (both taken from the
 * forward search, so the argmin is held fixed).  The distance is
 * d = ED(x^, y^) of the z-normalised windows (Eq. (4)-(5)); the gradient is
 * the chain rule through the z-normalisation Jacobian, written out below
 * from those definitions.  Accumulates g * gradient into grad (length n).
 * A zero distance or a flat window contributes nothing.
 */
int oracle_nn_grad(const double* T, int64_t n, int32_t m, int64_t i, int64_t j, double g, double* grad)
{
    if (!T || !grad || m < 3 || i < 0 || j < 0 || i > n - m || j > n - m) return OR_EINVAL;
    const double* x = T + i;
    const double* y = T + j;
    double sx = 0.0, sy = 0.0;
    for (int32_t k = 0; k < m; ++k) {
        sx += x[k];
        sy += y[k];
    }
    double mx = sx / m, my = sy / m;
    double vx = 0.0, vy = 0.0;
    for (int32_t k = 0; k < m; ++k) {
        vx += (x[k] - mx) * (x[k] - mx);
        vy += (y[k] - my) * (y[k] - my);
    }
    double sdx = sqrt(vx / m), sdy = sqrt(vy / m);
    double feps = flat_eps_of(T, n);
    if (sdx <= feps || sdy <= feps) return OR_OK;
    double d2 = 0.0;
    for (int32_t k = 0; k < m; ++k) {
        double dd = (x[k] - mx) / sdx - (y[k] - my) / sdy;
        d2 += dd * dd;
    }
    double d = sqrt(d2);
    if (!(d > 0.0)) return OR_OK;
    /* d = sqrt(sum_k (xh_k - yh_k)^2); dd/dxh_k = (xh_k - yh_k)/d.
       xh = (x - mx)/sdx, so the Jacobian of xh w.r.t. x is
       (I - 1 1^T/m - xh xh^T/m) / sdx.  Applying it to u = (xh - yh)/d:
       grad_x = (u - mean(u) - xh * (xh . u)/m) / sdx, and mean(u) = 0. */
    double xu = 0.0, yu = 0.0;
    for (int32_t k = 0; k < m; ++k) {
        double xh = (x[k] - mx) / sdx, yh = (y[k] - my) / sdy;
        double u = (xh - yh) / d;
        xu += xh * u;
        yu += yh * (-u);
    }
    for (int32_t k = 0; k < m; ++k) {
        double xh = (x[k] - mx) / sdx, yh = (y[k] - my) / sdy;
        double u = (xh - yh) / d;
        grad[i + k] += g * (u - xh * xu / m) / sdx;
        grad[j + k] += g * (-u - yh * yu / m) / sdy;
    }
    return OR_OK;
}
