"""Soundness of the FP32 selection sweep's guard band, checked on the CPU.

The selection sweep (Sec. 3.2) evaluates the Pearson correlation of every
pair in FP32 with the centred diagonal recurrence
    C(i, j) = C(i-1, j-1) + df[i-1] dg[j-1] + df[j-1] dg[i-1]
(df[i] = (t[i+m] - t[i]) / 2, dg[i] = (t[i+m] - mu[i+1]) + (t[i] - mu[i]),
both rounded to float32), started from exact FP64 values on a tile's first
column and top row (rounded to float32), and prunes a pair only when
rho~ = C * inv_i * inv_j (inv = 1 / (sqrt(m) sigma), float32) exceeds the
threshold by more than a guard band g.  Pruning is sound while
|rho~ - rho| stays below g.  The band the library uses at each length is
    g = max(1.25e-4, 4 * 2^-24 * sqrt(512) * gamma^2),
where gamma is the spread contrast of the series at that length: over blocks
of 256 windows, the largest sigma of the two blocks on either side over the
block's smallest sigma (windows with a small spread next to windows with a
large one amplify the covariance's absolute rounding error).  This test
replays the sweep's arithmetic on the CPU, operation by operation, on tiles
of the tallest height the sweep uses (512 rows, so chains of up to 511
recurrence steps), over the configured workloads (random walks and ECG-like
series, n = 1e4 .. 1e6), at tiles placed on the injected anomalies and at
random, and asserts the largest observed drift is below g / 4.

Each fused multiply-add is evaluated as a float64 product of the two float32
operands (exact: 48 significant bits) plus the float32 addend, rounded once
to float32; it equals the hardware's fused result except at double-rounding
ties, where it can differ by one float32 ulp, far below the margin asserted.
The exact correlations come from explicitly z-normalised windows in float64
(Eq. (4)) and one matrix product.
"""

import math

import numpy as np
import pytest

from paper_2304_01660_amd import synth

GUARD = 1.25e-4       # the library's default (smallest) guard band on rho
R = 512               # rows of the tallest sweep tile
NCOLS = 512           # columns replayed per tile


def _helpers(T, m):
    """Window statistics in FP64 (two-pass) and the sweep's FP32 helpers."""
    W = np.lib.stride_tricks.sliding_window_view(T, m)
    mu = W.mean(axis=1)
    sd = W.std(axis=1)
    N = W.shape[0]
    df = np.zeros(N)
    dg = np.zeros(N)
    df[:-1] = (T[m:m + N - 1] - T[:N - 1]) * 0.5
    dg[:-1] = (T[m:m + N - 1] - mu[1:]) + (T[:N - 1] - mu[:-1])
    inv = 1.0 / (math.sqrt(m) * sd)
    return mu, sd, df.astype(np.float32), dg.astype(np.float32), inv.astype(np.float32)


def contrast_guard(sd):
    """The guard band for window sigmas `sd`: the spread contrast over blocks
    of 256 windows, squared, times 4 * 2^-24 * sqrt(512), at least GUARD."""
    nb = (sd.shape[0] + 255) // 256
    pad = np.full(nb * 256, np.nan)
    pad[:sd.shape[0]] = sd
    blk = pad.reshape(nb, 256)
    bmax = np.nanmax(blk, axis=1)
    bmin = np.nanmin(blk, axis=1)
    hi = np.array([bmax[max(0, q - 2):q + 3].max() for q in range(nb)])
    gam2 = float(np.max((hi / bmin) ** 2))
    return max(GUARD, 4.0 * 2.0 ** -24 * math.sqrt(512.0) * gam2), gam2


def _zwin(T, m, mu, sd, lo, cnt):
    W = np.lib.stride_tricks.sliding_window_view(T, m)[lo:lo + cnt]
    return (W - mu[lo:lo + cnt, None]) / sd[lo:lo + cnt, None]


def _f32_fma(x, y, z):
    return (x.astype(np.float64) * y.astype(np.float64) + z.astype(np.float64)).astype(np.float32)


def _tile_drift(T, m, helpers, i0, j0):
    """Largest |rho~ - rho| over one R x NCOLS tile swept from (i0, j0)."""
    mu, sd, df, dg, inv = helpers
    Zr = _zwin(T, m, mu, sd, i0, R)
    Zc = _zwin(T, m, mu, sd, j0, NCOLS)
    rho = (Zr @ Zc.T) / m                                  # exact, FP64
    # exact covariances C = m sigma_i sigma_j rho on the first column and the
    # top row (the sweep's FP64 start and boundary values), rounded to float32
    cov = rho * (m * sd[i0:i0 + R, None] * sd[None, j0:j0 + NCOLS])
    C = np.empty((R, NCOLS), dtype=np.float32)
    C[0, :] = cov[0, :].astype(np.float32)
    C[:, 0] = cov[:, 0].astype(np.float32)
    dfj = df[j0:j0 + NCOLS - 1]     # df[j-1] for j = j0+1 ..
    dgj = dg[j0:j0 + NCOLS - 1]
    for r in range(1, R):
        ip = i0 + r - 1
        a = np.float32(df[ip]) * np.ones(NCOLS - 1, dtype=np.float32)
        b = np.float32(dg[ip]) * np.ones(NCOLS - 1, dtype=np.float32)
        inner = _f32_fma(dfj, b, C[r - 1, :-1])
        C[r, 1:] = _f32_fma(a, dgj, inner)
    rt = (C.astype(np.float64) * inv[i0:i0 + R, None].astype(np.float64)
          * inv[None, j0:j0 + NCOLS].astype(np.float64))
    return float(np.max(np.abs(rt - rho)))


def _tiles(w, rng, count_random):
    """Tile origins: one on every injected anomaly (rows there, columns to the
    right) plus random ones."""
    N = w.n - w.maxL + 1
    out = []
    for a in w.anomalies:
        i0 = int(min(max(0, a["position"] - R // 2), N - R - 1))
        j0 = int(rng.integers(i0, N - NCOLS))
        out.append((i0, j0))
    for _ in range(count_random):
        i0 = int(rng.integers(0, N - R - NCOLS))
        j0 = int(rng.integers(i0, N - NCOLS))
        out.append((i0, j0))
    return out


def _check(tag, w, lengths, count_random, seed):
    rng = np.random.default_rng(seed)
    tiles = _tiles(w, rng, count_random)
    for m in lengths:
        h = _helpers(w.T, m)
        g, gam2 = contrast_guard(h[1])
        worst = max(_tile_drift(w.T, m, h, i0, j0) for (i0, j0) in tiles)
        print(f"[fp32 drift] {tag} m={m}: max |rho32 - rho64| = {worst:.2e} over {len(tiles)} "
              f"tiles; gamma^2 = {gam2:.1f}, guard {g:.2e} ({g / worst:.1f}x)")
        assert worst <= g / 4, (tag, m, worst, g)


def test_fp32_drift_random_walk_100k():
    w = synth.config2()
    _check("c2", w, (w.minL, (w.minL + w.maxL) // 2, w.maxL), 4, 21)


def test_fp32_drift_ecg_1m():
    w = synth.config3()
    # 20 malformed beats: every anomaly tile at the two ends of the range
    _check("c3", w, (w.minL, w.maxL), 4, 22)


def test_fp32_drift_batch_series():
    ws = synth.config4()
    for s in (0, 7, 19, 31, 32, 40, 51, 63):   # random walks and ECG-like series
        w = ws[s]
        _check(f"c4[{s}]", w, (w.minL, w.maxL), 1, 230 + s)


def test_fp32_drift_random_walk_200k():
    w = synth.config5()
    _check("c5", w, (w.minL, w.maxL), 2, 24)


def test_guard_grows_with_spread_contrast():
    """A series whose windows alternate between a large and a tiny spread gets
    a guard band far above the default; a plain random walk keeps a band near
    the default."""
    rng = np.random.default_rng(9)
    t = np.arange(40000, dtype=np.float64)
    quiet = (t // 2000) % 2 == 0
    T = np.where(quiet, 1e-3, 1.0) * rng.standard_normal(t.shape[0])
    _, sd, _, _, _ = _helpers(T, 64)
    g, gam2 = contrast_guard(sd)
    assert gam2 > 1e5 and g > 0.1
    _, sd, _, _, _ = _helpers(synth.random_walk(rng, 40000), 64)
    g, _ = contrast_guard(sd)
    assert g < 1e-3


def test_drift_emulation_detects_a_wrong_helper():
    """The replay is sensitive: with dg rounded to bfloat16-like precision
    (8 significant bits) instead of float32 the drift exceeds the guard."""
    w = synth.config2()
    m = w.minL
    mu, sd, df, dg, inv = _helpers(w.T, m)
    coarse = dg.view(np.uint32) & np.uint32(0xFFFF0000)
    dgc = coarse.view(np.float32)
    d = _tile_drift(w.T, m, (mu, sd, df, dgc, inv), 20000, 50000)
    assert d > GUARD, d
