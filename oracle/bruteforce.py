"""TEST INFRASTRUCTURE ONLY: brute-force discords from the plain definition.

For every subsequence length m, P_m(i) is the smallest z-normalised Euclidean
distance from subsequence i to any non-self match j (|i - j| >= m), and the
top-k discords are the k indices with the largest P_m (Sec. 2.1, Eq. (3)-(5)).
This module evaluates that definition directly with numpy in float64:
explicit z-normalised windows (Eq. (4)), explicit squared differences
(Eq. (5)), an all-pairs matrix per row block, self matches masked.  No
pruning, no recurrences, no dot-product identity.

Only tests, the smoke check and the benchmark's CPU baseline import this.
Flat windows follow the same convention as the C oracle: sigma <= 1e-12 *
max(1, sigma of the series); flat-flat distance 0, flat-other sqrt(2m).
"""

from __future__ import annotations

import numpy as np
from numpy.lib.stride_tricks import sliding_window_view

FLAT_REL = 1e-12


def znorm_windows(T: np.ndarray, m: int):
    """All windows of length m, z-normalised (Eq. (4), population sigma)."""
    T = np.asarray(T, dtype=np.float64)
    W = sliding_window_view(T, m)
    mu = W.mean(axis=1)
    sd = W.std(axis=1)
    flat = sd <= FLAT_REL * max(1.0, float(np.std(T)))
    safe = np.where(flat, 1.0, sd)
    Z = (W - mu[:, None]) / safe[:, None]
    Z[flat] = 0.0
    return Z, mu, sd, flat


def profile(T: np.ndarray, m: int, block: int = 64):
    """Return (P, jstar): exact nearest-non-self-match distance per row."""
    Z, _, _, flat = znorm_windows(T, m)
    N = Z.shape[0]
    P = np.empty(N)
    J = np.empty(N, dtype=np.int64)
    cols = np.arange(N)
    for r0 in range(0, N, block):
        r1 = min(N, r0 + block)
        diff = Z[r0:r1, None, :] - Z[None, :, :]
        D2 = np.einsum("ijk,ijk->ij", diff, diff)
        rows = np.arange(r0, r1)
        # flat windows: distance 0 to another flat window, 2m to anything else
        fr = flat[r0:r1]
        if fr.any() or flat.any():
            both = fr[:, None] & flat[None, :]
            one = fr[:, None] ^ flat[None, :]
            D2 = np.where(both, 0.0, np.where(one, 2.0 * m, D2))
        self_match = np.abs(rows[:, None] - cols[None, :]) < m
        D2[self_match] = np.inf
        j = np.argmin(D2, axis=1)          # first minimum = smallest j
        J[r0:r1] = j
        P[r0:r1] = np.sqrt(D2[np.arange(r1 - r0), j])
    return P, J


def topk(P: np.ndarray, k: int):
    """Indices of the k largest P, ties broken by smaller index."""
    order = np.lexsort((np.arange(P.shape[0]), -P))
    return order[:k]


def discords(T: np.ndarray, minL: int, maxL: int, k: int):
    """Top-k discords for every length in [minL, maxL] by brute force.

    Returns dict with arrays idx[L*k], len[L*k], nn[L*k], nnidx[L*k], row
    q = (m - minL) * k + rank.
    """
    idx, lens, nn, nnidx = [], [], [], []
    for m in range(minL, maxL + 1):
        P, J = profile(T, m)
        top = topk(P, k)
        idx.extend(int(i) for i in top)
        lens.extend([m] * k)
        nn.extend(float(P[i]) for i in top)
        nnidx.extend(int(J[i]) for i in top)
    return {
        "idx": np.array(idx, dtype=np.int64),
        "len": np.array(lens, dtype=np.int32),
        "nn": np.array(nn, dtype=np.float64),
        "nnidx": np.array(nnidx, dtype=np.int64),
    }
