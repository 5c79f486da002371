"""Shared parity checks of the GPU tests (imported by the test modules).

Floating-point tolerance: the library evaluates distances in the Pearson
form ED^2 = 2m(1 - rho) in FP64 (Eq. (6)), the oracle on explicitly
z-normalised windows (Eq. (4)-(5)).  With rho carrying an absolute error of
about 1e-14, ED^2 may differ by 2m * 1e-12 absolutely plus 1e-9 relatively.
"""

import math

import numpy as np

import oracle
from oracle import bruteforce as bf

REL = 1e-9
RHO_ABS = 1e-12


def close_ed(a, b, m, rel=REL):
    """|a^2 - b^2| within 2m*RHO_ABS + rel*b^2 (elementwise, numpy)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a * a - b * b) <= 2.0 * m * RHO_ABS + 2.0 * rel * b * b + 1e-300


def check_against_profiles(T, out, minL, maxL, k, rel=REL):
    idx = out["idx"].cpu().numpy()
    ln = out["len"].cpu().numpy()
    nn = out["nn_dist"].cpu().numpy()
    nnj = out["nn_idx"].cpu().numpy()
    cnt = out["count"].cpu().numpy()
    assert np.all(cnt >= k)
    for m in range(minL, maxL + 1):
        P, J = bf.profile(T, m)
        rows = slice((m - minL) * k, (m - minL + 1) * k)
        exp = bf.topk(P, k)
        assert np.all(ln[rows] == m)
        for q in range(k):
            g, e = int(idx[rows][q]), int(exp[q])
            if g != e:
                assert close_ed(P[g], P[e], m, rel), (m, q, g, e, P[g], P[e])
            assert close_ed(nn[rows][q], P[g], m, rel), (m, q, nn[rows][q], P[g])
            j = int(nnj[rows][q])
            assert abs(j - g) >= m
            # the reported neighbour realises the nearest distance
            Zg = (T[g:g + m] - T[g:g + m].mean()) / T[g:g + m].std()
            Zj = (T[j:j + m] - T[j:j + m].mean()) / T[j:j + m].std()
            d = math.sqrt(((Zg - Zj) ** 2).sum())
            assert abs(d - P[g]) <= 1e-7 * max(1.0, P[g]), (m, q, j, J[g], d, P[g])


def match_rows(T, out, g, rel=REL):
    """Every row of a search result against a stored oracle result."""
    idx = out["idx"].cpu().numpy()
    ln = out["len"].cpu().numpy()
    nn = out["nn_dist"].cpu().numpy()
    nnj = out["nn_idx"].cpu().numpy()
    cnt = out["count"].cpu().numpy()
    gi = np.array(g["idx"])
    gn = np.array(g["nn"])
    gj = np.array(g["nnidx"])
    k = g["k"]
    assert idx.shape == gi.shape
    np.testing.assert_array_equal(ln, np.array(g["len"]))
    assert np.all(cnt >= k)
    ties = 0
    for q in range(gi.shape[0]):
        m = g["minL"] + q // k
        if idx[q] == gi[q]:
            assert nnj[q] == gj[q], (q, m, idx[q], nnj[q], gj[q])
        else:
            # near tie: the oracle's exact distance of the reported row
            d, j = oracle.nn_row(T, m, int(idx[q]))
            assert abs(d - gn[q]) <= rel * max(1.0, gn[q]), (q, idx[q], gi[q], d, gn[q])
            assert nnj[q] == j, (q, nnj[q], j)
            ties += 1
        assert abs(idx[q] - nnj[q]) >= m
        assert 0 < nn[q] <= 2 * math.sqrt(m) + 1e-12
    np.testing.assert_allclose(nn, gn, rtol=rel)
    return ties
