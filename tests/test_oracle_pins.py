"""Pins for the CPU oracle: it is checked against things other than itself.

* brute force over the plain definition (oracle/bruteforce.py) on many tiny
  seeded series -- MERLIN/DRAG must return exactly the top-k of P_m;
* DRAG at a fixed r must return exactly {i : P_m(i) >= r} (Alg. 2's range
  discord set, Sec. 2.1);
* library routines: numpy mean/std for Eq. (4), numpy.corrcoef for the
  Pearson form of Eq. (6);
* closed forms and special cases: exact copies inside / just outside the
  self-match zone, flat windows, distance bounds 0 <= ED <= 2 sqrt(m);
* invariances: affine maps of T, time reversal;
* the recurrences of Eq. (7)-(8) against direct two-pass statistics.
"""

import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import bruteforce as bf
from paper_2304_01660_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _tiny_cases(count=210):
    rng = np.random.default_rng(12345)
    kinds = ("rw", "noise", "ecg")
    for c in range(count):
        maxL = int(rng.integers(3, 21))
        minL = int(rng.integers(3, maxL + 1))
        minL = max(minL, maxL - 3)           # at most 4 lengths per case
        n = int(rng.integers(max(60, 3 * maxL - 1), 601))
        k = int((1, 3, 5)[c % 3])
        kind = kinds[c % 3]
        T = synth.small_random(1000 + c, n, kind)
        yield c, T, minL, maxL, k


def _check_topk(T, got_idx, got_nn, minL, maxL, k, rel=1e-12):
    for m in range(minL, maxL + 1):
        P, _ = bf.profile(T, m)
        rows = slice((m - minL) * k, (m - minL + 1) * k)
        gi = got_idx[rows]
        gn = got_nn[rows]
        exp = bf.topk(P, k)
        np.testing.assert_allclose(gn, P[exp], rtol=rel, atol=1e-12)
        for q in range(k):
            if gi[q] != exp[q]:
                # only a near-tie may reorder: the picked row's exact P must
                # equal the expected one to the tolerance
                assert abs(P[gi[q]] - P[exp[q]]) <= rel * max(1.0, P[exp[q]]), (m, q)
        np.testing.assert_allclose(P[gi], gn, rtol=rel, atol=1e-12)


def test_merlin_matches_bruteforce_on_tiny_series():
    n_cases = 0
    for c, T, minL, maxL, k in _tiny_cases():
        o = oracle.merlin(T, minL, maxL, k)
        _check_topk(T, o["idx"], o["nn"], minL, maxL, k)
        # nearest neighbour index: a true non-self match at exactly that distance
        for q in range(len(o["idx"])):
            m = int(o["len"][q])
            i, j = int(o["idx"][q]), int(o["nnidx"][q])
            assert abs(i - j) >= m
            d, jj = oracle.nn_row(T, m, i)
            assert jj == j
        n_cases += 1
    assert n_cases >= 200


@pytest.mark.parametrize("seed", range(12))
def test_drag_returns_exact_range_discord_set(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(150, 500))
    m = int(rng.integers(4, 25))
    T = synth.small_random(seed, n, ("rw", "noise", "ecg")[seed % 3])
    P, J = bf.profile(T, m)
    for qtl in (0.0, 0.5, 0.9, 0.99, 1.0):
        r = float(np.quantile(P, qtl)) * 0.999999
        idx, nn, nnidx, _ = oracle.drag(T, m, r)
        want = np.nonzero(P >= r)[0]
        np.testing.assert_array_equal(idx, want)
        np.testing.assert_allclose(nn, P[want], rtol=1e-12, atol=1e-12)
        np.testing.assert_array_equal(nnidx, J[want])
    # r above every distance: nothing survives; r <= 0: everything survives
    idx, _, _, _ = oracle.drag(T, m, 2.0 * math.sqrt(m) * 1.0001)
    assert idx.size == 0
    idx, nn, _, _ = oracle.drag(T, m, 0.0)
    np.testing.assert_array_equal(idx, np.arange(n - m + 1))
    np.testing.assert_allclose(nn, P, rtol=1e-12, atol=1e-12)
    idx, _, _, _ = oracle.drag(T, m, -1.0)
    assert idx.size == n - m + 1


def test_window_stats_match_numpy():
    T = synth.small_random(7, 3000, "rw") * 37.0 + 1e4
    for m in (3, 17, 128):
        mu, sd = oracle.window_stats(T, m)
        W = np.lib.stride_tricks.sliding_window_view(T, m)
        np.testing.assert_allclose(mu, W.mean(axis=1), rtol=1e-14)
        np.testing.assert_allclose(sd, W.std(axis=1), rtol=1e-9)


def test_recurrences_eq7_eq8_match_two_pass():
    """Eq. (7)-(8) (proved in the Appendix) reproduce the direct statistics."""
    T = synth.small_random(8, 5000, "rw")
    minL, maxL = 16, 80
    mu, sd = oracle.window_stats(T, minL)
    var = sd ** 2
    for m in range(minL, maxL):
        N1 = T.shape[0] - m          # windows of length m+1
        t = T[m:m + N1]              # t_{i+m}
        mu_n = (m * mu[:N1] + t) / (m + 1)
        var_n = m / (m + 1) * (var[:N1] + (mu[:N1] - t) ** 2 / (m + 1))
        mu, var = mu_n, var_n
        mu2, sd2 = oracle.window_stats(T, m + 1)
        scale = np.abs(T).max()
        np.testing.assert_allclose(mu, mu2, rtol=1e-12, atol=1e-13 * scale)
        np.testing.assert_allclose(np.sqrt(var), sd2, rtol=1e-10)


def test_pearson_identity_eq6():
    """ED^2 of z-normalised windows = 2m(1 - rho), rho from numpy.corrcoef."""
    T = synth.small_random(9, 800, "rw")
    rng = np.random.default_rng(0)
    for m in (5, 32, 100):
        N = T.shape[0] - m + 1
        for _ in range(40):
            i = int(rng.integers(0, N))
            d, j = oracle.nn_row(T, m, i)
            rho = np.corrcoef(T[i:i + m], T[j:j + m])[0, 1]
            assert abs(d * d - 2 * m * (1 - rho)) <= 1e-10 * (1 + d * d)


def test_distance_bounds():
    for seed in range(6):
        T = synth.small_random(20 + seed, 400, ("rw", "noise", "ecg")[seed % 3])
        for m in (3, 10, 40):
            P, _ = bf.profile(T, m)
            assert np.all(P >= 0) and np.all(P <= 2 * math.sqrt(m) + 1e-12)
            o = oracle.merlin(T, m, m, 3)
            assert np.all(o["nn"] >= 0) and np.all(o["nn"] <= 2 * math.sqrt(m) + 1e-12)


def test_self_match_exclusion_boundary():
    """A copy at offset m-1 is a self match (ignored); at offset m it is not."""
    rng = np.random.default_rng(3)
    m = 12
    for off, expect_zero in ((m - 1, False), (m, True)):
        T = rng.standard_normal(300)
        i = 100
        T[i + off:i + off + m] = T[i:i + m] * 3.0 + 5.0     # affine copy = same z-norm window
        d, j = oracle.nn_row(T, m, i)
        P, J = bf.profile(T, m)
        assert abs(P[i] - d) <= 1e-12
        if expect_zero:
            assert d < 1e-6 and j == i + off
        else:
            assert d > 0.1


def test_flat_windows_convention():
    rng = np.random.default_rng(4)
    T = rng.standard_normal(400)
    T[50:90] = 2.5            # flat run long enough for several flat windows
    T[250:262] = -1.0         # a second flat run
    m = 10
    P, J = bf.profile(T, m)
    idx, nn, nnidx, _ = oracle.drag(T, m, 0.0)
    np.testing.assert_allclose(nn, P, rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(nnidx, J)
    # window 50 is flat and has a flat non-self match (window 80 or 250)
    assert P[50] == 0.0


def test_affine_and_reversal_invariance():
    T = synth.small_random(30, 500, "rw")
    minL, maxL, k = 8, 11, 3
    base = oracle.merlin(T, minL, maxL, k)
    aff = oracle.merlin(-2.5 * T + 7.0, minL, maxL, k)
    np.testing.assert_array_equal(base["idx"], aff["idx"])
    np.testing.assert_allclose(base["nn"], aff["nn"], rtol=1e-9)
    for m in (minL, maxL):
        P, _ = bf.profile(T, m)
        Pr, _ = bf.profile(T[::-1].copy(), m)
        np.testing.assert_allclose(Pr[::-1], P, rtol=1e-10, atol=1e-12)


def test_r_schedule_does_not_change_result():
    """DRAG at r = exact k-th value, at r = 0 and MERLIN's schedule agree."""
    T = synth.small_random(31, 700, "ecg")
    m, k = 20, 5
    P, _ = bf.profile(T, m)
    kth = float(np.sort(P)[::-1][k - 1])
    a = oracle.merlin(T, m, m, k)
    for r in (kth, 0.0, 0.5 * kth):
        idx, nn, _, _ = oracle.drag(T, m, r)
        order = np.lexsort((idx, -nn))[:k]
        np.testing.assert_array_equal(idx[order], a["idx"])
        np.testing.assert_allclose(nn[order], a["nn"], rtol=1e-12)


def test_gradient_matches_finite_differences_and_invariants():
    T = synth.small_random(40, 400, "rw")
    m = 16
    rng = np.random.default_rng(5)
    for _ in range(6):
        i = int(rng.integers(0, T.shape[0] - m + 1))
        d, j = oracle.nn_row(T, m, i)
        g = oracle.nn_grad(T, m, i, j)

        def dist_fixed_j(S):
            x = S[i:i + m]
            y = S[j:j + m]
            xh = (x - x.mean()) / x.std()
            yh = (y - y.mean()) / y.std()
            return math.sqrt(((xh - yh) ** 2).sum())

        h = 1e-6
        for p in list(range(i, i + m)) + list(range(j, j + m)):
            Sp = T.copy(); Sp[p] += h
            Sm = T.copy(); Sm[p] -= h
            fd = (dist_fixed_j(Sp) - dist_fixed_j(Sm)) / (2 * h)
            assert abs(fd - g[p]) <= 1e-6 + 1e-5 * abs(g[p])
        # zero outside the two supports
        mask = np.ones(T.shape[0], bool)
        mask[i:i + m] = False
        mask[j:j + m] = False
        assert np.all(g[mask] == 0.0)
        # shift invariance and degree-0 homogeneity of each window's part
        for a0 in (i, j):
            part = g[a0:a0 + m]
            assert abs(part.sum()) <= 1e-10
            assert abs((part * T[a0:a0 + m]).sum()) <= 1e-8 * (1 + np.abs(T).max())
        # closed form through the Pearson correlation (Eq. (6)):
        # d P / d x_k = (rho * xh_k - yh_k) / (sigma_x * P)
        x, y = T[i:i + m], T[j:j + m]
        xh = (x - x.mean()) / x.std()
        yh = (y - y.mean()) / y.std()
        rho = float(np.corrcoef(x, y)[0, 1])
        np.testing.assert_allclose(g[i:i + m], (rho * xh - yh) / (x.std() * d), rtol=1e-8,
                                   atol=1e-12)


def test_config1_golden_is_regenerable_and_matches_bruteforce():
    path = os.path.join(GOLD, "c1_rw2k_m32-40_k1_fp64.json")
    with open(path) as f:
        g = json.load(f)
    w = synth.config1()
    assert synth.sha256(w.T) == g["sha256"]
    b = bf.discords(w.T, w.minL, w.maxL, w.k)
    np.testing.assert_array_equal(b["idx"], np.array(g["idx"]))
    np.testing.assert_allclose(b["nn"], np.array(g["nn"]), rtol=1e-12)
    np.testing.assert_array_equal(b["nnidx"], np.array(g["nnidx"]))


def _schedule_cases():
    """c1, twenty small series with 8-12 lengths each, and eight noisy sine
    waves whose period is much longer than the windows.  On the latter the
    nearest-neighbour distances fall as m grows (a longer window of a slow
    sine has a larger spread, so the same noise weighs less once
    z-normalised), which makes the r rules of the later lengths fail and
    retry."""
    w = synth.config1()
    yield "c1", w.T, w.minL, w.maxL, w.k
    rng = np.random.default_rng(777)
    for c in range(20):
        kind = ("rw", "noise", "ecg")[c % 3]
        minL = int(rng.integers(5, 13))
        maxL = minL + int(rng.integers(7, 12))
        n = int(rng.integers(3 * maxL + 40, 420))
        k = (1, 2, 3)[c % 3]
        yield f"s{c}", synth.small_random(2000 + c, n, kind), minL, maxL, k
    for c in range(8):
        g = np.random.default_rng(4000 + c)
        t = np.arange(420, dtype=np.float64)
        noise = (0.003, 0.01)[c % 2]
        T = np.sin(2 * math.pi * t / 150 + g.uniform(0, 2 * math.pi)) + noise * g.standard_normal(420)
        yield f"sine{c}", T, 8, 19, 2


def test_r_schedule_follows_alg1_on_bruteforce_values():
    """MERLIN's r per length and its DRAG call count follow Alg. 1's rules,
    with every success or failure decided by the brute-force profile.

    A DRAG call at range r finds #{i : P_m(i) >= r} discords (every row when
    r <= 0); it fails while that is below k.  The rules (readings of Alg. 1):
    at minL, r starts at 2 sqrt(minL) and halves after each failure; at the
    next four lengths it starts at 0.99 times the previous length's k-th
    largest P and is multiplied by 0.99 after each failure; later it starts
    at mean - 2 std of the last five lengths' k-th values (population std)
    and drops by that std after each failure (by 1 % when the std is 0).
    The call count, every failed r, and the successful r are checked.
    """
    retried = set()
    for name, T, minL, maxL, k in _schedule_cases():
        o = oracle.merlin(T, minL, maxL, k)
        kth = []
        for li, m in enumerate(range(minL, maxL + 1)):
            P, _ = bf.profile(T, m)
            N = P.shape[0]

            def found(r):
                return N if r <= 0 else int(np.count_nonzero(P >= r))

            if li == 0:
                r = 2.0 * math.sqrt(minL)
                lower = lambda r: 0.5 * r                       # noqa: E731
            elif li <= 4:
                r = 0.99 * kth[li - 1]
                lower = lambda r: 0.99 * r                      # noqa: E731
            else:
                h = np.array(kth[li - 5:li])
                mu, sd = float(h.mean()), float(h.std())
                r = mu - 2.0 * sd
                lower = (lambda r, sd=sd: r - sd) if sd > 0 else (lambda r: 0.99 * r)
            calls = 1
            while True:
                # no row of P may sit on the boundary r (the count would be
                # decided by rounding, not by the rule)
                assert np.all(np.abs(P - r) > 1e-9 * max(1.0, abs(r))), (name, m, r)
                if found(r) >= k:
                    break
                r = lower(r)
                calls += 1
                assert calls < 200, (name, m)
            assert int(o["calls"][li]) == calls, (name, m, int(o["calls"][li]), calls)
            if calls > 1:
                retried.add(0 if li == 0 else (1 if li <= 4 else 2))
            assert abs(float(o["r"][li]) - r) <= 1e-9 * max(1.0, abs(r)), (name, m, o["r"][li], r)
            kth.append(float(np.sort(P)[::-1][k - 1]))
            # the reported k-th value is the one the next length's rule reads
            assert abs(float(o["nn"][li * k + k - 1]) - kth[-1]) <= 1e-12 * max(1.0, kth[-1])
    # every rule's failure branch was exercised
    assert retried == {0, 1, 2}, retried


def test_openmp_build_matches_serial():
    """The OpenMP build of the oracle (phase 1's inner candidate loop split
    over threads, phase 2 one candidate per thread; used for the largest
    stored results) returns exactly what the serial build returns,
    evaluation counts included: MERLIN on config 1, and DRAG at a range
    small enough that hundreds of candidates stay alive, so the threaded
    branch of phase 1 runs too."""
    w = synth.config1()
    a = oracle.merlin(w.T, w.minL, w.maxL, w.k)
    b = oracle.merlin(w.T, w.minL, w.maxL, w.k, threads=4)
    for key in a:
        np.testing.assert_array_equal(np.asarray(a[key]), np.asarray(b[key]), err_msg=key)
    T = synth.small_random(77, 5000, "noise")
    P, _ = bf.profile(T, 16)
    Ps = np.sort(P)[::-1]
    r = float(0.5 * (Ps[600] + Ps[601]))    # between two rows: no rounding-decided boundary
    s = oracle.drag(T, 16, r)
    p = oracle.drag(T, 16, r, threads=4)
    assert s[0].shape[0] > 256          # the candidate list passed the threading threshold
    for x, y in zip(s[:3], p[:3]):
        np.testing.assert_array_equal(x, y)
    assert s[3] == p[3]
    np.testing.assert_array_equal(s[0], np.nonzero(P >= r)[0])
