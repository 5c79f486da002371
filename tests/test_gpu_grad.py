"""Gradient of reported nnDist with respect to the series (the adjoint path).

Checked against (a) the oracle's gradient (oracle_nn_grad: chain rule
through the z-normalisation Jacobian at the oracle's nearest neighbour),
(b) FP64 central finite differences of the oracle's exact row minimum, and
(c) invariants: zero outside the supports, sum of the gradient 0 (shift
invariance), sum of T * gradient 0 (scale invariance).
"""

import json
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2304_01660_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _oracle_grad(T, idx, ln, nnj, w):
    g = np.zeros(T.shape[0])
    for q in range(len(idx)):
        d, j = oracle.nn_row(T, int(ln[q]), int(idx[q]))
        assert j == int(nnj[q])
        oracle.nn_grad(T, int(ln[q]), int(idx[q]), j, float(w[q]), g)
    return g


def _fd_check(T, idx, ln, w, points, h=1e-4):
    """FP64 central differences of sum_q w[q] * nnDist_q at each point (the
    oracle's exact row minimum, recomputed on the perturbed series for every
    row whose windows cover the point).  Yields (point, fd, kink, rows):
    kink when a perturbation moves some row's nearest neighbour, rows = the
    number of rows covering the point."""
    base = [oracle.nn_row(T, int(ln[q]), int(idx[q])) for q in range(len(idx))]
    for p in points:
        fd = 0.0
        kink = False
        rows = 0
        for q in range(len(idx)):
            i, m = int(idx[q]), int(ln[q])
            d0, j0 = base[q]
            if not (i <= p < i + m or j0 <= p < j0 + m):
                continue
            rows += 1
            Tp = T.copy(); Tp[p] += h
            Tm = T.copy(); Tm[p] -= h
            dp, jp = oracle.nn_row(Tp, m, i)
            dm, jm = oracle.nn_row(Tm, m, i)
            if jp != j0 or jm != j0:
                kink = True
            fd += w[q] * (dp - dm) / (2 * h)
        yield p, fd, kink, rows


def test_gradient_small_matches_oracle_and_fd():
    dev = _dev()
    from paper_2304_01660_amd import api
    T = synth.small_random(321, 3000, "rw")
    minL, maxL, k = 20, 24, 3
    Tt = torch.from_numpy(T).to(dev).requires_grad_(True)
    _say("grad small forward")
    nn, idx, ln, nnj = api.DiscordNNDist.apply(Tt, minL, maxL, k, None)
    rng = np.random.default_rng(77)
    w = rng.standard_normal(nn.numel())
    loss = (nn * torch.from_numpy(w).to(dev)).sum()
    _say("grad small backward")
    loss.backward()
    g = Tt.grad.detach().cpu().numpy()
    idx_h, ln_h, nnj_h = idx.cpu().numpy(), ln.cpu().numpy(), nnj.cpu().numpy()
    ref = _oracle_grad(T, idx_h, ln_h, nnj_h, w)
    scale = np.abs(ref).max()
    np.testing.assert_allclose(g, ref, rtol=1e-8, atol=1e-10 * scale)
    # zero outside supports
    sup = np.zeros(T.shape[0], bool)
    for q in range(len(idx_h)):
        m = int(ln_h[q])
        sup[idx_h[q]:idx_h[q] + m] = True
        sup[nnj_h[q]:nnj_h[q] + m] = True
    assert np.all(g[~sup] == 0.0)
    assert abs(g.sum()) <= 1e-9 * scale * T.shape[0] ** 0.5
    assert abs((g * T).sum()) <= 1e-8 * scale * np.abs(T).max() * T.shape[0] ** 0.5
    pts = np.nonzero(sup)[0]
    pts = rng.choice(pts, size=12, replace=False)
    compared = 0
    for p, fd, kink, rows in _fd_check(T, idx_h, ln_h, w, pts):
        if kink:
            continue
        assert abs(fd - g[p]) <= 1e-6 + 1e-3 * abs(g[p]), (p, fd, g[p])
        compared += 1
    assert compared >= 8, compared


def test_backward_recomputes_neighbours_and_handles_invalid_rows():
    dev = _dev()
    from paper_2304_01660_amd import api
    T = synth.small_random(322, 2000, "ecg")
    Tt = torch.from_numpy(T).to(dev)
    _say("grad invalid rows")
    out = api.discords(Tt, 30, 32, 2)
    idx = torch.cat([out["idx"], torch.tensor([-5, 1990], device=dev)])
    ln = torch.cat([out["len"], torch.tensor([30, 30], dtype=torch.int32, device=dev)])
    gin = torch.ones(idx.numel(), dtype=torch.float64, device=dev)
    gT, nnj = api.discords_backward(Tt, idx, ln, gin, maxm=32, return_nn_idx=True)
    nnj = nnj.cpu().numpy()
    np.testing.assert_array_equal(nnj[:-2], out["nn_idx"].cpu().numpy())
    assert nnj[-1] == -1 and nnj[-2] == -1
    ref = _oracle_grad(T, out["idx"].cpu().numpy(), out["len"].cpu().numpy(),
                       out["nn_idx"].cpu().numpy(), np.ones(out["idx"].numel()))
    np.testing.assert_allclose(gT.cpu().numpy(), ref, rtol=1e-8, atol=1e-10 * np.abs(ref).max())


def test_config5_gradient():
    """n = 200,000, m in [96, 160], top-5; backward checked at 64 seeded points."""
    dev = _dev()
    from paper_2304_01660_amd import api
    w5 = synth.config5()
    T = w5.T
    Tt = torch.from_numpy(T).to(dev).requires_grad_(True)
    _say("config5 forward")
    nn, idx, ln, nnj = api.DiscordNNDist.apply(Tt, w5.minL, w5.maxL, w5.k, None)
    gold = None
    for f in sorted(os.listdir(GOLD)):
        if f.startswith("c5_") and f.endswith(".json"):
            gold = json.load(open(os.path.join(GOLD, f)))
    if gold is not None:
        assert synth.sha256(T) == gold["sha256"]
        np.testing.assert_allclose(nn.detach().cpu().numpy(), np.array(gold["nn"]), rtol=1e-9)
    rng = np.random.default_rng(5)
    wts = rng.standard_normal(nn.numel())
    _say("config5 backward")
    (nn * torch.from_numpy(wts).to(dev)).sum().backward()
    g = Tt.grad.detach().cpu().numpy()
    idx_h, ln_h, nnj_h = idx.cpu().numpy(), ln.cpu().numpy(), nnj.cpu().numpy()
    sup = np.zeros(T.shape[0], bool)
    for q in range(len(idx_h)):
        m = int(ln_h[q])
        sup[idx_h[q]:idx_h[q] + m] = True
        sup[nnj_h[q]:nnj_h[q] + m] = True
    inside = rng.choice(np.nonzero(sup)[0], size=56, replace=False)
    outside = rng.choice(np.nonzero(~sup)[0], size=8, replace=False)
    assert np.all(g[outside] == 0.0)
    # oracle gradient, restricted to the rows touching the sampled points
    ref = np.zeros(T.shape[0])
    for q in range(len(idx_h)):
        m = int(ln_h[q])
        i, j = int(idx_h[q]), int(nnj_h[q])
        if np.any((inside >= i) & (inside < i + m)) or np.any((inside >= j) & (inside < j + m)):
            oracle.nn_grad(T, m, i, j, float(wts[q]), ref)
    np.testing.assert_allclose(g[inside], ref[inside], rtol=1e-7,
                               atol=1e-10 * np.abs(ref[inside]).max())
    # finite differences at all 64 points: the 8 outside every support must
    # give 0 (no row covers them), the 56 inside must match away from kinks
    _say("config5 finite differences at 64 points")
    compared = kinks = 0
    for p, fd, kink, rows in _fd_check(T, idx_h, ln_h, wts, np.concatenate([inside, outside])):
        if rows == 0:
            assert fd == 0.0 and g[p] == 0.0, (p, fd, g[p])
            continue
        if kink:
            kinks += 1
            continue
        assert abs(fd - g[p]) <= 1e-6 + 1e-3 * abs(g[p]), (p, fd, g[p])
        compared += 1
    _say("config5 FD compared", compared, "kinks", kinks)
    assert compared >= 48, (compared, kinks)
