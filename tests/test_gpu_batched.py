"""Batched search: many series of uneven length, each with its own length
range, in one call (one round of launches serves every series).

Every series runs the same per-series arithmetic as the single-series entry
point, so the batched results must be identical to it bit for bit; the
single-series path is itself checked against the oracle, and the small
cases here are checked against brute force as well.  The full 64-series
workload is checked against the single-series path for every series and
against the oracle's exact nearest-neighbour distance on sampled rows.
"""

import json
import math
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2304_01660_amd import synth
from parity_helpers import check_against_profiles, match_rows

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KEYS = ("idx", "len", "nn_dist", "nn_idx", "count")


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _small_batch():
    rng = np.random.default_rng(4242)
    out = []
    for b in range(7):
        kind = ("rw", "noise", "ecg")[b % 3]
        maxL = int(rng.integers(8, 60))
        minL = max(3, maxL - int(rng.integers(0, 6)))
        n = int(rng.integers(3 * maxL, 3500))
        out.append((synth.small_random(900 + b, n, kind), minL, maxL))
    return out


@pytest.mark.parametrize("dist_bits", [64, 32])
def test_batched_equals_single_and_bruteforce(dist_bits):
    dev = _dev()
    from paper_2304_01660_amd import api
    cases = _small_batch()
    k = 2
    _say("batched small", dist_bits, [(T.shape[0], lo, hi) for T, lo, hi in cases])
    res = api.discords_batched([torch.from_numpy(T).to(dev) for T, _, _ in cases],
                               [lo for _, lo, _ in cases], [hi for _, _, hi in cases], k,
                               dist_bits=dist_bits)
    for b, (T, lo, hi) in enumerate(cases):
        _say("batched small series", b)
        one = api.discords(torch.from_numpy(T).to(dev), lo, hi, k, dist_bits=dist_bits)
        for key in KEYS:
            assert torch.equal(res[b][key], one[key]), (b, key)
        check_against_profiles(T, res[b], lo, hi, k)


def test_batched_graph_replay_and_direct_launch_agree():
    """The cached round graph (reused across calls on one workspace) and
    direct launches give the same result."""
    dev = _dev()
    from paper_2304_01660_amd import api
    cases = _small_batch()
    values = [torch.from_numpy(T).to(dev) for T, _, _ in cases]
    lo = [c[1] for c in cases]
    hi = [c[2] for c in cases]
    nbytes = api.batched_workspace_size([v.shape[0] for v in values], lo, hi, 3)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    _say("batched graph replay")
    a = api.discords_batched(values, lo, hi, 3, workspace=ws)
    b = api.discords_batched(values, lo, hi, 3, workspace=ws)
    c = api.discords_batched(values, lo, hi, 3, workspace=ws, graphs=False)
    d, st = api.discords_batched(values, lo, hi, 3, workspace=ws, time_kernels=True,
                                 return_stats=True)
    for s in range(len(cases)):
        for key in KEYS:
            assert torch.equal(a[s][key], b[s][key]), (s, key)
            assert torch.equal(a[s][key], c[s][key]), (s, key)
            assert torch.equal(a[s][key], d[s][key]), (s, key)
    assert st["range_searches"] >= sum(h - l + 1 for l, h in zip(lo, hi))
    assert st["kernel_launches"][0] > 0
    # every range discord was live when refinement started
    assert st["rows_after_far"] >= st["survivors"] >= sum(h - l + 1 for l, h in zip(lo, hi)) * 3


def test_batched_single_series_equals_plain():
    dev = _dev()
    from paper_2304_01660_amd import api
    T = torch.from_numpy(synth.small_random(31, 5000, "ecg")).to(dev)
    _say("batched B=1")
    a = api.discords_batched([T], 20, 26, 4)[0]
    b = api.discords(T, 20, 26, 4)
    for key in KEYS:
        assert torch.equal(a[key], b[key]), key


def test_batched_nonfinite_names_the_series():
    dev = _dev()
    from paper_2304_01660_amd import api
    from paper_2304_01660_amd._lib import PalmadError
    cases = _small_batch()
    bad = cases[3][0].copy()
    bad[17] = np.inf
    vals = [torch.from_numpy(T).to(dev) for T, _, _ in cases]
    vals[3] = torch.from_numpy(bad).to(dev)
    _say("batched nonfinite")
    with pytest.raises(PalmadError) as ei:
        api.discords_batched(vals, [c[1] for c in cases], [c[2] for c in cases], 1)
    assert ei.value.code == -2
    assert "series 3" in str(ei.value)


def test_config4_batched_full_size():
    """The 64-series workload in one batched call, in the tile geometry the
    benchmark times: every row of every series against the oracle's stored
    MERLIN result for that series (tests/golden/c4/, one file per series),
    and every series identical to a single-series call."""
    dev = _dev()
    from paper_2304_01660_amd import api, tuning
    ws = synth.config4()
    gold = {}
    gdir = os.path.join(os.path.dirname(__file__), "golden", "c4")
    for b, w in enumerate(ws):
        path = os.path.join(gdir, f"{b:02d}_{w.name}.json")
        if os.path.exists(path):
            gold[b] = json.load(open(path))
    if len(gold) < len(ws):
        pytest.skip(f"config-4 goldens incomplete ({len(gold)} of {len(ws)})")
    opts = tuning.batch_options()
    _say("config4 batched", len(ws), opts)
    res, st = api.discords_batched([torch.from_numpy(w.T).to(dev) for w in ws],
                                   [w.minL for w in ws], [w.maxL for w in ws], 1,
                                   return_stats=True, **opts)
    _say("config4 stats", st)
    ties = 0
    for b, w in enumerate(ws):
        assert synth.sha256(w.T) == gold[b]["sha256"], b
        ties += match_rows(w.T, res[b], gold[b])
        one = api.discords(torch.from_numpy(w.T).to(dev), w.minL, w.maxL, 1, **opts)
        for key in KEYS:
            assert torch.equal(res[b][key], one[key]), (b, w.name, key)
    _say("config4 near ties", ties)


def test_autotune_returns_valid_options_and_same_discords():
    """The tuner times the search on a probe and returns tile geometry; the
    search under any geometry reports the same discords (within the
    floating-point tolerance, checked against brute force)."""
    dev = _dev()
    from paper_2304_01660_amd import api
    cases = _small_batch()[:4]
    vals = [torch.from_numpy(T).to(dev) for T, _, _ in cases]
    lo = [c[1] for c in cases]
    hi = [c[2] for c in cases]
    _say("autotune small batch")
    opts, rep = api.autotune(vals, lo, hi, 2, probe_lengths=3, reps=1)
    _say("autotune", opts, rep)
    assert rep["evaluated"] >= 10
    assert rep["best_seconds"] <= rep["base_seconds"]
    assert opts["rows_near"] in (128, 256, 512) and opts["rows_far"] in (128, 256, 512)
    assert opts["rows_refine"] in (128, 256, 512)
    assert opts["chunk_cols"] >= 64 and opts["near_cols"] >= 64 and opts["far_grid"] >= 1
    res = api.discords_batched(vals, lo, hi, 2, **opts)
    for b, (T, l, h) in enumerate(cases):
        check_against_profiles(T, res[b], l, h, 2)
    # single series form
    opts1, rep1 = api.autotune(vals[0], lo[0], hi[0], 2, probe_lengths=2, reps=1, dist_bits=64)
    assert opts1["dist_bits"] == 64
    out = api.discords(vals[0], lo[0], hi[0], 2, **opts1)
    check_against_profiles(cases[0][0], out, lo[0], hi[0], 2)
