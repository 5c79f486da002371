"""Streaming series (palmad_stream_*): a series appended in pieces, with the
top-k discords of every length and the exact nearest-neighbour profiles
after each append, against the oracle (brute-force profiles, MERLIN's stored
result) and against the one-shot search on the same points."""

import json
import os
import sys

import numpy as np
import pytest

import oracle
from oracle import bruteforce as bf
from paper_2304_01660_amd import synth
from parity_helpers import check_against_profiles, close_ed, match_rows

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("kind,n,minL,maxL,k,pieces", [
    ("rw", 2600, 20, 26, 3, (700, 500, 900, 500)),
    ("ecg", 3100, 30, 33, 2, (1500, 1, 63, 1536)),
])
def test_stream_matches_bruteforce_after_every_append(kind, n, minL, maxL, k, pieces):
    dev = _dev()
    from paper_2304_01660_amd import api
    T = synth.small_random(900 + n, n, kind)
    assert sum(pieces) == n
    st = api.Stream(n, minL, maxL, k, device=0)
    try:
        done = 0
        for p in pieces:
            _say("stream append", kind, done, p)
            st.append(torch.from_numpy(T[done:done + p]).to(dev))
            done += p
            assert len(st) == done
            if done < 3 * maxL - 1:
                continue
            Tp = T[:done]
            out = st.discords()
            out["count"] = torch.full((maxL - minL + 1,), k, dtype=torch.int32)
            check_against_profiles(Tp, out, minL, maxL, k)
            # the exact profile of the shortest and the longest length
            for m in (minL, maxL):
                P, _ = bf.profile(Tp, m)
                got = st.profile(m).cpu().numpy()
                assert got.shape == P.shape
                assert np.all(close_ed(got, P, m)), m
            # the one-shot search over the same points
            one = api.discords(torch.from_numpy(Tp).to(dev), minL, maxL, k)
            for key in ("idx", "len", "nn_idx"):
                assert torch.equal(out[key], one[key]), key
            assert torch.equal(out["nn_dist"], one["nn_dist"])
    finally:
        st.close()


def test_stream_of_config2_in_three_appends_matches_golden():
    """The 100k random walk (m = 64..128, top-3) appended in three pieces:
    every row against the oracle's stored MERLIN result."""
    dev = _dev()
    from paper_2304_01660_amd import api
    w = synth.config2()
    g = None
    for f in sorted(os.listdir(GOLD)):
        if f.startswith("c2_") and f.endswith(".json"):
            g = json.load(open(os.path.join(GOLD, f)))
    assert g is not None and synth.sha256(w.T) == g["sha256"]
    st = api.Stream(w.n, w.minL, w.maxL, w.k, device=0)
    try:
        cuts = [0, 41_000, 70_500, w.n]
        for a, b in zip(cuts[:-1], cuts[1:]):
            _say("config2 stream append", a, b)
            st.append(torch.from_numpy(w.T[a:b]).to(dev))
        out = st.discords()
        out["count"] = torch.full((w.maxL - w.minL + 1,), w.k, dtype=torch.int32)
        ties = match_rows(w.T, out, g)
        _say("config2 stream near ties", ties)
    finally:
        st.close()


def test_stream_rejects_overflow_and_nonfinite_values():
    dev = _dev()
    from paper_2304_01660_amd import api, _lib
    T = synth.small_random(5, 400, "rw")
    st = api.Stream(400, 10, 12, 1, device=0)
    try:
        st.append(torch.from_numpy(T[:300]).to(dev))
        before = st.discords()
        bad = torch.from_numpy(T[300:350].copy()).to(dev)
        bad[7] = float("nan")
        with pytest.raises(_lib.PalmadError) as e:
            st.append(bad)
        assert e.value.code == -2
        assert len(st) == 300
        with pytest.raises(_lib.PalmadError) as e:
            st.append(torch.from_numpy(T[:101]).to(dev))
        assert e.value.code == -1
        assert len(st) == 300
        after = st.discords()
        for key in ("idx", "nn_dist", "nn_idx"):
            assert torch.equal(before[key], after[key]), key
        st.append(torch.from_numpy(T[300:]).to(dev))
        out = st.discords()
        out["count"] = torch.full((3,), 1, dtype=torch.int32)
        check_against_profiles(T, out, 10, 12, 1)
    finally:
        st.close()
