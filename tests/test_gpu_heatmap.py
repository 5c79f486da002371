"""GPU parity of the discord heatmap and discord interest (Sec. 5,
Eq. (11)-(12)) through the C ABI.

The heatmap row of length m holds every range discord of the successful
range search (nearest non-self match at distance >= r_m) with nnDist^2/(2m);
its pins are the brute-force matrix profile P_m of the oracle and the r_m of
the oracle's own MERLIN run (Alg. 1 with the same rules): membership must be
P_m(i) >= r_m except within the distance tolerance of r_m, values must be
P_m(i)^2 / (2m).  Interest is the per-column maximum over the lengths and the
k best columns, checked against numpy on the same heatmap and against the
maxima of the oracle-built heatmap.
"""

import sys

import numpy as np
import pytest

import oracle
from oracle import bruteforce as bf
from paper_2304_01660_amd import synth
from parity_helpers import close_ed
from parity_helpers import check_against_profiles as _check_against_profiles

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


CASES = [(0, "rw", 900, 16, 20, 1), (1, "noise", 1500, 24, 27, 3), (2, "ecg", 2600, 40, 43, 2),
         (3, "rw", 700, 8, 12, 5)]


@pytest.mark.parametrize("dist_bits", [64, 32])
@pytest.mark.parametrize("case", CASES)
def test_heatmap_matches_profiles_and_oracle_range(dist_bits, case):
    from paper_2304_01660_amd import api
    dev = _dev()
    c, kind, n, minL, maxL, k = case
    T = synth.small_random(9100 + c, n, kind)
    _say("heatmap", dist_bits, case)
    out = api.discord_heatmap(torch.from_numpy(T).to(dev), minL, maxL, k, dist_bits=dist_bits)
    _check_against_profiles(T, out, minL, maxL, k)
    heat = out["heat"].cpu().numpy()
    rng = out["range"].cpu().numpy()
    cnt = out["count"].cpu().numpy()
    ref = oracle.merlin(T, minL, maxL, k)
    np.testing.assert_allclose(rng, ref["r"], rtol=1e-7, atol=1e-12)
    assert heat.shape == (maxL - minL + 1, n - minL + 1)
    oracle_heat = np.zeros_like(heat)
    for m in range(minL, maxL + 1):
        li = m - minL
        N = n - m + 1
        P, _ = bf.profile(T, m)
        r = rng[li]
        assert np.all(heat[li, N:] == 0.0)
        row = heat[li, :N]
        if r <= 0:
            member = np.ones(N, dtype=bool)
            mem_o = member
        else:
            member = row > 0.0
            want = P >= r
            far = ~close_ed(P, np.full_like(P, r), m, 1e-9)
            np.testing.assert_array_equal(member[far], want[far])
            mem_o = np.where(far, want, member)  # near r either side is right
        assert int(member.sum()) == int(cnt[li])
        exp = P[member] ** 2 / (2.0 * m)
        np.testing.assert_allclose(row[member], exp, rtol=1e-8, atol=1e-11)
        oracle_heat[li, :N] = np.where(mem_o, P ** 2 / (2.0 * m), 0.0)
    # interest (Eq. (12)) on the device heatmap
    ht = out["heat"]
    col_score, col_len, top_idx, top_len, top_score = api.heatmap_interest(ht, minL, k)
    cs = col_score.cpu().numpy()
    cl = col_len.cpu().numpy()
    np.testing.assert_array_equal(cs, heat.max(axis=0))
    np.testing.assert_array_equal(cl, minL + heat.argmax(axis=0))
    order = np.lexsort((np.arange(heat.shape[1]), -cs))[:k]
    np.testing.assert_array_equal(top_idx.cpu().numpy(), order)
    np.testing.assert_array_equal(top_len.cpu().numpy(), cl[order])
    np.testing.assert_array_equal(top_score.cpu().numpy(), cs[order])
    # and the maxima agree with those of the heatmap built from the profiles
    np.testing.assert_allclose(cs, oracle_heat.max(axis=0), rtol=1e-8, atol=1e-11)


def test_heatmap_interest_rejects_bad_arguments():
    from paper_2304_01660_amd import api
    dev = _dev()
    h = torch.zeros((3, 10), dtype=torch.float64, device=dev)
    with pytest.raises(Exception):
        api.heatmap_interest(h, 8, 11)
    with pytest.raises(Exception):
        api.heatmap_interest(h, 8, 0)
