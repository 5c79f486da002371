"""GPU parity of the diagonal band pre-pass (option band_pass = 1): the
pre-pass tests every subsequence against its nearest non-self offsets on the
right, [m, m + 256), swept down the diagonals, before the first selection
pass.  It only prunes, so every result must equal brute force (and the
search without it) exactly; its pair counter shows that it ran.  Series are
seeded and synthetic; the periodic ECG-like kind is the one where most
subsequences die inside the band."""

import sys

import numpy as np
import pytest

from oracle import bruteforce as bf
from paper_2304_01660_amd import synth
from parity_helpers import close_ed
from parity_helpers import check_against_profiles as _check_against_profiles

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BAND = 256  # offsets per subsequence (64 lanes x 4 diagonals)
SEG = 256   # rows per work item


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _api():
    from paper_2304_01660_amd import api
    return api


def _items(n, m):
    """Work items of the pre-pass that run at length m (all columns inside)."""
    N = n - m + 1
    return sum(1 for i0 in range(0, N, SEG) if i0 + m + SEG + BAND - 1 <= N)


def _cases():
    rng = np.random.default_rng(4242)
    for c in range(12):
        kind = ("ecg", "rw", "noise")[c % 3]
        maxL = int(rng.integers(8, 90))
        minL = max(3, maxL - int(rng.integers(0, 4)))
        n = int(rng.integers(max(3 * maxL, 900), 5000))
        k = (1, 3, 2, 5)[c % 4]
        yield c, kind, n, minL, maxL, k


@pytest.mark.parametrize("dist_bits", [32, 64])
def test_band_pass_matches_bruteforce(dist_bits):
    dev = _dev()
    api = _api()
    ran = 0
    for c, kind, n, minL, maxL, k in _cases():
        T = synth.small_random(9100 + c, n, kind)
        _say("band", dist_bits, c, kind, n, minL, maxL, k)
        out = api.discords(torch.from_numpy(T).to(dev), minL, maxL, k, dist_bits=dist_bits,
                           band_pass=1, return_stats=True)
        _check_against_profiles(T, out, minL, maxL, k)
        ev = out["stats"]["kernel_evals"][5]
        if _items(n, minL) > 0:
            assert ev > 0
            ran += 1
        else:
            assert ev == 0
    assert ran >= 6


@pytest.mark.parametrize("dist_bits", [32, 64])
@pytest.mark.parametrize("seed,n,m", [(1, 2000, 16), (2, 4100, 60), (3, 3000, 3)])
def test_band_pass_range_search(dist_bits, seed, n, m):
    """Bare range searches over the whole range of r, including r <= 0
    (every pair passes the test) and r above the largest distance."""
    dev = _dev()
    api = _api()
    T = synth.small_random(9200 + seed, n, ("ecg", "rw", "noise")[seed % 3])
    P, _ = bf.profile(T, m)
    for qtl in (0.0, 0.3, 0.9, 0.999, 1.0):
        r = float(np.quantile(P, qtl)) * (1 - 1e-7)
        _say("band-range", dist_bits, seed, n, m, qtl)
        mask, nn, cnt = api.range_discords(torch.from_numpy(T).to(dev), m, r, dist_bits=dist_bits,
                                           band_pass=1)
        mask = mask.cpu().numpy()
        nn = nn.cpu().numpy()
        far = ~close_ed(P, np.full_like(P, r), m, 1e-9)
        np.testing.assert_array_equal(mask[far], (P >= r)[far])
        assert cnt == int(mask.sum())
        assert np.all(close_ed(nn[mask], P[mask], m))
    for r in (0.0, -1.0):
        mask, nn, cnt = api.range_discords(torch.from_numpy(T).to(dev), m, r, dist_bits=dist_bits,
                                           band_pass=1)
        assert cnt == n - m + 1
    mask, nn, cnt = api.range_discords(torch.from_numpy(T).to(dev), m, 2.0 * np.sqrt(m) * 1.001,
                                       dist_bits=dist_bits, band_pass=1)
    assert cnt == 0


def test_band_pass_equals_plain_search():
    """A 60,000-point ECG-like series over several tiles of both passes: the
    searches with and without the pre-pass agree bit for bit and take the
    same range searches."""
    dev = _dev()
    api = _api()
    T = torch.from_numpy(synth.small_random(9300, 60000, "ecg")).to(dev)
    _say("band-vs-plain ecg 60000 m 40..56")
    a = api.discords(T, 40, 56, 3, return_stats=True)
    b = api.discords(T, 40, 56, 3, band_pass=1, return_stats=True)
    for key in ("idx", "nn_dist", "nn_idx", "count"):
        assert torch.equal(a[key], b[key]), key
    sa, sb = a["stats"], b["stats"]
    assert sb["kernel_evals"][5] > 0 and sa["kernel_evals"][5] == 0
    assert sb["range_searches"] == sa["range_searches"]
