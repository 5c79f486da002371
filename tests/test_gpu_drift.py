"""Soundness of the FP32 selection sweep on the device: the largest drift
|rho_FP32 - rho_FP64| of the sweep's FP32 recurrence (the library's own
kernel arithmetic, side by side with FP64 from the same exact start), over
thousands of sampled 512-row tiles of the configured workloads and every
tile of the smallest batch series, stays below a quarter of the guard band
the selection sweep uses at that length."""

import sys

import pytest

from paper_2304_01660_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _cases():
    """(name, series, minL, lengths, items): 2048 sampled tiles on the large
    workloads, every tile (items = 0) of the smallest batch series."""
    w2, w3, w5 = synth.config2(), synth.config3(), synth.config5()
    b = synth.config4()
    rw = max((w for w in b if "rw" in w.name), key=lambda w: w.n)
    ecg = min((w for w in b if "ecg" in w.name), key=lambda w: w.minL)
    small_ecg = sorted((w for w in b if "ecg" in w.name), key=lambda w: w.n)[:3]
    small_rw = min((w for w in b if "rw" in w.name), key=lambda w: w.n)
    cases = [
        (w2.name, w2.T, w2.minL, (w2.minL, w2.maxL), 2048),
        (w3.name, w3.T, w3.minL, (w3.minL, (w3.minL + w3.maxL) // 2, w3.maxL), 2048),
        (w5.name, w5.T, w5.minL, (w5.minL, w5.maxL), 2048),
        (rw.name, rw.T, rw.minL, (rw.minL, rw.maxL), 2048),
        (ecg.name, ecg.T, ecg.minL, (ecg.minL, ecg.maxL), 2048),
        (small_rw.name, small_rw.T, small_rw.minL, (small_rw.minL, small_rw.maxL), 0),
    ]
    cases += [(w.name, w.T, w.minL, (w.minL, (w.minL + w.maxL) // 2, w.maxL), 0) for w in small_ecg]
    return cases


def test_fp32_selection_drift_is_within_a_quarter_of_the_band():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_01660_amd import api
    dev = torch.device("cuda:0")
    rows = []
    for name, T, minL, ms, items in _cases():
        Td = torch.from_numpy(T).to(dev)
        for m in ms:
            d, band = api.selection_drift(Td, minL, m, items=items, chunk=512)
            _say("drift", name, m, items or "all", d, band, d / band)
            rows.append((name, m, d, band))
    _say("worst drift / band", max(d / b for _, _, d, b in rows))
    for name, m, d, band in rows:
        assert 0.0 < d, (name, m)          # FP32 does differ from FP64
        assert band >= 1.2499e-4
        assert d <= band / 4, (name, m, d, band)
