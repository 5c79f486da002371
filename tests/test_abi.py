"""C ABI checks that need no GPU: the library loads, exports every symbol the
public header declares, and validates arguments on the host."""

import ctypes
import os
import re

import pytest

from paper_2304_01660_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "palmad.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(palmad_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    syms = declared_symbols()
    assert len(syms) >= 8
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(_lib.SIGNATURES), "binding and header disagree"


def test_version_string():
    v = _lib.lib().palmad_version().decode()
    assert "gfx950" in v


def _ws(n, minL, maxL, k, **kw):
    o = _lib.make_options(**kw)
    b = ctypes.c_size_t(0)
    rc = _lib.lib().palmad_workspace_size(n, minL, maxL, k, ctypes.byref(o), ctypes.byref(b))
    return rc, b.value


@pytest.mark.parametrize("n,minL,maxL,k,code", [
    (1000, 2, 10, 1, -1),        # minL < 3
    (1000, 20, 10, 1, -1),       # maxL < minL
    (100, 10, 34, 1, -1),        # n < 3*maxL - 1
    (1000, 10, 20, 0, -1),       # k < 1
    (1000, 10, 20, 65, -6),      # k above the supported maximum
    (10**6, 10, 3001, 1, -6),    # maxL above the supported maximum
])
def test_workspace_size_rejects_bad_arguments(n, minL, maxL, k, code):
    rc, _ = _ws(n, minL, maxL, k)
    assert rc == code
    assert _lib.lib().palmad_last_error(None)


def test_workspace_size_accepts_minimum_length_and_grows():
    rc, b1 = _ws(59, 10, 20, 1)   # n = 3*maxL - 1
    assert rc == 0 and b1 > 0
    rc, b2 = _ws(10**6, 128, 256, 3)
    assert rc == 0 and b2 > b1 and b2 < 512 * 2**20


def test_options_validation():
    rc, _ = _ws(1000, 10, 20, 1, dist_bits=16)
    assert rc == -1
    rc, _ = _ws(1000, 10, 20, 1, dist_bits=64)
    assert rc == 0
    rc, _ = _ws(1000, 10, 20, 1, rows_near=300)
    assert rc == -1
    rc, _ = _ws(1000, 10, 20, 1, rows_near=128, rows_far=256, rows_refine=512)
    assert rc == 0
    o = _lib.make_options()
    o.reserved[1] = 1
    b = ctypes.c_size_t(0)
    assert _lib.lib().palmad_workspace_size(1000, 10, 20, 1, ctypes.byref(o), ctypes.byref(b)) == -1
    rc, _ = _ws(1000, 10, 20, 1, band_pass=2)
    assert rc == -1
    rc, _ = _ws(1000, 10, 20, 1, band_pass=1)
    assert rc == 0


def test_null_pointer_arguments_are_rejected():
    L = _lib.lib()
    assert L.palmad_workspace_size(1000, 10, 20, 1, None, None) == -1
    assert L.palmad_create(None, 0) == -1
    assert L.palmad_discords(None, None, 1000, 10, 20, 1, None, None, 0, None, None, None,
                             None, None, None, None) == -1
    assert L.palmad_discord_heatmap(None, None, 1000, 10, 20, 1, None, None, 0, None, None,
                                    None, None, None, None, 991, None, None, None) == -1
    assert L.palmad_heatmap_interest(None, None, 11, 991, 991, 10, 1, None, None, None, None,
                                     None, None) == -1
    L.palmad_destroy(None)


def _bws(lengths, lo, hi, k, **kw):
    B = len(lengths)
    offs = (ctypes.c_int64 * (B + 1))()
    for b, n in enumerate(lengths):
        offs[b + 1] = offs[b] + n
    c_lo = (ctypes.c_int32 * max(B, 1))(*lo)
    c_hi = (ctypes.c_int32 * max(B, 1))(*hi)
    o = _lib.make_options(**kw)
    b = ctypes.c_size_t(0)
    rc = _lib.lib().palmad_batched_workspace_size(B, offs, c_lo, c_hi, k, ctypes.byref(o),
                                                  ctypes.byref(b))
    return rc, b.value


def test_batched_workspace_size():
    rc, one = _ws(20000, 50, 100, 1)
    assert rc == 0
    rc, b1 = _bws([20000], [50], [100], 1)
    assert rc == 0 and b1 >= one
    rc, b3 = _bws([20000, 5000, 70000], [50, 10, 60], [100, 30, 110], 1)
    assert rc == 0 and b3 > b1
    # the per-series regions dominate: the batch needs about the sum
    parts = [_ws(n, lo, hi, 1)[1] for n, lo, hi in ((20000, 50, 100), (5000, 10, 30),
                                                     (70000, 60, 110))]
    assert abs(b3 - sum(parts)) <= 64 * 1024


@pytest.mark.parametrize("lengths,lo,hi,k,code", [
    ([], [], [], 1, -1),                         # B = 0
    ([1000, 50], [10, 10], [20, 20], 1, -1),     # second series too short for maxL
    ([1000, 1000], [10, 2], [20, 20], 1, -1),    # minL < 3
    ([1000, 1000], [10, 10], [20, 20], 65, -6),  # k above the supported maximum
])
def test_batched_workspace_size_rejects_bad_arguments(lengths, lo, hi, k, code):
    rc, _ = _bws(lengths, lo, hi, k)
    assert rc == code
    msg = _lib.lib().palmad_last_error(None).decode()
    assert msg
    if len(lengths) == 2 and code == -1:
        assert "series 1" in msg


def test_batched_offsets_must_start_at_zero():
    offs = (ctypes.c_int64 * 2)(5, 2005)
    lo = (ctypes.c_int32 * 1)(10)
    hi = (ctypes.c_int32 * 1)(20)
    b = ctypes.c_size_t(0)
    assert _lib.lib().palmad_batched_workspace_size(1, offs, lo, hi, 1, None, ctypes.byref(b)) == -1
    assert _lib.lib().palmad_batched_workspace_size(1, None, lo, hi, 1, None, ctypes.byref(b)) == -1


def test_stream_workspace_size_validates_and_grows_with_lengths():
    L = _lib.lib()
    o = _lib.make_options()
    b = ctypes.c_size_t(0)
    assert L.palmad_stream_workspace_size(100, 10, 34, 1, ctypes.byref(o), ctypes.byref(b)) == -1
    assert L.palmad_stream_workspace_size(10**5, 2, 34, 1, ctypes.byref(o), ctypes.byref(b)) == -1
    assert L.palmad_stream_workspace_size(10**5, 64, 64, 3, ctypes.byref(o), ctypes.byref(b)) == 0
    one = b.value
    assert L.palmad_stream_workspace_size(10**5, 64, 128, 3, ctypes.byref(o), ctypes.byref(b)) == 0
    # one profile of 8 bytes per subsequence and length beyond a search's workspace
    assert b.value - one >= 8 * 64 * (10**5 - 128)
    ws = ctypes.c_size_t(0)
    assert L.palmad_workspace_size(10**5, 64, 128, 3, ctypes.byref(o), ctypes.byref(ws)) == 0
    assert b.value > ws.value


def test_stream_calls_reject_null_handles():
    L = _lib.lib()
    assert L.palmad_stream_append(None, None, 1, None) == -1
    assert L.palmad_stream_discords(None, None, None, None, None, None) == -1
    assert L.palmad_stream_profile(None, 10, None, None) == -1
    assert L.palmad_stream_length(None) == -1
    L.palmad_stream_destroy(None)
