"""The allocation-free entry point (palmad_discords_static, workspace in a
static device array) against palmad_discords with a caller workspace,
called through the C ABI: identical outputs on two calls in a row, the
second on a smaller series with another length range (the array keeps the
first call's contents, so anything the search failed to initialise would
show), and a host-side rejection of a search too large for the array."""

import ctypes
import sys

import numpy as np
import pytest

from paper_2304_01660_amd import _lib, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

OUT_KEYS = ("idx", "len", "nn", "nnidx", "count")


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _outputs(dev, L, k):
    return {
        "idx": torch.full((L * k,), -7, dtype=torch.int64, device=dev),
        "len": torch.full((L * k,), -7, dtype=torch.int32, device=dev),
        "nn": torch.full((L * k,), -7.0, dtype=torch.float64, device=dev),
        "nnidx": torch.full((L * k,), -7, dtype=torch.int64, device=dev),
        "count": torch.full((L,), -7, dtype=torch.int32, device=dev),
    }


def _ptrs(o):
    return [o[key].data_ptr() for key in OUT_KEYS]


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L = _lib.lib()
    c = ctypes.c_void_p()
    _lib.check(L.palmad_create(ctypes.byref(c), 0))
    yield c
    L.palmad_destroy(c)


def _with_workspace(ctx, T, minL, maxL, k, opts):
    L = _lib.lib()
    dev = T.device
    n = T.shape[0]
    nb = ctypes.c_size_t(0)
    _lib.check(L.palmad_workspace_size(n, minL, maxL, k, ctypes.byref(opts), ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    o = _outputs(dev, maxL - minL + 1, k)
    st = torch.cuda.current_stream().cuda_stream
    _lib.check(L.palmad_discords(ctx, T.data_ptr(), n, minL, maxL, k, ctypes.byref(opts),
                                 ws.data_ptr(), nb.value, *_ptrs(o), None, st), ctx)
    torch.cuda.synchronize()
    return o, nb.value


def _static(ctx, T, minL, maxL, k, opts):
    L = _lib.lib()
    o = _outputs(T.device, maxL - minL + 1, k)
    st = torch.cuda.current_stream().cuda_stream
    _lib.check(L.palmad_discords_static(ctx, T.data_ptr(), T.shape[0], minL, maxL, k,
                                        ctypes.byref(opts), *_ptrs(o), None, st), ctx)
    torch.cuda.synchronize()
    return o


def test_static_workspace_matches_caller_workspace(ctx):
    dev = torch.device("cuda:0")
    cases = [
        # (series, minL, maxL, k): the second is smaller, with another range
        (synth.config2().T, 64, 128, 3),
        (synth.small_random(77, 20000, "ecg"), 40, 60, 2),
    ]
    for dist_bits in (32, 64):
        opts = _lib.make_options(dist_bits=dist_bits)
        for T_np, minL, maxL, k in cases:
            T = torch.from_numpy(np.ascontiguousarray(T_np)).to(dev)
            _say("static workspace", dist_bits, T.shape[0], minL, maxL, k)
            ref, need = _with_workspace(ctx, T, minL, maxL, k, opts)
            assert need <= _lib.STATIC_WORKSPACE_BYTES
            got = _static(ctx, T, minL, maxL, k, opts)
            for key in OUT_KEYS:
                assert torch.equal(got[key], ref[key]), (dist_bits, T.shape[0], key)
            assert int(ref["count"].min().item()) >= k


def test_static_workspace_rejects_searches_that_do_not_fit(ctx):
    L = _lib.lib()
    dev = torch.device("cuda:0")
    n, minL, maxL, k = 1_000_000, 128, 256, 3
    opts = _lib.make_options()
    nb = ctypes.c_size_t(0)
    _lib.check(L.palmad_workspace_size(n, minL, maxL, k, ctypes.byref(opts), ctypes.byref(nb)))
    assert nb.value > _lib.STATIC_WORKSPACE_BYTES
    T = torch.zeros(n, dtype=torch.float64, device=dev)
    o = _outputs(dev, maxL - minL + 1, k)
    _say("static workspace too small", n)
    rc = L.palmad_discords_static(ctx, T.data_ptr(), n, minL, maxL, k, ctypes.byref(opts),
                                  *_ptrs(o), None, torch.cuda.current_stream().cuda_stream)
    assert rc == -3
    assert b"static workspace" in L.palmad_last_error(ctx)
    torch.cuda.synchronize()
    assert int((o["idx"] != -7).sum().item()) == 0  # nothing written
