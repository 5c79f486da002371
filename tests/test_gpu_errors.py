"""Error paths of the C ABI that need a context (hence a GPU): an undersized
workspace (PALMAD_EWORKSPACE, rejected on the host before any launch) and
device-side failures forced from the host through PALMAD_FAULT
(PALMAD_EDEVICE): "hip" fails before any device work, "converge" lets the
search run with one range search per length, so every kernel exits normally
and the driver reports the range search that did not converge.  After each
failure the context still works and gives the normal result."""

import ctypes
import os
import sys

import numpy as np
import pytest

from paper_2304_01660_amd import _lib, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KEYS = ("idx", "len", "nn", "nnidx", "count")


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L = _lib.lib()
    c = ctypes.c_void_p()
    _lib.check(L.palmad_create(ctypes.byref(c), 0))
    yield c
    L.palmad_destroy(c)


@pytest.fixture()
def fault():
    def set_(site):
        if site is None:
            os.environ.pop("PALMAD_FAULT", None)
        else:
            os.environ["PALMAD_FAULT"] = site
    yield set_
    os.environ.pop("PALMAD_FAULT", None)


def _case():
    T = synth.small_random(5, 3000, "rw")
    return T, 20, 26, 2


def _call(ctx, T, minL, maxL, k, ws_bytes=None):
    L = _lib.lib()
    dev = torch.device("cuda:0")
    Td = torch.from_numpy(np.ascontiguousarray(T)).to(dev)
    n = Td.shape[0]
    opts = _lib.make_options()
    nb = ctypes.c_size_t(0)
    _lib.check(L.palmad_workspace_size(n, minL, maxL, k, ctypes.byref(opts), ctypes.byref(nb)))
    size = nb.value if ws_bytes is None else ws_bytes(nb.value)
    ws = torch.empty(max(size, 256), dtype=torch.uint8, device=dev)
    Lc = maxL - minL + 1
    o = {
        "idx": torch.full((Lc * k,), -7, dtype=torch.int64, device=dev),
        "len": torch.full((Lc * k,), -7, dtype=torch.int32, device=dev),
        "nn": torch.full((Lc * k,), -7.0, dtype=torch.float64, device=dev),
        "nnidx": torch.full((Lc * k,), -7, dtype=torch.int64, device=dev),
        "count": torch.full((Lc,), -7, dtype=torch.int32, device=dev),
    }
    rc = L.palmad_discords(ctx, Td.data_ptr(), n, minL, maxL, k, ctypes.byref(opts),
                           ws.data_ptr(), size, *[o[key].data_ptr() for key in KEYS], None,
                           torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    msg = (L.palmad_last_error(ctx) or b"").decode()
    return rc, msg, o


def _untouched(o):
    return all(bool((o[key] == -7).all().item()) for key in KEYS)


def test_undersized_workspace(ctx):
    T, minL, maxL, k = _case()
    _say("undersized workspace")
    rc, msg, o = _call(ctx, T, minL, maxL, k, ws_bytes=lambda need: need - 256)
    assert rc == -3, msg
    assert "workspace" in msg
    assert _untouched(o)
    rc, msg, o = _call(ctx, T, minL, maxL, k)
    assert rc == 0, msg


def test_injected_hip_failure(ctx, fault):
    T, minL, maxL, k = _case()
    fault("hip")
    _say("PALMAD_FAULT=hip")
    rc, msg, o = _call(ctx, T, minL, maxL, k)
    assert rc == -4, msg
    assert "PALMAD_FAULT" in msg
    assert _untouched(o)
    fault(None)
    rc, msg, good = _call(ctx, T, minL, maxL, k)
    assert rc == 0, msg
    assert int(good["count"].min().item()) >= k


def test_injected_non_convergence(ctx, fault):
    T, minL, maxL, k = _case()
    _, _, ref = _call(ctx, T, minL, maxL, k)
    fault("converge")
    _say("PALMAD_FAULT=converge")
    rc, msg, o = _call(ctx, T, minL, maxL, k)
    assert rc == -4, msg
    assert "did not converge" in msg
    # the first length failed on its first range search: no row of it was written
    assert bool((o["idx"][:k] == -7).all().item())
    fault(None)
    rc, msg, again = _call(ctx, T, minL, maxL, k)
    assert rc == 0, msg
    for key in KEYS:
        assert torch.equal(again[key], ref[key]), key
