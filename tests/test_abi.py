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
    o.reserved[2] = 1
    b = ctypes.c_size_t(0)
    assert _lib.lib().palmad_workspace_size(1000, 10, 20, 1, ctypes.byref(o), ctypes.byref(b)) == -1


def test_null_pointer_arguments_are_rejected():
    L = _lib.lib()
    assert L.palmad_workspace_size(1000, 10, 20, 1, None, None) == -1
    assert L.palmad_create(None, 0) == -1
    assert L.palmad_discords(None, None, 1000, 10, 20, 1, None, None, 0, None, None, None,
                             None, None, None, None) == -1
    L.palmad_destroy(None)
