"""The HIP sources are built without packed FP32 instructions, and their
kernels make no function calls.

The build passes the target feature that disables them to hipcc.  The host
compilation passes print a warning that they do not know the feature; the
device pass does honour it.  This test compiles a small float2 kernel both
ways to show that the flag removes packed FP32 arithmetic, then compiles
every library source to gfx950 assembly with the build's own flags and
checks that none contains a packed FP32 add, multiply or fused multiply-add.
The same assembly must hold no call: the device library's work-item and
work-group queries are inlined only when the kernels share its floating-point
mode attributes (building with the IEEE mode bit off turned each of them into
a call, and the call's register convention into extra registers in every
kernel).
"""

import os
import re
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import __graft_entry__ as ge  # noqa: E402

PACKED = re.compile(r"\bv_pk_(add|mul|fma)_f32\b")
CALL = re.compile(r"\bs_(swappc|setpc)_b64\b")
TOY = """#include <hip/hip_runtime.h>
__global__ void k(float2* a, const float2* b, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) { float2 x = a[i], y = b[i]; x.x = x.x * y.x + y.y; x.y = x.y * y.y + y.x; a[i] = x; }
}
"""

pytestmark = pytest.mark.skipif(not os.path.exists(ge.HIPCC) and shutil.which("hipcc") is None,
                                reason="hipcc not available")


def _device_asm(src, flags, workdir):
    out = os.path.join(workdir, os.path.basename(src) + ".s")
    subprocess.check_call([ge.HIPCC, *flags, "--cuda-device-only", "-S", "-o", out, src],
                          stderr=subprocess.DEVNULL)
    with open(out) as f:
        return f.read()


def _flags(extra=()):
    return [f for f in ge.HIP_FLAGS if f not in ("-shared", "-fPIC")] + list(extra)


def test_flag_removes_packed_fp32_from_a_float2_kernel():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "toy.hip")
        with open(src, "w") as f:
            f.write(TOY)
        base = [f for f in _flags() if f not in ("-Xclang", "-target-feature", "-packed-fp32-ops")]
        assert PACKED.search(_device_asm(src, base, d))          # packed without the flag
        assert not PACKED.search(_device_asm(src, _flags(), d))  # none with it


@pytest.mark.parametrize("src", sorted(ge.SOURCES))
def test_library_sources_have_no_packed_fp32_and_no_calls(src):
    with tempfile.TemporaryDirectory() as d:
        asm = _device_asm(os.path.join(ge.CSRC, src), _flags(ge.SOURCES[src]), d)
        hits = sorted(set(m.group(0) for m in PACKED.finditer(asm)))
        assert not hits, (src, hits)
        calls = sorted(set(m.group(0) for m in CALL.finditer(asm)))
        assert not calls, (src, calls)
