"""ctypes binding of libpalmad.so (the C ABI declared in include/palmad.h).

Argument marshalling only.  The library must have been built in-tree
(``python -c "import __graft_entry__ as g; g.build()"``); if it is missing
this module raises instead of falling back to anything else.
"""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# PALMAD_LIBRARY may point at another build of the same library (profiling
# builds); by default the in-tree build is loaded.
LIB_PATH = os.environ.get("PALMAD_LIBRARY") or os.path.join(_HERE, "libpalmad.so")

PALMAD_OK = 0
STATUS = {
    0: "PALMAD_OK",
    -1: "PALMAD_EINVAL",
    -2: "PALMAD_ENONFINITE",
    -3: "PALMAD_EWORKSPACE",
    -4: "PALMAD_EDEVICE",
    -5: "PALMAD_ENOMEM",
    -6: "PALMAD_EUNSUPPORTED",
}


class Options(ctypes.Structure):
    _fields_ = [
        ("dist_bits", ctypes.c_int32),
        ("guard", ctypes.c_float),
        ("near_cols", ctypes.c_int32),
        ("chunk_cols", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("rows_near", ctypes.c_int32),
        ("rows_far", ctypes.c_int32),
        ("rows_refine", ctypes.c_int32),
        ("far_grid", ctypes.c_int32),
        ("band_pass", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 2),
    ]


# PALMAD_KERNEL_CLASSES: near, far, refine, polish, length, band
KERNEL_CLASSES = 6


class Stats(ctypes.Structure):
    _fields_ = [
        ("evals_select", ctypes.c_uint64),
        ("evals_refine", ctypes.c_uint64),
        ("evals_polish", ctypes.c_uint64),
        ("range_searches", ctypes.c_uint64),
        ("survivors", ctypes.c_uint64),
        ("seconds", ctypes.c_double),
        ("kernel_evals", ctypes.c_uint64 * KERNEL_CLASSES),
        ("kernel_launches", ctypes.c_uint64 * KERNEL_CLASSES),
        ("kernel_ms", ctypes.c_double * KERNEL_CLASSES),
        ("rows_after_near", ctypes.c_uint64),
        ("rows_after_far", ctypes.c_uint64),
    ]

    def as_dict(self):
        d = {}
        for f, _ in self._fields_:
            v = getattr(self, f)
            d[f] = list(v) if hasattr(v, "__len__") else v
        return d


class TuneReport(ctypes.Structure):
    _fields_ = [
        ("evaluated", ctypes.c_int32),
        ("probe_lengths", ctypes.c_int32),
        ("base_seconds", ctypes.c_double),
        ("best_seconds", ctypes.c_double),
    ]


# PALMAD_STATIC_WORKSPACE_BYTES: the static workspace of palmad_discords_static
STATIC_WORKSPACE_BYTES = 32 << 20
FLAG_TIME_KERNELS = 1
FLAG_NO_GRAPH = 2
KERNEL_CLASSES = ("select_near", "select_far", "refine", "polish")


class PalmadError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32

# name -> (restype, argtypes); every exported symbol of include/palmad.h
SIGNATURES = {
    "palmad_version": (ctypes.c_char_p, []),
    "palmad_last_error": (ctypes.c_char_p, [_vp]),
    "palmad_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int]),
    "palmad_destroy": (None, [_vp]),
    "palmad_workspace_size": (ctypes.c_int, [_i64, _i32, _i32, _i32, ctypes.POINTER(Options),
                                             ctypes.POINTER(ctypes.c_size_t)]),
    "palmad_discords": (ctypes.c_int, [_vp, _vp, _i64, _i32, _i32, _i32, ctypes.POINTER(Options),
                                       _vp, ctypes.c_size_t, _vp, _vp, _vp, _vp, _vp,
                                       ctypes.POINTER(Stats), _vp]),
    "palmad_batched_workspace_size": (ctypes.c_int, [_i32, _vp, _vp, _vp, _i32,
                                                     ctypes.POINTER(Options),
                                                     ctypes.POINTER(ctypes.c_size_t)]),
    "palmad_discords_batched": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _vp, _i32,
                                               ctypes.POINTER(Options), _vp, ctypes.c_size_t, _vp,
                                               _vp, _vp, _vp, _vp, ctypes.POINTER(Stats), _vp]),
    "palmad_autotune_workspace_size": (ctypes.c_int, [_i32, _vp, _vp, _vp, _i32, _i32,
                                                      ctypes.POINTER(ctypes.c_size_t)]),
    "palmad_autotune": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _vp, _i32,
                                       ctypes.POINTER(Options), _i32, _i32, _vp, ctypes.c_size_t,
                                       ctypes.POINTER(Options), ctypes.POINTER(TuneReport), _vp]),
    "palmad_range_discords": (ctypes.c_int, [_vp, _vp, _i64, _i32, ctypes.c_double,
                                             ctypes.POINTER(Options), _vp, ctypes.c_size_t, _vp,
                                             _vp, ctypes.POINTER(_i64), ctypes.POINTER(Stats),
                                             _vp]),
    "palmad_discord_heatmap": (ctypes.c_int, [_vp, _vp, _i64, _i32, _i32, _i32,
                                              ctypes.POINTER(Options), _vp, ctypes.c_size_t, _vp,
                                              _vp, _vp, _vp, _vp, _vp, _i64, _vp,
                                              ctypes.POINTER(Stats), _vp]),
    "palmad_heatmap_interest": (ctypes.c_int, [_vp, _vp, _i32, _i64, _i64, _i32, _i32, _vp, _vp,
                                               _vp, _vp, _vp, _vp]),
    "palmad_window_stats": (ctypes.c_int, [_vp, _vp, _i64, _i32, _i32, _vp, ctypes.c_size_t, _vp,
                                           _vp, _vp]),
    "palmad_selection_drift_workspace_size": (ctypes.c_int, [_i64, _i32, _i32,
                                                             ctypes.POINTER(ctypes.c_size_t)]),
    "palmad_selection_drift": (ctypes.c_int, [_vp, _vp, _i64, _i32, _i32, _i64, _i32,
                                              ctypes.c_float, _vp, ctypes.c_size_t,
                                              ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_double), _vp]),
    "palmad_stream_workspace_size": (ctypes.c_int, [_i64, _i32, _i32, _i32, ctypes.POINTER(Options),
                                                    ctypes.POINTER(ctypes.c_size_t)]),
    "palmad_stream_create": (ctypes.c_int, [_vp, _i64, _i32, _i32, _i32, ctypes.POINTER(Options),
                                            _vp, ctypes.c_size_t, ctypes.POINTER(_vp), _vp]),
    "palmad_stream_append": (ctypes.c_int, [_vp, _vp, _i64, _vp]),
    "palmad_stream_discords": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "palmad_stream_profile": (ctypes.c_int, [_vp, _i32, _vp, _vp]),
    "palmad_stream_length": (_i64, [_vp]),
    "palmad_stream_destroy": (None, [_vp]),
    "palmad_discords_static": (ctypes.c_int, [_vp, _vp, _i64, _i32, _i32, _i32,
                                              ctypes.POINTER(Options), _vp, _vp, _vp, _vp, _vp,
                                              ctypes.POINTER(Stats), _vp]),
    "palmad_backward_workspace_size": (ctypes.c_int, [_i64, _i64, _i32,
                                                      ctypes.POINTER(ctypes.c_size_t)]),
    "palmad_discords_backward": (ctypes.c_int, [_vp, _vp, _i64, _i64, _i32, _vp, _vp, _vp, _vp,
                                                ctypes.c_size_t, _vp, _vp, _vp]),
}

_lib = None


def lib():
    """Load libpalmad.so once; raise if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc: int, ctx=None):
    if rc != PALMAD_OK:
        msg = lib().palmad_last_error(ctx)
        raise PalmadError(rc, msg.decode() if msg else "")


def make_options(dist_bits=0, guard=0.0, near_cols=0, chunk_cols=0, time_kernels=False,
                 rows_near=0, rows_far=0, rows_refine=0, far_grid=0, graphs=True,
                 band_pass=0) -> Options:
    o = Options()
    o.far_grid = int(far_grid)
    o.band_pass = int(band_pass)
    o.rows_near = int(rows_near)
    o.rows_far = int(rows_far)
    o.rows_refine = int(rows_refine)
    o.dist_bits = int(dist_bits)
    o.guard = float(guard)
    o.near_cols = int(near_cols)
    o.chunk_cols = int(chunk_cols)
    o.flags = (FLAG_TIME_KERNELS if time_kernels else 0) | (0 if graphs else FLAG_NO_GRAPH)
    return o
