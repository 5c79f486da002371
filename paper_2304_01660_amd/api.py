"""Python API over the C ABI: torch tensors in, torch tensors out.

Torch supplies device memory (inputs, outputs, workspace) and the current
HIP stream; every step of the search runs in the library's kernels.
"""

from __future__ import annotations

import ctypes
import threading

import torch

from . import _lib

_ctx_lock = threading.Lock()
_ctxs = {}


def context(device: int):
    """The library context of a device (created once per process)."""
    with _ctx_lock:
        c = _ctxs.get(device)
        if c is None:
            p = ctypes.c_void_p()
            _lib.check(_lib.lib().palmad_create(ctypes.byref(p), int(device)))
            c = p
            _ctxs[device] = c
        return c


def workspace_size(n: int, minL: int, maxL: int, k: int, **opts) -> int:
    o = _lib.make_options(**opts)
    nbytes = ctypes.c_size_t(0)
    _lib.check(_lib.lib().palmad_workspace_size(int(n), int(minL), int(maxL), int(k),
                                                ctypes.byref(o), ctypes.byref(nbytes)))
    return int(nbytes.value)


def _series(T: torch.Tensor) -> torch.Tensor:
    if not isinstance(T, torch.Tensor):
        raise TypeError("T must be a torch tensor on a GPU")
    if T.device.type != "cuda":
        raise ValueError("T must live on a GPU device")
    if T.dim() != 1:
        raise ValueError("T must be one-dimensional")
    return T.to(torch.float64).contiguous()


def _stream(dev) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _workspace(nbytes: int, dev) -> torch.Tensor:
    # torch's caching allocator returns 256-byte aligned blocks
    ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dev)
    assert ws.data_ptr() % 256 == 0
    return ws


def discords(T: torch.Tensor, minL: int, maxL: int, k: int, *, dist_bits: int = 0,
             guard: float = 0.0, near_cols: int = 0, chunk_cols: int = 0, workspace=None,
             return_stats: bool = False, time_kernels: bool = False, rows_near: int = 0,
             rows_far: int = 0, rows_refine: int = 0, far_grid: int = 0, graphs: bool = True,
             band_pass: int = 0):
    """Top-k discords of every length in [minL, maxL].

    Returns a dict of device tensors: idx int64[L*k], len int32[L*k],
    nn_dist float64[L*k], nn_idx int64[L*k], count int32[L]; row
    (m - minL) * k + rank.  With ``return_stats`` also the call's counters.
    """
    T = _series(T)
    dev = T.device
    n = T.shape[0]
    L = maxL - minL + 1
    o = _lib.make_options(dist_bits, guard, near_cols, chunk_cols, time_kernels, rows_near,
                          rows_far, rows_refine, far_grid, graphs, band_pass)
    nbytes = workspace_size(n, minL, maxL, k, dist_bits=dist_bits, guard=guard,
                            near_cols=near_cols, chunk_cols=chunk_cols)
    ws = workspace if workspace is not None else _workspace(nbytes, dev)
    if ws.numel() < nbytes:
        raise ValueError(f"workspace has {ws.numel()} bytes, needs {nbytes}")
    out = {
        "idx": torch.empty(L * k, dtype=torch.int64, device=dev),
        "len": torch.empty(L * k, dtype=torch.int32, device=dev),
        "nn_dist": torch.empty(L * k, dtype=torch.float64, device=dev),
        "nn_idx": torch.empty(L * k, dtype=torch.int64, device=dev),
        "count": torch.empty(L, dtype=torch.int32, device=dev),
    }
    st = _lib.Stats()
    ctx = context(dev.index if dev.index is not None else torch.cuda.current_device())
    rc = _lib.lib().palmad_discords(
        ctx, ctypes.c_void_p(T.data_ptr()), n, minL, maxL, k, ctypes.byref(o),
        ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(out["idx"].data_ptr()),
        ctypes.c_void_p(out["len"].data_ptr()), ctypes.c_void_p(out["nn_dist"].data_ptr()),
        ctypes.c_void_p(out["nn_idx"].data_ptr()), ctypes.c_void_p(out["count"].data_ptr()),
        ctypes.byref(st), _stream(dev))
    _lib.check(rc, ctx)
    if return_stats:
        out["stats"] = st.as_dict()
    return out


def discord_heatmap(T: torch.Tensor, minL: int, maxL: int, k: int, *, dist_bits: int = 0,
                    guard: float = 0.0, near_cols: int = 0, chunk_cols: int = 0,
                    return_stats: bool = False, rows_near: int = 0, rows_far: int = 0,
                    rows_refine: int = 0, far_grid: int = 0, graphs: bool = True,
                    band_pass: int = 0):
    """Top-k discords of every length plus the discord heatmap (Eq. (11)).

    Returns the dict of ``discords`` plus ``heat`` float64[L, n - minL + 1]
    (row m - minL: nnDist^2 / (2m) = 1 - rho of every range discord of length
    m, 0 elsewhere) and ``range`` float64[L] (r of each length's successful
    range search).
    """
    T = _series(T)
    dev = T.device
    n = T.shape[0]
    L = maxL - minL + 1
    ld = n - minL + 1
    o = _lib.make_options(dist_bits, guard, near_cols, chunk_cols, False, rows_near, rows_far,
                          rows_refine, far_grid, graphs, band_pass)
    nbytes = workspace_size(n, minL, maxL, k, dist_bits=dist_bits, guard=guard,
                            near_cols=near_cols, chunk_cols=chunk_cols)
    ws = _workspace(nbytes, dev)
    out = {
        "idx": torch.empty(L * k, dtype=torch.int64, device=dev),
        "len": torch.empty(L * k, dtype=torch.int32, device=dev),
        "nn_dist": torch.empty(L * k, dtype=torch.float64, device=dev),
        "nn_idx": torch.empty(L * k, dtype=torch.int64, device=dev),
        "count": torch.empty(L, dtype=torch.int32, device=dev),
        "heat": torch.empty((L, ld), dtype=torch.float64, device=dev),
        "range": torch.empty(L, dtype=torch.float64, device=dev),
    }
    st = _lib.Stats()
    ctx = context(dev.index if dev.index is not None else torch.cuda.current_device())
    rc = _lib.lib().palmad_discord_heatmap(
        ctx, ctypes.c_void_p(T.data_ptr()), n, minL, maxL, k, ctypes.byref(o),
        ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(out["idx"].data_ptr()),
        ctypes.c_void_p(out["len"].data_ptr()), ctypes.c_void_p(out["nn_dist"].data_ptr()),
        ctypes.c_void_p(out["nn_idx"].data_ptr()), ctypes.c_void_p(out["count"].data_ptr()),
        ctypes.c_void_p(out["heat"].data_ptr()), ld, ctypes.c_void_p(out["range"].data_ptr()),
        ctypes.byref(st), _stream(dev))
    _lib.check(rc, ctx)
    if return_stats:
        out["stats"] = st.as_dict()
    return out


def heatmap_interest(heat: torch.Tensor, minL: int, k: int):
    """Discord interest (Eq. (12)) of a heatmap [L, ncols] from discord_heatmap.

    Returns (col_score float64[ncols], col_len int32[ncols], top_idx int64[k],
    top_len int32[k], top_score float64[k]) as device tensors: per column the
    largest value over the lengths and its length, and the k best columns.
    """
    if heat.dim() != 2 or heat.dtype != torch.float64 or not heat.is_cuda:
        raise ValueError("heat must be a 2-D float64 CUDA tensor")
    heat = heat.contiguous()
    dev = heat.device
    L, ncols = heat.shape
    col_score = torch.empty(ncols, dtype=torch.float64, device=dev)
    col_len = torch.empty(ncols, dtype=torch.int32, device=dev)
    top_idx = torch.empty(k, dtype=torch.int64, device=dev)
    top_len = torch.empty(k, dtype=torch.int32, device=dev)
    top_score = torch.empty(k, dtype=torch.float64, device=dev)
    ctx = context(dev.index if dev.index is not None else torch.cuda.current_device())
    rc = _lib.lib().palmad_heatmap_interest(
        ctx, ctypes.c_void_p(heat.data_ptr()), L, ncols, ncols, minL, k,
        ctypes.c_void_p(col_score.data_ptr()), ctypes.c_void_p(col_len.data_ptr()),
        ctypes.c_void_p(top_idx.data_ptr()), ctypes.c_void_p(top_len.data_ptr()),
        ctypes.c_void_p(top_score.data_ptr()), _stream(dev))
    _lib.check(rc, ctx)
    return col_score, col_len, top_idx, top_len, top_score


def batched_workspace_size(lengths, minL, maxL, k: int, **opts) -> int:
    """Workspace bytes of discords_batched for series of the given lengths."""
    B = len(lengths)
    offs = (ctypes.c_int64 * (B + 1))()
    for b, n in enumerate(lengths):
        offs[b + 1] = offs[b] + int(n)
    lo = (ctypes.c_int32 * B)(*[int(v) for v in minL])
    hi = (ctypes.c_int32 * B)(*[int(v) for v in maxL])
    o = _lib.make_options(**opts)
    nbytes = ctypes.c_size_t(0)
    _lib.check(_lib.lib().palmad_batched_workspace_size(B, offs, lo, hi, int(k), ctypes.byref(o),
                                                        ctypes.byref(nbytes)))
    return int(nbytes.value)


def discords_batched(series, minL, maxL, k: int, *, dist_bits: int = 0, guard: float = 0.0,
                     near_cols: int = 0, chunk_cols: int = 0, return_stats: bool = False,
                     time_kernels: bool = False, rows_near: int = 0, rows_far: int = 0,
                     rows_refine: int = 0, far_grid: int = 0, graphs: bool = True,
                     band_pass: int = 0,
                     workspace=None):
    """Top-k discords of every length of several series in one search.

    ``series`` is a list of 1-D GPU tensors (or one flat tensor plus
    ``offsets`` given as a list of lengths via a (values, lengths) tuple);
    ``minL``/``maxL`` are ints or per-series sequences.  Returns a list with
    one dict per series, laid out as the result of :func:`discords`.
    """
    if isinstance(series, tuple):
        values, lengths = series
        values = _series(values)
        lengths = [int(v) for v in lengths]
    else:
        parts = [_series(t) for t in series]
        if not parts:
            raise ValueError("no series given")
        values = torch.cat(parts) if len(parts) > 1 else parts[0]
        lengths = [int(t.shape[0]) for t in parts]
    dev = values.device
    B = len(lengths)
    lo = [int(minL)] * B if isinstance(minL, int) else [int(v) for v in minL]
    hi = [int(maxL)] * B if isinstance(maxL, int) else [int(v) for v in maxL]
    if len(lo) != B or len(hi) != B:
        raise ValueError("minL and maxL need one entry per series")
    offs = (ctypes.c_int64 * (B + 1))()
    for b, n in enumerate(lengths):
        offs[b + 1] = offs[b] + n
    if offs[B] != values.shape[0]:
        raise ValueError("series lengths do not add up to the values")
    c_lo = (ctypes.c_int32 * B)(*lo)
    c_hi = (ctypes.c_int32 * B)(*hi)
    o = _lib.make_options(dist_bits, guard, near_cols, chunk_cols, time_kernels, rows_near,
                          rows_far, rows_refine, far_grid, graphs, band_pass)
    nbytes = ctypes.c_size_t(0)
    _lib.check(_lib.lib().palmad_batched_workspace_size(B, offs, c_lo, c_hi, int(k),
                                                        ctypes.byref(o), ctypes.byref(nbytes)))
    nbytes = int(nbytes.value)
    ws = workspace if workspace is not None else _workspace(nbytes, dev)
    if ws.numel() < nbytes:
        raise ValueError(f"workspace has {ws.numel()} bytes, needs {nbytes}")
    Ls = [h - l + 1 for l, h in zip(lo, hi)]
    rows = sum(Ls) * k
    idx = torch.empty(rows, dtype=torch.int64, device=dev)
    ln = torch.empty(rows, dtype=torch.int32, device=dev)
    nn = torch.empty(rows, dtype=torch.float64, device=dev)
    nnj = torch.empty(rows, dtype=torch.int64, device=dev)
    cnt = torch.empty(sum(Ls), dtype=torch.int32, device=dev)
    st = _lib.Stats()
    ctx = context(dev.index if dev.index is not None else torch.cuda.current_device())
    rc = _lib.lib().palmad_discords_batched(
        ctx, ctypes.c_void_p(values.data_ptr()), offs, B, c_lo, c_hi, int(k), ctypes.byref(o),
        ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(idx.data_ptr()),
        ctypes.c_void_p(ln.data_ptr()), ctypes.c_void_p(nn.data_ptr()),
        ctypes.c_void_p(nnj.data_ptr()), ctypes.c_void_p(cnt.data_ptr()), ctypes.byref(st),
        _stream(dev))
    _lib.check(rc, ctx)
    res = []
    r0 = c0 = 0
    for L in Ls:
        res.append({"idx": idx[r0:r0 + L * k], "len": ln[r0:r0 + L * k],
                    "nn_dist": nn[r0:r0 + L * k], "nn_idx": nnj[r0:r0 + L * k],
                    "count": cnt[c0:c0 + L]})
        r0 += L * k
        c0 += L
    if return_stats:
        return res, st.as_dict()
    return res


TUNED_KEYS = ("dist_bits", "guard", "near_cols", "chunk_cols", "rows_near", "rows_far",
              "rows_refine", "far_grid", "band_pass")


def autotune(series, minL, maxL, k: int, *, probe_lengths: int = 6, reps: int = 2, **base):
    """Pick the sweeps' tile geometry by timing probes of the search itself.

    ``series`` is one 1-D GPU tensor or a list of them (as for
    :func:`discords_batched`); ``base`` holds starting options.  Returns
    (options dict for :func:`discords` / :func:`discords_batched`, report).
    """
    if isinstance(series, torch.Tensor):
        parts = [_series(series)]
    else:
        parts = [_series(t) for t in series]
    values = torch.cat(parts) if len(parts) > 1 else parts[0]
    dev = values.device
    B = len(parts)
    lo = [int(minL)] * B if isinstance(minL, int) else [int(v) for v in minL]
    hi = [int(maxL)] * B if isinstance(maxL, int) else [int(v) for v in maxL]
    offs = (ctypes.c_int64 * (B + 1))()
    for b, t in enumerate(parts):
        offs[b + 1] = offs[b] + int(t.shape[0])
    c_lo = (ctypes.c_int32 * B)(*lo)
    c_hi = (ctypes.c_int32 * B)(*hi)
    nbytes = ctypes.c_size_t(0)
    _lib.check(_lib.lib().palmad_autotune_workspace_size(B, offs, c_lo, c_hi, int(k),
                                                         int(probe_lengths),
                                                         ctypes.byref(nbytes)))
    ws = _workspace(int(nbytes.value), dev)
    o = _lib.make_options(**base)
    best = _lib.Options()
    rep = _lib.TuneReport()
    ctx = context(dev.index if dev.index is not None else torch.cuda.current_device())
    rc = _lib.lib().palmad_autotune(ctx, ctypes.c_void_p(values.data_ptr()), offs, B, c_lo, c_hi,
                                    int(k), ctypes.byref(o), int(probe_lengths), int(reps),
                                    ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                    ctypes.byref(best), ctypes.byref(rep), _stream(dev))
    _lib.check(rc, ctx)
    opts = {key: getattr(best, key) for key in TUNED_KEYS}
    report = {f: getattr(rep, f) for f, _ in rep._fields_}
    return opts, report


def range_discords(T: torch.Tensor, m: int, r: float, *, dist_bits: int = 0, guard: float = 0.0,
                   near_cols: int = 0, chunk_cols: int = 0, return_stats: bool = False,
                   time_kernels: bool = False, rows_near: int = 0, rows_far: int = 0,
                   rows_refine: int = 0, far_grid: int = 0, band_pass: int = 0):
    """All subsequences of length m whose nearest non-self match is >= r away.

    Returns (mask bool[N] on the device, nn_dist float64[N] valid where mask,
    count); with ``return_stats`` also the counters.
    """
    T = _series(T)
    dev = T.device
    n = T.shape[0]
    N = n - m + 1
    o = _lib.make_options(dist_bits, guard, near_cols, chunk_cols, time_kernels, rows_near,
                          rows_far, rows_refine, far_grid, True, band_pass)
    nbytes = workspace_size(n, m, m, 1, dist_bits=dist_bits, guard=guard, near_cols=near_cols,
                            chunk_cols=chunk_cols)
    ws = _workspace(nbytes, dev)
    words = torch.empty((N + 63) // 64, dtype=torch.int64, device=dev)
    nn = torch.empty(N, dtype=torch.float64, device=dev)
    cnt = ctypes.c_int64(0)
    st = _lib.Stats()
    ctx = context(dev.index if dev.index is not None else torch.cuda.current_device())
    rc = _lib.lib().palmad_range_discords(
        ctx, ctypes.c_void_p(T.data_ptr()), n, m, float(r), ctypes.byref(o),
        ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(words.data_ptr()),
        ctypes.c_void_p(nn.data_ptr()), ctypes.byref(cnt), ctypes.byref(st), _stream(dev))
    _lib.check(rc, ctx)
    bits = torch.arange(64, device=dev, dtype=torch.int64)
    mask = ((words[:, None] >> bits[None, :]) & 1).reshape(-1)[:N].bool()
    res = (mask, nn, int(cnt.value))
    if return_stats:
        return res + (st.as_dict(),)
    return res


def window_stats(T: torch.Tensor, minL: int, m: int):
    """(mu, sigma) of every window of length m, from Eq. (4) at minL then Eq. (7)-(8)."""
    T = _series(T)
    dev = T.device
    n = T.shape[0]
    N = n - m + 1
    nbytes = workspace_size(n, minL, m, 1)
    ws = _workspace(nbytes, dev)
    mu = torch.empty(N, dtype=torch.float64, device=dev)
    sg = torch.empty(N, dtype=torch.float64, device=dev)
    ctx = context(dev.index if dev.index is not None else torch.cuda.current_device())
    rc = _lib.lib().palmad_window_stats(ctx, ctypes.c_void_p(T.data_ptr()), n, minL, m,
                                        ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                        ctypes.c_void_p(mu.data_ptr()),
                                        ctypes.c_void_p(sg.data_ptr()), _stream(dev))
    _lib.check(rc, ctx)
    return mu, sg


def discords_backward(T: torch.Tensor, idx: torch.Tensor, length: torch.Tensor,
                      grad_nn: torch.Tensor, maxm: int | None = None, grad_T=None,
                      return_nn_idx: bool = False):
    """grad_T += sum_q grad_nn[q] * d nnDist(idx[q], len[q]) / dT (FP64).

    The nearest neighbour of every row is recomputed on the device; see
    palmad_discords_backward in include/palmad.h.
    """
    T = _series(T)
    dev = T.device
    n = T.shape[0]
    idx = idx.to(device=dev, dtype=torch.int64).contiguous()
    length = length.to(device=dev, dtype=torch.int32).contiguous()
    g = grad_nn.to(device=dev, dtype=torch.float64).contiguous()
    K = idx.numel()
    if maxm is None:
        maxm = int(length.max().item()) if K else 3
    nbytes = ctypes.c_size_t(0)
    _lib.check(_lib.lib().palmad_backward_workspace_size(n, K, int(maxm), ctypes.byref(nbytes)))
    ws = _workspace(int(nbytes.value), dev)
    if grad_T is None:
        grad_T = torch.zeros(n, dtype=torch.float64, device=dev)
    nnj = torch.empty(max(K, 1), dtype=torch.int64, device=dev)
    ctx = context(dev.index if dev.index is not None else torch.cuda.current_device())
    rc = _lib.lib().palmad_discords_backward(
        ctx, ctypes.c_void_p(T.data_ptr()), n, K, int(maxm), ctypes.c_void_p(idx.data_ptr()),
        ctypes.c_void_p(length.data_ptr()), ctypes.c_void_p(g.data_ptr()),
        ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(grad_T.data_ptr()),
        ctypes.c_void_p(nnj.data_ptr()), _stream(dev))
    _lib.check(rc, ctx)
    if return_nn_idx:
        return grad_T, nnj[:K]
    return grad_T


class DiscordNNDist(torch.autograd.Function):
    """nnDist of the top-k discords of every length, differentiable in T.

    forward(T, minL, maxL, k, options dict) -> (nn_dist, idx, len, nn_idx);
    only nn_dist carries a gradient.  The backward pass recomputes each
    reported row's nearest neighbour on the device and scatters the
    closed-form derivative (held at that neighbour) into dL/dT.
    """

    @staticmethod
    def forward(ctx, T, minL, maxL, k, options=None):
        out = discords(T.detach(), int(minL), int(maxL), int(k), **(options or {}))
        ctx.save_for_backward(T.detach(), out["idx"], out["len"])
        ctx.maxL = int(maxL)
        ctx.mark_non_differentiable(out["idx"], out["len"], out["nn_idx"])
        return out["nn_dist"], out["idx"], out["len"], out["nn_idx"]

    @staticmethod
    def backward(ctx, g_nn, g_idx=None, g_len=None, g_nnidx=None):
        T, idx, ln = ctx.saved_tensors
        gT = discords_backward(T, idx, ln, g_nn, maxm=ctx.maxL)
        return gT.to(T.dtype), None, None, None, None


def discord_nn_dist(T: torch.Tensor, minL: int, maxL: int, k: int, **options):
    """Differentiable nnDist[L*k] of the top-k discords (see DiscordNNDist)."""
    return DiscordNNDist.apply(T, minL, maxL, k, options)[0]


def selection_drift(T: torch.Tensor, minL: int, m: int, *, items: int = 2048, chunk: int = 512,
                    guard: float = 0.0):
    """(drift, band): the largest |rho_FP32 - rho_FP64| of the FP32 selection
    recurrence over `items` sampled 512-row tiles of `chunk` columns at
    length m, and the guard band the selection sweep uses there."""
    T = _series(T)
    dev = T.device
    n = T.shape[0]
    nb = ctypes.c_size_t(0)
    _lib.check(_lib.lib().palmad_selection_drift_workspace_size(n, int(minL), int(m),
                                                                ctypes.byref(nb)))
    ws = _workspace(int(nb.value), dev)
    d, b = ctypes.c_double(0.0), ctypes.c_double(0.0)
    ctx = context(dev.index if dev.index is not None else torch.cuda.current_device())
    rc = _lib.lib().palmad_selection_drift(ctx, ctypes.c_void_p(T.data_ptr()), n, int(minL), int(m),
                                           int(items), int(chunk), float(guard),
                                           ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                           ctypes.byref(d), ctypes.byref(b), _stream(dev))
    _lib.check(rc, ctx)
    return d.value, b.value


class Stream:
    """A series that grows by appends (palmad_stream_*): after any append,
    the top-k discords of every length of the series so far, equal to
    ``discords`` on the same points, and the exact nearest-neighbour profile
    of any length.  The device workspace is held until ``close``."""

    def __init__(self, capacity: int, minL: int, maxL: int, k: int, device=None, **opts):
        dev = torch.device("cuda", device if device is not None else torch.cuda.current_device())
        self.device = dev
        self.minL, self.maxL, self.k = int(minL), int(maxL), int(k)
        o = _lib.make_options(**opts)
        nbytes = ctypes.c_size_t(0)
        _lib.check(_lib.lib().palmad_stream_workspace_size(int(capacity), self.minL, self.maxL,
                                                            self.k, ctypes.byref(o),
                                                            ctypes.byref(nbytes)))
        self._ws = _workspace(int(nbytes.value), dev)
        self._ctx = context(dev.index)
        h = ctypes.c_void_p()
        rc = _lib.lib().palmad_stream_create(self._ctx, int(capacity), self.minL, self.maxL, self.k,
                                             ctypes.byref(o), ctypes.c_void_p(self._ws.data_ptr()),
                                             self._ws.numel(), ctypes.byref(h), _stream(dev))
        _lib.check(rc, self._ctx)
        self._h = h

    def __len__(self) -> int:
        return int(_lib.lib().palmad_stream_length(self._h))

    def append(self, values: torch.Tensor) -> None:
        v = _series(values)
        rc = _lib.lib().palmad_stream_append(self._h, ctypes.c_void_p(v.data_ptr()), v.shape[0],
                                             _stream(self.device))
        _lib.check(rc, self._ctx)

    def discords(self) -> dict:
        L = self.maxL - self.minL + 1
        dev = self.device
        out = {
            "idx": torch.empty(L * self.k, dtype=torch.int64, device=dev),
            "len": torch.empty(L * self.k, dtype=torch.int32, device=dev),
            "nn_dist": torch.empty(L * self.k, dtype=torch.float64, device=dev),
            "nn_idx": torch.empty(L * self.k, dtype=torch.int64, device=dev),
        }
        rc = _lib.lib().palmad_stream_discords(
            self._h, *[ctypes.c_void_p(out[key].data_ptr()) for key in ("idx", "len", "nn_dist", "nn_idx")],
            _stream(dev))
        _lib.check(rc, self._ctx)
        return out

    def profile(self, m: int) -> torch.Tensor:
        nn = torch.empty(len(self) - int(m) + 1, dtype=torch.float64, device=self.device)
        rc = _lib.lib().palmad_stream_profile(self._h, int(m), ctypes.c_void_p(nn.data_ptr()),
                                              _stream(self.device))
        _lib.check(rc, self._ctx)
        return nn

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.lib().palmad_stream_destroy(self._h)
            self._h = None
            self._ws = None

    def __del__(self):
        self.close()
