"""Benchmark: top-k range discords over a length range on one MI355X.

Headline workload (one "step" = one full search, every length, through the
C ABI): a seeded ECG-like series of n = 1,000,000 points (beats of three
Gaussian bumps, period U(240, 260) samples, N(0, 0.05^2) noise, 20 malformed
beats; FP32-canonical values), lengths m = 128..256 (129 lengths), top-3
discords per length; FP32 selection sweep, FP64 refinement and exact FP64
distances.  Inputs are resident in HBM before the timed region.

Prints one JSON line: lengths/s as `value`, plus device-counted distance
evaluations/s, the roofline of the dominant kernel (from HIP events recorded
around its launches on the library's stream during instrumented steps), the
per-length statistics kernel against the HBM roofline, legs on the other
workloads (the 100k random walk, the 64-series batch against the plain
per-series loop, forward + backward on the 200k random walk, the discord
heatmap, the dense matrix profile and the streaming series) and the CPU
oracle on a bounded sample of the headline workload.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "z-norm distance evals/sec + lengths/sec over [minL,maxL]; batched vs plain"
# VALU issue rate of MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz lane-ops/s
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBPS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# Minimal VALU lane-operations per pair evaluation of a sweep step: two FMAs
# for the covariance update, one multiply by 1/(sqrt(m) sigma_j), one compare
# (selection) or max (refinement).
OPS_PER_EVAL = 4
# Algorithmic HBM bytes of the per-length statistics step per subsequence
# and length: the series value (8), mean and sigma read and written (32),
# three FP32 helpers (12), two bitmaps (1/4, rounded into the 52).
LENGTH_BYTES_PER_SUBSEQ = 52
KERNEL_NAMES = {
    "select_near": "k_select_near",
    "select_far": "k_select_far",
    "refine": "k_refine",
    "polish": "k_polish",
    "length": "k_length",
    "select_band": "k_select_band",
}
CLASS_NAMES = ("select_near", "select_far", "refine", "polish", "length", "select_band")
SERIES_TEXT = {
    "c2": "seeded random walk with 5 injected sine bursts/level shifts (seed 1)",
    "c3": ("seeded ECG-like beat train (3 Gaussian bumps per beat, period U(240, 260), "
           "N(0, 0.05^2) noise) with 20 malformed beats (seed 2)"),
    "c5": "seeded random walk with 10 injected sine bursts (seed 4)",
}


def host_cpu():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model or "unknown", "logical_cpus": os.cpu_count()}


def workload(synth, tag):
    return {"c2": synth.config2, "c3": synth.config3, "c5": synth.config5}[tag]()


def golden_of(tag, w):
    path = os.path.join(ROOT, "tests", "golden", f"{tag}_{w.name}.json")
    return json.load(open(path)) if os.path.exists(path) else None


def merlin_calls(w, golden):
    """Every DRAG call of the oracle's MERLIN run on this workload, as
    (length index, r), rebuilt from the stored per-length results with the
    rules of Alg. 1 (first length: 2 sqrt(minL), halved after a failure;
    next four: 0.99 nnDist(m - 1), times 0.99 after a failure; later: mean -
    2 sd of the last five nnDist, lowered by sd after a failure; nnDist(m) =
    the k-th reported distance).  Each length's last r is checked against
    the stored one."""
    import math

    L = w.maxL - w.minL + 1
    k = w.k
    hist = [golden["nn"][li * k + k - 1] for li in range(L)]
    calls = []
    for li in range(L):
        nc = golden["calls"][li]
        if li == 0:
            rs = [2.0 * math.sqrt(w.minL) * 0.5 ** c for c in range(nc)]
        elif li <= 4:
            rs = [0.99 * hist[li - 1] * 0.99 ** c for c in range(nc)]
        else:
            last = hist[li - 5:li]
            mu = sum(last) / 5.0
            sd = math.sqrt(sum((x - mu) ** 2 for x in last) / 5.0)
            r, rs = mu - 2.0 * sd, []
            for c in range(nc):
                rs.append(r)
                r = r - sd if sd > 0.0 else 0.99 * r
        if abs(rs[-1] - golden["r"][li]) > 1e-9 * max(1.0, abs(golden["r"][li])):
            return None
        calls += [(li, r) for r in rs]
    return calls


def cpu_baseline(w, golden, budget_s: float):
    """The oracle (serial FP64 DRAG, oracle/merlin.c) on a stratified sample
    of the DRAG calls its MERLIN run makes on this workload (failed attempts
    and the first length's range halving included, rebuilt from the stored
    result), until the time budget is spent; lengths/s = lengths / (mean
    sampled call time x number of calls).  The full run's own wall time,
    taken when the stored result was written, is reported beside it."""
    import oracle

    if golden is None:
        return None
    L = w.maxL - w.minL + 1
    calls = merlin_calls(w, golden)
    if calls is None:
        return None
    # stratified order over the calls: middle, then halves, quarters, ...
    order, seen = [], set()
    for step in (2, 4, 8, 16, 32, 64, 128, 256):
        for q in range(1, step, 2):
            c = min(len(calls) - 1, q * len(calls) // step)
            if c not in seen:
                seen.add(c)
                order.append(c)
    order = [0] + [c for c in order if c != 0]  # the first call (largest r) too
    t0 = time.perf_counter()
    done = []
    for c in order:
        li, r = calls[c]
        oracle.drag(w.T, w.minL + li, r)
        done.append((w.minL + li, round(r, 4)))
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    est = dt / len(done) * len(calls)
    full_s = golden.get("oracle_seconds")
    return {
        "value": L / est,
        "unit": "lengths/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"serial FP64 DRAG of the oracle (oracle/merlin.c): {len(done)} of the "
                   f"{len(calls)} DRAG calls of its MERLIN run on the same series, as (m, r) "
                   f"{done}, {dt:.1f} s; lengths/s = {L} lengths / (mean call time x "
                   f"{len(calls)} calls)"),
        "host_cpu": host_cpu(),
        "full_run": {
            "seconds": full_s,
            "lengths_per_s": (L / full_s) if full_s else None,
            "what": "the oracle's complete MERLIN on this workload (every length, every DRAG "
                    "call), timed when the stored result was written",
            "host_cpu": (golden.get("oracle_host") or {}).get("cpu"),
            "threads": (golden.get("oracle_host") or {}).get("threads_used", 1),
        },
    }


def check_golden(out, golden):
    import numpy as np
    if golden is None:
        return "no-golden"
    idx = out["idx"].cpu().numpy()
    nn = out["nn_dist"].cpu().numpy()
    gi = np.array(golden["idx"])
    gn = np.array(golden["nn"])
    if not np.allclose(nn, gn, rtol=1e-9):
        return "nn-mismatch"
    if not np.array_equal(idx, gi):
        return "index-near-tie"
    return "exact"


def search_leg(api, torch, dev, w, tuned, steps, warmup):
    """Time the full search (production path: graph replay, no events), then
    the same steps with HIP events around every kernel class on the
    library's stream."""
    T = torch.from_numpy(w.T).to(dev)
    L = w.maxL - w.minL + 1
    ws = torch.empty(api.workspace_size(w.n, w.minL, w.maxL, w.k), dtype=torch.uint8, device=dev)
    for _ in range(warmup):
        api.discords(T, w.minL, w.maxL, w.k, workspace=ws, **tuned)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = api.discords(T, w.minL, w.maxL, w.k, workspace=ws, return_stats=True, **tuned)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt / steps * 1e3
    st_prod = out["stats"]
    agg = None
    t1 = time.perf_counter()
    for _ in range(steps):
        out_t = api.discords(T, w.minL, w.maxL, w.k, workspace=ws, return_stats=True,
                             time_kernels=True, **tuned)
        st = out_t["stats"]
        if agg is None:
            agg = {k: (list(v) if isinstance(v, list) else v) for k, v in st.items()}
        else:
            for k, v in st.items():
                if isinstance(v, list):
                    agg[k] = [a + b for a, b in zip(agg[k], v)]
                else:
                    agg[k] += v
    torch.cuda.synchronize()
    ms_instrumented = (time.perf_counter() - t1) / steps * 1e3
    for key in ("idx", "nn_dist", "nn_idx", "count"):
        if not torch.equal(out[key], out_t[key]):
            raise SystemExit("instrumented and production runs disagree")
    evals = st_prod["evals_select"] + st_prod["evals_refine"] + st_prod["evals_polish"]
    kernels = {}
    for ci, name in enumerate(CLASS_NAMES):
        launches = agg["kernel_launches"][ci]
        ms = agg["kernel_ms"][ci]
        kernels[name] = {
            "launches_per_step": launches / steps,
            "ms_per_step": ms / steps,
            "evals_per_step": agg["kernel_evals"][ci] / steps,
            "avg_launch_us": (ms / launches * 1e3) if launches else None,
        }
    dom = max(("select_near", "select_far", "refine", "select_band"),
              key=lambda k: kernels[k]["ms_per_step"])
    dk = kernels[dom]
    achieved = None
    if dk["ms_per_step"] > 0:
        # evals per launch / average launch duration == evals / summed duration
        achieved = dk["evals_per_step"] * OPS_PER_EVAL / (dk["ms_per_step"] * 1e-3) / 1e12
    # per-length statistics kernel against HBM: algorithmic bytes of every
    # length's statistics over the kernel's summed time (retry rounds only
    # reset bitmaps and add time, not algorithmic bytes)
    lk = kernels["length"]
    len_bytes = sum(LENGTH_BYTES_PER_SUBSEQ * (w.n - m + 1) for m in range(w.minL, w.maxL + 1))
    len_gbps = len_bytes / (lk["ms_per_step"] * 1e-3) / 1e9 if lk["ms_per_step"] > 0 else None
    return {
        "out": out,
        "T": T,
        "ms_per_step": ms_per_step,
        "seconds": dt,
        "lengths_per_s": L / (ms_per_step * 1e-3),
        "evals_per_s": evals / (ms_per_step * 1e-3),
        "range_searches_per_step": st_prod["range_searches"],
        "ms_per_step_instrumented": ms_instrumented,
        "kernels": kernels,
        "dominant": dom,
        "achieved": achieved,
        "length_kernel_hbm": {
            "bytes_per_step": len_bytes,
            "ms_per_step": lk["ms_per_step"],
            "launches_per_step": lk["launches_per_step"],
            "achieved_GBps": len_gbps,
            "peak_GBps": HBM_PEAK_GBPS,
            "frac": len_gbps / HBM_PEAK_GBPS if len_gbps else None,
            "bytes_per_subsequence": LENGTH_BYTES_PER_SUBSEQ,
        },
    }


def batched_vs_plain(api, synth, tuning, torch, dev, reps: int, retune: bool):
    """64 uneven series (lengths log-uniform in [1e4, 2e5], each with its own
    length range of 51 lengths, top-1): one batched call against a loop of
    single-series calls over the same series.  The batched call uses tile
    geometry from the autotuner (tuned on the batch, outside the timing); the
    loop gets the best of: default geometry with graph replay, default
    geometry with direct launches, and the tuned geometry."""
    ws = synth.config4()
    vals = [torch.from_numpy(w.T).to(dev) for w in ws]
    lo = [w.minL for w in ws]
    hi = [w.maxL for w in ws]
    lengths = sum(h - l + 1 for l, h in zip(lo, hi))
    nb = api.batched_workspace_size([v.shape[0] for v in vals], lo, hi, 1)
    wsb = torch.empty(nb, dtype=torch.uint8, device=dev)
    flat = torch.cat(vals)
    sizes = [v.shape[0] for v in vals]
    tuned, report = tuning.batch_options(), "stored"
    if retune:
        probe, treps = tuning.PROBES["batch"]
        tuned, report = api.autotune(vals, lo, hi, 1, probe_lengths=probe, reps=treps)
    res = api.discords_batched((flat, sizes), lo, hi, 1, workspace=wsb, **tuned)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        res, st = api.discords_batched((flat, sizes), lo, hi, 1, workspace=wsb,
                                       return_stats=True, **tuned)
    torch.cuda.synchronize()
    t_batched = (time.perf_counter() - t0) / reps
    evals_b = st["evals_select"] + st["evals_refine"] + st["evals_polish"]
    wss = [torch.empty(api.workspace_size(w.n, w.minL, w.maxL, 1), dtype=torch.uint8, device=dev)
           for w in ws]
    plain = {}
    variants = {"default_graph": dict(graphs=True), "default_direct": dict(graphs=False)}
    if tuned:
        variants["tuned_graph"] = dict(tuned)
    for name, kw in variants.items():
        for b, w in enumerate(ws):  # warm-up
            api.discords(vals[b], w.minL, w.maxL, 1, workspace=wss[b], **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            outs = [api.discords(vals[b], w.minL, w.maxL, 1, workspace=wss[b], **kw)
                    for b, w in enumerate(ws)]
        torch.cuda.synchronize()
        plain[name] = (time.perf_counter() - t0) / reps
    same = all(torch.equal(res[b][key], outs[b][key]) for b in range(len(ws))
               for key in ("idx", "len", "nn_dist", "nn_idx", "count"))
    t_plain = min(plain.values())
    return {
        "workload": tuning.BATCH_NAME,
        "series": len(ws),
        "points": int(sum(sizes)),
        "lengths": lengths,
        "batched_s": t_batched,
        "batched_lengths_per_s": lengths / t_batched,
        "batched_evals_per_s": evals_b / t_batched,
        "plain_loop_s": t_plain,
        "plain_loop_lengths_per_s": lengths / t_plain,
        "plain_loop_variants_s": plain,
        "speedup": t_plain / t_batched,
        "results_identical_to_last_loop_variant": bool(same),
        "tuned_options": tuned,
        "tune_report": report,
        "reps": reps,
    }


def heatmap_leg(api, torch, dev, w, T, tuned, ms_plain, plain_out, reps: int = 3):
    """The discord heatmap search (Eq. (11)) on the same workload, and the
    interest kernels (Eq. (12)) on its heatmap, timed on the GPU."""
    opts = dict(tuned or {})
    L = w.maxL - w.minL + 1
    api.discord_heatmap(T, w.minL, w.maxL, w.k, **opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        hm = api.discord_heatmap(T, w.minL, w.maxL, w.k, **opts)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    same = bool(torch.equal(hm["idx"], plain_out["idx"]))
    heat = hm["heat"]
    ncols = heat.shape[1]
    api.heatmap_interest(heat, w.minL, w.k)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    ir = 10
    for _ in range(ir):
        api.heatmap_interest(heat, w.minL, w.k)
    e1.record(st)
    torch.cuda.synchronize()
    ims = e0.elapsed_time(e1) / ir
    nbytes = L * ncols * 8 + ncols * 12 + w.k * 20
    return {
        "workload": w.name,
        "ms_per_search": ms,
        "lengths_per_s": L / (ms * 1e-3),
        "slowdown_vs_top_k_only": ms / ms_plain,
        "top_k_identical_to_plain_search": same,
        "range_discords_total": int(hm["count"].sum().item()),
        "interest": {
            "ms": ims,
            "columns": ncols,
            "algorithmic_bytes": nbytes,
            "achieved_GBps": nbytes / (ims * 1e-3) / 1e9,
            "peak_GBps": 8000.0,
            "frac": nbytes / (ims * 1e-3) / 8e12,
            "bound": "hbm",
        },
    }


def dense_leg(api, torch, w, T, tuned, ms_plain, reps: int = 3):
    """The dense exact matrix profile at one length (a range search with
    r = 0: no pruning, every pair swept in FP64 on both sides), against the
    pruned search's time per length: whether pruning pays on this GPU."""
    m = (w.minL + w.maxL) // 2
    opts = dict(tuned or {})
    api.range_discords(T, m, 0.0, **opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        api.range_discords(T, m, 0.0, **opts)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    _, _, cnt, st = api.range_discords(T, m, 0.0, return_stats=True, time_kernels=True, **opts)
    ev = st["kernel_evals"][2]
    kms = st["kernel_ms"][2]
    lanes = ev * OPS_PER_EVAL / (kms * 1e-3) / 1e12 if kms > 0 else None
    L = w.maxL - w.minL + 1
    return {
        "m": m,
        "ms": ms,
        "subsequences": cnt,
        "pair_evaluations": ev,
        "refine_kernel_ms": kms,
        "refine_Tlane_ops_per_s": lanes,
        "refine_frac_of_valu_peak": lanes / VALU_PEAK_TOPS if lanes else None,
        "pruned_search_ms_per_length": ms_plain / L,
        "pruning_speedup": ms / (ms_plain / L),
    }


def ordered_pairs(n: int, m: int) -> int:
    """Ordered non-self-match pairs (i, j), |i - j| >= m, among the
    subsequences of length m of n points."""
    N = n - m + 1
    if N <= m:
        return 0
    return N * (N - 1) - 2 * ((m - 1) * N - m * (m - 1) // 2)


def stream_leg(api, torch, dev, w, cuts, reps: int = 2):
    """The series appended in pieces (streaming series): wall time of the
    appends and of one top-k query, the pairs the appends add (every
    ordered non-self pair of the final series, each evaluated once by the
    FP64 band sweeps) and their rate against the VALU issue ceiling."""
    T = torch.from_numpy(w.T).to(dev)
    L = w.maxL - w.minL + 1
    app_ms, q_ms = [], []
    for rep in range(reps + 1):
        st = api.Stream(w.n, w.minL, w.maxL, w.k, device=dev.index or 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a, b in zip(cuts[:-1], cuts[1:]):
            st.append(T[a:b])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        out = st.discords()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        st.close()
        if rep:  # the first pass warms up
            app_ms.append((t1 - t0) * 1e3)
            q_ms.append((t2 - t1) * 1e3)
    pairs = sum(ordered_pairs(w.n, m) for m in range(w.minL, w.maxL + 1))
    a = min(app_ms)
    rate = pairs * OPS_PER_EVAL / (a * 1e-3) / 1e12
    return {
        "workload": w.name,
        "appends": [b - a_ for a_, b in zip(cuts[:-1], cuts[1:])],
        "append_ms_total": a,
        "query_ms": min(q_ms),
        "lengths_per_s_query": L / (min(q_ms) * 1e-3),
        "pairs_added": pairs,
        "pairs_per_s": pairs / (a * 1e-3),
        "Tlane_ops_per_s": rate,
        "frac_of_valu_peak": rate / VALU_PEAK_TOPS,
        "top_k_as_oracle": None,
        "_out": out,
    }


def kernel_build_flags() -> list:
    """The hipcc flags the library's kernels are built with."""
    import __graft_entry__ as ge

    return [f for f in ge.HIP_FLAGS if f not in ("-shared", "-I", os.path.join(ROOT, "include"))] + \
        list(ge.SOURCES["kernels.hip"])


def measured_traffic(kernel: str, workload: str, options: dict):
    """HBM bytes per launch of `kernel` from the stored hardware-counter
    summary under profiles/, if it was taken on this exact kernel source,
    build flags, workload and tile geometry (None otherwise)."""
    import glob
    import hashlib

    src = os.path.join(ROOT, "paper_2304_01660_amd", "csrc", "kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    flags = kernel_build_flags()
    for path in glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json")):
        rec = json.load(open(path))
        if (rec.get("kernel") == kernel and rec.get("workload") == workload
                and rec.get("tile_options") == options and rec.get("kernels_hip_sha256") == sha
                and rec.get("build_flags") == flags):
            return rec["bytes_per_launch"], os.path.relpath(path, ROOT)
    return None, None


def grad_leg(api, torch, dev, synth, tuning, reps: int = 3):
    """Forward + backward on the 200k random walk (m 96..160, top-5): the
    search, then the gradient of sum_q w_q nnDist_q with respect to the
    series (w ~ N(0, 1), seed 5) through the adjoint kernels, each timed
    with events on the caller's stream (the library orders its own stream
    inside the call)."""
    import numpy as np

    w = synth.config5()
    L = w.maxL - w.minL + 1
    T = torch.from_numpy(w.T).to(dev)
    opts = tuning.options_for(w.n, w.minL, w.maxL)
    wts = torch.from_numpy(np.random.default_rng(5).standard_normal(L * w.k)).to(dev)
    out = api.discords(T, w.minL, w.maxL, w.k, **opts)
    api.discords_backward(T, out["idx"], out["len"], wts, maxm=w.maxL)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    fwd = bwd = 0.0
    for _ in range(reps):
        ev[0].record(st)
        out = api.discords(T, w.minL, w.maxL, w.k, **opts)
        ev[1].record(st)
        api.discords_backward(T, out["idx"], out["len"], wts, maxm=w.maxL)
        ev[2].record(st)
        torch.cuda.synchronize()
        fwd += ev[0].elapsed_time(ev[1])
        bwd += ev[1].elapsed_time(ev[2])
    fwd /= reps
    bwd /= reps
    lens = out["len"].cpu().numpy().astype(np.int64)
    # the adjoint recomputes every reported row against every column: one
    # FP64 fused multiply-add per window element and pair (the centred dot
    # product), the column's own statistics besides
    flops = float(sum(2.0 * m * (w.n - m + 1) for m in lens))
    return {
        "workload": w.name,
        "forward_ms": fwd,
        "backward_ms": bwd,
        "lengths_per_s_fwd_bwd": L / ((fwd + bwd) * 1e-3),
        "rows": int(lens.shape[0]),
        "backward_pair_flops": flops,
        "backward_TFLOPs": flops / (bwd * 1e-3) / 1e12,
        "backward_frac_fp64_peak": flops / (bwd * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=("c2", "c3", "c5"),
                    help="headline workload (default: the million-point ECG-like series)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0,
                    help="seconds of oracle work in the CPU baseline sample")
    ap.add_argument("--no-legs", action="store_true", help="headline workload only")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--no-heatmap", action="store_true",
                    help="skip the discord heatmap / interest leg")
    ap.add_argument("--no-dense", action="store_true",
                    help="skip the dense matrix-profile leg")
    ap.add_argument("--no-stream", action="store_true",
                    help="skip the streaming-series leg")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run one plain device-to-device copy of MIB MiB (a known-size "
                         "reference for hardware traffic counters) and exit")
    ap.add_argument("--retune", action="store_true",
                    help="run the autotuner now instead of using the stored tile options")
    ap.add_argument("--batch-reps", type=int, default=2)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the library has no "
              "multi-GPU path (sharding across GPUs is described, not implemented)",
              file=sys.stderr)
        return 2

    import torch

    from paper_2304_01660_amd import api, synth, tuning

    dev = torch.device("cuda:0")
    if args.copy_probe:
        a = torch.ones(args.copy_probe * 2**20 // 8, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel() * 8}), flush=True)
        return 0
    w = workload(synth, args.workload)
    L = w.maxL - w.minL + 1
    golden = golden_of(args.workload, w)
    # tile geometry chosen by the autotuner (stored, or tuned now, untimed)
    tuned, tune_report = tuning.options_for(w.n, w.minL, w.maxL), "stored"
    if args.retune:
        probe, treps = tuning.PROBES["single"]
        tuned, tune_report = api.autotune(torch.from_numpy(w.T).to(dev), w.minL, w.maxL, w.k,
                                          probe_lengths=probe, reps=treps)
    head = search_leg(api, torch, dev, w, tuned, args.steps, args.warmup)
    parity = check_golden(head["out"], golden)
    dk = head["kernels"][head["dominant"]]
    achieved = head["achieved"]
    traffic, traffic_src = measured_traffic(KERNEL_NAMES[head["dominant"]], w.name, tuned)
    roofline = {
        "bound": "alu",
        "achieved": achieved,
        "peak": VALU_PEAK_TOPS,
        "unit": "Top/s",
        "frac": (achieved / VALU_PEAK_TOPS) if achieved else None,
        "traffic": traffic,
        "traffic_unit": "bytes per launch (HBM, counter-measured)",
        "traffic_source": traffic_src,
        "kernel": KERNEL_NAMES[head["dominant"]],
        "ops_per_eval": OPS_PER_EVAL,
        "avg_launch_us": dk["avg_launch_us"],
        "evals_per_launch": (dk["evals_per_step"] / dk["launches_per_step"]
                             if dk["launches_per_step"] else None),
        "frac_of_fp32_peak": (achieved * 2 / 157.3) if achieved else None,
    }
    legs = {}
    if not args.no_legs:
        if args.workload != "c2":
            w2 = synth.config2()
            leg = search_leg(api, torch, dev, w2, tuning.options_for(w2.n, w2.minL, w2.maxL),
                             max(5, args.steps), 1)
            d2 = leg["kernels"][leg["dominant"]]
            legs["rw100k"] = {
                "workload": w2.name,
                "lengths_per_s": leg["lengths_per_s"],
                "ms_per_step": leg["ms_per_step"],
                "evals_per_s": leg["evals_per_s"],
                "parity_vs_oracle": check_golden(leg["out"], golden_of("c2", w2)),
                "dominant_kernel": KERNEL_NAMES[leg["dominant"]],
                "dominant_avg_launch_us": d2["avg_launch_us"],
                "dominant_frac_valu": (leg["achieved"] / VALU_PEAK_TOPS) if leg["achieved"] else None,
                "length_kernel_hbm_frac": leg["length_kernel_hbm"]["frac"],
                "kernels": leg["kernels"],
            }
            plain2 = leg
        else:
            w2, plain2 = w, head
        if not args.no_batched:
            legs["batched"] = batched_vs_plain(api, synth, tuning, torch, dev, args.batch_reps,
                                               args.retune)
        if not args.no_grad:
            legs["fwd_bwd"] = grad_leg(api, torch, dev, synth, tuning)
        opts2 = tuning.options_for(w2.n, w2.minL, w2.maxL)
        if not args.no_heatmap:
            legs["heatmap"] = heatmap_leg(api, torch, dev, w2, plain2["T"], opts2,
                                          plain2["ms_per_step"], plain2["out"])
        if not args.no_dense:
            legs["dense_matrix_profile"] = dense_leg(api, torch, w2, plain2["T"], opts2,
                                                     plain2["ms_per_step"])
        if not args.no_stream:
            sl = stream_leg(api, torch, dev, w2, [0, 41_000, 70_500, w2.n])
            out = sl.pop("_out")
            out["count"] = torch.full((w2.maxL - w2.minL + 1,), w2.k, dtype=torch.int32)
            sl["top_k_as_oracle"] = check_golden(out, golden_of("c2", w2))
            legs["stream"] = sl
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, golden, args.cpu_budget)

    line = {
        "metric": METRIC,
        "value": head["lengths_per_s"],
        "unit": "lengths/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "n": w.n, "minL": w.minL, "maxL": w.maxL, "k": w.k, "lengths": L,
            "series": SERIES_TEXT[args.workload],
            "tile_options": tuned or "defaults",
        },
        "tune_report": tune_report,
        "evals_per_s": head["evals_per_s"],
        "range_searches_per_step": head["range_searches_per_step"],
        "ms_per_step_instrumented": head["ms_per_step_instrumented"],
        "kernels": head["kernels"],
        "length_kernel_hbm": head["length_kernel_hbm"],
        "parity_vs_oracle": parity,
        "roofline": roofline,
        "legs": legs,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
