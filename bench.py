"""Benchmark: top-k range discords over a length range on one MI355X.

Workload (one "step" = one full search, every length, through the C ABI):
a seeded random walk of n = 100,000 points (FP32-canonical values) with five
injected sine bursts or level shifts; lengths m = 64..128 (65 lengths),
top-3 discords per length; FP32 selection sweep, FP64 refinement and exact
FP64 distances.  Inputs are resident in HBM before the timed region.

Prints one JSON line: lengths/s as `value`, plus device-counted distance
evaluations/s, the roofline of the dominant kernel (from HIP events recorded
around its launches during the timed steps) and the CPU oracle on a bounded
sample of the same workload.
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "z-norm distance evals/sec + lengths/sec over [minL,maxL]; batched vs plain"
# VALU issue rate of MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz lane-ops/s
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# Minimal VALU lane-operations per pair evaluation of a sweep step: two FMAs
# for the covariance update, one multiply by 1/(sqrt(m) sigma_j), one compare
# (selection) or max (refinement).
OPS_PER_EVAL = 4
KERNEL_NAMES = {
    "select_near": "k_select_near",
    "select_far": "k_select_far",
    "refine": "k_refine",
    "polish": "k_polish",
}


def cpu_baseline(w, golden, n_lengths: int):
    """Time the oracle's range search at MERLIN's final r for a few lengths."""
    import oracle

    if golden is None:
        return None
    L = w.maxL - w.minL + 1
    picks = [int(round(x)) for x in
             [1 + i * (L - 2) / max(1, n_lengths - 1) for i in range(n_lengths)]]
    t0 = time.perf_counter()
    for li in picks:
        m = w.minL + li
        oracle.drag(w.T, m, golden["r"][li])
    dt = time.perf_counter() - t0
    return {
        "value": len(picks) / dt,
        "unit": "lengths/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"serial FP64 DRAG of the oracle at MERLIN's final r for lengths "
                   f"{[w.minL + li for li in picks]} of the same series ({dt:.1f} s); excludes "
                   f"the first length's r-halving rounds (about 300 s alone for the oracle)"),
        "host_cpu": platform.processor() or platform.machine(),
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
    tuned, report = tuning.options(tuning.BATCH_NAME), "stored"
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


def measured_traffic(kernel: str, workload: str, options: dict):
    """HBM bytes per launch of `kernel` from the stored hardware-counter
    summary under profiles/, if it was taken on this exact kernel source,
    workload and tile geometry (None otherwise)."""
    import glob
    import hashlib

    src = os.path.join(ROOT, "paper_2304_01660_amd", "csrc", "kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for path in glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json")):
        rec = json.load(open(path))
        if (rec.get("kernel") == kernel and rec.get("workload") == workload
                and rec.get("tile_options") == options and rec.get("kernels_hip_sha256") == sha):
            return rec["bytes_per_launch"], os.path.relpath(path, ROOT)
    return None, None


def check_golden(out, golden, T):
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-lengths", type=int, default=12)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run one plain device-to-device copy of MIB MiB (a known-size "
                         "reference for hardware traffic counters) and exit")
    ap.add_argument("--retune", action="store_true",
                    help="run the autotuner now instead of using the stored tile options")
    ap.add_argument("--batch-reps", type=int, default=2)
    ap.add_argument("--no-heatmap", action="store_true",
                    help="skip the discord heatmap / interest leg")
    ap.add_argument("--no-dense", action="store_true",
                    help="skip the dense matrix-profile leg")
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
    w = synth.config2()
    L = w.maxL - w.minL + 1
    gpath = os.path.join(ROOT, "tests", "golden", "c2_rw100k_m64-128_k3_fp32.json")
    golden = json.load(open(gpath)) if os.path.exists(gpath) else None
    T = torch.from_numpy(w.T).to(dev)
    ws = torch.empty(api.workspace_size(w.n, w.minL, w.maxL, w.k), dtype=torch.uint8, device=dev)
    # tile geometry chosen by the autotuner (stored, or tuned now, untimed)
    tuned, tune_report = tuning.options(w.name), "stored"
    if args.retune:
        probe, treps = tuning.PROBES["single"]
        tuned, tune_report = api.autotune(T, w.minL, w.maxL, w.k, probe_lengths=probe, reps=treps)
    for _ in range(args.warmup):
        api.discords(T, w.minL, w.maxL, w.k, workspace=ws, **tuned)
    torch.cuda.synchronize()

    # timed region: the production path (round graphs replayed, no events)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = api.discords(T, w.minL, w.maxL, w.k, workspace=ws, return_stats=True, **tuned)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt / args.steps * 1e3
    st_prod = out["stats"]

    # the same steps again with HIP events around every sweep launch, on the
    # library's stream where the kernels run: per-kernel device time
    agg = None
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
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
    ms_instrumented = (time.perf_counter() - t1) / args.steps * 1e3
    for key in ("idx", "nn_dist", "nn_idx", "count"):
        if not torch.equal(out[key], out_t[key]):
            raise SystemExit("instrumented and production runs disagree")
    parity = check_golden(out, golden, w.T)

    evals = (st_prod["evals_select"] + st_prod["evals_refine"] + st_prod["evals_polish"]) * args.steps
    kernels = {}
    for ci, name in enumerate(("select_near", "select_far", "refine", "polish")):
        launches = agg["kernel_launches"][ci]
        ms = agg["kernel_ms"][ci]
        kernels[name] = {
            "launches_per_step": launches / args.steps,
            "ms_per_step": ms / args.steps,
            "evals_per_step": agg["kernel_evals"][ci] / args.steps,
            "avg_launch_us": (ms / launches * 1e3) if launches else None,
        }
    dom = max(("select_near", "select_far", "refine"), key=lambda k: kernels[k]["ms_per_step"])
    dk = kernels[dom]
    achieved = None
    if dk["ms_per_step"] > 0:
        # evals per launch / average launch duration == evals / summed duration
        achieved = dk["evals_per_step"] * OPS_PER_EVAL / (dk["ms_per_step"] * 1e-3) / 1e12
    traffic, traffic_src = measured_traffic(KERNEL_NAMES[dom], w.name, tuned)
    roofline = {
        "bound": "alu",
        "achieved": achieved,
        "peak": VALU_PEAK_TOPS,
        "unit": "Top/s",
        "frac": (achieved / VALU_PEAK_TOPS) if achieved else None,
        "traffic": traffic,
        "traffic_unit": "bytes per launch (HBM, counter-measured)",
        "traffic_source": traffic_src,
        "kernel": KERNEL_NAMES[dom],
        "ops_per_eval": OPS_PER_EVAL,
        "avg_launch_us": dk["avg_launch_us"],
        "evals_per_launch": (dk["evals_per_step"] / dk["launches_per_step"]
                             if dk["launches_per_step"] else None),
    }
    batched = None
    if not args.no_batched:
        batched = batched_vs_plain(api, synth, tuning, torch, dev, args.batch_reps, args.retune)
    heat = None
    if not args.no_heatmap:
        heat = heatmap_leg(api, torch, dev, w, T, tuned, ms_per_step, out)
    dense = None
    if not args.no_dense:
        dense = dense_leg(api, torch, w, T, tuned, ms_per_step)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, golden, args.cpu_lengths)

    line = {
        "metric": METRIC,
        "value": L / (ms_per_step * 1e-3),
        "unit": "lengths/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "n": w.n, "minL": w.minL, "maxL": w.maxL, "k": w.k, "lengths": L,
            "series": "seeded random walk with 5 injected sine bursts/level shifts (seed 1)",
            "tile_options": tuned or "defaults",
        },
        "tune_report": tune_report,
        "evals_per_s": evals / dt,
        "range_searches_per_step": st_prod["range_searches"],
        "ms_per_step_instrumented": ms_instrumented,
        "kernels": kernels,
        "parity_vs_oracle": parity,
        "roofline": roofline,
        "batched": batched,
        "heatmap": heat,
        "dense_matrix_profile": dense,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
