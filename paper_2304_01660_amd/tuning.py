"""Stored tile geometry, chosen by the autotuner, keyed by problem size.

The sweeps' tile geometry (row-tile heights, first-pass width, chunk
length, queued-pass grid, and whether the diagonal band pre-pass runs)
changes only the order of floating-point work,
never the result beyond the documented tolerance, but it decides how well
a problem fills the GPU.  The stored table (``tuned_gfx950.json``, beside
this module) holds one entry per bucket of series length n and window
length m; each entry was chosen by :func:`api.autotune` on an MI355X for a
representative synthetic series of that bucket.  :func:`options_for` returns
the entry of the bucket holding (n, m) -- or, when no bucket holds it, of
the nearest bucket in (log n, log m) -- so every input gets tuned geometry.
:func:`batch_options` returns the entry tuned on the 64-series batch.

``python -m paper_2304_01660_amd.tuning [OUT] [--only 0,5,batch]`` re-runs
the autotuner for every bucket (or the listed ones) on the current GPU and
writes the table.
"""

from __future__ import annotations

import json
import math
import os
import sys

TUNED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_gfx950.json")

# (probe lengths, timed runs per configuration).  The probe is the whole
# length range: a probe of a series' first lengths is dominated by the first
# length's range-halving searches and chose worse geometry than full runs.
PROBES = {"single": (4096, 2), "batch": (4096, 1)}

BATCH_NAME = "batch64_rw+ecg_n1e4-2e5_m(50..100)+50_k1_fp32"

# Buckets: [n_lo, n_hi) x [m_lo, m_hi) of series length n and mid window
# length m, each with the representative workload the autotuner runs for it
# (a generator of synth, or a seeded random walk of n points over the
# lengths lo..hi with top-k); its (n, m) is the bucket's centre.
BUCKETS = [
    {"n": [0, 60_000], "m": [3, 96], "probe": ("rw", 30_000, 48, 80, 3)},
    {"n": [0, 60_000], "m": [96, 3001], "probe": ("rw", 40_000, 128, 192, 3)},
    {"n": [60_000, 400_000], "m": [3, 112], "probe": ("config2", 100_000, 64, 128, 3)},
    {"n": [60_000, 400_000], "m": [112, 3001], "probe": ("config5", 200_000, 96, 160, 5)},
    {"n": [400_000, 2**31], "m": [3, 160], "probe": ("rw", 1_000_000, 64, 128, 3)},
    {"n": [400_000, 2**31], "m": [160, 3001], "probe": ("config3", 1_000_000, 128, 256, 3)},
]


def _table() -> dict:
    if not os.path.exists(TUNED):
        return {}
    with open(TUNED) as f:
        return json.load(f)


def bucket_of(n: int, m: int, buckets) -> int:
    """Index of the bucket holding (n, m) among those with stored options,
    else of the one whose centre is nearest in (log n, log m); -1 if none
    has options."""
    live = [q for q, b in enumerate(buckets) if b.get("options")]
    for q in live:
        b = buckets[q]
        if b["n"][0] <= n < b["n"][1] and b["m"][0] <= m < b["m"][1]:
            return q
    best, bq = None, -1
    for q in live:
        cn, cm = buckets[q]["centre"]
        d = math.log(n / cn) ** 2 + math.log(m / cm) ** 2
        if best is None or d < best:
            best, bq = d, q
    return bq


def options_for(n: int, minL: int, maxL: int) -> dict:
    """Stored options for a series of length n searched over [minL, maxL]
    ({} -- the library defaults -- when no table is stored)."""
    tab = _table().get("buckets")
    if not tab:
        return {}
    q = bucket_of(int(n), (int(minL) + int(maxL)) // 2, tab)
    return dict(tab[q]["options"]) if q >= 0 else {}


def batch_options() -> dict:
    """Stored options of the 64-series batch."""
    return dict(_table().get("batch", {}).get("options", {}))


def _probe_series(probe):
    from . import synth

    kind, n, lo, hi, k = probe
    if kind.startswith("config"):
        w = getattr(synth, kind)()
        return w.name, w.T, w.minL, w.maxL, w.k
    import numpy as np

    T = synth.fp32_canonical(synth.random_walk(np.random.default_rng(n), n))
    return f"rw{n}_m{lo}-{hi}_k{k}", T, lo, hi, k


def tune_all(out_path: str, only=None) -> dict:
    """Tune every bucket (or the bucket indices in ``only``, keeping the
    stored entries of the others) and the batch, and write the table."""
    import torch

    from . import api, synth

    dev = torch.device("cuda:0")
    old = _table()
    rec = {"buckets": []}
    probe, reps = PROBES["single"]
    for q, b in enumerate(BUCKETS):
        if only is not None and q not in only:
            prev = old.get("buckets", [])
            rec["buckets"].append(prev[q] if q < len(prev) else {"n": b["n"], "m": b["m"]})
            continue
        name, T, lo, hi, k = _probe_series(b["probe"])
        opts, rep = api.autotune(torch.from_numpy(T).to(dev), lo, hi, k, probe_lengths=probe,
                                 reps=reps)
        rec["buckets"].append({"n": b["n"], "m": b["m"], "centre": [int(T.shape[0]), (lo + hi) // 2],
                               "tuned_on": name, "options": opts, "report": rep})
        print(name, opts, rep, flush=True)
    if only is None or "batch" in only:
        ws = synth.config4()
        probe, reps = PROBES["batch"]
        opts, rep = api.autotune([torch.from_numpy(x.T).to(dev) for x in ws],
                                 [x.minL for x in ws], [x.maxL for x in ws], 1,
                                 probe_lengths=probe, reps=reps)
        rec["batch"] = {"tuned_on": BATCH_NAME, "options": opts, "report": rep}
        print(BATCH_NAME, opts, rep, flush=True)
    else:
        rec["batch"] = old.get("batch", {})
    with open(out_path, "w") as f:
        json.dump(rec, f, indent=1)
    return rec


if __name__ == "__main__":
    # python -m paper_2304_01660_amd.tuning [OUT] [--only 0,5,batch]
    argv = sys.argv[1:]
    only = None
    if "--only" in argv:
        i = argv.index("--only")
        only = [x if x == "batch" else int(x) for x in argv[i + 1].split(",")]
        del argv[i:i + 2]
    tune_all(argv[0] if argv else TUNED, only)
