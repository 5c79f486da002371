"""Stored tile geometry for named workloads, chosen by the autotuner.

The sweeps' tile geometry (row-tile heights, first-pass width, chunk
length, queued-pass grid) changes only the order of floating-point work,
never the result beyond the documented tolerance, but it decides how well
a workload fills the GPU.  ``python -m paper_2304_01660_amd.tuning OUT``
runs :func:`api.autotune` on the benchmark workloads on the current GPU and
writes the chosen options to OUT (JSON); the file committed beside this
module, ``tuned_gfx950.json``, came from that command on an MI355X.
:func:`options` returns the stored options of a workload (an empty dict,
i.e. the library defaults, when none are stored).
"""

from __future__ import annotations

import json
import os
import sys

TUNED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_gfx950.json")

# workload name -> (probe lengths, timed runs per configuration)
PROBES = {"single": (8, 2), "batch": (12, 1)}


def options(name: str) -> dict:
    """Stored options of workload ``name`` ({} when none are stored)."""
    if not os.path.exists(TUNED):
        return {}
    with open(TUNED) as f:
        rec = json.load(f)
    return dict(rec.get(name, {}).get("options", {}))


def tune_all(out_path: str) -> dict:
    import torch

    from . import api, synth

    dev = torch.device("cuda:0")
    rec = {}
    w = synth.config2()
    probe, reps = PROBES["single"]
    opts, rep = api.autotune(torch.from_numpy(w.T).to(dev), w.minL, w.maxL, w.k,
                             probe_lengths=probe, reps=reps)
    rec[w.name] = {"options": opts, "report": rep}
    print(w.name, opts, rep, flush=True)
    ws = synth.config4()
    probe, reps = PROBES["batch"]
    opts, rep = api.autotune([torch.from_numpy(x.T).to(dev) for x in ws], [x.minL for x in ws],
                             [x.maxL for x in ws], 1, probe_lengths=probe, reps=reps)
    rec[BATCH_NAME] = {"options": opts, "report": rep}
    print(BATCH_NAME, opts, rep, flush=True)
    with open(out_path, "w") as f:
        json.dump(rec, f, indent=1)
    return rec


BATCH_NAME = "batch64_rw+ecg_n1e4-2e5_m(50..100)+50_k1_fp32"

if __name__ == "__main__":
    tune_all(sys.argv[1] if len(sys.argv) > 1 else TUNED)
