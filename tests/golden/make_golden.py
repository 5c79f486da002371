"""Write the stored expected results under tests/golden/ (calls only oracle/).

Each golden file is JSON: the workload name and parameters, the SHA-256 of
the float64 input series (regenerated from the seeded generator, never
stored), and the oracle's MERLIN output.  The values come from the CPU
oracle in ``oracle/merlin.c`` and nothing else.

Usage:  python tests/golden/make_golden.py c1 [c2 ...]
"""

from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2304_01660_amd import synth  # noqa: E402

CONFIGS = {
    "c1": synth.config1,
    "c2": synth.config2,
    "c5": synth.config5,
}


def write(tag: str) -> str:
    w = CONFIGS[tag]()
    t0 = time.time()
    o = oracle.merlin(w.T, w.minL, w.maxL, w.k)
    dt = time.time() - t0
    rec = {
        "workload": w.name,
        "source": "oracle/merlin.c oracle_merlin (serial FP64 MERLIN + DRAG)",
        "n": w.n, "minL": w.minL, "maxL": w.maxL, "k": w.k,
        "sha256": synth.sha256(w.T),
        "idx": [int(v) for v in o["idx"]],
        "len": [int(v) for v in o["len"]],
        "nn": [float(v) for v in o["nn"]],
        "nnidx": [int(v) for v in o["nnidx"]],
        "calls": [int(v) for v in o["calls"]],
        "r": [float(v) for v in o["r"]],
        "evals": int(o["evals"]),
        "oracle_seconds": dt,
    }
    path = os.path.join(HERE, f"{tag}_{w.name}.json")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    return path


if __name__ == "__main__":
    for tag in sys.argv[1:]:
        print(write(tag), flush=True)
