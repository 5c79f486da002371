"""Write the stored expected results under tests/golden/ (calls only oracle/).

Each golden file is JSON: the workload name and parameters, the SHA-256 of
the float64 input series (regenerated from the seeded generator, never
stored), and the oracle's MERLIN output.  The values come from the CPU
oracle in ``oracle/merlin.c`` and nothing else.

Usage:
    python tests/golden/make_golden.py c1 [c2 c3 c5 ...] [--threads T]
    python tests/golden/make_golden.py c4 [--jobs J] [--series 0,5,7]

``--threads T`` runs the OpenMP build of the same oracle source (identical
results, tested against the serial build) on T threads; the million-point
workload needs it to finish in hours rather than days.

``c4`` writes one file per series of the 64-series batch under
``tests/golden/c4/`` (the series are independent problems), J series at a
time in separate processes; series whose file already exists are skipped.
"""

from __future__ import annotations

import json
import multiprocessing
import os
import platform
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
    "c3": synth.config3,
    "c5": synth.config5,
}
C4_DIR = os.path.join(HERE, "c4")


def _host(threads=None):
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu": model or platform.machine(), "threads_used": threads or 1,
            "nproc": os.cpu_count()}


def record(w, threads=None):
    t0 = time.time()
    o = oracle.merlin(w.T, w.minL, w.maxL, w.k, threads=threads)
    dt = time.time() - t0
    return {
        "workload": w.name,
        "source": ("oracle/merlin.c oracle_merlin (FP64 MERLIN + DRAG, "
                   + (f"OpenMP build, {threads} threads)" if threads else "serial)")),
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
        "oracle_host": _host(threads),
    }


def write(tag: str, threads=None) -> str:
    w = CONFIGS[tag]()
    rec = record(w, threads)
    path = os.path.join(HERE, f"{tag}_{w.name}.json")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    return path


def c4_path(s: int, w) -> str:
    return os.path.join(C4_DIR, f"{s:02d}_{w.name}.json")


def _c4_one(s: int) -> str:
    w = synth.config4()[s]
    rec = record(w)
    rec["series_index"] = s
    path = c4_path(s, w)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(rec, f, indent=1)
    os.replace(tmp, path)
    return f"{path} {rec['oracle_seconds']:.1f}s"


def write_c4(jobs: int, series=None):
    os.makedirs(C4_DIR, exist_ok=True)
    ws = synth.config4()
    todo = [s for s in (series if series is not None else range(len(ws)))
            if not os.path.exists(c4_path(s, ws[s]))]
    # largest series first so the pool drains evenly
    todo.sort(key=lambda s: -ws[s].n)
    with multiprocessing.Pool(jobs) as pool:
        for msg in pool.imap_unordered(_c4_one, todo):
            print(msg, flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    jobs, series, threads = 1, None, None
    if "--threads" in args:
        i = args.index("--threads")
        threads = int(args[i + 1])
        del args[i:i + 2]
    if "--jobs" in args:
        i = args.index("--jobs")
        jobs = int(args[i + 1])
        del args[i:i + 2]
    if "--series" in args:
        i = args.index("--series")
        series = [int(x) for x in args[i + 1].split(",")]
        del args[i:i + 2]
    for tag in args:
        if tag == "c4":
            write_c4(jobs, series)
        else:
            print(write(tag, threads), flush=True)
