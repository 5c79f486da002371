"""Seeded synthetic time series shaped like the paper's workloads.

The paper evaluates on a random-walk model and on real electrocardiograms
(Sec. 4.1, Tab. 1).  The real recordings are not available, so these
generators produce stand-ins: Gaussian random walks and quasi-periodic
ECG-like beat trains, each with injected subsequence anomalies.

This module is shared by the tests, the benchmark and the oracle's golden
script.  It holds only input generation: no z-normalisation, no distances and
no part of the discord search itself.

Every generator works in float64 with ``numpy.random.default_rng(seed)``.
Series that feed an FP32 pipeline are canonicalised as
``float64(float32(T))`` so that the oracle and the GPU see identical values.
"""

from __future__ import annotations

import dataclasses
import hashlib
import math

import numpy as np

__all__ = [
    "Workload",
    "random_walk",
    "ecg_like",
    "config1",
    "config2",
    "config3",
    "config4",
    "config5",
    "small_random",
    "fp32_canonical",
    "sha256",
]


@dataclasses.dataclass
class Workload:
    """One discord-search problem: a series plus its length range and k."""

    name: str
    T: np.ndarray            # float64 [n]
    minL: int
    maxL: int
    k: int
    dist_bits: int           # 64 = FP64 distances end to end, 32 = FP32 sweep
    anomalies: list          # list of dicts: position, length, kind
    seed: int

    @property
    def n(self) -> int:
        return int(self.T.shape[0])


def fp32_canonical(T: np.ndarray) -> np.ndarray:
    """Round a float64 series through float32 and back."""
    return np.asarray(T, dtype=np.float64).astype(np.float32).astype(np.float64)


def sha256(T: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(T, dtype=np.float64).tobytes()).hexdigest()


def _local_std(base: np.ndarray, p: int, L: int) -> float:
    """Population std of the pre-injection series over [p - L, p + 2L)."""
    lo = max(0, p - L)
    hi = min(base.shape[0], p + 2 * L)
    return float(np.std(base[lo:hi]))


def _place(rng, n: int, lengths, maxL: int):
    """Sequentially place intervals of the given lengths by rejection.

    Each interval [p, p+L) keeps at least maxL samples from both ends of the
    series and at least 2*maxL samples from every interval placed before it.
    """
    placed = []
    for L in lengths:
        for _ in range(100000):
            lo = maxL
            hi = n - maxL - L
            if hi <= lo:
                raise ValueError("series too short for the requested anomalies")
            p = int(rng.integers(lo, hi + 1))
            ok = True
            for (q, Lq) in placed:
                gap = max(q - (p + L), p - (q + Lq))
                if gap < 2 * maxL:
                    ok = False
                    break
            if ok:
                placed.append((p, L))
                break
        else:
            raise ValueError("could not place anomalies; series too short")
    return placed


def random_walk(rng, n: int) -> np.ndarray:
    """Cumulative sum of N(0, 1) steps (the random-walk model of Sec. 4.1)."""
    return np.cumsum(rng.standard_normal(n))


def inject_bursts(rng, base: np.ndarray, count: int, maxL: int,
                  len_range=(50, 150), amp_range=(2.0, 4.0),
                  kinds=("sine", "shift"), fixed_len=None, fixed_amp=None,
                  sine_period=None):
    """Inject sine bursts or level shifts into a copy of ``base``.

    Lengths are uniform integers in ``len_range`` (or ``fixed_len``), the
    amplitude is ``a * local_std`` with ``a`` uniform in ``amp_range`` (or
    ``fixed_amp``).  A sine burst spans two full cycles over its length unless
    ``sine_period`` is given; a level shift adds a constant of random sign.
    """
    T = base.copy()
    lengths = []
    for _ in range(count):
        lengths.append(int(fixed_len) if fixed_len is not None
                       else int(rng.integers(len_range[0], len_range[1] + 1)))
    spots = _place(rng, base.shape[0], lengths, maxL)
    meta = []
    for (p, L) in spots:
        kind = kinds[0] if len(kinds) == 1 else (kinds[int(rng.integers(0, len(kinds)))])
        a = float(fixed_amp) if fixed_amp is not None else float(rng.uniform(*amp_range))
        s_loc = _local_std(base, p, L)
        u = np.arange(L, dtype=np.float64)
        if kind == "sine":
            period = float(sine_period) if sine_period is not None else L / 2.0
            T[p:p + L] += a * s_loc * np.sin(2.0 * math.pi * u / period)
        else:
            sign = 1.0 if rng.uniform() < 0.5 else -1.0
            T[p:p + L] += sign * a * s_loc
        meta.append({"position": int(p), "length": int(L), "kind": kind, "amp": a})
    return T, meta


# Gaussian bump parameters of one synthetic heartbeat: (amplitude, centre
# offset from the beat onset, width), all in samples.
_BUMPS = ((0.15, 50.0, 8.0), (1.0, 100.0, 4.0), (0.35, 175.0, 12.0))


def ecg_like(rng, n: int, malformed: int, maxL: int, period=(240.0, 260.0),
             noise_std=0.05):
    """Quasi-periodic ECG-like series with malformed beats.

    Beat onsets advance by a period drawn uniformly from ``period``; a beat is
    the sum of three Gaussian bumps.  ``malformed`` beats, at least four beats
    apart and at least ``maxL`` samples from either end, either lose one bump
    or have one bump widened twofold.  N(0, noise_std^2) noise is added last.
    """
    onsets = []
    b = 0.0
    while b < n:
        onsets.append(b)
        b += float(rng.uniform(period[0], period[1]))
    nb = len(onsets)
    eligible = [q for q in range(nb)
                if onsets[q] >= maxL and onsets[q] + period[1] <= n - maxL]
    chosen = []
    tries = 0
    while len(chosen) < malformed:
        tries += 1
        if tries > 1000000:
            raise ValueError("could not place malformed beats")
        q = eligible[int(rng.integers(0, len(eligible)))]
        if all(abs(q - c) >= 4 for c in chosen):
            chosen.append(q)
    chosen.sort()
    defects = {}
    meta = []
    for q in chosen:
        bump = int(rng.integers(0, 3))
        kind = "drop" if rng.uniform() < 0.5 else "widen"
        defects[q] = (bump, kind)
        meta.append({"position": int(onsets[q]), "length": int(period[1]),
                     "kind": f"{kind}{bump}"})
    T = np.zeros(n, dtype=np.float64)
    t = np.arange(n, dtype=np.float64)
    for q, b0 in enumerate(onsets):
        for bi, (A, c, w) in enumerate(_BUMPS):
            if q in defects and defects[q][0] == bi:
                if defects[q][1] == "drop":
                    continue
                w = 2.0 * w
            centre = b0 + c
            lo = max(0, int(math.floor(centre - 8.0 * w)))
            hi = min(n, int(math.ceil(centre + 8.0 * w)) + 1)
            if hi <= lo:
                continue
            x = t[lo:hi] - centre
            T[lo:hi] += A * np.exp(-(x * x) / (2.0 * w * w))
    T += noise_std * rng.standard_normal(n)
    return T, meta


def config1() -> Workload:
    """Random walk n=2,000 with two 40-point sine bursts; m in [32, 40], top-1, FP64."""
    rng = np.random.default_rng(0)
    base = random_walk(rng, 2000)
    T, meta = inject_bursts(rng, base, 2, maxL=40, fixed_len=40, fixed_amp=3.0,
                            kinds=("sine",), sine_period=20.0)
    return Workload("rw2k_m32-40_k1_fp64", T, 32, 40, 1, 64, meta, 0)


def config2() -> Workload:
    """Random walk n=100,000 with five bursts or shifts; m in [64, 128], top-3, FP32."""
    rng = np.random.default_rng(1)
    base = random_walk(rng, 100_000)
    T, meta = inject_bursts(rng, base, 5, maxL=128)
    return Workload("rw100k_m64-128_k3_fp32", fp32_canonical(T), 64, 128, 3, 32, meta, 1)


def config3() -> Workload:
    """ECG-like n=1,000,000 with 20 malformed beats; m in [128, 256], top-3, FP32."""
    rng = np.random.default_rng(2)
    T, meta = ecg_like(rng, 1_000_000, 20, maxL=256)
    return Workload("ecg1m_m128-256_k3_fp32", fp32_canonical(T), 128, 256, 3, 32, meta, 2)


def config4(count: int = 64):
    """Batch of uneven series: lengths log-uniform in [1e4, 2e5].

    The first half are random walks with 1-5 bursts or shifts, the second
    half ECG-like with 1-5 malformed beats.  Each series has its own
    minL uniform in [50, 100] and maxL = minL + 50; top-1; FP32.
    """
    master = np.random.default_rng(3)
    out = []
    for s in range(count):
        n_s = int(round(math.exp(master.uniform(math.log(1e4), math.log(2e5)))))
        minL = int(master.integers(50, 101))
        maxL = minL + 50
        rng = np.random.default_rng(3000 + s)
        cnt = int(rng.integers(1, 6))
        if s < count // 2:
            base = random_walk(rng, n_s)
            T, meta = inject_bursts(rng, base, cnt, maxL=maxL)
            kind = "rw"
        else:
            T, meta = ecg_like(rng, n_s, cnt, maxL=maxL)
            kind = "ecg"
        out.append(Workload(f"batch{s}_{kind}{n_s}_m{minL}-{maxL}", fp32_canonical(T),
                            minL, maxL, 1, 32, meta, 3000 + s))
    return out


def config5() -> Workload:
    """Random walk n=200,000 with ten sine bursts; m in [96, 160], top-5, FP32 forward."""
    rng = np.random.default_rng(4)
    base = random_walk(rng, 200_000)
    T, meta = inject_bursts(rng, base, 10, maxL=160, kinds=("sine",))
    return Workload("rw200k_m96-160_k5_grad", fp32_canonical(T), 96, 160, 5, 32, meta, 4)


def small_random(seed: int, n: int, kind: str = "rw") -> np.ndarray:
    """Tiny seeded series for parity sweeps (random walk, ECG-like or white noise)."""
    rng = np.random.default_rng(seed)
    if kind == "rw":
        return random_walk(rng, n)
    if kind == "noise":
        return rng.standard_normal(n)
    if kind == "ecg":
        T, _ = ecg_like(rng, n, 0, maxL=1)
        return T
    raise ValueError(kind)
