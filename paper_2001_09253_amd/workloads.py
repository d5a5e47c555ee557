"""Seeded synthetic workloads for the spline hot path.

This module only draws numbers: knots, values, end derivatives, instance sizes
and arrival times.  It holds none of the spline arithmetic (no rows, no solve,
no query positions, no evaluation), so both the FP64 oracle under ``oracle/``
and the HIP path may be fed from it without sharing any of the method.

Distributions follow the paper's benchmark generator (section "Curve
Interpolation", step 5 of the methodology list): every new knot is the previous
one plus an increment drawn from U(0,1), with a zero increment replaced by
1e-4, and every value is a fresh U(0,1) draw.  An increment that does not move
the knot in floating point (below half a unit in the last place of a large
knot: at 2^28 knots, draws below about 1e-8) counts as zero, so that the
knots stay strictly increasing.  The paper does not state the
first knot; it is 0 here, as in its own test curves.  The increment and the
value are two independent draws.  Random numbers come from NumPy's PCG64
(``numpy.random.default_rng``).

End conditions cycle through the three cases of the "Quality Checks" section:
natural (derivative sentinel 1e32, i.e. above 0.99e30), flat (0, 0) and twist
(-1, 1).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

NATURAL = 1e32          # any value above 0.99e30 selects a natural end
BC_CASES = (
    ("natural", NATURAL, NATURAL),
    ("flat", 0.0, 0.0),
    ("twist", -1.0, 1.0),
)

# The hand-made 13-knot curve of the "Quality Checks" section.
HAND_KNOTS = np.array([0, 0.5, 1, 1.01, 1.25, 1.5, 1.58, 1.79, 2.12, 2.30,
                       2.402, 2.451, 2.5], dtype=np.float64)
HAND_VALUES = np.array([1, 1.2, 2, 0.25, 0.25, 0.25, 0.63, 0.96, 1.17, 1.23,
                        1.245, 1.249, 1.25], dtype=np.float64)

# Sizes of the worked example: 13 knots, 2048 uniform display points.
BASE_N = 13
BASE_M = 2048


def paper_curve(rng: np.random.Generator, n: int, x0: float = 0.0):
    """Knots and values of one random curve drawn the paper's way."""
    if n < 0:
        raise ValueError("n must be non-negative")
    inc = rng.random(n)
    val = rng.random(n)
    inc[inc == 0.0] = 1e-4
    x = np.empty(n, dtype=np.float64)
    if n:
        inc[0] = x0
        # add.accumulate sums strictly left to right, so every knot is exactly
        # the previous knot plus its own increment
        np.add.accumulate(inc, out=x)
        while True:
            stuck = np.nonzero(x[1:] <= x[:-1])[0] + 1
            if stuck.size == 0:
                break
            inc[stuck] = 1e-4
            np.add.accumulate(inc, out=x)
    return x, val.astype(np.float64)


def alternating_curve(rng: np.random.Generator, n: int, small: float = 1e-3, scale: float = 1.0):
    """Knots whose widths alternate 1, small, 1, small, ... from x_0 = 0 and
    standard-normal values times scale: a stress shape for the halo of the
    block solves (the widths alone set how fast a dropped coupling decays)."""
    widths = np.where(np.arange(n - 1) % 2 == 0, 1.0, small)
    x = np.concatenate([[0.0], np.cumsum(widths)])
    y = rng.standard_normal(n) * scale
    return x, y


def spacing_curve(rng: np.random.Generator, n: int, kind: str):
    """Knots with adversarial spacing and standard-normal values, x_0 = 0:
      "sawtooth_down": runs of widths 1, 0.1, ..., 1e-7 (each much narrower
          than the one before it);
      "sawtooth_up":   runs of widths 1e-7, ..., 0.1, 1;
      "loguniform":    widths log-uniform over 12 orders of magnitude;
      "clustered":     U(0,1) widths with every 97th width shrunk by 1e-6."""
    k = np.arange(n - 1)
    if kind == "sawtooth_down":
        w = 10.0 ** (-(k % 8).astype(np.float64))
    elif kind == "sawtooth_up":
        w = 10.0 ** ((k % 8).astype(np.float64) - 7.0)
    elif kind == "loguniform":
        w = 10.0 ** rng.uniform(-12.0, 0.0, n - 1)
    elif kind == "clustered":
        w = rng.random(n - 1)
        w[::97] *= 1e-6
        w[w == 0] = 1.0
    else:
        raise ValueError(kind)
    x = np.concatenate([[0.0], np.cumsum(w)])
    return x, rng.standard_normal(n)


def bc_for(i: int):
    """(name, start_deriv, end_deriv) of the i-th instance in the cycle."""
    return BC_CASES[i % len(BC_CASES)]


@dataclass
class Instance:
    x: np.ndarray
    y: np.ndarray
    start_deriv: float
    end_deriv: float
    m: int

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def single(seed: int, n: int, m: int, bc: int = 0) -> Instance:
    """One seeded curve with n knots and m uniform queries; bc indexes BC_CASES."""
    rng = np.random.default_rng(seed)
    x, y = paper_curve(rng, n)
    _, sd, ed = BC_CASES[bc % len(BC_CASES)]
    return Instance(x, y, sd, ed, int(m))


def config_small(seed: int = 0, bc: int = 0) -> Instance:
    """Smallest worked size of the paper: 13 knots, 2048 uniform points."""
    return single(seed, BASE_N, BASE_M, bc)


def config_large(seed: int = 0, bc: int = 0) -> Instance:
    """The worked size scaled 1000x: 13,000 knots, 2,048,000 uniform points."""
    return single(seed, BASE_N * 1000, BASE_M * 1000, bc)


def log_uniform_sizes(rng: np.random.Generator, count: int, lo: float, hi: float,
                      base_n: int = BASE_N, base_m: int = BASE_M):
    """Instance sizes scaled by s ~ logU(lo, hi) from the worked size."""
    s = np.exp(rng.uniform(np.log(lo), np.log(hi), size=count))
    n = np.maximum(3, np.rint(base_n * s)).astype(np.int64)
    m = np.maximum(2, np.rint(base_m * s)).astype(np.int64)
    return n, m


@dataclass
class Batch:
    """Many curves in CSR form: instance i owns knots koff[i]:koff[i+1] and
    queries qoff[i]:qoff[i+1]."""
    koff: np.ndarray      # int64[count+1]
    qoff: np.ndarray      # int64[count+1]
    x: np.ndarray         # float64[sum n]
    y: np.ndarray         # float64[sum n]
    sd: np.ndarray        # float64[count]
    ed: np.ndarray        # float64[count]

    @property
    def count(self) -> int:
        return int(self.koff.shape[0] - 1)

    @property
    def n(self) -> np.ndarray:
        return np.diff(self.koff)

    @property
    def m(self) -> np.ndarray:
        return np.diff(self.qoff)

    def instance(self, i: int) -> Instance:
        a, b = int(self.koff[i]), int(self.koff[i + 1])
        return Instance(self.x[a:b], self.y[a:b], float(self.sd[i]), float(self.ed[i]),
                        int(self.qoff[i + 1] - self.qoff[i]))


def batch_from_sizes(seed: int, n: np.ndarray, m: np.ndarray) -> Batch:
    rng = np.random.default_rng(seed)
    count = int(len(n))
    koff = np.zeros(count + 1, dtype=np.int64)
    qoff = np.zeros(count + 1, dtype=np.int64)
    koff[1:] = np.cumsum(n)
    qoff[1:] = np.cumsum(m)
    x = np.empty(int(koff[-1]), dtype=np.float64)
    y = np.empty(int(koff[-1]), dtype=np.float64)
    sd = np.empty(count, dtype=np.float64)
    ed = np.empty(count, dtype=np.float64)
    for i in range(count):
        xi, yi = paper_curve(rng, int(n[i]))
        x[koff[i]:koff[i + 1]] = xi
        y[koff[i]:koff[i + 1]] = yi
        _, sd[i], ed[i] = bc_for(i)
    return Batch(koff, qoff, x, y, sd, ed)


def batch(seed: int = 0, count: int = 4096, lo: float = 0.1, hi: float = 10.0) -> Batch:
    """The batched workload: sizes log-uniform between lo and hi times the
    worked size (4096 instances, 0.1x..10x by default)."""
    rng = np.random.default_rng(seed)
    n, m = log_uniform_sizes(rng, count, lo, hi)
    return batch_from_sizes(seed + 1, n, m)


@dataclass
class Trace:
    """Open-loop arrival trace: request r arrives at t[r] seconds."""
    t: np.ndarray
    n: np.ndarray
    m: np.ndarray


def poisson_trace(seed: int, rate: float, duration: float, lo: float = 0.1,
                  hi: float = 100.0) -> Trace:
    """Poisson arrivals (exponential gaps of mean 1/rate) over `duration`
    seconds, sizes log-uniform between lo and hi times the worked size."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=int(rate * duration * 1.5) + 16)
    t = np.cumsum(gaps)
    t = t[t < duration]
    n, m = log_uniform_sizes(rng, len(t), lo, hi)
    return Trace(t, n, m)


def sweep_sizes(seed: int, count: int, nmax: int = 1 << 20, nmin: int = 4) -> np.ndarray:
    """The paper's benchmark size list: r on a uniform grid in [0,1] mapped
    through (r(sqrt(nmax)-sqrt(nmin)) + sqrt(nmin))^2, then shuffled."""
    r = np.linspace(0.0, 1.0, count)
    sizes = np.rint((r * (np.sqrt(nmax) - np.sqrt(nmin)) + np.sqrt(nmin)) ** 2).astype(np.int64)
    rng = np.random.default_rng(seed)
    rng.shuffle(sizes)
    return sizes
