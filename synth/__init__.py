"""Seeded synthetic workloads for the batched Mallows-distance path.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic (no costs, no transport, no normalisation). Both the
HIP path and the CPU oracle are fed from here, and nothing else is shared
between them.

Objects are discrete distributions ("bags of weighted vectors", Sec. 1.1 and
Sec. 2.2 of the paper): a support of t points in R^d with non-negative weights.
A set of n such objects is stored ragged:

    offsets  int64   [n+1]        offsets[i]..offsets[i+1] index object i
    points   f64|f32 [offsets[n], d] row-major
    weights  f64|f32 [offsets[n]]

The paper's experiments use image, video and protein descriptors that are not
available here; every workload below is synthetic with the sizes, support
ranges and weight laws of the five measured configurations.

Random streams: ``numpy.random.default_rng([13020435, cfg, stream])`` with
stream 0 = mixture means, 1 = data bags, 2 = centroids, 3 = arrivals,
4 = parity samples.  Weights are Dirichlet(alpha * 1_t), drawn as independent
Gamma(alpha, 1) variates divided by their bag's sum (a bag of one atom gets
weight 1 exactly).  Gaussian-mixture points pick a component uniformly per
point and add sigma * N(0, I_d) to its mean; means are U[-box, box]^d.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SEED = 13020435
STREAM_MEANS, STREAM_DATA, STREAM_CENTROIDS, STREAM_ARRIVALS, STREAM_SAMPLE = 0, 1, 2, 3, 4


@dataclasses.dataclass
class RaggedSet:
    offsets: np.ndarray
    points: np.ndarray
    weights: np.ndarray

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def d(self) -> int:
        return int(self.points.shape[1])

    @property
    def sizes(self) -> np.ndarray:
        return np.diff(self.offsets)

    @property
    def max_support(self) -> int:
        return int(self.sizes.max()) if self.n > 0 else 0

    def bag(self, i: int):
        a, b = int(self.offsets[i]), int(self.offsets[i + 1])
        return self.points[a:b], self.weights[a:b]

    def astype(self, dtype) -> "RaggedSet":
        return RaggedSet(self.offsets.copy(), self.points.astype(dtype), self.weights.astype(dtype))

    def subset(self, idx) -> "RaggedSet":
        """Ragged set holding objects ``idx`` (in that order)."""
        idx = np.asarray(idx, dtype=np.int64)
        sizes = self.sizes[idx]
        off = np.zeros(idx.size + 1, dtype=np.int64)
        np.cumsum(sizes, out=off[1:])
        rows = np.concatenate([np.arange(self.offsets[i], self.offsets[i + 1]) for i in idx]) \
            if idx.size else np.zeros(0, dtype=np.int64)
        return RaggedSet(off, self.points[rows], self.weights[rows])


def from_bags(bags, dtype=np.float64) -> RaggedSet:
    """Ragged set from a list of (points[t,d], weights[t]) pairs."""
    sizes = [int(np.asarray(w).shape[0]) for _, w in bags]
    off = np.zeros(len(bags) + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    d = int(np.asarray(bags[0][0]).reshape(sizes[0], -1).shape[1]) if bags else 1
    pts = np.concatenate([np.asarray(p, dtype=dtype).reshape(-1, d) for p, _ in bags]) if bags \
        else np.zeros((0, d), dtype)
    w = np.concatenate([np.asarray(w, dtype=dtype).reshape(-1) for _, w in bags]) if bags \
        else np.zeros(0, dtype)
    return RaggedSet(off, pts, w)


def rng_for(cfg: int, stream: int, *extra: int) -> np.random.Generator:
    return np.random.default_rng([SEED, cfg, stream, *extra])


def _offsets(sizes: np.ndarray) -> np.ndarray:
    off = np.zeros(sizes.size + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    return off


def dirichlet_ragged(rng: np.random.Generator, alpha: float, sizes: np.ndarray) -> np.ndarray:
    """Dirichlet(alpha * 1_t) weights for every bag, as Gamma variates over bag sums."""
    off = _offsets(sizes)
    g = rng.gamma(alpha, 1.0, size=int(off[-1]))
    sums = np.add.reduceat(g, off[:-1]) if sizes.size else np.zeros(0)
    return g / np.repeat(sums, sizes)


def gmm_points(rng, means: np.ndarray, sigma: float, total: int) -> np.ndarray:
    comp = rng.integers(0, means.shape[0], size=total)
    return means[comp] + sigma * rng.standard_normal((total, means.shape[1]))


def unit_gaussian_points(rng, d: int, total: int) -> np.ndarray:
    x = rng.standard_normal((total, d))
    return x / np.linalg.norm(x, axis=1, keepdims=True)


# The five measured configurations.  "law" names the point distribution.
CONFIGS = {
    1: dict(name="c1_plain_fp64", n=200, d=3, t_range=(4, 8), law="gmm", comps=5, sigma=1.0,
            box=5.0, alpha=1.0, k=10, s=8, dtype="f64", kind="assign"),
    2: dict(name="c2_assign_100k_x512_d8", n=100_000, d=8, t_range=(1, 16), law="gmm", comps=20,
            sigma=1.0, box=5.0, alpha=0.5, k=512, s=16, dtype="f32", kind="assign"),
    3: dict(name="c3_assign_50k_x256_d128", n=50_000, d=128, t_range=(8, 32), law="unit", comps=0,
            sigma=0.0, box=0.0, alpha=1.0, k=256, s=32, dtype="f32", kind="assign"),
    4: dict(name="c4_pairwise_4096_d16", n=4096, d=16, t_range=(2, 64), law="gmm", comps=20,
            sigma=1.0, box=5.0, alpha=0.3, k=0, s=0, dtype="f64", kind="pairwise",
            single_atom=410),
    5: dict(name="c5_serve_d32_x1024", n=0, d=32, t_range=(4, 64), law="gmm", comps=20, sigma=1.0,
            box=5.0, alpha=1.0, k=1024, s=32, dtype="f64", kind="serve",
            rates=(2000, 10000, 50000), duration_s=60.0),
}


def _means(cfg: int, spec) -> Optional[np.ndarray]:
    if spec["law"] != "gmm":
        return None
    rng = rng_for(cfg, STREAM_MEANS)
    return rng.uniform(-spec["box"], spec["box"], size=(spec["comps"], spec["d"]))


def _points(rng, cfg, spec, means, total):
    if spec["law"] == "gmm":
        return gmm_points(rng, means, spec["sigma"], total)
    return unit_gaussian_points(rng, spec["d"], total)


def _store(spec, s: RaggedSet) -> RaggedSet:
    return s.astype(np.float32) if spec["dtype"] == "f32" else s


def make_data(cfg: int, n: Optional[int] = None, chunk: Optional[int] = None) -> RaggedSet:
    """The data bags of configuration ``cfg`` (stream 1).

    ``n`` overrides the object count (same law, different draw).  ``chunk``
    selects an independent sub-stream, used to draw serving queries in pieces.
    """
    spec = CONFIGS[cfg]
    n = spec["n"] if n is None else int(n)
    rng = rng_for(cfg, STREAM_DATA) if chunk is None else rng_for(cfg, STREAM_DATA, chunk)
    lo, hi = spec["t_range"]
    if cfg == 4:
        u = rng.uniform(math.log(lo), math.log(hi + 1), size=n)
        sizes = np.minimum(hi, np.floor(np.exp(u))).astype(np.int64)
        n_single = min(n, int(round(spec["single_atom"] * n / spec["n"])))
        single = rng.choice(n, size=n_single, replace=False)
        sizes[single] = 1
    else:
        sizes = rng.integers(lo, hi + 1, size=n).astype(np.int64)
    off = _offsets(sizes)
    pts = _points(rng, cfg, spec, _means(cfg, spec), int(off[-1]))
    w = dirichlet_ragged(rng, spec["alpha"], sizes)
    return _store(spec, RaggedSet(off, pts, w))


def make_centroids(cfg: int, k: Optional[int] = None) -> RaggedSet:
    """K centroids of fixed support s drawn from the same law (stream 2)."""
    spec = CONFIGS[cfg]
    k = spec["k"] if k is None else int(k)
    rng = rng_for(cfg, STREAM_CENTROIDS)
    sizes = np.full(k, spec["s"], dtype=np.int64)
    off = _offsets(sizes)
    pts = _points(rng, cfg, spec, _means(cfg, spec), int(off[-1]))
    w = dirichlet_ragged(rng, spec["alpha"], sizes)
    return _store(spec, RaggedSet(off, pts, w))


def arrivals(cfg: int, rate: float, duration_s: float) -> np.ndarray:
    """Open-loop Poisson arrival times (seconds) on [0, duration_s) (stream 3)."""
    rng = rng_for(cfg, STREAM_ARRIVALS, int(rate))
    n_guess = int(rate * duration_s * 1.2 + 100)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_guess))
    while t[-1] < duration_s:
        more = t[-1] + np.cumsum(rng.exponential(1.0 / rate, size=n_guess))
        t = np.concatenate([t, more])
    return t[t < duration_s]


def sample_pairs(cfg: int, n_rows: int, n_cols: int, count: int, tag: int = 0) -> np.ndarray:
    """``count`` distinct (row, col) index pairs, seeded (stream 4)."""
    rng = rng_for(cfg, STREAM_SAMPLE, tag)
    total = n_rows * n_cols
    flat = rng.choice(total, size=min(count, total), replace=False)
    return np.stack([flat // n_cols, flat % n_cols], axis=1).astype(np.int64)


def sample_rows(cfg: int, n_rows: int, count: int, tag: int = 0) -> np.ndarray:
    rng = rng_for(cfg, STREAM_SAMPLE, 1000 + tag)
    return np.sort(rng.choice(n_rows, size=min(count, n_rows), replace=False)).astype(np.int64)


def make_degenerate(seed: int, n: int, t: int, s: int, d: int = 2, grid: int = 4,
                    identical_every: int = 4) -> tuple:
    """A family of highly degenerate transport problems: ``n`` pairs of bags
    with equal weights (all 1, so with t and s powers of two the normalised
    weights and every flow are exact binary fractions) and points on the
    integer grid {0..grid-1}^d (exact costs, many ties).  Every
    ``identical_every``-th pair is one bag against itself, where every pivot
    from the north-west corner is degenerate.  Returns (A, B, pairs) with
    pair k = (k, k)."""
    rng = np.random.default_rng([SEED, 900, seed, t, s, d])
    bags_a, bags_b = [], []
    for k in range(n):
        xa = rng.integers(0, grid, size=(t, d)).astype(np.float64)
        if identical_every and k % identical_every == 0 and s == t:
            xb = xa.copy()
        else:
            xb = rng.integers(0, grid, size=(s, d)).astype(np.float64)
        bags_a.append((xa, np.ones(t)))
        bags_b.append((xb, np.ones(s)))
    pairs = np.stack([np.arange(n), np.arange(n)], axis=1).astype(np.int64)
    return from_bags(bags_a), from_bags(bags_b), pairs
