"""Hierarchical D2-clustering of Alg. 3 on one GPU.

The paper runs each level as three synchronised steps between a master and
slave processors.  Here the master's segment bookkeeping is host control
over small integer arrays.  All distance and update work of the slaves, the
segmentation's, and the merge, runs in the library on the GPU, every
segment of a level at once:

* ``d2_assign_segmented`` labels each object among its own segment's
  centroids;
* ``d2_centroid_update_free`` with object weights solves Alg. 1's Step 1
  program for every cluster (the centroid weights free) and moves every
  centroid by Eq. (4); the binary splits use ``d2_centroid_update`` (the
  centroid weights held);
* ``d2_merge_level`` keeps the centroids with members, sums their weights
  and lets every original object inherit its new label.

Per level:

1. **Segmentation (Sec. 2.2).**  Segments larger than tau are split in two
   by constrained D2-clustering with two centroids, repeated until none is
   larger.  All oversize segments split in the same round: a split depends
   only on its own segment, so the result is the one the largest-first
   order gives.
2. **Clustering.**  Every segment is clustered into ceil(n_mu / e) groups
   (tau = c e, Sec. 2.5) by weighted D2-clustering: Alg. 1 with Eq. (3),
   (4), the centroid weights free (``update="constrained"`` holds them at
   their starting values instead).
3. **Merge.**  The segments' centroids are concatenated in segment order,
   labels are offset (Eq. (5)) and inherited (Eq. (6)), and a centroid's
   weight is the sum of its members' weights.  A centroid becomes an object
   of the next level with the atom weights its last update left.  The hierarchy stops at the
   first level with at most k centroids.

The random choices (initial centroids) consume a caller-given stream of
uniforms in a fixed order:

* a split takes positions floor(u |S|) and then floor(u' (|S| - 1)) among
  the rest;
* a segment's picks are a partial Fisher-Yates shuffle.

Each clustering runs ``rounds`` rounds of (labelling, ``passes`` weighted
update passes) and then labels once more.  A split that leaves a side empty
halves the segment instead.  A cluster left without members is dropped at
the merge.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np
import torch

from .api import (DeviceSet, Handle, Opts, d2_assign_segmented, d2_centroid_update,
                  d2_centroid_update_free, d2_merge_level, free_basis_buffer)


class _Stream:
    """Caller-given uniforms, consumed in order."""

    def __init__(self, u):
        self._u = np.asarray(u, dtype=np.float64).ravel()
        self._k = 0

    def take(self) -> float:
        if self._k == self._u.size:
            raise RuntimeError("the stream of uniforms ran out")
        self._k += 1
        return float(self._u[self._k - 1])


def _gather(G: DeviceSet, g_off: np.ndarray, objs) -> tuple:
    """A set made of the atoms of objects `objs` of G (in that order), with
    uniform weights (the starting centroids of a clustering); returns
    (DeviceSet, host offsets)."""
    objs = np.asarray(objs, dtype=np.int64)
    sizes = g_off[1:][objs] - g_off[:-1][objs]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    # atom rows of the picked objects, object after object
    rows = np.repeat(g_off[:-1][objs] - off[:-1], sizes) + np.arange(int(off[-1]), dtype=np.int64)
    dev = G.points.device
    rows_d = torch.as_tensor(rows, device=dev)
    pts = G.points.index_select(0, rows_d)
    w = torch.as_tensor(np.repeat(1.0 / np.maximum(sizes, 1), sizes), device=dev)
    Z = DeviceSet(torch.as_tensor(off, device=dev), pts.contiguous(), w.contiguous(),
                  int(sizes.max()) if len(objs) else 1)
    return Z, off


def _count(stats, G, g_off, z_off, segments, starts, rounds, passes, free):
    """Adds the LPs this clustering solves, and their pivot-free FP64 work
    (3 t s d + 3 t s per member and centroid), to `stats`.  A free update
    solves one program per cluster, a constrained one one per member."""
    t = (g_off[1:] - g_off[:-1]).astype(np.float64)
    s = (z_off[1:] - z_off[:-1]).astype(np.float64)
    d = G.d
    n_seg = np.array([len(S) for S in segments], dtype=np.float64)
    k_seg = np.array([len(st) for st in starts], dtype=np.int64)
    t_seg = np.add.reduceat(t[np.concatenate(segments)], np.concatenate([[0], np.cumsum(n_seg)[:-1]]).astype(np.int64))
    z_first = np.concatenate([[0], np.cumsum(k_seg)[:-1]]).astype(np.int64)
    s_sum = np.add.reduceat(s, z_first)
    s_max = np.maximum.reduceat(s, z_first)
    add = {
        # labelling: every member against every centroid of its segment
        "lps_label": float(((rounds + 1) * n_seg * k_seg).sum()),
        "flops_label": float(((rounds + 1) * t_seg * s_sum * (3 * d + 3)).sum()),
        # update: every member against one centroid (bounded by the largest)
        "lps_update": float((rounds * passes * (k_seg if free else n_seg)).sum()),
        "flops_update": float((rounds * passes * t_seg * s_max * (3 * d + 3)).sum()),
    }
    add["lps"] = add["lps_label"] + add["lps_update"]
    add["flops"] = add["flops_label"] + add["flops_update"]
    for key, v in add.items():
        stats[key] = stats.get(key, 0.0) + v


def _cluster_segments(h, G, g_off, omega, segments, starts, rounds, passes, opts, stats=None,
                      free=False):
    """Weighted D2-clustering of every segment at once, the centroid weights
    free (Alg. 1) when `free`, else held; segment mu starts from its objects
    starts[mu].  Returns (centroids, their host offsets, the centroid range
    of each segment, labels over G)."""
    order = [o for s in starts for o in s]
    Z, z_off = _gather(G, g_off, order)
    if stats is not None:
        _count(stats, G, g_off, z_off, segments, starts, rounds, passes, free)
    zseg = np.concatenate([[0], np.cumsum([len(s) for s in starts])]).astype(np.int64)
    seg = np.full(G.n, -1, dtype=np.int32)
    if segments:
        seg[np.concatenate(segments)] = np.repeat(np.arange(len(segments), dtype=np.int32),
                                                  [len(S) for S in segments])
    dev = G.points.device
    seg_d = torch.as_tensor(seg, device=dev)
    zseg_d = torch.as_tensor(zseg, device=dev)
    worst = torch.zeros((), dtype=torch.int32, device=dev)
    # each cluster's optimal basis starts its next pass (the same members
    # within a round; a changed membership is detected and starts cold)
    basis = free_basis_buffer(G, Z, max(len(S) for S in segments)) if free and segments else None
    for _ in range(rounds):
        labels, _, _ = d2_assign_segmented(h, G, Z, seg_d, zseg_d, opts)
        for _ in range(passes):
            if free:
                z_new, w_new, _, _, _, _, cst = d2_centroid_update_free(h, G, Z, labels, opts,
                                                                        weights=omega, basis=basis)
                if cst.numel():
                    worst = torch.maximum(worst, cst.max())
                Z = DeviceSet(Z.offsets, z_new, w_new, Z.max_support)
            else:
                z_new = d2_centroid_update(h, G, Z, labels, opts, weights=omega)[0]
                Z = Z.with_points(z_new)
    labels, _, _ = d2_assign_segmented(h, G, Z, seg_d, zseg_d, opts)
    if int(worst.item()) != 0:
        raise RuntimeError(f"a cluster's centroid program failed (status {int(worst.item())})")
    return Z, z_off, zseg, labels


def hierarchical_d2(h: Handle, X: DeviceSet, tau: int, e: int, k: int, uniforms,
                    rounds: int = 3, passes: int = 2, opts: Optional[Opts] = None,
                    max_levels: int = 16, stats: Optional[dict] = None, update: str = "free"):
    """Alg. 3 on one GPU.  Returns (centroids as a DeviceSet, labels of X as
    a host int32 array, their weights, per-level statistics).  `stats`, when
    given, receives the count of LPs solved ("lps") and their pivot-free
    FP64 work ("flops"; the update's is bounded by the largest centroid).
    ``update``: "free" (Alg. 1 in Step 2, the paper's) or "constrained"."""
    if tau < 2 or e < 1 or k < 1:
        raise ValueError("need tau >= 2, e >= 1 and k >= 1")
    if update not in ("free", "constrained"):
        raise ValueError("update is 'free' or 'constrained'")
    if X.n < 1:
        raise ValueError("no objects to cluster")
    opts = opts or Opts()
    U = _Stream(uniforms)
    G = X if X.points.dtype == torch.float64 else X.with_points(X.points.double())
    g_off = G.offsets.cpu().numpy()
    omega = torch.ones(G.n, dtype=torch.float64, device=G.points.device)
    C = torch.arange(G.n, dtype=torch.int32, device=G.points.device)
    levels = []
    for _ in range(max_levels):
        # Step 1: segmentation by binary splits
        segments = [np.arange(G.n)]
        while max(len(S) for S in segments) > tau:
            split = [q for q, S in enumerate(segments) if len(S) > tau]
            starts = []
            for q in split:
                S = segments[q]
                a = math.floor(U.take() * len(S))
                b = math.floor(U.take() * (len(S) - 1))
                b += b >= a                       # the b-th position other than a
                starts.append([int(S[a]), int(S[b])])
            _, _, zseg, labels = _cluster_segments(h, G, g_off, omega, [segments[q] for q in split],
                                                   starts, rounds, passes, opts, stats)
            labels = labels.cpu().numpy()
            out = []
            where = {q: mu for mu, q in enumerate(split)}
            for q, S in enumerate(segments):
                if q not in where:
                    out.append(S)
                    continue
                on_first = labels[S] == zseg[where[q]]
                A, B = S[on_first], S[~on_first]
                if A.size == 0 or B.size == 0:
                    A, B = S[:S.size // 2], S[S.size // 2:]
                out += [A, B]
            segments = out
        # Step 2: every segment into ceil(n_mu / e) clusters
        starts = []
        for S in segments:
            pos = np.arange(S.size)
            for q in range(math.ceil(S.size / e)):
                r = q + math.floor(U.take() * (S.size - q))
                pos[q], pos[r] = pos[r], pos[q]
            starts.append([int(S[p]) for p in pos[:math.ceil(S.size / e)]])
        Z, z_off, zseg, labels = _cluster_segments(h, G, g_off, omega, segments, starts, rounds, passes,
                                                   opts, stats, free=update == "free")
        if int(labels.min().item()) < 0:
            raise RuntimeError("an object's transport problem failed; check its weights and points")
        # Step 3: merge (Eq. (5)), weights, inheritance (Eq. (6)); a
        # segment's centroids are a contiguous range, so index order is
        # segment order
        n_level = G.n
        G, omega, C, g_off = d2_merge_level(h, Z, labels, omega, C)
        levels.append({"objects": n_level, "segments": len(segments), "centroids": G.n,
                       "max_segment": int(max(S.size for S in segments))})
        if G.n <= k or G.n == n_level:
            break
    return G, C.cpu().numpy(), omega.cpu().numpy(), levels
