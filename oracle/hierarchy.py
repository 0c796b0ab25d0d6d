"""Plain FP64 one-GPU-scale version of the hierarchical clustering of Alg. 3
(TEST INFRASTRUCTURE ONLY: used by the tests, never by the product path).

Written from Sec. 2 of the paper, level by level:

  Step 1  segmentation (Sec. 2.2): starting from one segment holding every
          object of the level, a segment with more than tau objects is split
          in two by constrained D2-clustering with two centroids, until no
          segment is larger than tau.  A split depends only on the segment it
          splits, so splitting every oversize segment in the same round gives
          the segments that splitting the largest one first would give.
  Step 2  each segment mu is clustered on its own into k_mu = ceil(n_mu / e)
          groups (tau = c e, Sec. 2.5) by weighted D2-clustering (Eq. (3),
          (4)): Alg. 1's centroid update with the centroid weights free
          (``free_update``); ``update="constrained"`` holds them at their
          starting values instead (Alg. 2's Step 3*).
  Step 3  the segments' centroids are concatenated in segment order, every
          object's level label is offset by the centroids before its segment
          (Eq. (5)), each original object inherits the label of its ancestor
          (Eq. (6)), and a centroid's weight is the sum of its members'
          weights.  The hierarchy stops once at most k centroids remain.

Readings where the paper is silent:
  * random choices (the two initial centroids of a split, the k_mu initial
    centroids of a segment) consume a given stream of uniforms U in a fixed
    order: a split picks position floor(u |S|) of the segment, then
    floor(u' (|S| - 1)) among the others; a segment's k_mu picks are a
    partial Fisher-Yates shuffle of its positions;
  * an initial centroid is the picked object's atoms with uniform weights;
  * the binary splits of Step 1 use the constrained update (the paper's
    segmentation is constrained D2-clustering with two centroids);
  * a centroid carries the weights its last update left (free weights,
    zeros included) into the next level, where it is an object;
  * each clustering runs `rounds` rounds of (labelling within segments,
    `passes` passes of the weighted update), then labels once more;
  * a split that leaves one side empty falls back to halving the segment in
    index order;
  * a cluster left without members is dropped at the merge (it represents
    no data);
  * objects are listed in increasing index inside every segment, and the
    two halves of a split keep that order (the first centroid's side
    first).
"""
from __future__ import annotations

import math

import numpy as np

from . import INIT_NWC, emd_batch
from .free_update import free_update
from .update import centroid_update


class _Uniforms:
    def __init__(self, u):
        self.u = np.asarray(u, dtype=np.float64)
        self.k = 0

    def next(self) -> float:
        if self.k >= self.u.size:
            raise RuntimeError("uniform stream exhausted")
        v = float(self.u[self.k])
        self.k += 1
        return v


class _Ragged:
    def __init__(self, offsets, points, weights):
        self.offsets = np.asarray(offsets, dtype=np.int64)
        self.points = np.asarray(points, dtype=np.float64)
        self.weights = np.asarray(weights, dtype=np.float64)

    @property
    def n(self):
        return self.offsets.size - 1

    def bag(self, i):
        a, b = int(self.offsets[i]), int(self.offsets[i + 1])
        return self.points[a:b], self.weights[a:b]


def split_positions(n: int, U: _Uniforms):
    """The two starting objects of a binary split of a segment of n > 1
    objects (positions within the segment): position floor(u n), then
    position floor(u' (n - 1)) among the n - 1 others, in increasing order."""
    a = int(math.floor(U.next() * n))
    rest = [x for x in range(n) if x != a]
    b = rest[int(math.floor(U.next() * (n - 1)))]
    return a, b


def segment_positions(n: int, e: int, U: _Uniforms):
    """The starting objects of a segment of n objects clustered into
    k_mu = ceil(n / e) groups (tau = c e): the first k_mu entries of a
    partial Fisher-Yates shuffle of 0..n-1, step q swapping entry q with entry
    q + floor(u (n - q))."""
    kmu = int(math.ceil(n / e))
    pos = list(range(n))
    for q in range(kmu):
        r = q + int(math.floor(U.next() * (n - q)))
        pos[q], pos[r] = pos[r], pos[q]
    return pos[:kmu]


def split_sides(S, labels, first):
    """The two halves of a binary split: the members labelled with the
    split's first centroid, then the rest, each in increasing index; when
    either side is empty, the segment is halved in index order instead."""
    S = np.asarray(S, dtype=np.int64)
    A = S[np.asarray(labels)[S] == first]
    B = S[np.asarray(labels)[S] != first]
    if len(A) == 0 or len(B) == 0:
        A, B = S[:len(S) // 2], S[len(S) // 2:]
    return A, B


def merge_level(segs, zoff, labels, omega, C):
    """Step 3 of Alg. 3 for one level.  Segment mu's centroids are
    zoff[mu] .. zoff[mu+1] of the level's centroid list, which concatenates
    the segments' centroids in segment order, so a member's label already
    carries the offset |Z^(mu-1)| of Eq. (5).  Centroids without members are
    dropped and the kept ones renumbered in order (keep[new] = old index).
    Returns (keep, the level label of every object Ct, the new weights as
    member-weight sums, and the inherited labels C' = Ct[C] of the original
    objects, Eq. (6))."""
    n = len(labels)
    keep = []
    Ct = np.full(n, -1, dtype=np.int64)
    for mu, S in enumerate(segs):
        S = np.asarray(S, dtype=np.int64)
        for j in range(int(zoff[mu]), int(zoff[mu + 1])):
            members = S[np.asarray(labels)[S] == j]
            if len(members):
                Ct[members] = len(keep)
                keep.append(j)
    new_omega = np.zeros(len(keep))
    for i in range(n):
        new_omega[Ct[i]] += omega[i]
    return keep, Ct, new_omega, Ct[np.asarray(C, dtype=np.int64)]


def _centroids_from(G, picks):
    """Centroids made of the picked objects' atoms with uniform weights."""
    pts, wts, off = [], [], [0]
    for i in picks:
        x, _ = G.bag(int(i))
        pts.append(np.asarray(x, dtype=np.float64))
        wts.append(np.full(x.shape[0], 1.0 / x.shape[0]))
        off.append(off[-1] + x.shape[0])
    return pts, wts, off


def assign_segmented(X, Z, seg, zoff, init: int = INIT_NWC):
    """For every object, the nearest centroid among zoff[seg[i]] .. zoff[seg[i]+1]
    (ties: lowest index); label -1 with status 5 when the segment is invalid
    or empty, label -1 with the worst status when a pair fails."""
    n = X.offsets.shape[0] - 1
    seg = np.asarray(seg)
    zoff = np.asarray(zoff)
    pairs = []
    for i in range(n):
        s = int(seg[i])
        if 0 <= s < zoff.size - 1:
            for j in range(int(zoff[s]), int(zoff[s + 1])):
                pairs.append((i, j))
    pairs = np.array(pairs, dtype=np.int64).reshape(-1, 2)
    dist, st, _ = emd_batch(X, Z, pairs, init=init) if len(pairs) else (np.zeros(0), np.zeros(0), None)
    labels = np.full(n, -1, dtype=np.int32)
    best = np.full(n, np.nan)
    status = np.full(n, 5, dtype=np.int32)
    for i in range(n):
        rows = np.flatnonzero(pairs[:, 0] == i) if len(pairs) else np.zeros(0, dtype=int)
        if rows.size == 0:
            continue
        worst = int(st[rows].max())
        status[i] = worst
        if worst == 0:
            k = rows[int(np.argmin(dist[rows]))]   # first minimum: lowest centroid
            labels[i] = int(pairs[k, 1])
            best[i] = dist[k]
    return labels, best, status


def _cluster(G, omega, segs, picks, rounds, passes, init, free=False):
    """Weighted D2-clustering of every segment in `segs` at once, segment mu
    starting from the objects picks[mu]; the centroid weights are free
    (Alg. 1) when `free`, else held (constrained).  Returns (centroid ragged
    set, its segment offsets, final labels over G, -1 outside)."""
    pts, wts, off = [], [], [0]
    zoff = [0]
    for p in picks:
        a, b, o = _centroids_from(G, p)
        pts += a
        wts += b
        zoff.append(zoff[-1] + len(p))
    sizes = [x.shape[0] for x in pts]
    off = np.concatenate([[0], np.cumsum(sizes)])
    Z = _Ragged(off, np.concatenate(pts), np.concatenate(wts))
    seg = np.full(G.n, -1, dtype=np.int32)
    for mu, S in enumerate(segs):
        seg[S] = mu
    for _ in range(rounds):
        labels, _, _ = assign_segmented(G, Z, seg, zoff, init)
        for _ in range(passes):
            if free:
                z_new, p_new, _, _, _ = free_update(G, Z, labels, omega)
                Z = _Ragged(Z.offsets, z_new, p_new)
            else:
                z_new, _, _, _ = centroid_update(G, Z, labels, init=init, weights=omega)
                Z = _Ragged(Z.offsets, z_new, Z.weights)
    labels, _, _ = assign_segmented(G, Z, seg, zoff, init)
    return Z, np.asarray(zoff), labels


def hierarchy(X, tau: int, e: int, k: int, uniforms, rounds: int = 3, passes: int = 2,
              init: int = INIT_NWC, max_levels: int = 16, update: str = "free"):
    """Returns (centroids as (offsets, points, weights), labels of X, levels)
    with levels a list of dicts (objects, segments, centroids).  ``update``:
    "free" (Alg. 1 in Step 2, the paper's) or "constrained"."""
    if update not in ("free", "constrained"):
        raise ValueError("update is 'free' or 'constrained'")
    U = _Uniforms(uniforms)
    G = _Ragged(X.offsets, X.points, X.weights)
    omega = np.ones(G.n)
    C = np.arange(G.n)
    levels = []
    for _ in range(max_levels):
        # Step 1: binary splits until every segment holds at most tau objects
        segs = [np.arange(G.n)]
        while any(len(S) > tau for S in segs):
            big = [q for q, S in enumerate(segs) if len(S) > tau]
            picks = []
            for q in big:
                S = segs[q]
                a, b = split_positions(len(S), U)
                picks.append([S[a], S[b]])
            _, zoff, labels = _cluster(G, omega, [segs[q] for q in big], picks, rounds, passes, init)
            new = []
            for q, S in enumerate(segs):
                if q not in big:
                    new.append(S)
                    continue
                mu = big.index(q)
                A, B = split_sides(S, labels, int(zoff[mu]))
                new += [A, B]
            segs = new
        # Step 2: each segment into ceil(n_mu / e) clusters
        picks = [[S[p] for p in segment_positions(len(S), e, U)] for S in segs]
        Z, zoff, labels = _cluster(G, omega, segs, picks, rounds, passes, init, free=update == "free")
        if labels.min() < 0:
            raise RuntimeError("a transport problem failed")
        # Step 3: merge in segment order (Eq. (5)), inherit labels (Eq. (6))
        keep, Ct, new_omega, C = merge_level(segs, zoff, labels, omega, C)
        pts = [Z.bag(j)[0] for j in keep]
        wts = [Z.bag(j)[1] for j in keep]
        off = np.concatenate([[0], np.cumsum([p.shape[0] for p in pts])])
        levels.append({"objects": G.n, "segments": len(segs), "centroids": len(keep),
                       "max_segment": max(len(S) for S in segs)})
        G = _Ragged(off, np.concatenate(pts), np.concatenate(wts))
        omega = new_omega
        if len(keep) <= k or len(keep) == levels[-1]["objects"]:
            break
    return (G.offsets, G.points, G.weights), C.astype(np.int32), levels, omega
