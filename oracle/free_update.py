"""Plain FP64 centroid update of D2-clustering with free centroid weights
(TEST INFRASTRUCTURE ONLY: used by the tests, never by the product path).

Alg. 1 (Sec. 1.1) updates a cluster's centroid z = {(z^(r), p_z^(r))} from
its members v_i = {(v_i^(a), p_i^(a))} by repeating:

  Step 1  with the atoms z^(r) fixed, solve the linear program of Eq. (1)
          over the centroid weights p_z and every member's matching w^(i):
              minimise  sum_i omega_i sum_{r,a} w^(i)_{r a} |z^(r) - v_i^(a)|^2
              subject to sum_a w^(i)_{r a} = p_z^(r)   for every member i, atom r,
                         sum_r w^(i)_{r a} = p_i^(a)   for every member i, atom a,
                         sum_r p_z^(r) = 1,  p_z >= 0,  w >= 0;
          omega_i is the member's weight of weighted D2-clustering (Eq. (3)),
          all 1 without weights;
  Step 2  with p_z and the w^(i) fixed, every atom moves to the mean of the
          member atoms weighted by omega_i times their flows to it, Eq. (2)
          (Eq. (4) with weights);
  Step 3  the objective of Eq. (1) with the moved atoms and the same p_z, w.

This module does one pass of Steps 1-3 for every cluster.  Step 1 is solved
by ``lp_simplex``: a plain dense two-phase tableau simplex with Bland's rule
(lowest-index entering column with a negative reduced cost, lowest-index
basic variable among ratio-test ties), which terminates on every LP.

Readings where the paper is silent:
  * member weights p_i and the centroid weights p_z are probability vectors
    (the member's weights are divided by their sum, as everywhere);
  * a member whose weights or omega are invalid (negative, not finite, zero
    sum) is left out with status 1, one whose label is outside [0, K) with
    status 5; a member of weight omega = 0 costs and moves nothing and is
    left out of the LP;
  * an atom that receives no mass keeps its coordinates, with weight 0;
  * a flow or weight of the Step 1 solution at or below FLOW_EPS = 1e-14 (of
    the unit mass every member carries) is rounding noise of a zero and is
    set to 0 before Steps 2-3, so an atom left without mass by the exact
    solution is not moved to a mean of noise;
  * a cluster without members keeps its atoms and weights.
"""
from __future__ import annotations

import numpy as np

LABEL_OUT_OF_RANGE = 5
FLOW_EPS = 1e-14


def _pivot(T, basis, k, q):
    T[k] /= T[k, q]
    for i in range(T.shape[0]):
        if i != k and T[i, q] != 0.0:
            T[i] -= T[i, q] * T[k]
    basis[k] = q


def _bland(T, basis, ncols, tol, max_iter):
    """Minimise the objective row of T (last row) over the first ncols columns
    with Bland's rule; the last column is the right-hand side."""
    m = T.shape[0] - 1
    for _ in range(max_iter):
        neg = np.flatnonzero(T[m, :ncols] < -tol)
        if neg.size == 0:
            return True
        q = int(neg[0])
        col = T[:m, q]
        rows = np.flatnonzero(col > tol)
        if rows.size == 0:
            raise ArithmeticError("unbounded linear program")
        ratios = T[rows, -1] / col[rows]
        best = ratios.min()
        ties = rows[ratios <= best]
        k = int(ties[np.argmin(np.asarray(basis)[ties])])
        _pivot(T, basis, k, q)
    return False


def lp_simplex(c, A, b, tol=1e-12, max_iter=100000):
    """min c.x subject to A x = b, x >= 0, with b >= 0 and rows possibly
    linearly dependent.  Phase I minimises the sum of one artificial variable
    per row; artificials left in the basis at zero are pivoted out on any
    non-zero original column, or their row is dropped as redundant.
    Returns (value, x)."""
    c = np.asarray(c, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    m, n = A.shape
    scale = max(1.0, float(np.abs(c).max()) if c.size else 1.0)
    # phase I
    T = np.zeros((m + 1, n + m + 1))
    T[:m, :n] = A
    T[:m, n:n + m] = np.eye(m)
    T[:m, -1] = b
    T[m, :n] = -A.sum(axis=0)
    T[m, -1] = -b.sum()
    basis = list(range(n, n + m))
    if not _bland(T, basis, n + m, tol, max_iter):
        raise ArithmeticError("phase I iteration limit")
    if T[m, -1] < -1e-9:
        raise ArithmeticError("infeasible linear program")
    keep = []
    for k in range(m):
        if basis[k] >= n:
            nz = np.flatnonzero(np.abs(T[k, :n]) > 1e-9)
            if nz.size:
                _pivot(T, basis, k, int(nz[0]))
                keep.append(k)
        else:
            keep.append(k)
    # phase II over the original columns, redundant rows dropped
    T2 = np.zeros((len(keep) + 1, n + 1))
    T2[:-1, :n] = T[keep, :n]
    T2[:-1, -1] = T[keep, -1]
    basis2 = [basis[k] for k in keep]
    T2[-1, :n] = c
    for k, j in enumerate(basis2):
        T2[-1] -= c[j] * T2[k]
    if not _bland(T2, basis2, n, tol * scale, max_iter):
        raise ArithmeticError("phase II iteration limit")
    x = np.zeros(n)
    for k, j in enumerate(basis2):
        x[j] = max(T2[k, -1], 0.0)
    return float(c @ x), x


def cluster_lp(members, zpts):
    """The LP of Step 1 for one cluster: members is a list of (points[t,d],
    probabilities p[t], omega); zpts the s fixed atoms.  Variables: each
    member's w[a, r] (member by member, a-major), then p_z[s].  Returns
    (c, A, b, layout) with layout[i] = offset of member i's block."""
    s = zpts.shape[0]
    layout, off = [], 0
    for x, p, om in members:
        layout.append(off)
        off += len(p) * s
    nvar = off + s
    rows_A, rows_b = [], []
    c = np.zeros(nvar)
    for (x, p, om), o in zip(members, layout):
        t = len(p)
        for a in range(t):
            for r in range(s):
                diff = x[a] - zpts[r]
                c[o + a * s + r] = om * float(np.dot(diff, diff))
        for a in range(t):                  # sum_r w[a, r] = p[a]
            row = np.zeros(nvar)
            row[o + a * s:o + (a + 1) * s] = 1.0
            rows_A.append(row)
            rows_b.append(p[a])
        for r in range(s):                  # sum_a w[a, r] - p_z[r] = 0
            row = np.zeros(nvar)
            row[o + r:o + t * s:s] = 1.0
            row[off + r] = -1.0
            rows_A.append(row)
            rows_b.append(0.0)
    row = np.zeros(nvar)                    # sum_r p_z[r] = 1
    row[off:] = 1.0
    rows_A.append(row)
    rows_b.append(1.0)
    return c, np.array(rows_A), np.array(rows_b), layout


def free_update(X, Z, labels, weights=None):
    """One pass of Alg. 1 (Steps 1-3) with free centroid weights for every
    cluster.  Returns (z_new [Z.offsets[K], d], p_new [Z.offsets[K]],
    eps_step1 [K] (the Step 1 LP value), eps_step3 [K], status [n])."""
    zoff = np.asarray(Z.offsets, dtype=np.int64)
    K = zoff.shape[0] - 1
    zpts = np.asarray(Z.points, dtype=np.float64)
    zw = np.asarray(Z.weights, dtype=np.float64)
    labels = np.asarray(labels).reshape(-1)
    n = int(np.asarray(X.offsets).shape[0] - 1)
    z_new = zpts.copy()
    p_new = zw.copy()
    eps1 = np.zeros(K)
    eps3 = np.zeros(K)
    status = np.zeros(n, dtype=np.int32)
    groups = [[] for _ in range(K)]
    for i in range(n):
        j = int(labels[i])
        if j < 0 or j >= K:
            status[i] = LABEL_OUT_OF_RANGE
            continue
        om = 1.0 if weights is None else float(weights[i])
        x, p = X.bag(i)
        p = np.asarray(p, dtype=np.float64)
        if not (np.isfinite(om) and om >= 0.0) or not np.all(np.isfinite(p)) or np.any(p < 0) \
                or not p.sum() > 0:
            status[i] = 1
            continue
        if om > 0.0:
            groups[j].append((np.asarray(x, dtype=np.float64), p / p.sum(), om))
    for j in range(K):
        if not groups[j]:
            continue
        a0, a1 = int(zoff[j]), int(zoff[j + 1])
        z = zpts[a0:a1]
        s = z.shape[0]
        c, A, b, layout = cluster_lp(groups[j], z)
        value, x = lp_simplex(c, A, b)
        eps1[j] = value
        x = np.where(x > FLOW_EPS, x, 0.0)
        pz = x[len(c) - s:]
        # Step 2: omega- and flow-weighted means (Eq. (2), Eq. (4))
        num = np.zeros_like(z)
        den = np.zeros(s)
        plans = []
        for (xi, p, om), o in zip(groups[j], layout):
            w = x[o:o + len(p) * s].reshape(len(p), s)
            plans.append((xi, w, om))
            num += om * (w.T @ xi)
            den += om * w.sum(axis=0)
        zn = z.copy()
        moved = den > 0
        zn[moved] = num[moved] / den[moved, None]
        z_new[a0:a1] = zn
        p_new[a0:a1] = pz
        # Step 3: the objective with the moved atoms, the same matchings
        for xi, w, om in plans:
            diff = xi[:, None, :] - zn[None, :, :]
            eps3[j] += om * float((w * (diff * diff).sum(axis=2)).sum())
    return z_new, p_new, eps1, eps3, status
