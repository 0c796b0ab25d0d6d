"""Plain FP64 centroid update of constrained D2-clustering (TEST INFRASTRUCTURE
ONLY: used by the tests, the smoke check and the benchmark's CPU baseline;
never by the product path).

Constrained D2-clustering (Alg. 2, Step 3*) holds every centroid's weights
fixed (uniform 1/s_j in the paper) and runs the centroid update of Alg. 1
with them.  With the weights fixed, the LP of Step 1 separates into one
transport problem per member (Sec. 2.2), so one pass is:

  Step 1  for every object i with label j = C(i): the optimal plan w^(i)
          between z_j and v_i, i.e. Eq. (1) with z_j fixed (``emd_pair``);
  Step 2  every centroid atom moves to the flow-weighted mean of the member
          atoms it receives mass from, Eq. (2):
              z_j^(r) = sum_i sum_a w^(i)_{a r} v_i^(a) / sum_i sum_a w^(i)_{a r};
  Step 3  the objective of Eq. (1) with the moved atoms and the same plans:
              eps_j = sum_i sum_{a,r} w^(i)_{a r} |z_j^(r) - v_i^(a)|^2.

Weighted D2-clustering (Eq. (3)-(4)) gives each object a weight omega_i:
its D^2 counts omega_i times in the objective, and its flows count omega_i
times in both sums of the mean (Eq. (4)).  Without weights every omega_i = 1.

Readings where the paper is silent:
  * any fixed centroid weights are accepted (uniform is the paper's case);
    they are normalised by their sum like every weight vector;
  * an atom that receives no flow (empty cluster, zero weight) keeps its
    coordinates;
  * an object whose label is outside [0, K) is left out (status 5), and so
    is one whose transport problem fails (its oracle status) or whose
    weight is negative or not finite (status 1);
  * eps_step1[j] is the Step 1 objective (sum of the members' D^2 against the
    old atoms), reported beside the Step 3 value.

Sums run over members in increasing object index, atoms in increasing order.
"""
from __future__ import annotations

import numpy as np

from . import INIT_NWC, emd_pair

LABEL_OUT_OF_RANGE = 5


def centroid_update(X, Z, labels, init: int = INIT_NWC, return_plans: bool = False, weights=None):
    """One pass of Steps 1-3 for every cluster (weights: the objects' omega).

    Returns (z_new[Z.offsets[K], d], eps_step1[K], eps_step3[K], status[n])
    and, with ``return_plans``, the list of (i, j, plan[t_i, s_j]) used.
    """
    zoff = np.asarray(Z.offsets, dtype=np.int64)
    K = zoff.shape[0] - 1
    zpts = np.asarray(Z.points, dtype=np.float64)
    zw = np.asarray(Z.weights, dtype=np.float64)
    labels = np.asarray(labels).reshape(-1)
    n = int(np.asarray(X.offsets).shape[0] - 1)
    d = zpts.shape[1]
    num = np.zeros((zpts.shape[0], d))
    den = np.zeros(zpts.shape[0])
    eps1 = np.zeros(K)
    eps3 = np.zeros(K)
    status = np.zeros(n, dtype=np.int32)
    plans = []
    # Step 1: one transport problem per member, against its own centroid
    for i in range(n):
        j = int(labels[i])
        if j < 0 or j >= K:
            status[i] = LABEL_OUT_OF_RANGE
            continue
        om = 1.0 if weights is None else float(weights[i])
        if not (np.isfinite(om) and om >= 0.0):
            status[i] = 1
            continue
        x, p = X.bag(i)
        a0, a1 = int(zoff[j]), int(zoff[j + 1])
        try:
            d2, plan, _, _, _ = emd_pair(x, p, zpts[a0:a1], zw[a0:a1], init)
        except ArithmeticError as e:
            status[i] = getattr(e, "status", 3)
            continue
        plans.append((i, j, plan, om))
        eps1[j] += om * d2
        x = np.asarray(x, dtype=np.float64)
        # numerator and denominator of Eq. (2) / (4): plan[a, r] weights v_i^(a)
        num[a0:a1] += om * (plan.T @ x)
        den[a0:a1] += om * plan.sum(axis=0)
    # Step 2: Eq. (2); atoms without flow stay where they are
    z_new = zpts.copy()
    moved = den > 0
    z_new[moved] = num[moved] / den[moved, None]
    # Step 3: the objective with the moved atoms and the Step 1 plans
    for i, j, plan, om in plans:
        x = np.asarray(X.bag(i)[0], dtype=np.float64)
        a0, a1 = int(zoff[j]), int(zoff[j + 1])
        diff = x[:, None, :] - z_new[None, a0:a1, :]
        eps3[j] += om * float((plan * (diff * diff).sum(axis=2)).sum())
    if return_plans:
        return z_new, eps1, eps3, status, [(i, j, plan) for i, j, plan, _ in plans]
    return z_new, eps1, eps3, status
