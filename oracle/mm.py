"""Plain FP64 MM distance between two sets of centroids (TEST INFRASTRUCTURE
ONLY: used by the tests and the benchmark's CPU baseline, never by the
product path).

Eq. (10) of Sec. 3.1: for centroid sets Z = {z_1..z_k} and Z' = {z'_1..z'_k'}
with cluster proportions p and p', the squared MM distance is the transport
LP over the clusters whose ground cost is the squared Mallows distance
between centroids:

    MM^2(Z, Z') = min_w sum_i sum_j w_ij D^2(z_i, z'_j),
                  sum_j w_ij = p_i,  sum_i w_ij = p'_j,  w >= 0.

Steps, in that order: every D^2(z_i, z'_j) (Eq. (1) with both sides fixed),
then the outer LP on that matrix.  p and p' are normalised by their sums like
every weight vector.
"""
from __future__ import annotations

from . import INIT_NWC, assign, emd_cost


def mm_distance(Z1, p1, Z2, p2, init: int = INIT_NWC):
    """Returns (MM^2, M[k, k'] of squared Mallows distances, plan[k, k'])."""
    _, _, M, status, _ = assign(Z1, Z2, init=init, want_all=True)
    if status.max() != 0:
        raise ArithmeticError("a centroid pair failed")
    value, plan, _, _, _ = emd_cost(M, p1, p2, init)
    return value, M, plan
