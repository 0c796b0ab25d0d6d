"""Plain FP64 labelling under the combined distance of Eq. (9) (TEST
INFRASTRUCTURE ONLY: used by the tests, never by the product path).

Sec. 3 describes an image by several distributions, one per feature type
(a colour bag U and a texture bag V), and compares two images by the root of
the sum of the per-type squared Mallows distances.  Labelling with it
(Alg. 2 Step 2 on that distance) is written out as: every per-type D^2
matrix, their sum, the argmin of each row (ties to the lowest centroid), and
label -1 for a row in which any pair of any type failed.
"""
from __future__ import annotations

import numpy as np

from . import INIT_NWC, assign


def assign_multi(Xs, Zs, init: int = INIT_NWC):
    """Returns (labels, best, all[n, K] summed over types, status)."""
    total = None
    worst = None
    for X, Z in zip(Xs, Zs):
        _, _, allv, st, _ = assign(X, Z, init=init, want_all=True)
        total = allv.copy() if total is None else total + allv
        worst = st.copy() if worst is None else np.maximum(worst, st)
    labels = np.full(total.shape[0], -1, dtype=np.int32)
    best = np.full(total.shape[0], np.nan)
    for i in range(total.shape[0]):
        if worst[i] == 0:
            labels[i] = int(np.argmin(total[i]))   # first minimum: lowest index
            best[i] = total[i, labels[i]]
    return labels, best, total, worst
