"""Shared parity helpers for the GPU tests (tolerances of the FP64 path).

A device value g passes against the oracle value o when
    |g - o| <= 1e-10 * max(|o|, 1e-4 * S)
with S = sum_ab p_a q_b |x_a - y_b|^2 the independent-coupling cost of the
pair (an upper bound on D^2), which gives identical distributions (D^2 = 0)
an absolute floor of 1e-14 * S.
"""
import numpy as np

REL = 1e-10


def coupling_cost(x, p, y, q) -> float:
    x = np.asarray(x, np.float64).reshape(len(p), -1)
    y = np.asarray(y, np.float64).reshape(len(q), -1)
    p = np.asarray(p, np.float64); q = np.asarray(q, np.float64)
    p = p / p.sum(); q = q / q.sum()
    C = ((x[:, None, :] - y[None, :, :]) ** 2).sum(-1)
    return float(p @ C @ q)


def pair_tolerance(A, B, pairs) -> np.ndarray:
    tol = np.empty(len(pairs))
    for k, (i, j) in enumerate(pairs):
        x, p = A.bag(int(i)); y, q = B.bag(int(j))
        tol[k] = REL * 1e-4 * coupling_cost(x, p, y, q)
    return tol


def assert_close(g, o, floor_abs):
    g = np.asarray(g, np.float64); o = np.asarray(o, np.float64)
    bound = np.maximum(REL * np.abs(o), floor_abs)
    bad = ~(np.abs(g - o) <= bound)
    if bad.any():
        k = int(np.flatnonzero(bad)[0])
        raise AssertionError(f"{int(bad.sum())} of {g.size} values out of tolerance; first at {k}: "
                             f"gpu={g.flat[k]!r} oracle={o.flat[k]!r} bound={bound.flat[k]!r}")


def assert_labels(g_lab, o_lab, o_all, floor_abs_rows):
    """Labels equal, or the device's pick is within tolerance of the oracle's
    minimum (a near-tie under the c9 rule)."""
    g_lab = np.asarray(g_lab); o_lab = np.asarray(o_lab)
    diff = np.flatnonzero(g_lab != o_lab)
    for i in diff:
        gi, oi = int(g_lab[i]), int(o_lab[i])
        assert gi >= 0, f"row {i}: device label {gi}, oracle {oi}"
        gap = o_all[i, gi] - o_all[i, oi]
        assert gap <= max(REL * abs(o_all[i, oi]), floor_abs_rows[i]), \
            f"row {i}: label {gi} vs {oi}, oracle gap {gap}"
    return diff.size
