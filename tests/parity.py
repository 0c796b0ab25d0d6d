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


def coupling_moments(S):
    """Per object i of a ragged set: m2_i = sum_a p_a |x_a|^2 and
    mu_i = sum_a p_a x_a with p normalised, so that the independent-coupling
    cost of (i, j) is m2_i + m2_j' - 2 mu_i . mu_j' (for the tolerance floor
    of many pairs at once)."""
    off = np.asarray(S.offsets)
    x = np.asarray(S.points, np.float64).reshape(off[-1], -1)
    w = np.asarray(S.weights, np.float64)
    seg = np.repeat(np.arange(len(off) - 1), np.diff(off))
    tot = np.bincount(seg, weights=w, minlength=len(off) - 1)
    p = w / tot[seg]
    m2 = np.bincount(seg, weights=p * (x * x).sum(1), minlength=len(off) - 1)
    mu = np.stack([np.bincount(seg, weights=p * x[:, k], minlength=len(off) - 1)
                   for k in range(x.shape[1])], 1)
    return m2, mu


def pair_tolerance_fast(A, B, pairs) -> np.ndarray:
    """pair_tolerance from the per-object moments (no per-pair Python loop)."""
    ma, ua = coupling_moments(A)
    mb, ub = (ma, ua) if B is A else coupling_moments(B)
    i, j = pairs[:, 0], pairs[:, 1]
    s = ma[i] + mb[j] - 2.0 * np.einsum("kd,kd->k", ua[i], ub[j])
    return REL * 1e-4 * np.maximum(s, 0.0)


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
