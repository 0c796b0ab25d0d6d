"""Plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``emd_oracle.c`` (a plain transportation
simplex, see that file's header for the steps and their source in the paper)
with ctypes, and widens every input to FP64 exactly before the call.

    emd_pair(x, p, y, q)              -> (D^2, plan[t,s], u[t], v[s], pivots)
    emd_batch(A, B, pairs)            -> (D^2[npairs], status, pivots)
    emd_batch_stats(A, B, pairs)      -> (D^2[npairs], status, pivots, Bland pivots)
    assign(X, Z)                      -> (labels, best, all[n,K], status, pivots)
    pairwise(X)                       -> (condensed D^2, status, pivots)
    centroid_update(X, Z, labels)     -> (z_new, eps_step1, eps_step3, status)
                                         (``update.py``: Alg. 2 Step 3*)
    emd_cost(C, p, q)                 -> (value, plan, u, v, pivots), given cost
    mm_distance(Z1, p1, Z2, p2)       -> (MM^2, D^2 matrix, plan)  (``mm.py``: Eq. (10))
    assign_multi(Xs, Zs)              -> (labels, best, summed all, status)  (``multi.py``: Eq. (9))

Sets are ``synth.RaggedSet``-like objects with ``offsets``, ``points``,
``weights``.  Labels follow Alg. 2 Step 2 (argmin over centroids, ties to the
lowest index, -1 when any pair of the row failed).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "emd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

INIT_NWC = 0
INIT_VOGEL = 1

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, -O2, pthreads)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-pthread",
                               "-o", tmp, _SRC, "-lm"], cwd=_HERE)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    lib.oracle_emd_pair.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P, P,
                                    ctypes.c_int, ctypes.c_int, P, P, P, P, P, P]
    lib.oracle_emd_cost.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int,
                                    ctypes.c_int, P, P, P, P, P, P]
    lib.oracle_emd_batch.argtypes = [ctypes.c_int, P, P, P, I64, P, P, P, I64, P, I64,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P, P]
    lib.oracle_assign.argtypes = [ctypes.c_int, P, P, P, I64, P, P, P, I64, ctypes.c_int,
                                  ctypes.c_int, P, P, P, P, P, P]
    lib.oracle_pairwise.argtypes = [ctypes.c_int, P, P, P, I64, ctypes.c_int, ctypes.c_int,
                                    P, P, P, P]
    for f in (lib.oracle_emd_pair, lib.oracle_emd_cost, lib.oracle_emd_batch, lib.oracle_assign,
              lib.oracle_pairwise):
        f.restype = ctypes.c_int
    _lib = lib
    return lib


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return max(1, os.cpu_count() or 1)


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _set(S):
    off = np.ascontiguousarray(S.offsets, dtype=np.int64)
    pts = _f64(S.points)
    d = pts.shape[1] if pts.ndim == 2 else 1
    return off, pts.reshape(-1, d), _f64(S.weights).reshape(-1), off.shape[0] - 1, d


def emd_pair(x, p, y, q, init: int = INIT_NWC, stats: bool = False, bland_after: int = 0):
    """(D^2, plan[t,s], u[t], v[s], pivots); with ``stats`` also the number of
    pivots taken under Bland's rule.  ``bland_after``: the run of degenerate
    pivots that switches to Bland's rule (0 = the default 2(t+s))."""
    lib = _load()
    x = _f64(x); y = _f64(y)
    x = x.reshape(x.shape[0], -1); y = y.reshape(y.shape[0], -1)
    p = _f64(p).reshape(-1); q = _f64(q).reshape(-1)
    t, d = x.shape
    s = y.shape[0]
    if y.shape[1] != d or p.size != t or q.size != s:
        raise ValueError("shape mismatch")
    d2 = np.zeros(1)
    plan = np.zeros((t, s))
    u = np.zeros(t)
    v = np.zeros(s)
    piv = np.zeros(1, dtype=np.int64)
    bl = np.zeros(1, dtype=np.int64)
    st = lib.oracle_emd_pair(t, s, d, _p(x), _p(p), _p(y), _p(q), init, bland_after, _p(d2),
                             _p(plan), _p(u), _p(v), _p(piv), _p(bl))
    if st != 0:
        err = ArithmeticError(f"oracle status {st}")
        err.status = st
        raise err
    if stats:
        return float(d2[0]), plan, u, v, int(piv[0]), int(bl[0])
    return float(d2[0]), plan, u, v, int(piv[0])


def emd_cost(C, p, q, init: int = INIT_NWC, stats: bool = False, bland_after: int = 0):
    """The transport LP with the given t x s cost matrix (any finite values):
    (value, plan[t,s], u[t], v[s], pivots); with ``stats`` also the number of
    pivots taken under Bland's rule."""
    lib = _load()
    C = _f64(C)
    t, s = C.shape
    p = _f64(p).reshape(-1); q = _f64(q).reshape(-1)
    if p.size != t or q.size != s:
        raise ValueError("shape mismatch")
    val = np.zeros(1)
    plan = np.zeros((t, s))
    u = np.zeros(t)
    v = np.zeros(s)
    piv = np.zeros(1, dtype=np.int64)
    bl = np.zeros(1, dtype=np.int64)
    st = lib.oracle_emd_cost(t, s, _p(C), _p(p), _p(q), init, bland_after, _p(val), _p(plan),
                             _p(u), _p(v), _p(piv), _p(bl))
    if st != 0:
        err = ArithmeticError(f"oracle status {st}")
        err.status = st
        raise err
    if stats:
        return float(val[0]), plan, u, v, int(piv[0]), int(bl[0])
    return float(val[0]), plan, u, v, int(piv[0])


def emd_batch(A, B, pairs, init: int = INIT_NWC, threads: int | None = None):
    dist, status, piv, _ = emd_batch_stats(A, B, pairs, init, threads)
    return dist, status, piv


def emd_batch_stats(A, B, pairs, init: int = INIT_NWC, threads: int | None = None,
                    bland_after: int = 0):
    """(D^2[npairs], status, pivots, pivots taken under Bland's rule)."""
    lib = _load()
    oa, xa, wa, na, d = _set(A)
    ob, xb, wb, nb, db = _set(B)
    if d != db:
        raise ValueError("dimension mismatch")
    pairs = np.ascontiguousarray(pairs, dtype=np.int64).reshape(-1, 2)
    m = pairs.shape[0]
    dist = np.full(m, np.nan)
    status = np.zeros(m, dtype=np.int32)
    piv = np.zeros(m, dtype=np.int64)
    bl = np.zeros(m, dtype=np.int64)
    rc = lib.oracle_emd_batch(d, _p(oa), _p(xa), _p(wa), na, _p(ob), _p(xb), _p(wb), nb,
                              _p(pairs), m, init, bland_after, threads or default_threads(),
                              _p(dist), _p(status), _p(piv), _p(bl))
    if rc != 0:
        raise RuntimeError(f"oracle_emd_batch failed ({rc})")
    return dist, status, piv, bl


def assign(X, Z, init: int = INIT_NWC, threads: int | None = None, want_all: bool = True):
    lib = _load()
    ox, xx, wx, nx, d = _set(X)
    oz, xz, wz, nz, dz = _set(Z)
    if d != dz:
        raise ValueError("dimension mismatch")
    labels = np.zeros(nx, dtype=np.int32)
    best = np.zeros(nx)
    allv = np.full((nx, nz), np.nan) if want_all else None
    status = np.zeros(nx, dtype=np.int32)
    piv = np.zeros((nx, nz), dtype=np.int64) if want_all else None
    rc = lib.oracle_assign(d, _p(ox), _p(xx), _p(wx), nx, _p(oz), _p(xz), _p(wz), nz, init,
                           threads or default_threads(), _p(labels), _p(best), _p(allv),
                           _p(status), _p(piv), None)
    if rc != 0:
        raise RuntimeError(f"oracle_assign failed ({rc})")
    return labels, best, allv, status, piv


def pairwise(X, init: int = INIT_NWC, threads: int | None = None):
    lib = _load()
    ox, xx, wx, nx, d = _set(X)
    m = nx * (nx - 1) // 2
    out = np.full(m, np.nan)
    status = np.zeros(m, dtype=np.int32)
    piv = np.zeros(m, dtype=np.int64)
    rc = lib.oracle_pairwise(d, _p(ox), _p(xx), _p(wx), nx, init, threads or default_threads(),
                             _p(out), _p(status), _p(piv), None)
    if rc != 0:
        raise RuntimeError(f"oracle_pairwise failed ({rc})")
    return out, status, piv


def independent_coupling_cost(x, p, y, q) -> float:
    """S = sum_a sum_b p_a q_b |x_a - y_b|^2 (normalised weights): the cost of
    the product plan, an upper bound on D^2 used as the parity floor scale."""
    x = _f64(x).reshape(len(p), -1); y = _f64(y).reshape(len(q), -1)
    p = _f64(p) / _f64(p).sum(); q = _f64(q) / _f64(q).sum()
    diff = x[:, None, :] - y[None, :, :]
    C = np.einsum("abk,abk->ab", diff, diff)
    return float(p @ C @ q)


from .update import centroid_update  # noqa: E402  (uses emd_pair above)
from .mm import mm_distance  # noqa: E402  (uses assign and emd_cost above)
from .multi import assign_multi  # noqa: E402  (uses assign above)
