"""Python binding of libd2 with the C ABI's names.

Argument marshalling only: tensors are turned into device pointers and the
current torch stream is passed down; every step of the computation runs in
the HIP kernels.  Torch provides the device memory (outputs, workspace) and
the stream.

    h = Handle(0)
    X = DeviceSet.from_ragged(ragged, device)          # offsets/points/weights on the GPU
    labels, best, all_, status = d2_assign(h, X, Z)
    dist, status = d2_emd_batch(h, A, B, pairs)[:2]
    condensed, status = d2_pairwise(h, X)
    tiles, tile_offsets = d2_cost_tiles(h, A, B, pairs)
    z_new, eps1, eps3, counts, status = d2_centroid_update(h, X, Z, labels)
    Z, labels, history = constrained_d2(h, X, Z0)      # Alg. 2 with Step 3*
    dist, status, (plan, plan_off) = d2_emd_cost_batch(h, row_off, row_w, col_off, col_w,
                                                       costs, cost_off)
    mm2, M, plan = d2_mm_distance(h, Z1, p1, Z2, p2)   # Eq. (10)
    labels, best, all_, status = d2_assign_multi(h, [X_colour, X_texture], [Z_colour, Z_texture])
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional

import torch

from . import _ffi
from ._ffi import check


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


@dataclasses.dataclass
class DeviceSet:
    """A ragged set resident on the GPU (see d2_set in include/d2.h)."""
    offsets: torch.Tensor   # int64 [n+1]
    points: torch.Tensor    # float64|float32 [offsets[n], d]
    weights: torch.Tensor   # same dtype [offsets[n]]
    max_support: int

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0]) - 1

    @property
    def d(self) -> int:
        return int(self.points.shape[1])

    @classmethod
    def from_ragged(cls, s, device="cuda:0") -> "DeviceSet":
        """From any object with numpy ``offsets``, ``points``, ``weights``."""
        off = torch.as_tensor(s.offsets, dtype=torch.int64)
        sizes = off[1:] - off[:-1]
        ms = int(sizes.max()) if sizes.numel() else 1
        pts = torch.as_tensor(s.points)
        if pts.dtype not in (torch.float32, torch.float64):
            pts = pts.to(torch.float64)
        w = torch.as_tensor(s.weights).to(pts.dtype)
        return cls(off.to(device), pts.reshape(off[-1].item() if off.numel() else 0, -1)
                   .contiguous().to(device), w.contiguous().to(device), max(ms, 1))

    def with_points(self, points: torch.Tensor) -> "DeviceSet":
        """The same supports and weights at new atom coordinates (the weights
        are converted to the points' dtype)."""
        return DeviceSet(self.offsets, points.contiguous(),
                         self.weights.to(points.dtype).contiguous(), self.max_support)

    def c(self) -> _ffi.d2_set:
        if self.points.dtype == torch.float64:
            dt = _ffi.D2_F64
        elif self.points.dtype == torch.float32:
            dt = _ffi.D2_F32
        else:
            raise TypeError("points must be float32 or float64")
        if self.weights.dtype != self.points.dtype:
            raise TypeError("weights and points must share a dtype")
        for t in (self.offsets, self.points, self.weights):
            if not t.is_contiguous():
                raise ValueError("set tensors must be contiguous")
        return _ffi.d2_set(self.n, self.d, dt, self.offsets.data_ptr(), self.points.data_ptr(),
                           self.weights.data_ptr(), int(self.max_support), 0)


@dataclasses.dataclass
class Opts:
    cost_mode: int = _ffi.D2_COST_F64_DIRECT
    init: int = _ffi.D2_INIT_AUTO
    max_pivots: int = 0
    want_sqrt: int = 0
    opt_tol: float = 0.0
    schedule: int = _ffi.D2_SCHED_AUTO
    flags: int = 0
    bland_after: int = 0

    def c(self) -> _ffi.d2_opts:
        return _ffi.d2_opts(self.cost_mode, self.init, self.max_pivots, self.want_sqrt,
                            self.opt_tol, self.schedule, self.flags, self.bland_after)


class Handle:
    """Owns a d2_handle bound to one GPU."""

    def __init__(self, device: int = 0):
        self.device = device
        h = ctypes.c_void_p()
        check(_ffi.lib().d2_create(ctypes.byref(h), device), "d2_create")
        self._h = h

    @property
    def ptr(self):
        return self._h

    def close(self):
        if self._h:
            _ffi.lib().d2_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dev(h: Handle) -> torch.device:
    return torch.device("cuda", h.device)


def d2_workspace_bytes(h: Handle, which: int, A: DeviceSet, B: Optional[DeviceSet] = None,
                       npairs: int = 0, opts: Optional[Opts] = None) -> int:
    a = A.c()
    b = B.c() if B is not None else None
    o = (opts or Opts()).c()
    return int(_ffi.lib().d2_workspace_bytes(h.ptr, which, ctypes.byref(a),
                                              ctypes.byref(b) if b is not None else None, npairs,
                                              ctypes.byref(o)))


def _workspace(h, which, A, B, npairs, opts):
    nbytes = d2_workspace_bytes(h, which, A, B, npairs, opts)
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=_dev(h))
    return ws, nbytes


def d2_assign(h: Handle, X: DeviceSet, Z: DeviceSet, opts: Optional[Opts] = None,
              want_all: bool = False):
    """labels[n] int32, best[n] f64, all[n,K] f64 or None, row_status[n] int32."""
    opts = opts or Opts()
    dev = _dev(h)
    n, K = X.n, Z.n
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    best = torch.empty(n, dtype=torch.float64, device=dev)
    allv = torch.empty((n, K), dtype=torch.float64, device=dev) if want_all else None
    status = torch.empty(n, dtype=torch.int32, device=dev)
    ws, nbytes = _workspace(h, _ffi.WHICH_ASSIGN, X, Z, 0, opts)
    x, z, o = X.c(), Z.c(), opts.c()
    check(_ffi.lib().d2_assign(h.ptr, ctypes.byref(x), ctypes.byref(z), ctypes.byref(o),
                               _ptr(labels), _ptr(best), _ptr(allv), _ptr(status), _ptr(ws),
                               nbytes, _stream(dev)), "d2_assign")
    return labels, best, allv, status


def d2_assign_into(h: Handle, X: DeviceSet, Z: DeviceSet, opts: Optional[Opts],
                   labels: torch.Tensor, best: torch.Tensor, all_: Optional[torch.Tensor],
                   status: Optional[torch.Tensor], ws: Optional[torch.Tensor], ws_bytes: int):
    """d2_assign into caller-provided tensors, on the current torch stream."""
    opts = opts or Opts()
    x, z, o = X.c(), Z.c(), opts.c()
    check(_ffi.lib().d2_assign(h.ptr, ctypes.byref(x), ctypes.byref(z), ctypes.byref(o),
                               _ptr(labels), _ptr(best), _ptr(all_), _ptr(status), _ptr(ws),
                               ws_bytes, _stream(_dev(h))), "d2_assign")


def _pair_sizes(A: DeviceSet, B: DeviceSet, pairs: torch.Tensor):
    sa = (A.offsets[1:] - A.offsets[:-1])[pairs[:, 0]]
    sb = (B.offsets[1:] - B.offsets[:-1])[pairs[:, 1]]
    return sa, sb


def _offsets_of(sizes: torch.Tensor) -> torch.Tensor:
    off = torch.zeros(sizes.numel() + 1, dtype=torch.int64, device=sizes.device)
    off[1:] = torch.cumsum(sizes, 0)
    return off


def d2_emd_batch(h: Handle, A: DeviceSet, B: DeviceSet, pairs: torch.Tensor,
                 opts: Optional[Opts] = None, want_plan: bool = False, want_duals: bool = False,
                 want_pivots: bool = False):
    """dist[m], status[m], and (plan, plan_offsets), (duals, dual_offsets) when asked;
    with ``want_pivots`` a fifth item, pivots[m, 2] int32 (pivots taken, of which
    under Bland's rule)."""
    opts = opts or Opts()
    dev = _dev(h)
    pairs = pairs.to(device=dev, dtype=torch.int64).reshape(-1, 2).contiguous()
    m = int(pairs.shape[0])
    dist = torch.empty(m, dtype=torch.float64, device=dev)
    status = torch.empty(m, dtype=torch.int32, device=dev)
    plan = plan_off = duals = dual_off = None
    if want_plan or want_duals:
        sa, sb = _pair_sizes(A, B, pairs)
        if want_plan:
            plan_off = _offsets_of(sa * sb)
            plan = torch.empty(int(plan_off[-1].item()) if m else 0, dtype=torch.float64,
                               device=dev)
        if want_duals:
            dual_off = _offsets_of(sa + sb)
            duals = torch.empty(int(dual_off[-1].item()) if m else 0, dtype=torch.float64,
                                device=dev)
    piv = torch.empty((m, 2), dtype=torch.int32, device=dev) if want_pivots else None
    ws, nbytes = _workspace(h, _ffi.WHICH_EMD_BATCH, A, B, m, opts)
    a, b, o = A.c(), B.c(), opts.c()
    check(_ffi.lib().d2_emd_batch(h.ptr, ctypes.byref(a), ctypes.byref(b), _ptr(pairs), m,
                                  ctypes.byref(o), _ptr(dist), _ptr(plan_off), _ptr(plan),
                                  _ptr(dual_off), _ptr(duals), _ptr(status), _ptr(piv), _ptr(ws),
                                  nbytes, _stream(dev)), "d2_emd_batch")
    if want_pivots:
        return dist, status, (plan, plan_off), (duals, dual_off), piv
    return dist, status, (plan, plan_off), (duals, dual_off)


def d2_emd_batch_basis(h: Handle, A: DeviceSet, B: DeviceSet, pairs: torch.Tensor,
                       opts: Optional[Opts] = None):
    """dist[m], status[m], and each pair's optimal basis: cells [c, 2] int32
    (A atom, B atom), flows [c] f64 and offsets [m + 1] int64, pair k's
    t + s - 1 cells at offsets[k] (sorted; see d2_emd_batch_basis in d2.h)."""
    opts = opts or Opts()
    dev = _dev(h)
    pairs = pairs.to(device=dev, dtype=torch.int64).reshape(-1, 2).contiguous()
    m = int(pairs.shape[0])
    dist = torch.empty(m, dtype=torch.float64, device=dev)
    status = torch.empty(m, dtype=torch.int32, device=dev)
    sa, sb = _pair_sizes(A, B, pairs)
    off = _offsets_of(sa + sb - 1)
    cells = int(off[-1].item()) if m else 0
    ij = torch.full((cells, 2), -1, dtype=torch.int32, device=dev)
    w = torch.full((cells,), float("nan"), dtype=torch.float64, device=dev)
    a, b, o = A.c(), B.c(), opts.c()
    check(_ffi.lib().d2_emd_batch_basis(h.ptr, ctypes.byref(a), ctypes.byref(b), _ptr(pairs), m,
                                        ctypes.byref(o), _ptr(dist), _ptr(off), _ptr(ij), _ptr(w),
                                        _ptr(status), _stream(dev)), "d2_emd_batch_basis")
    return dist, status, ij, w, off


def d2_pairwise(h: Handle, X: DeviceSet, opts: Optional[Opts] = None):
    """condensed[n(n-1)/2] f64 (squareform order), status (same shape)."""
    opts = opts or Opts()
    dev = _dev(h)
    m = X.n * (X.n - 1) // 2
    out = torch.empty(m, dtype=torch.float64, device=dev)
    status = torch.empty(m, dtype=torch.int32, device=dev)
    ws, nbytes = _workspace(h, _ffi.WHICH_PAIRWISE, X, None, 0, opts)
    x, o = X.c(), opts.c()
    check(_ffi.lib().d2_pairwise(h.ptr, ctypes.byref(x), ctypes.byref(o), _ptr(out),
                                 _ptr(status), _ptr(ws), nbytes, _stream(dev)), "d2_pairwise")
    return out, status


def d2_tune_pairwise(h: Handle, X: DeviceSet, opts: Optional[Opts] = None):
    """Autotune the pairwise schedule for this workload shape (synchronous).
    Returns (condensed, status, best_ms) of the fastest run."""
    opts = opts or Opts()
    dev = _dev(h)
    m = X.n * (X.n - 1) // 2
    out = torch.empty(m, dtype=torch.float64, device=dev)
    status = torch.empty(m, dtype=torch.int32, device=dev)
    ws, nbytes = _workspace(h, _ffi.WHICH_PAIRWISE, X, None, 0, opts)
    x, o = X.c(), opts.c()
    best = ctypes.c_double()
    check(_ffi.lib().d2_tune_pairwise(h.ptr, ctypes.byref(x), ctypes.byref(o), _ptr(out),
                                      _ptr(status), _ptr(ws), nbytes, _stream(dev),
                                      ctypes.byref(best)), "d2_tune_pairwise")
    return out, status, best.value


def d2_cost_tiles(h: Handle, A: DeviceSet, B: DeviceSet, pairs: torch.Tensor,
                  cost_mode: int = _ffi.D2_COST_F64_DIRECT):
    """tiles (ragged, row-major t_i x s_j per pair), tile_offsets[m+1]."""
    dev = _dev(h)
    pairs = pairs.to(device=dev, dtype=torch.int64).reshape(-1, 2).contiguous()
    m = int(pairs.shape[0])
    sa, sb = _pair_sizes(A, B, pairs)
    off = _offsets_of(sa * sb)
    tiles = torch.empty(int(off[-1].item()) if m else 0, dtype=torch.float64, device=dev)
    ws, nbytes = _workspace(h, _ffi.WHICH_COST_TILES, A, B, m, None)
    a, b = A.c(), B.c()
    check(_ffi.lib().d2_cost_tiles(h.ptr, ctypes.byref(a), ctypes.byref(b), _ptr(pairs), m,
                                   cost_mode, _ptr(tiles), _ptr(off), _ptr(ws), nbytes,
                                   _stream(dev)), "d2_cost_tiles")
    return tiles, off


def d2_centroid_update(h: Handle, X: DeviceSet, Z: DeviceSet, labels: torch.Tensor,
                       opts: Optional[Opts] = None, weights: Optional[torch.Tensor] = None):
    """One pass of the constrained D2 centroid update (Alg. 2 Step 3*), with
    optional object weights (weighted D2-clustering, Eq. (3)-(4)).

    Returns z_new [Z.offsets[K], d] f64, eps_step1 [K] f64, eps_step3 [K] f64,
    counts [K] int32, status [n] int32 (see d2_centroid_update in d2.h)."""
    opts = opts or Opts()
    dev = _dev(h)
    labels = labels.to(device=dev, dtype=torch.int32).contiguous()
    if weights is not None:
        weights = weights.to(device=dev, dtype=torch.float64).contiguous()
    K = Z.n
    z_new = torch.empty((int(Z.points.shape[0]), Z.d), dtype=torch.float64, device=dev)
    eps1 = torch.empty(K, dtype=torch.float64, device=dev)
    eps3 = torch.empty(K, dtype=torch.float64, device=dev)
    counts = torch.empty(K, dtype=torch.int32, device=dev)
    status = torch.empty(X.n, dtype=torch.int32, device=dev)
    ws, nbytes = _workspace(h, _ffi.WHICH_UPDATE, X, Z, 0, opts)
    x, z, o = X.c(), Z.c(), opts.c()
    check(_ffi.lib().d2_centroid_update(h.ptr, ctypes.byref(x), ctypes.byref(z), _ptr(labels),
                                        _ptr(weights), ctypes.byref(o), _ptr(z_new), _ptr(eps1),
                                        _ptr(eps3),
                                        _ptr(counts), _ptr(status), _ptr(ws), nbytes,
                                        _stream(dev)), "d2_centroid_update")
    return z_new, eps1, eps3, counts, status


def d2_centroid_update_free(h: Handle, X: DeviceSet, Z: DeviceSet, labels: torch.Tensor,
                            opts: Optional[Opts] = None, weights: Optional[torch.Tensor] = None,
                            max_members: Optional[int] = None, want_pivots: bool = False,
                            basis: Optional[torch.Tensor] = None):
    """One pass of the centroid update of Alg. 1 with free centroid weights
    (Steps 1-3; object weights as in Eq. (3)-(4)).

    max_members bounds the members of one cluster (None: the largest count
    among the labels, read back once).  Returns z_new [Z.offsets[K], d] f64,
    w_new [Z.offsets[K]] f64, eps_step1 [K], eps_step3 [K] f64, counts [K],
    obj_status [n], cluster_status [K] int32 (see d2_centroid_update_free in
    d2.h); with ``want_pivots`` also the simplex pivots of each cluster
    [K] int32.  ``basis`` (device int32 [K, stride], see free_basis_buffer)
    carries each cluster's optimal basis to the next call as its start."""
    opts = opts or Opts()
    dev = _dev(h)
    labels = labels.to(device=dev, dtype=torch.int32).contiguous()
    if weights is not None:
        weights = weights.to(device=dev, dtype=torch.float64).contiguous()
    K = Z.n
    if max_members is None:
        inr = labels[(labels >= 0) & (labels < K)].to(torch.int64)
        max_members = int(torch.bincount(inr, minlength=1).max().item()) if inr.numel() else 1
    max_members = max(1, int(max_members))
    z_new = torch.empty((int(Z.points.shape[0]), Z.d), dtype=torch.float64, device=dev)
    w_new = torch.empty(int(Z.points.shape[0]), dtype=torch.float64, device=dev)
    eps1 = torch.empty(K, dtype=torch.float64, device=dev)
    eps3 = torch.empty(K, dtype=torch.float64, device=dev)
    counts = torch.empty(K, dtype=torch.int32, device=dev)
    status = torch.empty(X.n, dtype=torch.int32, device=dev)
    cstatus = torch.empty(K, dtype=torch.int32, device=dev)
    piv = torch.empty(K, dtype=torch.int32, device=dev) if want_pivots else None
    ws, nbytes = _workspace(h, _ffi.WHICH_UPDATE_FREE, X, Z, max_members, opts)
    if basis is not None:
        if basis.dtype != torch.int32 or basis.dim() != 2 or basis.shape[0] != K or not basis.is_contiguous():
            raise ValueError("basis must be a contiguous int32 [K, stride] tensor")
    stride = int(basis.shape[1]) if basis is not None else 0
    x, z, o = X.c(), Z.c(), opts.c()
    check(_ffi.lib().d2_centroid_update_free(h.ptr, ctypes.byref(x), ctypes.byref(z), _ptr(labels),
                                             _ptr(weights), max_members, ctypes.byref(o),
                                             _ptr(z_new), _ptr(w_new), _ptr(eps1), _ptr(eps3),
                                             _ptr(counts), _ptr(status), _ptr(cstatus), _ptr(piv),
                                             _ptr(basis), stride, _ptr(ws), nbytes, _stream(dev)),
          "d2_centroid_update_free")
    if want_pivots:
        return z_new, w_new, eps1, eps3, counts, status, cstatus, piv
    return z_new, w_new, eps1, eps3, counts, status, cstatus


def free_basis_buffer(X: DeviceSet, Z: DeviceSet, max_members: int) -> torch.Tensor:
    """Starting-basis rows for d2_centroid_update_free, all -1 (no kept
    basis): one row per centroid, wide enough for a program of up to
    max_members members (max_members (max_support(X) + max_support(Z) - 1)
    + 1 rows, plus the count)."""
    stride = int(max_members) * (X.max_support + Z.max_support - 1) + 2
    return torch.full((Z.n, stride), -1, dtype=torch.int32, device=Z.points.device)


def d2_merge_level(h: Handle, Z: DeviceSet, labels: torch.Tensor, omega: Optional[torch.Tensor],
                   C: torch.Tensor):
    """One level's merge of Alg. 3 Step 3 (Eq. (5)-(6)): the centroids of Z
    with members among the level objects (labels [n]) become the next
    level's objects, renumbered in index order, each weighted by the sum of
    its members' omega (None: 1 each); C [n0] (the level object of every
    original object) is replaced by the inherited labels.  Returns (the next
    level's objects as a DeviceSet, their weights [kept] f64, the new C
    [n0] int32, host offsets [kept + 1] int64)."""
    dev = _dev(h)
    labels = labels.to(device=dev, dtype=torch.int32).contiguous()
    if omega is not None:
        omega = omega.to(device=dev, dtype=torch.float64).contiguous()
    C = C.to(device=dev, dtype=torch.int32).clone()
    K = Z.n
    kept = torch.empty(1, dtype=torch.int64, device=dev)
    off = torch.empty(K + 1, dtype=torch.int64, device=dev)
    pts = torch.empty_like(Z.points)
    wts = torch.empty(int(Z.points.shape[0]), dtype=Z.points.dtype, device=dev)
    new_omega = torch.empty(max(K, 1), dtype=torch.float64, device=dev)
    ws, nbytes = _workspace(h, _ffi.WHICH_MERGE, Z, None, labels.numel(), None)
    z = Z.c()
    check(_ffi.lib().d2_merge_level(h.ptr, ctypes.byref(z), labels.numel(), _ptr(labels), _ptr(omega),
                                    C.numel(), _ptr(C), _ptr(kept), _ptr(off), _ptr(pts), _ptr(wts),
                                    _ptr(new_omega), _ptr(ws), nbytes, _stream(dev)),
          "d2_merge_level")
    q = int(kept.item())
    off_h = off[:q + 1].cpu().numpy()
    sizes = off_h[1:] - off_h[:-1]
    na = int(off_h[-1])
    G = DeviceSet(off[:q + 1].clone(), pts[:na].clone(), wts[:na].clone(), int(sizes.max()) if q else 1)
    return G, new_omega[:q].clone(), C, off_h


def constrained_d2(h: Handle, X: DeviceSet, Z: DeviceSet, opts: Optional[Opts] = None,
                   max_rounds: int = 20, max_passes: int = 10, rtol: float = 1e-9):
    """Constrained D2-clustering (Alg. 2 with Step 3* in place of Step 3).

    Each round labels every object by its nearest centroid (Step 2, d2_assign),
    then repeats the fixed-weight centroid update (Step 3*, d2_centroid_update)
    until its objective changes by at most rtol relative (Alg. 1 Step 3); the
    rounds stop when the clustering objective eps(C) = sum_j eps_j does
    (Step 4).  The centroid weights are kept as given (uniform in the paper).
    Host control only: every step runs in the library.  FP32 inputs are
    widened to FP64 once, since the moved atoms are FP64.

    Returns (Z, labels, history) with history a list of (round, passes,
    eps(C)) tuples.
    """
    if X.points.dtype != torch.float64:
        X = X.with_points(X.points.double())
    if Z.points.dtype != torch.float64:
        Z = Z.with_points(Z.points.double())
    history = []
    labels = None
    prev_round = None
    for rnd in range(max_rounds):
        labels, _, _, row_status = d2_assign(h, X, Z, opts)                 # Step 2
        prev = None
        passes = 0
        eps = None
        for passes in range(1, max_passes + 1):                              # Step 3*
            z_new, _, eps3, _, _ = d2_centroid_update(h, X, Z, labels, opts)
            Z = Z.with_points(z_new)
            eps = float(eps3.sum().item())
            if prev is not None and abs(prev - eps) <= rtol * max(abs(eps), 1e-300):
                break
            prev = eps
        history.append((rnd, passes, eps))
        if prev_round is not None and abs(prev_round - eps) <= rtol * max(abs(eps), 1e-300):
            break                                                            # Step 4
        prev_round = eps
    return Z, labels, history


def d2_emd_cost_batch(h: Handle, row_offsets: torch.Tensor, row_weights: torch.Tensor,
                      col_offsets: torch.Tensor, col_weights: torch.Tensor, costs: torch.Tensor,
                      cost_offsets: torch.Tensor, max_rows: Optional[int] = None,
                      max_cols: Optional[int] = None, opts: Optional[Opts] = None,
                      want_plan: bool = False):
    """Transport LPs over given FP64 cost matrices (see d2_emd_cost_batch in
    d2.h).  Returns dist[m], status[m], (plan, plan_offsets)."""
    opts = opts or Opts()
    dev = _dev(h)

    def prep(t, dt):
        return t.to(device=dev, dtype=dt).contiguous()

    roff, coff = prep(row_offsets, torch.int64), prep(col_offsets, torch.int64)
    rw, cw = prep(row_weights, torch.float64), prep(col_weights, torch.float64)
    C, moff = prep(costs, torch.float64).reshape(-1), prep(cost_offsets, torch.int64)
    m = int(roff.numel()) - 1
    rs = roff[1:] - roff[:-1]
    cs = coff[1:] - coff[:-1]
    if max_rows is None:
        max_rows = int(rs.max().item()) if m > 0 else 1
    if max_cols is None:
        max_cols = int(cs.max().item()) if m > 0 else 1
    dist = torch.empty(m, dtype=torch.float64, device=dev)
    status = torch.empty(m, dtype=torch.int32, device=dev)
    plan = plan_off = None
    if want_plan:
        plan_off = _offsets_of(rs * cs)
        plan = torch.empty(int(plan_off[-1].item()) if m else 0, dtype=torch.float64, device=dev)
    o = opts.c()
    check(_ffi.lib().d2_emd_cost_batch(h.ptr, m, _ptr(roff), _ptr(rw), _ptr(coff), _ptr(cw), _ptr(C),
                                       _ptr(moff), int(max_rows), int(max_cols), ctypes.byref(o),
                                       _ptr(dist), _ptr(plan_off), _ptr(plan), _ptr(status), None, 0,
                                       _stream(dev)), "d2_emd_cost_batch")
    return dist, status, (plan, plan_off)


def d2_mm_distance(h: Handle, Z1: DeviceSet, p1: torch.Tensor, Z2: DeviceSet, p2: torch.Tensor,
                   opts: Optional[Opts] = None):
    """Squared MM distance of Eq. (10) between two centroid sets with cluster
    proportions p1, p2: every D^2(z_i, z'_j) by d2_assign, then the transport
    LP over the clusters on that matrix by d2_emd_cost_batch (both set sizes
    at most 64).  Returns (MM^2 as a 0-d tensor, M [k1, k2], plan [k1, k2])."""
    opts = opts or Opts()
    dev = _dev(h)
    k1, k2 = Z1.n, Z2.n
    _, _, M, st = d2_assign(h, Z1, Z2, opts, want_all=True)
    off1 = torch.tensor([0, k1], dtype=torch.int64, device=dev)
    off2 = torch.tensor([0, k2], dtype=torch.int64, device=dev)
    zero = torch.zeros(1, dtype=torch.int64, device=dev)
    dist, status, (plan, _) = d2_emd_cost_batch(h, off1, p1, off2, p2, M, zero, k1, k2, opts,
                                                want_plan=True)
    return dist[0], M, plan.reshape(k1, k2)


def d2_assign_multi(h: Handle, Xs, Zs, opts: Optional[Opts] = None, want_all: bool = False):
    """Nearest-centroid labels under the combined distance of Eq. (9): the sum
    over feature types of the per-type D^2.  Xs, Zs: lists of DeviceSet, one
    per type.  Returns labels[n], best[n], all[n, K] or None, row_status[n]."""
    opts = opts or Opts()
    dev = _dev(h)
    m = len(Xs)
    if m != len(Zs) or m < 1:
        raise ValueError("one centroid set per object set")
    xs = (_ffi.d2_set * m)(*[X.c() for X in Xs])
    zs = (_ffi.d2_set * m)(*[Z.c() for Z in Zs])
    n, K = Xs[0].n, Zs[0].n
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    best = torch.empty(n, dtype=torch.float64, device=dev)
    allv = torch.empty((n, K), dtype=torch.float64, device=dev) if want_all else None
    status = torch.empty(n, dtype=torch.int32, device=dev)
    o = opts.c()
    nbytes = int(_ffi.lib().d2_workspace_bytes(h.ptr, _ffi.WHICH_MULTI, xs, zs, m, ctypes.byref(o)))
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    check(_ffi.lib().d2_assign_multi(h.ptr, m, xs, zs, ctypes.byref(o), _ptr(labels), _ptr(best),
                                     _ptr(allv), _ptr(status), _ptr(ws), nbytes, _stream(dev)),
          "d2_assign_multi")
    return labels, best, allv, status


def d2_assign_segmented(h: Handle, X: DeviceSet, Z: DeviceSet, seg: torch.Tensor,
                        zseg_offsets: torch.Tensor, opts: Optional[Opts] = None):
    """Nearest centroid of each object among its own segment's centroids
    (Alg. 3 Step 2).  seg[n]: segment of each object; zseg_offsets[nseg+1]:
    each segment's range of Z.  Returns labels[n] (global centroid index),
    best[n], row_status[n]."""
    opts = opts or Opts()
    dev = _dev(h)
    seg = seg.to(device=dev, dtype=torch.int32).contiguous()
    zoff = zseg_offsets.to(device=dev, dtype=torch.int64).contiguous()
    n = X.n
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    best = torch.empty(n, dtype=torch.float64, device=dev)
    status = torch.empty(n, dtype=torch.int32, device=dev)
    x, z, o = X.c(), Z.c(), opts.c()
    check(_ffi.lib().d2_assign_segmented(h.ptr, ctypes.byref(x), ctypes.byref(z), _ptr(seg),
                                         int(zoff.numel()) - 1, _ptr(zoff), ctypes.byref(o),
                                         _ptr(labels), _ptr(best), _ptr(status), _stream(dev)),
          "d2_assign_segmented")
    return labels, best, status
