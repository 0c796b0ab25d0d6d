"""GPU parity of d2_emd_batch_basis: each pair's optimal basis as sorted
(A atom, B atom, flow) cells, through the C ABI.

What is compared:
* the value is d2_emd_batch's, bit for bit (the same solver), and the
  oracle's within the parity tolerance;
* the cells are t + s - 1 distinct cells, sorted, forming a spanning tree
  of the t + s atoms (the shape of a transportation basis), with flows >= 0
  that meet both marginals and whose cost is the value;
* the dense plan d2_emd_batch returns holds exactly these flows on these
  cells (bitwise) and zeros elsewhere;
* on inputs in general position the optimal vertex is unique, so the
  oracle's positive plan cells are basis cells with the same flows.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.parity import REL

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"


@pytest.fixture(scope="module")
def d2():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests selected but no GPU is visible")
    import paper_1302_0435_amd as m
    m._ffi.lib()
    return m


@pytest.fixture(scope="module")
def h(d2):
    return d2.Handle(0)


def sets(seed, na, nb, lo_a, hi_a, lo_b, hi_b, d, grid=False):
    rng = np.random.default_rng([5151, seed])

    def bags(n, lo, hi):
        out = []
        for _ in range(n):
            t = int(rng.integers(lo, hi + 1))
            x = rng.normal(size=(t, d))
            w = rng.dirichlet(np.ones(t))
            if grid:
                x = np.round(x * 2.0)
                w = np.full(t, 1.0 / t)
            out.append((x, w))
        return synth.from_bags(out, np.float64)
    return bags(na, lo_a, hi_a), bags(nb, lo_b, hi_b)


def is_spanning_tree(cells, t, s):
    parent = list(range(t + s))

    def find(u):
        while parent[u] != u:
            parent[u] = parent[parent[u]]
            u = parent[u]
        return u
    for a, b in cells:
        ra, rb = find(int(a)), find(t + int(b))
        if ra == rb:
            return False
        parent[ra] = rb
    return len(cells) == t + s - 1


def check(d2, h, A, B, pairs, unique):
    Ad = d2.DeviceSet.from_ragged(A, DEV)
    Bd = d2.DeviceSet.from_ragged(B, DEV)
    P = torch.as_tensor(pairs, device=DEV)
    dist, st, ij, w, off = d2.d2_emd_batch_basis(h, Ad, Bd, P)
    dist2, st2, (plan, poff), _ = d2.d2_emd_batch(h, Ad, Bd, P, want_plan=True)
    torch.cuda.synchronize()
    dist, st, ij, w, off = (t.cpu().numpy() for t in (dist, st, ij, w, off))
    dist2, st2, plan, poff = (t.cpu().numpy() for t in (dist2, st2, plan, poff))
    assert np.all(st == 0) and np.array_equal(st, st2)
    assert np.array_equal(dist, dist2)
    for k, (i, j) in enumerate(pairs):
        x, p = A.bag(i)
        y, q = B.bag(j)
        t, s = len(p), len(q)
        c = ij[off[k]:off[k + 1]]
        f = w[off[k]:off[k + 1]]
        assert len(c) == t + s - 1
        assert np.all((c[:, 0] >= 0) & (c[:, 0] < t) & (c[:, 1] >= 0) & (c[:, 1] < s))
        keys = c[:, 0].astype(np.int64) * s + c[:, 1]
        assert np.all(np.diff(keys) > 0), "cells not sorted or repeated"
        assert is_spanning_tree(c, t, s)
        assert np.all(f >= 0.0)
        pn = np.asarray(p, np.float64) / np.sum(p)
        qn = np.asarray(q, np.float64) / np.sum(q)
        assert np.allclose(np.bincount(c[:, 0], weights=f, minlength=t), pn, rtol=0, atol=1e-12)
        assert np.allclose(np.bincount(c[:, 1], weights=f, minlength=s), qn, rtol=0, atol=1e-12)
        C = ((np.asarray(x, np.float64)[:, None, :] - np.asarray(y, np.float64)[None, :, :]) ** 2).sum(-1)
        dense = np.zeros((t, s))
        dense[c[:, 0], c[:, 1]] = f
        assert np.array_equal(plan[poff[k]:poff[k + 1]].reshape(t, s), dense)
        o_val, o_plan = oracle.emd_pair(x, p, y, q)[:2]
        scale = max(abs(o_val), 1e-4 * float((pn[:, None] * qn[None, :] * C).sum()))
        assert abs(dist[k] - o_val) <= REL * scale, (k, dist[k], o_val)
        assert abs(float((f * C[c[:, 0], c[:, 1]]).sum()) - o_val) <= REL * scale
        if unique:
            pos = np.argwhere(o_plan > 1e-13)
            assert np.all(dense[pos[:, 0], pos[:, 1]] > 0.0), k
            np.testing.assert_allclose(dense, o_plan, rtol=0, atol=1e-12)


@pytest.mark.parametrize("lo,hi,d", [(1, 16, 3), (17, 32, 4), (33, 64, 2)])
def test_basis_general_position(d2, h, lo, hi, d):
    A, B = sets(lo, 12, 9, lo, hi, 1, hi, d)
    pairs = np.array([(i, j) for i in range(A.n) for j in range(B.n)][::2], dtype=np.int64)
    check(d2, h, A, B, pairs, unique=True)


def test_basis_swapped_orientation_and_wide_pairs(d2, h):
    # A's objects smaller than B's: the solver swaps the sides
    A, B = sets(7, 10, 10, 1, 8, 33, 64, 3)
    pairs = np.array([(i, j) for i in range(A.n) for j in range(B.n)][::3], dtype=np.int64)
    check(d2, h, A, B, pairs, unique=True)


def test_basis_degenerate_grid(d2, h):
    # equal weights on integer points: many optimal plans and degenerate
    # (zero-flow) basic cells; the basis is still a spanning tree
    A, B = sets(9, 10, 10, 2, 24, 2, 24, 2, grid=True)
    pairs = np.array([(i, j) for i in range(A.n) for j in range(B.n)][::2], dtype=np.int64)
    check(d2, h, A, B, pairs, unique=False)


def test_basis_bad_pairs_and_errors(d2, h):
    import ctypes
    A, B = sets(11, 4, 4, 2, 6, 2, 6, 2)
    Ad = d2.DeviceSet.from_ragged(A, DEV)
    Bd = d2.DeviceSet.from_ragged(B, DEV)
    # an index out of range: status 2, its cells untouched
    bad = torch.tensor([[0, 0], [0, 0]], dtype=torch.int64, device=DEV)
    bad[1, 1] = 4
    dist_b = torch.empty(2, dtype=torch.float64, device=DEV)
    st_b = torch.empty(2, dtype=torch.int32, device=DEV)
    offb = torch.tensor([0, 12, 24], dtype=torch.int64, device=DEV)   # t + s - 1 <= 11
    ijb = torch.full((24, 2), -1, dtype=torch.int32, device=DEV)
    wb = torch.full((24,), float("nan"), dtype=torch.float64, device=DEV)
    L, F = d2._ffi.lib(), d2._ffi
    a, b, o = Ad.c(), Bd.c(), d2.Opts().c()
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    assert L.d2_emd_batch_basis(h.ptr, ctypes.byref(a), ctypes.byref(b), p(bad), 2, ctypes.byref(o), p(dist_b),
                                p(offb), p(ijb), p(wb), p(st_b), None) == F.D2_OK
    torch.cuda.synchronize()
    assert st_b.cpu().tolist()[1] == F.D2_PAIR_TOO_LARGE
    assert np.isnan(dist_b.cpu().numpy()[1])
    assert np.all(ijb[12:].cpu().numpy() == -1) and np.all(np.isnan(wb[12:].cpu().numpy()))
    t0, s0 = len(A.bag(0)[1]), len(B.bag(0)[1])
    assert np.all(ijb[:t0 + s0 - 1].cpu().numpy() >= 0)
    # null outputs, supports past the lane-group shapes
    assert L.d2_emd_batch_basis(h.ptr, ctypes.byref(a), ctypes.byref(b), p(bad), 2, ctypes.byref(o), p(dist_b),
                                None, p(ijb), p(wb), p(st_b), None) == F.D2_EINVAL
    big = synth.from_bags([(np.zeros((70, 2)), np.full(70, 1 / 70))], np.float64)
    Gd = d2.DeviceSet.from_ragged(big, DEV)
    g = Gd.c()
    assert L.d2_emd_batch_basis(h.ptr, ctypes.byref(g), ctypes.byref(b), p(bad), 1, ctypes.byref(o), p(dist_b),
                                p(offb), p(ijb), p(wb), p(st_b), None) == F.D2_EUNSUPPORTED
