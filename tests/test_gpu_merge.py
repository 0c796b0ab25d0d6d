"""GPU parity of one level's merge (Alg. 3 Step 3, Eq. (5)-(6)) through the C
ABI, against the oracle's merge_level.

Everything here is exact: the kept centroids, their atoms and atom weights
(copied), the new offsets and the inherited labels are integers or copies,
and each new centroid weight is its members' omega added in increasing
member index on both sides, so all of it is compared bit for bit."""
import numpy as np
import pytest

import synth
from oracle.hierarchy import merge_level

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


def make_level(seed, n, nseg, k_per, smax, d, n0, empty_frac, dtype=np.float64):
    """n level objects cut into nseg segments, segment mu owning k_per[mu]
    consecutive centroids of up to smax atoms; a fraction of the centroids
    gets no members.  C maps n0 original objects onto the level objects."""
    rng = np.random.default_rng([9102, seed, n, nseg, smax, d])
    seg_of = np.sort(rng.integers(0, nseg, n))
    segs = [np.flatnonzero(seg_of == mu) for mu in range(nseg)]
    zoff = np.concatenate([[0], np.cumsum(k_per)]).astype(np.int64)
    K = int(zoff[-1])
    alive = rng.random(K) >= empty_frac
    labels = np.full(n, -1, dtype=np.int32)
    for mu, S in enumerate(segs):
        cand = np.arange(zoff[mu], zoff[mu + 1])
        cand = cand[alive[cand]] if alive[cand].any() else cand
        if len(cand) and len(S):
            labels[S] = rng.choice(cand, len(S))
    sizes = rng.integers(1, smax + 1, K)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pts = rng.normal(size=(int(off[-1]), d)).astype(dtype)
    wts = np.concatenate([rng.dirichlet(np.ones(s)) for s in sizes]).astype(dtype) if K else \
        np.zeros(0, dtype)
    Z = synth.RaggedSet(off, pts, wts)
    omega = rng.uniform(0.1, 4.0, n)
    C = rng.integers(0, max(n, 1), n0).astype(np.int32) if n else np.zeros(n0, np.int32)
    return segs, zoff, labels, omega, C, Z


def check_against_oracle(d2, h, segs, zoff, labels, omega, C, Z, with_omega=True):
    Zd = d2.DeviceSet.from_ragged(Z, DEV)
    om = omega if with_omega else np.ones(len(labels))
    keep, _, o_omega, o_C = merge_level(segs, zoff, labels, om, C)
    G, g_omega, g_C, g_off = d2.d2_merge_level(
        h, Zd, torch.as_tensor(labels, device=DEV),
        torch.as_tensor(omega, device=DEV) if with_omega else None,
        torch.as_tensor(C, device=DEV))
    torch.cuda.synchronize()
    keep = np.asarray(keep, dtype=np.int64)
    assert G.n == len(keep)
    sizes = Z.offsets[1:][keep] - Z.offsets[:-1][keep]
    assert np.array_equal(g_off, np.concatenate([[0], np.cumsum(sizes)]))
    assert np.array_equal(G.offsets.cpu().numpy(), g_off)
    sub = Z.subset(keep) if len(keep) else None
    if sub is not None:
        assert np.array_equal(G.points.cpu().numpy(), sub.points)
        assert np.array_equal(G.weights.cpu().numpy(), sub.weights)
        assert G.max_support == int(sizes.max())
    assert np.array_equal(g_omega.cpu().numpy(), np.asarray(o_omega))
    assert np.array_equal(g_C.cpu().numpy(), np.asarray(o_C))
    return G


@pytest.mark.parametrize("seed,n,nseg,smax,d,n0,empty", [
    (0, 70, 2, 5, 3, 150, 0.3),           # a ragged tail of a 64-object tile
    (1, 5000, 11, 9, 16, 20000, 0.25),    # many tiles, a scan over several blocks
    (2, 40000, 40, 64, 2, 100000, 0.1),   # the shape of a hierarchy level
])
def test_merge_matches_oracle(d2, h, seed, n, nseg, smax, d, n0, empty):
    rng = np.random.default_rng(seed)
    k_per = rng.integers(1, max(2, n // nseg // 4), nseg)
    check_against_oracle(d2, h, *make_level(seed, n, nseg, k_per, smax, d, n0, empty))


def test_merge_f32_and_unit_weights(d2, h):
    segs, zoff, labels, omega, C, Z = make_level(3, 900, 3, [40, 1, 77], 12, 5, 3000, 0.4,
                                                 dtype=np.float32)
    G = check_against_oracle(d2, h, segs, zoff, labels, omega, C, Z, with_omega=False)
    assert G.points.dtype == torch.float32


def test_merge_edge_cases(d2, h):
    # every centroid kept, and supports past the lane-group limit
    segs, zoff, labels, omega, C, Z = make_level(4, 300, 1, [300], 200, 2, 500, 0.0)
    labels = np.arange(300, dtype=np.int32)
    check_against_oracle(d2, h, segs, zoff, labels, omega, C, Z)
    # one centroid takes everything
    labels = np.zeros(300, dtype=np.int32)
    check_against_oracle(d2, h, segs, zoff, labels, omega, C, Z)
    # no original objects, then no level objects (nothing kept)
    check_against_oracle(d2, h, segs, zoff, labels, omega, np.zeros(0, np.int32), Z)
    G, g_omega, g_C, g_off = d2.d2_merge_level(
        h, d2.DeviceSet.from_ragged(Z, DEV), torch.zeros(0, dtype=torch.int32, device=DEV), None,
        torch.tensor([0, 5, -1], dtype=torch.int32, device=DEV))
    assert G.n == 0 and g_omega.numel() == 0 and list(g_off) == [0]
    assert g_C.cpu().tolist() == [-1, -1, -1]


def test_merge_unlabelled_objects_and_bad_entries(d2, h):
    """Objects whose label is out of range belong to no centroid; an entry
    of C outside the level objects, or naming such an object, inherits -1."""
    segs, zoff, labels, omega, C, Z = make_level(5, 400, 4, [20, 20, 20, 20], 7, 3, 800, 0.2)
    labels[::9] = -1
    labels[5::13] = 80 + 7                      # beyond the 80 centroids
    C[::17] = -3
    C[3::19] = 400                              # past the level objects
    keep_mask = (labels >= 0) & (labels < 80)
    # the oracle's merge takes only member objects: compare on them
    inr = np.flatnonzero(keep_mask)
    remap = np.full(400, -1, dtype=np.int64)
    remap[inr] = np.arange(len(inr))
    segs_in = [remap[S[keep_mask[S]]] for S in segs]
    okC = (C >= 0) & (C < 400)
    okC[okC] &= keep_mask[C[okC]]
    keep, _, o_omega, o_C = merge_level(segs_in, zoff, labels[inr], omega[inr], remap[C[okC]])
    Zd = d2.DeviceSet.from_ragged(Z, DEV)
    G, g_omega, g_C, _ = d2.d2_merge_level(h, Zd, torch.as_tensor(labels, device=DEV),
                                           torch.as_tensor(omega, device=DEV), torch.as_tensor(C, device=DEV))
    gC = g_C.cpu().numpy()
    assert G.n == len(keep)
    assert np.array_equal(g_omega.cpu().numpy(), np.asarray(o_omega))
    assert np.array_equal(gC[okC], np.asarray(o_C))
    assert np.all(gC[~okC] == -1)


def test_merge_repeatable_and_rejects_bad_calls(d2, h):
    import ctypes
    segs, zoff, labels, omega, C, Z = make_level(6, 3000, 5, [100] * 5, 10, 4, 5000, 0.2)
    Zd = d2.DeviceSet.from_ragged(Z, DEV)
    lab = torch.as_tensor(labels, device=DEV)
    om = torch.as_tensor(omega, device=DEV)
    Cd = torch.as_tensor(C, device=DEV)
    a = d2.d2_merge_level(h, Zd, lab, om, Cd)
    b = d2.d2_merge_level(h, Zd, lab, om, Cd)
    assert torch.equal(a[1], b[1]) and torch.equal(a[2], b[2]) and torch.equal(a[0].points, b[0].points)
    L, F = d2._ffi.lib(), d2._ffi
    z = Zd.c()
    out = torch.empty(Zd.points.shape, dtype=Zd.points.dtype, device=DEV)
    one = torch.empty(Zd.n + 1, dtype=torch.int64, device=DEV)
    ws = torch.empty(1 << 20, dtype=torch.uint8, device=DEV)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    # outputs over Z's own atoms
    assert L.d2_merge_level(h.ptr, ctypes.byref(z), lab.numel(), p(lab), p(om), 0, None, p(one), p(one),
                            ctypes.c_void_p(z.points), p(out), p(om), p(ws), ws.numel(), None) == F.D2_EINVAL
    # a workspace below the query
    need = L.d2_workspace_bytes(h.ptr, F.WHICH_MERGE, ctypes.byref(z), None, lab.numel(), None)
    assert need > 0
    assert L.d2_merge_level(h.ptr, ctypes.byref(z), lab.numel(), p(lab), p(om), 0, None, p(one), p(one),
                            p(out), p(out), p(om), p(ws), need - 1, None) == F.D2_EWORKSPACE
    # negative sizes
    assert L.d2_merge_level(h.ptr, ctypes.byref(z), -1, p(lab), p(om), 0, None, p(one), p(one),
                            p(out), p(out), p(om), p(ws), ws.numel(), None) == F.D2_EINVAL
