"""GPU parity of the constrained D2 centroid update (Alg. 2 Step 3*) through
the C ABI, against the FP64 oracle on the same seeded inputs.

Tolerances (derived from the arithmetic):
* moved atoms: a flow-weighted mean lies in the convex hull of the member
  atoms, and the flows carry a few ulps of the unit mass each, so
  |g - o| <= 1e-10 * M_j with M_j the largest coordinate magnitude among the
  cluster's member atoms and its old atoms;
* the Step 1 and Step 3 objectives are sums of per-member transport costs:
  |g - o| <= 1e-10 * max(|o|, 1e-4 * S_j), S_j the sum of the members'
  independent-coupling costs (the floor of the pair rule, summed);
* counts and statuses are integers: equal.
Inputs are seeded: labels are either the oracle's nearest-centroid labels or
seeded random labels; centroid weights are uniform (the paper's case) unless
a test says otherwise.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.parity import REL, coupling_cost

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


def uniform(Z):
    w = np.concatenate([np.full(int(s), 1.0 / int(s)) for s in Z.sizes]) if Z.n else np.zeros(0)
    return synth.RaggedSet(Z.offsets, Z.points, w.astype(Z.points.dtype))


def run(d2, h, X, Z, labels, init=0, xmax=None, zmax=None):
    Xd = d2.DeviceSet.from_ragged(X, DEV)
    Zd = d2.DeviceSet.from_ragged(Z, DEV)
    if xmax is not None:
        Xd.max_support = xmax
    if zmax is not None:
        Zd.max_support = zmax
    lab = torch.as_tensor(np.asarray(labels, dtype=np.int32), device=DEV)
    z, e1, e3, cnt, st = d2.d2_centroid_update(h, Xd, Zd, lab, d2.Opts(init=init))
    torch.cuda.synchronize()
    return (z.cpu().numpy(), e1.cpu().numpy(), e3.cpu().numpy(), cnt.cpu().numpy(),
            st.cpu().numpy())


def check(X, Z, labels, got, clusters=None):
    """Compare the device's pass with the oracle's on the same inputs."""
    z, e1, e3, cnt, st = got
    oz, oe1, oe3, ost = oracle.centroid_update(X, Z, labels)
    labels = np.asarray(labels)
    K = Z.n
    clusters = range(K) if clusters is None else clusters
    np.testing.assert_array_equal(st, ost)
    for j in clusters:
        a0, a1 = int(Z.offsets[j]), int(Z.offsets[j + 1])
        mem = [i for i in range(X.n) if labels[i] == j and ost[i] == 0]
        assert cnt[j] == len(mem)
        pts = [np.abs(np.asarray(X.bag(i)[0], np.float64)).max() for i in mem]
        M = max([np.abs(np.asarray(Z.points[a0:a1], np.float64)).max(initial=0.0)] + pts)
        err = np.abs(z[a0:a1] - oz[a0:a1]).max(initial=0.0)
        assert err <= REL * max(M, 1e-300), f"cluster {j}: atom error {err} (scale {M})"
        zo = np.asarray(Z.points[a0:a1], np.float64)
        zw = np.asarray(Z.weights[a0:a1], np.float64)
        s_old = sum(coupling_cost(*X.bag(i), zo, zw) for i in mem)
        s_new = sum(coupling_cost(*X.bag(i), oz[a0:a1], zw) for i in mem)
        assert abs(e1[j] - oe1[j]) <= REL * max(abs(oe1[j]), 1e-4 * s_old), \
            f"cluster {j}: eps1 {e1[j]!r} vs {oe1[j]!r}"
        assert abs(e3[j] - oe3[j]) <= REL * max(abs(oe3[j]), 1e-4 * s_new), \
            f"cluster {j}: eps3 {e3[j]!r} vs {oe3[j]!r}"
    return oz, oe1, oe3


@pytest.mark.parametrize("init", [0, 1, 2, 3])
def test_config1_nearest_labels(d2, h, init):
    X = synth.make_data(1)
    Z = uniform(synth.make_centroids(1))
    labels = oracle.assign(X, Z)[0]
    got = run(d2, h, X, Z, labels, init=init)
    check(X, Z, labels, got)
    assert np.all(got[2] <= got[1] + 1e-12 * np.maximum(got[1], 1.0))   # Step 2 descends


@pytest.mark.parametrize("tlo,thi,s,d,f32", [
    (1, 8, 8, 3, False),      # class 0
    (5, 30, 16, 5, True),     # class 1
    (20, 64, 24, 4, False),   # class 2
    (33, 64, 64, 2, True),    # class 3
    (1, 16, 40, 70, False),   # class 2 with s > t, two coordinate passes in the mean
])
def test_every_class_random_labels(d2, h, tlo, thi, s, d, f32):
    rng = np.random.default_rng(100 + s + d)
    n, K = 90, 7
    bags = [(rng.normal(size=(t, d)) * 3.0, rng.dirichlet(np.full(t, 0.6)))
            for t in rng.integers(tlo, thi + 1, size=n)]
    X = synth.from_bags(bags)
    Z = synth.from_bags([(rng.normal(size=(s, d)) * 3.0, np.full(s, 1.0 / s)) for _ in range(K)])
    if f32:
        X, Z = X.astype(np.float32), Z.astype(np.float32)
    labels = rng.integers(0, K, size=n)
    check(X, Z, labels, run(d2, h, X, Z, labels))


def test_fixed_nonuniform_weights(d2, h):
    rng = np.random.default_rng(7)
    X = synth.from_bags([(rng.normal(size=(t, 3)), rng.dirichlet(np.ones(t)))
                         for t in rng.integers(2, 12, size=60)])
    Z = synth.from_bags([(rng.normal(size=(6, 3)), rng.dirichlet(np.ones(6))) for _ in range(4)])
    labels = rng.integers(0, 4, size=60)
    check(X, Z, labels, run(d2, h, X, Z, labels))


def test_edge_cases(d2, h):
    """Empty cluster, labels outside [0, K), a bag with bad weights, a
    zero-weight centroid atom, single-atom objects, identical bags."""
    rng = np.random.default_rng(8)
    bags = [(rng.normal(size=(t, 2)), rng.dirichlet(np.ones(t))) for t in [3, 1, 4, 2, 5, 1, 6, 3]]
    bags[4] = (bags[4][0], np.array([0.2, -0.1, 0.3, 0.3, 0.3]))   # bad weights
    zb = [(rng.normal(size=(3, 2)), [0.5, 0.0, 0.5]), (rng.normal(size=(4, 2)), np.full(4, 0.25)),
          (rng.normal(size=(2, 2)), [0.5, 0.5])]
    bags.append((zb[1][0].copy(), np.full(4, 0.25)))                 # identical to centroid 1
    X = synth.from_bags(bags)
    Z = synth.from_bags(zb)
    labels = np.array([0, 0, 1, -1, 0, 5, 1, 0, 1])                 # cluster 2 is empty
    got = run(d2, h, X, Z, labels)
    z, e1, e3, cnt, st = got
    np.testing.assert_array_equal(st, [0, 0, 0, 5, 1, 5, 0, 0, 0])
    np.testing.assert_array_equal(z[7:9], Z.points[7:9])              # empty cluster keeps its atoms
    np.testing.assert_array_equal(z[1], Z.points[1])                  # zero-weight atom keeps its place
    assert cnt[2] == 0 and e1[2] == 0.0 and e3[2] == 0.0
    check(X, Z, labels, got)


def test_no_objects_keeps_every_atom(d2, h):
    Z = uniform(synth.make_centroids(1))
    Xd = d2.DeviceSet(torch.zeros(1, dtype=torch.int64, device=DEV),
                      torch.zeros((0, 3), dtype=torch.float64, device=DEV),
                      torch.zeros(0, dtype=torch.float64, device=DEV), 1)
    Zd = d2.DeviceSet.from_ragged(Z, DEV)
    z, e1, e3, cnt, st = d2.d2_centroid_update(h, Xd, Zd, torch.zeros(0, dtype=torch.int32, device=DEV))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(z.cpu().numpy(), Z.points)
    assert (e1.cpu().numpy() == 0).all() and (e3.cpu().numpy() == 0).all()
    assert (cnt.cpu().numpy() == 0).all()


def test_repeatable_bits(d2, h):
    X = synth.make_data(1)
    Z = uniform(synth.make_centroids(1))
    labels = np.random.default_rng(9).integers(0, Z.n, size=X.n)
    a = run(d2, h, X, Z, labels)
    b = run(d2, h, X, Z, labels)
    for u, v in zip(a, b):
        assert np.array_equal(u, v, equal_nan=True)


def test_rejects_aliasing_and_bad_modes(d2, h):
    X = synth.make_data(1)
    Z = uniform(synth.make_centroids(1))
    Xd = d2.DeviceSet.from_ragged(X, DEV)
    Zd = d2.DeviceSet.from_ragged(Z, DEV)
    lab = torch.zeros(X.n, dtype=torch.int32, device=DEV)
    with pytest.raises(d2.D2Error) as e:
        d2.d2_centroid_update(h, Xd, Zd, lab, d2.Opts(cost_mode=d2.D2_COST_BF16_MFMA))
    assert e.value.code == 3
    # z_new may not be Z's own points
    import ctypes
    x, z, o = Xd.c(), Zd.c(), d2.Opts().c()
    nb = d2.d2_workspace_bytes(h, 4, Xd, Zd)
    ws = torch.empty(nb, dtype=torch.uint8, device=DEV)
    rc = d2._ffi.lib().d2_centroid_update(h.ptr, ctypes.byref(x), ctypes.byref(z),
                                          ctypes.c_void_p(lab.data_ptr()), None, ctypes.byref(o),
                                          ctypes.c_void_p(Zd.points.data_ptr()), None, None, None,
                                          None, ctypes.c_void_p(ws.data_ptr()), nb, None)
    assert rc == 1
    rc = d2._ffi.lib().d2_centroid_update(h.ptr, ctypes.byref(x), ctypes.byref(z),
                                          ctypes.c_void_p(lab.data_ptr()), None, ctypes.byref(o),
                                          ctypes.c_void_p(ws.data_ptr()), None, None, None,
                                          None, ctypes.c_void_p(ws.data_ptr()), nb - 1, None)
    assert rc == 2


def test_full_config2_sampled_clusters(d2, h):
    """100,000 objects (d=8, t up to 16) with seeded labels over 512
    centroids of 16 uniform atoms; the oracle recomputes 6 whole clusters."""
    X = synth.make_data(2)
    Z = uniform(synth.make_centroids(2))
    labels = synth.rng_for(2, synth.STREAM_SAMPLE, 77).integers(0, Z.n, size=X.n)
    got = run(d2, h, X, Z, labels)
    assert got[4].max() == 0
    assert got[3].sum() == X.n
    pick = synth.rng_for(2, synth.STREAM_SAMPLE, 78).choice(Z.n, size=6, replace=False)
    rows = np.flatnonzero(np.isin(labels, pick))
    sub = X.subset(rows)
    sub_lab = labels[rows]
    z, e1, e3, cnt, st = got
    check(sub, Z, sub_lab, (z, e1, e3, cnt, st[rows]), clusters=[int(j) for j in pick])


def test_constrained_d2_driver_matches_oracle_loop(d2, h):
    """Three rounds of Alg. 2 with Step 3* (two update passes each), on the
    device through constrained_d2 and on the CPU through the oracle."""
    X = synth.make_data(1)
    Z0 = uniform(synth.make_centroids(1))
    Zg, lab_g, hist = d2.constrained_d2(h, d2.DeviceSet.from_ragged(X, DEV),
                                        d2.DeviceSet.from_ragged(Z0, DEV), max_rounds=3,
                                        max_passes=2, rtol=0.0)
    torch.cuda.synchronize()
    assert [r[1] for r in hist] == [2, 2, 2]
    Z = Z0
    for _ in range(3):
        lab = oracle.assign(X, Z)[0]
        for _ in range(2):
            zn, _, e3, _ = oracle.centroid_update(X, Z, lab)
            Z = synth.RaggedSet(Z.offsets, zn, Z.weights)
    np.testing.assert_array_equal(lab_g.cpu().numpy(), lab)
    M = np.abs(X.points).max()
    assert np.abs(Zg.points.cpu().numpy() - Z.points).max() <= REL * M
    assert abs(hist[-1][2] - e3.sum()) <= REL * e3.sum()
