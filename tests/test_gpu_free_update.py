"""GPU parity of the centroid update with free centroid weights (Alg. 1,
Steps 1-3, Step 1 as the LP of Eq. (1) over the centroid weights and every
member's matching) through the C ABI, against the FP64 oracle.

What is compared:
* the Step 1 optimum (unique): |g - o| <= 1e-10 * max(|o|, 1e-4 S_j), S_j
  the sum over members of omega times the independent-coupling cost to the
  old centroid (an upper bound on the optimum);
* on inputs in general position the optimal vertex is unique, so the new
  weights (|g - o| <= 1e-9) and atoms (|g - o| <= 1e-9 times the cluster's
  coordinate scale) and the Step 3 objective (as Step 1) are compared too;
* on degenerate inputs (integer grids, repeated members), where several
  optima exist, the device's weights are checked to be optimal on their own:
  a probability vector whose fixed-weight transport problems, summed with
  the omegas, reach the Step 1 optimum; and Step 2 cannot raise it;
* counts and statuses are integers: equal.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle.free_update import free_update
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


def make_case(seed, K, per, tlo, thi, s, d=2, extra_labels=(), dtype=np.float64):
    """K clusters of ``per`` members around separate centres, centroids of s
    atoms near each centre with uniform weights; ``extra_labels`` appends
    objects with those (possibly out-of-range) labels."""
    rng = np.random.default_rng([7301, seed, K, per, s, d])
    centres = rng.normal(size=(K, d)) * 6.0
    bags, labels = [], []
    for j in range(K):
        for _ in range(per):
            t = int(rng.integers(tlo, thi + 1))
            bags.append((centres[j] + rng.normal(size=(t, d)), rng.dirichlet(np.ones(t)) * 3.0))
            labels.append(j)
    for lab in extra_labels:
        t = int(rng.integers(tlo, thi + 1))
        bags.append((rng.normal(size=(t, d)), rng.dirichlet(np.ones(t))))
        labels.append(lab)
    zb = [(centres[j] + rng.normal(size=(s, d)) * 0.8, np.full(s, 1.0 / s)) for j in range(K)]
    return (synth.from_bags(bags, dtype), synth.from_bags(zb, dtype),
            np.asarray(labels, dtype=np.int32))


def run(d2, h, X, Z, labels, weights=None, max_members=None, opts=None):
    Xd = d2.DeviceSet.from_ragged(X, DEV)
    Zd = d2.DeviceSet.from_ragged(Z, DEV)
    lab = torch.as_tensor(labels, device=DEV)
    w = None if weights is None else torch.as_tensor(np.asarray(weights, np.float64), device=DEV)
    out = d2.d2_centroid_update_free(h, Xd, Zd, lab, opts, weights=w, max_members=max_members)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


def members_of(X, labels, ost, weights, j):
    return [i for i in range(X.n) if labels[i] == j and ost[i] == 0
            and (weights is None or weights[i] > 0)]


def scale_S(X, Z, mem, weights, j):
    a0, a1 = int(Z.offsets[j]), int(Z.offsets[j + 1])
    zo = np.asarray(Z.points[a0:a1], np.float64)
    zw = np.full(a1 - a0, 1.0)
    return sum((1.0 if weights is None else weights[i]) * coupling_cost(*X.bag(i), zo, zw) for i in mem)


def check_unique(X, Z, labels, got, weights=None):
    z, w, e1, e3, cnt, st, cst = got
    oz, ow, oe1, oe3, ost = free_update(X, Z, labels, weights)
    np.testing.assert_array_equal(st, ost)
    for j in range(Z.n):
        a0, a1 = int(Z.offsets[j]), int(Z.offsets[j + 1])
        mem = members_of(X, labels, ost, weights, j)
        assert cst[j] == 0 and cnt[j] == len(mem), (j, cst[j], cnt[j], len(mem))
        S = scale_S(X, Z, mem, weights, j)
        for g, o, what in ((e1[j], oe1[j], "step 1"), (e3[j], oe3[j], "step 3")):
            assert abs(g - o) <= REL * max(abs(o), 1e-4 * S), (j, what, g, o)
        np.testing.assert_allclose(w[a0:a1], ow[a0:a1], rtol=0, atol=1e-9, err_msg=f"weights {j}")
        M = max([np.abs(np.asarray(Z.points[a0:a1], np.float64)).max()] +
                [np.abs(np.asarray(X.bag(i)[0], np.float64)).max() for i in mem])
        np.testing.assert_allclose(z[a0:a1], oz[a0:a1], rtol=0, atol=1e-9 * M, err_msg=f"atoms {j}")


def check_optimal(X, Z, labels, got, weights=None):
    """For inputs with several optima: the value is the oracle's, and the
    device's weights reach it with fixed-weight transport problems."""
    z, w, e1, e3, cnt, st, cst = got
    _, _, oe1, _, ost = free_update(X, Z, labels, weights)
    np.testing.assert_array_equal(st, ost)
    for j in range(Z.n):
        a0, a1 = int(Z.offsets[j]), int(Z.offsets[j + 1])
        mem = members_of(X, labels, ost, weights, j)
        assert cst[j] == 0 and cnt[j] == len(mem)
        S = scale_S(X, Z, mem, weights, j)
        tol = REL * max(abs(oe1[j]), 1e-4 * S)
        assert abs(e1[j] - oe1[j]) <= tol, (j, e1[j], oe1[j])
        if not mem:
            continue
        pz = w[a0:a1]
        assert np.all(pz >= 0.0) and abs(pz.sum() - 1.0) <= 1e-12
        zo = np.asarray(Z.points[a0:a1], np.float64)
        keep = pz > 0.0
        total = sum((1.0 if weights is None else weights[i]) *
                    oracle.emd_pair(*X.bag(i), zo[keep], pz[keep])[0] for i in mem)
        assert abs(total - oe1[j]) <= tol + 1e-12 * abs(oe1[j]), (j, total, oe1[j])
        assert e3[j] <= e1[j] + tol


def test_free_update_matches_oracle(d2, h):
    X, Z, labels = make_case(1, K=5, per=6, tlo=2, thi=7, s=5)
    check_unique(X, Z, labels, run(d2, h, X, Z, labels))


def test_free_update_several_tiles_and_wide_centroids(d2, h):
    # 140 objects (three counting-sort tiles), s = 12, d = 3
    X, Z, labels = make_case(2, K=7, per=20, tlo=3, thi=9, s=12, d=3)
    check_unique(X, Z, labels, run(d2, h, X, Z, labels))


def test_free_update_object_weights_and_statuses(d2, h):
    X, Z, labels = make_case(3, K=4, per=5, tlo=2, thi=6, s=4, extra_labels=(-1, 4, 1))
    n = X.n
    rng = np.random.default_rng(11)
    weights = rng.uniform(0.5, 3.0, n)
    weights[2] = 0.0            # takes no part
    weights[7] = -1.0           # invalid: status 1
    weights[9] = np.nan         # invalid: status 1
    got = run(d2, h, X, Z, labels, weights=weights)
    assert got[5][n - 3] == 5 and got[5][n - 2] == 5 and got[5][7] == 1 and got[5][9] == 1
    check_unique(X, Z, labels, got, weights)


def test_free_update_float32_inputs(d2, h):
    X, Z, labels = make_case(4, K=3, per=6, tlo=2, thi=8, s=6, dtype=np.float32)
    check_unique(X, Z, labels, run(d2, h, X, Z, labels))


def test_free_update_degenerate_grid(d2, h):
    # integer points, equal weights, repeated members: many optimal vertices
    rng = np.random.default_rng(5)
    bags, labels = [], []
    for j in range(4):
        base = [(rng.integers(0, 3, size=(4, 2)).astype(np.float64), np.ones(4)) for _ in range(3)]
        for k in range(8):
            bags.append(base[k % 3])
            labels.append(j)
    zb = [(rng.integers(0, 3, size=(4, 2)).astype(np.float64), np.full(4, 0.25)) for _ in range(4)]
    X, Z = synth.from_bags(bags), synth.from_bags(zb)
    labels = np.asarray(labels, np.int32)
    check_optimal(X, Z, labels, run(d2, h, X, Z, labels))


def test_free_update_empty_and_oversized_clusters(d2, h):
    X, Z, labels = make_case(6, K=4, per=4, tlo=2, thi=5, s=3)
    labels = labels.copy()
    labels[labels == 2] = 1       # cluster 2 empty, cluster 1 has 8 members
    z, w, e1, e3, cnt, st, cst = run(d2, h, X, Z, labels, max_members=6)
    # cluster 2: no members, unchanged
    a0, a1 = int(Z.offsets[2]), int(Z.offsets[3])
    assert cst[2] == 0 and cnt[2] == 0 and e1[2] == 0.0 and e3[2] == 0.0
    np.testing.assert_array_equal(z[a0:a1], Z.points[a0:a1])
    np.testing.assert_array_equal(w[a0:a1], Z.weights[a0:a1])
    # cluster 1: over the bound, unchanged, every member flagged
    a0, a1 = int(Z.offsets[1]), int(Z.offsets[2])
    assert cst[1] == 2 and cnt[1] == 0 and np.isnan(e1[1]) and np.isnan(e3[1])
    assert np.all(st[labels == 1] == 2)
    np.testing.assert_array_equal(z[a0:a1], Z.points[a0:a1])
    np.testing.assert_array_equal(w[a0:a1], Z.weights[a0:a1])
    # clusters 0 and 3 as the oracle
    oz, ow, oe1, oe3, ost = free_update(X, Z, labels)
    for j in (0, 3):
        b0, b1 = int(Z.offsets[j]), int(Z.offsets[j + 1])
        assert cst[j] == 0 and abs(e1[j] - oe1[j]) <= 1e-10 * abs(oe1[j])
        np.testing.assert_allclose(w[b0:b1], ow[b0:b1], rtol=0, atol=1e-9)


def test_free_update_repeatable_bits_and_pivot_cap(d2, h):
    X, Z, labels = make_case(7, K=3, per=6, tlo=3, thi=7, s=6)
    a = run(d2, h, X, Z, labels)
    b = run(d2, h, X, Z, labels)
    for x, y in zip(a, b):
        assert np.array_equal(x, y, equal_nan=True)
    capped = run(d2, h, X, Z, labels, opts=d2.Opts(max_pivots=1))
    assert np.all(capped[6] == 3)
    assert np.all(capped[5] == 3)
    np.testing.assert_array_equal(capped[1], Z.weights)
    assert np.all(np.isnan(capped[2]))


def test_free_update_warm_start_from_kept_bases(d2, h):
    """A second pass over the same members (moved atoms, so other costs)
    starts from the first pass's optimal bases: same results as a cold
    start and as the oracle, in fewer pivots.  Rows that do not fit the
    program (another membership, garbage) are ignored."""
    X, Z, labels = make_case(8, K=4, per=8, tlo=3, thi=8, s=6)
    Xd = d2.DeviceSet.from_ragged(X, DEV)
    Zd = d2.DeviceSet.from_ragged(Z, DEV)
    lab = torch.as_tensor(labels, device=DEV)
    basis = d2.free_basis_buffer(Xd, Zd, 8)
    first = d2.d2_centroid_update_free(h, Xd, Zd, lab, want_pivots=True, basis=basis)
    torch.cuda.synchronize()
    kept = basis.cpu().numpy()
    assert np.all(kept[:, 0] > 0)
    # the moved atoms with the new weights: the next pass's centroids
    Z2 = synth.RaggedSet(Z.offsets, first[0].cpu().numpy(), first[1].cpu().numpy())
    Z2d = d2.DeviceSet.from_ragged(Z2, DEV)
    cold = [t.cpu().numpy() for t in d2.d2_centroid_update_free(h, Xd, Z2d, lab, want_pivots=True)]
    warm = [t.cpu().numpy() for t in d2.d2_centroid_update_free(h, Xd, Z2d, lab, want_pivots=True,
                                                                basis=basis)]
    torch.cuda.synchronize()
    check_unique(X, Z2, labels, warm[:7])
    for a, b in zip(cold[:7], warm[:7]):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-12)
    assert warm[7].sum() < cold[7].sum(), (warm[7], cold[7])
    # another membership with the same kept rows, and garbage rows
    lab2 = labels.copy()
    lab2[0], lab2[9] = lab2[9], lab2[0]
    junk = torch.randint(-5, 10**6, basis.shape, dtype=torch.int32, device=DEV)
    junk[:, 0] = basis[:, 0]
    for rows in (basis, junk):
        got = [t.cpu().numpy() for t in d2.d2_centroid_update_free(
            h, Xd, Z2d, torch.as_tensor(lab2, device=DEV), basis=rows.clone())]
        torch.cuda.synchronize()
        check_unique(X, Z2, lab2, got)


@pytest.mark.parametrize("max_members", [None, 100])
def test_free_update_large_programs(d2, h, max_members):
    """Two clusters of 48 members (m about 1,300 rows): with the members'
    own bound the program's vectors fit in LDS; with a bound of 100 they do
    not and the slab-resident kernel runs.  Both past the periodic
    reinversion (over 256 pivots), against the LP optimum from HiGHS on the
    oracle's program (scipy's linprog), and the device's weights checked to
    reach it with fixed-weight transport problems; the two variants give
    the same bits."""
    from scipy.optimize import linprog
    from oracle.free_update import cluster_lp
    X, Z, labels = make_case(9, K=2, per=48, tlo=8, thi=16, s=16, d=8)
    Xd = d2.DeviceSet.from_ragged(X, DEV)
    Zd = d2.DeviceSet.from_ragged(Z, DEV)
    lab = torch.as_tensor(labels, device=DEV)
    out = d2.d2_centroid_update_free(h, Xd, Zd, lab, want_pivots=True, max_members=max_members)
    torch.cuda.synchronize()
    z, w, e1, e3, cnt, st, cst, piv = [t.cpu().numpy() for t in out]
    if max_members is not None:
        ref_lds = [t.cpu().numpy() for t in d2.d2_centroid_update_free(h, Xd, Zd, lab, want_pivots=True)]
        for a, b in zip(ref_lds, (z, w, e1, e3, cnt, st, cst, piv)):
            assert np.array_equal(a, b)
    assert np.all(st == 0) and np.all(cst == 0) and np.all(cnt == 48)
    assert piv.max() > 256, piv
    for j in range(Z.n):
        a0, a1 = int(Z.offsets[j]), int(Z.offsets[j + 1])
        zo = np.asarray(Z.points[a0:a1], np.float64)
        mem = [i for i in range(X.n) if labels[i] == j]
        members = []
        for i in mem:
            x, p = X.bag(i)
            p = np.asarray(p, np.float64)
            members.append((np.asarray(x, np.float64), p / p.sum(), 1.0))
        c, A, b, _ = cluster_lp(members, zo)
        ref = linprog(c, A_eq=A, b_eq=b, bounds=(0, None), method="highs")
        assert ref.status == 0
        S = scale_S(X, Z, mem, None, j)
        tol = REL * max(abs(ref.fun), 1e-4 * S)
        assert abs(e1[j] - ref.fun) <= tol, (j, e1[j], ref.fun)
        pz = w[a0:a1]
        assert np.all(pz >= 0.0) and abs(pz.sum() - 1.0) <= 1e-12
        keep = pz > 0.0
        total = sum(oracle.emd_pair(*X.bag(i), zo[keep], pz[keep])[0] for i in mem)
        assert abs(total - ref.fun) <= tol + 1e-12 * abs(ref.fun), (j, total, ref.fun)
        assert e3[j] <= e1[j] + tol
