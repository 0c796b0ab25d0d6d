"""Pins for the oracle's centroid update with free centroid weights (Alg. 1,
Step 1 as the LP of Eq. (1) over the centroid weights and every member's
matching; Steps 2-3 as for the constrained update), no GPU.

Each check is derived here, not from the oracle's code:

* ``lp_simplex`` against HiGHS on random standard-form LPs with dependent
  rows;
* the Step 1 value against HiGHS on the cluster LP assembled here
  independently (Kronecker products, another variable order);
* one member: the optimal matching sends each atom to its nearest centroid
  atom, so the value is sum_a p_a min_r C_ar and the weights are the
  nearest atoms' collected mass;
* identical members: the value is sum(omega) times the one-member value;
* with the optimal weights fed back as fixed centroid weights, the
  per-member transport problems (the constrained update's LPs) sum to the
  same value; any other fixed weights (uniform) cannot do better;
* Eq. (3): doubling a member's omega equals listing it twice;
* a one-atom centroid forces every matching (weight 1), so the moved atom is
  the omega-weighted mean of the member means;
* Step 2 cannot raise the objective (eps_step3 <= eps_step1), and the
  weights form a probability vector.
Planted mistakes in the oracle (a dropped mass constraint, unweighted
costs, a flipped coupling sign, unweighted means) fail these checks.
"""
import numpy as np
import pytest

import synth


def cost(x, y):
    x = np.asarray(x, float); y = np.asarray(y, float)
    return ((x[:, None, :] - y[None, :, :]) ** 2).sum(-1)


def rand_cluster(rng, n, tlo, thi, s, d):
    members = []
    for _ in range(n):
        t = int(rng.integers(tlo, thi + 1))
        members.append((rng.normal(size=(t, d)) * 1.5, rng.dirichlet(np.ones(t)), float(rng.integers(1, 4))))
    z = rng.normal(size=(s, d)) * 1.5
    return members, z


def highs_value(members, z):
    """The Step 1 LP assembled independently: variables ordered by centroid
    atom r, then member, then member atom a; then p_z."""
    from scipy.optimize import linprog
    s = z.shape[0]
    ts = [len(p) for _, p, _ in members]
    T = sum(ts)
    nvar = s * T + s
    c = np.zeros(nvar)
    col = {}
    k = 0
    for r in range(s):
        for i, (x, p, om) in enumerate(members):
            for a in range(len(p)):
                col[(r, i, a)] = k
                c[k] = om * float(((x[a] - z[r]) ** 2).sum())
                k += 1
    A, b = [], []
    for i, (x, p, om) in enumerate(members):
        for a in range(len(p)):
            row = np.zeros(nvar)
            for r in range(s):
                row[col[(r, i, a)]] = 1.0
            A.append(row); b.append(p[a] / p.sum())
        for r in range(s):
            row = np.zeros(nvar)
            for a in range(len(p)):
                row[col[(r, i, a)]] = 1.0
            row[s * T + r] = -1.0
            A.append(row); b.append(0.0)
    row = np.zeros(nvar); row[s * T:] = 1.0
    A.append(row); b.append(1.0)
    res = linprog(c, A_eq=np.array(A), b_eq=np.array(b), bounds=(0, None), method="highs",
                  options={"primal_feasibility_tolerance": 1e-10, "dual_feasibility_tolerance": 1e-10})
    assert res.status == 0
    return res.fun


def as_sets(members, z, zw=None):
    X = synth.from_bags([(x, p) for x, p, _ in members])
    Z = synth.from_bags([(z, np.full(z.shape[0], 1.0 / z.shape[0]) if zw is None else zw)])
    om = np.array([o for _, _, o in members])
    return X, Z, om


def test_lp_simplex_against_highs():
    from scipy.optimize import linprog
    from oracle.free_update import lp_simplex
    rng = np.random.default_rng(11)
    for _ in range(40):
        m, n = int(rng.integers(2, 10)), int(rng.integers(6, 24))
        A = rng.integers(-2, 3, size=(m, n)).astype(float)
        b = A @ rng.random(n)
        A = np.vstack([A, 2 * A[0] - A[-1]]); b = np.append(b, 2 * b[0] - b[-1])   # a dependent row
        flip = b < 0
        A[flip] *= -1; b[flip] *= -1
        c = rng.normal(size=n) + 2.0
        v, x = lp_simplex(c, A, b)
        r = linprog(c, A_eq=A, b_eq=b, bounds=(0, None), method="highs")
        if r.status == 3:
            continue
        assert abs(v - r.fun) <= 1e-9 * max(1.0, abs(r.fun))
        assert np.abs(A @ x - b).max() <= 1e-9 and x.min() >= 0


@pytest.mark.parametrize("seed", range(6))
def test_step1_value_against_highs(seed):
    from oracle.free_update import free_update
    rng = np.random.default_rng(100 + seed)
    members, z = rand_cluster(rng, int(rng.integers(1, 5)), 1, 5, int(rng.integers(1, 5)), 3)
    X, Z, om = as_sets(members, z)
    _, pz, e1, e3, st = free_update(X, Z, np.zeros(X.n, int), weights=om)
    want = highs_value(members, z)
    assert st.max() == 0
    assert abs(e1[0] - want) <= 1e-9 * max(1.0, want)
    assert abs(pz.sum() - 1.0) <= 1e-12 and pz.min() >= 0.0
    assert e3[0] <= e1[0] * (1 + 1e-12) + 1e-15


def test_one_member_closed_form():
    from oracle.free_update import free_update
    rng = np.random.default_rng(7)
    for _ in range(10):
        t, s = int(rng.integers(1, 7)), int(rng.integers(1, 6))
        x = rng.normal(size=(t, 2)) * 2
        p = rng.dirichlet(np.ones(t))
        z = rng.normal(size=(s, 2)) * 2
        X, Z, _ = as_sets([(x, p, 1.0)], z)
        _, pz, e1, _, _ = free_update(X, Z, [0])
        C = cost(x, z)
        assert abs(e1[0] - float((p * C.min(axis=1)).sum())) <= 1e-12 * max(1.0, C.max())
        want = np.zeros(s)
        np.add.at(want, C.argmin(axis=1), p)
        assert np.allclose(pz, want, atol=1e-12)


def test_identical_members_scale_the_one_member_value():
    from oracle.free_update import free_update
    rng = np.random.default_rng(8)
    x = rng.normal(size=(5, 3)); p = rng.dirichlet(np.ones(5)); z = rng.normal(size=(4, 3))
    X1, Z, _ = as_sets([(x, p, 1.0)], z)
    _, _, one, _, _ = free_update(X1, Z, [0])
    oms = [1.0, 2.0, 0.5]
    X3, _, om = as_sets([(x, p, o) for o in oms], z)
    _, _, three, _, _ = free_update(X3, Z, [0, 0, 0], weights=om)
    assert abs(three[0] - sum(oms) * one[0]) <= 1e-12 * max(1.0, three[0])


@pytest.mark.parametrize("seed", range(4))
def test_optimal_weights_as_fixed_weights_give_the_same_value(seed):
    import oracle
    from oracle.free_update import free_update
    rng = np.random.default_rng(300 + seed)
    members, z = rand_cluster(rng, 4, 2, 6, 4, 2)
    X, Z, om = as_sets(members, z)
    _, pz, e1, _, _ = free_update(X, Z, np.zeros(X.n, int), weights=om)
    fixed = sum(o * oracle.emd_pair(x, p, z, np.maximum(pz, 0.0))[0] for x, p, o in members)
    assert abs(fixed - e1[0]) <= 1e-10 * max(1.0, e1[0])
    uniform = sum(o * oracle.emd_pair(x, p, z, np.full(z.shape[0], 1.0))[0] for x, p, o in members)
    assert e1[0] <= uniform * (1 + 1e-12)


def test_doubled_weight_equals_a_listed_twice_member():
    from oracle.free_update import free_update
    rng = np.random.default_rng(9)
    members, z = rand_cluster(rng, 3, 2, 5, 3, 2)
    (x0, p0, _), rest = members[0], members[1:]
    XA, Z, omA = as_sets([(x0, p0, 2.0)] + [(x, p, 1.0) for x, p, _ in rest], z)
    XB, _, omB = as_sets([(x0, p0, 1.0), (x0, p0, 1.0)] + [(x, p, 1.0) for x, p, _ in rest], z)
    _, _, a, _, _ = free_update(XA, Z, np.zeros(XA.n, int), weights=omA)
    _, _, b, _, _ = free_update(XB, Z, np.zeros(XB.n, int), weights=omB)
    assert abs(a[0] - b[0]) <= 1e-12 * max(1.0, a[0])


def test_one_atom_centroid_moves_to_the_weighted_mean():
    from oracle.free_update import free_update
    rng = np.random.default_rng(10)
    members, _ = rand_cluster(rng, 5, 1, 6, 1, 3)
    z = rng.normal(size=(1, 3))
    X, Z, om = as_sets(members, z)
    zn, pz, e1, e3, _ = free_update(X, Z, np.zeros(X.n, int), weights=om)
    means = np.array([p @ x for x, p, _ in members])
    want = (om[:, None] * means).sum(0) / om.sum()
    assert np.allclose(zn[0], want, atol=1e-12) and abs(pz[0] - 1.0) <= 1e-15
    want3 = sum(o * float(p @ ((x - want) ** 2).sum(1)) for x, p, o in members)
    assert abs(e3[0] - want3) <= 1e-12 * max(1.0, want3)


def test_labels_statuses_and_empty_clusters():
    from oracle.free_update import free_update
    rng = np.random.default_rng(12)
    members, z = rand_cluster(rng, 4, 1, 4, 3, 2)
    X = synth.from_bags([(x, p) for x, p, _ in members])
    Z = synth.from_bags([(z, np.full(3, 1 / 3)), (z + 5.0, np.full(3, 1 / 3))])
    zn, pz, e1, e3, st = free_update(X, Z, [0, 0, 7, -1])
    assert list(st) == [0, 0, 5, 5]
    assert np.array_equal(zn[3:], Z.points[3:]) and e1[1] == 0.0   # the empty cluster keeps its atoms
    assert np.allclose(pz[3:], Z.weights[3:])


def test_member_weights_are_probability_vectors():
    """Eq. (1) needs each member's weights to sum to one: scaling a member's
    weights by any positive factor changes nothing."""
    from oracle.free_update import free_update
    rng = np.random.default_rng(13)
    members, z = rand_cluster(rng, 3, 2, 5, 3, 2)
    X, Z, om = as_sets(members, z)
    scaled = synth.from_bags([(x, p * f) for (x, p, _), f in zip(members, (3.0, 0.25, 7.5))])
    a = free_update(X, Z, np.zeros(X.n, int), weights=om)
    b = free_update(scaled, Z, np.zeros(X.n, int), weights=om)
    assert abs(a[2][0] - b[2][0]) <= 1e-12 * max(1.0, a[2][0])
    assert np.allclose(a[0], b[0], atol=1e-12)
