"""Pins for the oracle's centroid update of constrained D2-clustering
(Alg. 2 Step 3*, i.e. Alg. 1 with the centroid weights held fixed), no GPU.

Each check is derived here from the mathematics, not from the oracle's code:

* one-atom centroids: every plan is forced (w_a1 = p_a), so the new atom is
  the mean of the members' weighted means and both objectives have closed
  forms;
* one-atom members: every centroid atom receives mass from the member point
  only, so every atom moves to the mean of the member points;
* equal weights and equal supports: the optimal plan is a permutation
  (Birkhoff), found here by brute force over all of them;
* Eq. (2) is the minimiser of a quadratic in z for fixed plans: moving the
  new atoms by any delta raises the Step 3 objective by exactly
  sum_r (sum of r's flows) |delta_r|^2;
* Step 2 cannot raise the objective and Step 1 of the next pass cannot raise
  it either (the monotone descent of Alg. 1);
* translating every point moves every new atom by the same vector;
* empty clusters, labels outside [0, K) and fixed non-uniform weights.
"""
import itertools

import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle


def norm(w):
    w = np.asarray(w, float)
    return w / w.sum()


def sqdist(a, b):
    a = np.asarray(a, float); b = np.asarray(b, float)
    return float(((a - b) ** 2).sum())


def random_bags(rng, n, tlo, thi, d, alpha=1.0):
    return [(rng.normal(size=(t, d)) * 2.0, rng.dirichlet(np.full(t, alpha)))
            for t in rng.integers(tlo, thi + 1, size=n)]


def test_one_atom_centroids_closed_form(oracle_mod):
    rng = np.random.default_rng(1)
    X = synth.from_bags(random_bags(rng, 30, 1, 7, 3))
    K = 4
    Z = synth.from_bags([(rng.normal(size=(1, 3)), [1.0]) for _ in range(K)])
    labels = rng.integers(0, K, size=X.n)
    z, e1, e3, st = oracle_mod.centroid_update(X, Z, labels)
    assert st.max() == 0
    for j in range(K):
        mem = [i for i in range(X.n) if labels[i] == j]
        means = [norm(X.bag(i)[1]) @ X.bag(i)[0] for i in mem]
        want = np.mean(means, axis=0)
        np.testing.assert_allclose(z[j], want, rtol=1e-13, atol=1e-13)
        old = Z.points[j]
        w1 = sum(norm(p) @ np.array([sqdist(a, old) for a in x]) for x, p in map(X.bag, mem))
        w3 = sum(norm(p) @ np.array([sqdist(a, want) for a in x]) for x, p in map(X.bag, mem))
        assert e1[j] == pytest.approx(w1, rel=1e-12)
        assert e3[j] == pytest.approx(w3, rel=1e-12)


def test_one_atom_members_collapse_every_atom_to_their_mean(oracle_mod):
    rng = np.random.default_rng(2)
    d = 4
    X = synth.from_bags([(rng.normal(size=(1, d)), [0.3]) for _ in range(25)])
    K, s = 3, 5
    Z = synth.from_bags([(rng.normal(size=(s, d)), rng.dirichlet(np.ones(s))) for _ in range(K)])
    labels = np.arange(X.n) % K
    z, e1, e3, st = oracle_mod.centroid_update(X, Z, labels)
    assert st.max() == 0
    for j in range(K):
        pts = X.points[labels == j]
        mean = pts.mean(axis=0)
        np.testing.assert_allclose(z[j * s:(j + 1) * s], np.tile(mean, (s, 1)), rtol=1e-13,
                                   atol=1e-13)
        assert e3[j] == pytest.approx(sum(sqdist(p, mean) for p in pts), rel=1e-12)


def test_equal_weights_permutation_bruteforce(oracle_mod):
    rng = np.random.default_rng(3)
    t, d, K, per = 3, 2, 3, 2
    X = synth.from_bags([(rng.normal(size=(t, d)), np.full(t, 1.0 / t)) for _ in range(K * per)])
    Z = synth.from_bags([(rng.normal(size=(t, d)), np.full(t, 1.0 / t)) for _ in range(K)])
    labels = np.repeat(np.arange(K), per)
    z, e1, e3, st = oracle_mod.centroid_update(X, Z, labels)
    assert st.max() == 0
    for j in range(K):
        zj = Z.points[j * t:(j + 1) * t]
        matched = []
        best_total = 0.0
        for i in np.flatnonzero(labels == j):
            x = X.bag(i)[0]
            costs = {sig: sum(sqdist(zj[r], x[sig[r]]) for r in range(t)) / t
                     for sig in itertools.permutations(range(t))}
            sig = min(costs, key=costs.get)
            best_total += costs[sig]
            matched.append(x[list(sig)])
        want = np.mean(matched, axis=0)
        np.testing.assert_allclose(z[j * t:(j + 1) * t], want, rtol=1e-13, atol=1e-13)
        assert e1[j] == pytest.approx(best_total, rel=1e-12)
        w3 = sum(sqdist(want[r], m[r]) for m in matched for r in range(t)) / t
        assert e3[j] == pytest.approx(w3, rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("seed", [4, 5])
def test_quadratic_identity_around_the_new_atoms(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    d, K, s = 3, 3, 4
    X = synth.from_bags(random_bags(rng, 24, 2, 6, d, alpha=0.7))
    Z = synth.from_bags([(rng.normal(size=(s, d)), np.full(s, 1.0 / s)) for _ in range(K)])
    labels = rng.integers(0, K, size=X.n)
    z, e1, e3, st, plans = oracle_mod.centroid_update(X, Z, labels, return_plans=True)
    assert st.max() == 0

    def objective(zz, j):
        tot = 0.0
        for i, jj, plan in plans:
            if jj != j:
                continue
            x = X.bag(i)[0]
            for a in range(x.shape[0]):
                for r in range(s):
                    tot += plan[a, r] * sqdist(x[a], zz[r])
        return tot

    for j in range(K):
        zj = z[j * s:(j + 1) * s]
        flow = np.zeros(s)
        for i, jj, plan in plans:
            if jj == j:
                flow += plan.sum(axis=0)
        base = objective(zj, j)
        assert e3[j] == pytest.approx(base, rel=1e-12)
        for _ in range(3):
            delta = rng.normal(size=zj.shape) * 0.1
            rise = objective(zj + delta, j) - base
            assert rise == pytest.approx(float(flow @ (delta ** 2).sum(axis=1)), rel=1e-8)


def test_descent_over_two_passes(oracle_mod):
    X = synth.make_data(1)
    Z0 = synth.make_centroids(1)
    labels = oracle_mod.assign(X, Z0)[0]
    z1, e1, e3, st = oracle_mod.centroid_update(X, Z0, labels)
    assert st.max() == 0
    scale = max(1.0, float(np.abs(X.points).max()) ** 2)
    assert np.all(e3 <= e1 + 1e-12 * scale)
    Z1 = synth.RaggedSet(Z0.offsets, z1, Z0.weights)
    _, f1, f3, st = oracle_mod.centroid_update(X, Z1, labels)
    assert np.all(f1 <= e3 + 1e-12 * scale)
    assert np.all(f3 <= f1 + 1e-12 * scale)
    # with K = 10 centroids of 8 atoms every cluster moved, and the
    # objective strictly decreased somewhere
    assert (e3 < e1).any()


def test_translation_moves_every_atom(oracle_mod):
    X = synth.make_data(1)
    Z = synth.make_centroids(1)
    labels = oracle_mod.assign(X, Z)[0]
    z, e1, e3, _ = oracle_mod.centroid_update(X, Z, labels)
    c = np.array([4.0, -2.0, 0.5])
    Xs = synth.RaggedSet(X.offsets, X.points + c, X.weights)
    Zs = synth.RaggedSet(Z.offsets, Z.points + c, Z.weights)
    zs, f1, f3, _ = oracle_mod.centroid_update(Xs, Zs, labels)
    np.testing.assert_allclose(zs - c, z, rtol=0, atol=1e-11)
    np.testing.assert_allclose(f1, e1, rtol=1e-10)
    np.testing.assert_allclose(f3, e3, rtol=1e-10)


def test_empty_cluster_and_bad_labels(oracle_mod):
    rng = np.random.default_rng(6)
    X = synth.from_bags(random_bags(rng, 10, 1, 5, 2))
    Z = synth.from_bags([(rng.normal(size=(3, 2)), np.full(3, 1 / 3)) for _ in range(3)])
    labels = np.array([0, 0, 2, -1, 2, 3, 0, 2, 0, -7])
    z, e1, e3, st = oracle_mod.centroid_update(X, Z, labels)
    np.testing.assert_array_equal(st, [0, 0, 0, 5, 0, 5, 0, 0, 0, 5])
    np.testing.assert_array_equal(z[3:6], Z.points[3:6])   # cluster 1 is empty
    assert e1[1] == 0.0 and e3[1] == 0.0
    assert not np.array_equal(z[0:3], Z.points[0:3])


def test_zero_weight_atom_keeps_its_place(oracle_mod):
    rng = np.random.default_rng(7)
    X = synth.from_bags(random_bags(rng, 6, 2, 4, 2))
    Z = synth.from_bags([(rng.normal(size=(3, 2)), [0.5, 0.0, 0.5])])
    z, e1, e3, st = oracle_mod.centroid_update(X, Z, np.zeros(6, dtype=int))
    assert st.max() == 0
    np.testing.assert_array_equal(z[1], Z.points[1])


def test_fixed_nonuniform_weights_flow_sums(oracle_mod):
    """With fixed centroid weights q, every member sends exactly q_r to atom
    r, so the denominator of Eq. (2) is n_j q_r and the new atom is the mean
    over members of (sum_a w_ar v^(a)) / q_r."""
    rng = np.random.default_rng(8)
    X = synth.from_bags(random_bags(rng, 12, 2, 6, 3))
    q = np.array([0.1, 0.2, 0.3, 0.4])
    Z = synth.from_bags([(rng.normal(size=(4, 3)), q * 5.0)])   # normalised inside
    z, e1, e3, st, plans = oracle_mod.centroid_update(X, Z, np.zeros(12, dtype=int),
                                                      return_plans=True)
    for _, _, plan in plans:
        np.testing.assert_allclose(plan.sum(axis=0), q, rtol=0, atol=1e-15)
    want = np.mean([(plan.T @ X.bag(i)[0]) / q[:, None] for i, _, plan in plans], axis=0)
    np.testing.assert_allclose(z, want, rtol=1e-12, atol=1e-12)
