"""Pins for the oracle's labelling under the combined distance of Eq. (9)
(sum over feature types of the per-type squared Mallows distance), no GPU.

* one-atom bags in every type: the combined D^2 is the squared Euclidean
  distance between the concatenated points, computed here directly;
* two identical types: every combined value is exactly twice the single
  type's, and the labels are the single type's;
* the root of the combined D^2 is a metric on the product space: triangle
  inequality on random triples;
* a failed pair in any type gives the row label -1.
"""
import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle


def test_one_atom_types_are_concatenated_points(oracle_mod):
    rng = np.random.default_rng(21)
    n, K, dims = 30, 7, [2, 5, 3]
    xs = [rng.normal(size=(n, d)) for d in dims]
    zs = [rng.normal(size=(K, d)) for d in dims]
    Xs = [synth.from_bags([(x[i:i + 1], [1.0]) for i in range(n)]) for x in xs]
    Zs = [synth.from_bags([(z[j:j + 1], [1.0]) for j in range(K)]) for z in zs]
    lab, best, total, st = oracle_mod.assign_multi(Xs, Zs)
    X = np.concatenate(xs, 1); Z = np.concatenate(zs, 1)
    want = ((X[:, None, :] - Z[None, :, :]) ** 2).sum(-1)
    np.testing.assert_allclose(total, want, rtol=1e-13)
    np.testing.assert_array_equal(lab, np.argmin(want, 1))
    assert st.max() == 0


def test_identical_types_double_every_value(oracle_mod):
    X = synth.make_data(1)
    Z = synth.make_centroids(1)
    lab1, best1, all1, _, _ = oracle_mod.assign(X, Z)
    lab, best, total, st = oracle_mod.assign_multi([X, X], [Z, Z])
    assert np.array_equal(total, 2.0 * all1)
    np.testing.assert_array_equal(lab, lab1)
    np.testing.assert_array_equal(best, 2.0 * best1)


def test_combined_root_is_a_metric(oracle_mod):
    rng = np.random.default_rng(22)

    def obj():
        return [(rng.normal(size=(t, d)), rng.dirichlet(np.ones(t)))
                for t, d in zip(rng.integers(1, 6, size=2), [3, 4])]

    objs = [obj() for _ in range(6)]
    A = [synth.from_bags([o[m] for o in objs]) for m in range(2)]
    _, _, total, _ = oracle_mod.assign_multi(A, A)
    D = np.sqrt(np.maximum(total, 0.0))
    assert np.all(np.diag(total) == 0.0)
    np.testing.assert_allclose(D, D.T, rtol=1e-12)
    for a in range(6):
        for b in range(6):
            for c in range(6):
                assert D[a, c] <= D[a, b] + D[b, c] + 1e-12


def test_a_failed_type_fails_the_row(oracle_mod):
    rng = np.random.default_rng(23)
    X1 = synth.from_bags([(rng.normal(size=(3, 2)), rng.dirichlet(np.ones(3))) for _ in range(4)])
    bags = [(rng.normal(size=(2, 3)), rng.dirichlet(np.ones(2))) for _ in range(4)]
    bags[2] = (bags[2][0], np.array([-1.0, 2.0]))
    X2 = synth.from_bags(bags)
    Z1 = synth.from_bags([(rng.normal(size=(3, 2)), np.ones(3)) for _ in range(3)])
    Z2 = synth.from_bags([(rng.normal(size=(2, 3)), np.ones(2)) for _ in range(3)])
    lab, best, total, st = oracle_mod.assign_multi([X1, X2], [Z1, Z2])
    np.testing.assert_array_equal(st, [0, 0, 1, 0])
    assert lab[2] == -1 and np.isnan(best[2])
    assert (lab[[0, 1, 3]] >= 0).all()
