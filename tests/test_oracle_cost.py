"""Pins for the oracle's transport LP with a given cost matrix and for the MM
distance of Eq. (10) built on it, no GPU.

The given-cost LP is pinned by an independent LP solver (HiGHS through
scipy) on costs of both signs, by the assignment solver for equal weights,
and by the exact invariance of transport LPs under C_ab + a_a + b_b.  The MM
distance is pinned on one-atom centroids, where every D^2(z_i, z'_j) is a
plain squared distance and the outer LP goes to HiGHS; and by the metric
properties the MM distance inherits as a Wasserstein distance over the
Mallows metric (zero on itself, symmetry, triangle inequality on its root).
"""
import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment, linprog

import synth


@pytest.fixture(scope="module")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle


def highs(C, p, q):
    C = np.asarray(C, float)
    t, s = C.shape
    p = np.asarray(p, float) / np.sum(p)
    q = np.asarray(q, float) / np.sum(q)
    A = np.zeros((t + s, t * s))
    for a in range(t):
        A[a, a * s:(a + 1) * s] = 1.0
    for b in range(s):
        A[t + b, b::s] = 1.0
    res = linprog(C.ravel(), A_eq=A, b_eq=np.concatenate([p, q]), bounds=(0, None),
                  method="highs", options={"primal_feasibility_tolerance": 1e-10,
                                           "dual_feasibility_tolerance": 1e-10})
    assert res.status == 0
    return res.fun


@pytest.mark.parametrize("seed", range(8))
def test_given_cost_against_highs(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    t, s = rng.integers(1, 12, size=2)
    C = rng.normal(size=(t, s)) * rng.choice([0.01, 1.0, 100.0])
    p = rng.dirichlet(np.full(t, 0.5))
    q = rng.dirichlet(np.full(s, 0.5))
    for init in (oracle_mod.INIT_NWC, oracle_mod.INIT_VOGEL):
        v, plan, u, vv, _ = oracle_mod.emd_cost(C, p, q, init)
        assert v == pytest.approx(highs(C, p, q), rel=1e-8, abs=1e-9 * np.abs(C).max())
        np.testing.assert_allclose(plan.sum(axis=1), p / p.sum(), atol=1e-13)
        np.testing.assert_allclose(plan.sum(axis=0), q / q.sum(), atol=1e-13)
        assert plan.min() >= 0.0
        assert float((plan * C).sum()) == pytest.approx(v, rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("n", [2, 5, 9])
def test_equal_weights_assignment(oracle_mod, n):
    rng = np.random.default_rng(n)
    C = rng.uniform(-3, 7, size=(n, n))
    r, c = linear_sum_assignment(C)
    v = oracle_mod.emd_cost(C, np.ones(n), np.ones(n))[0]
    assert v == pytest.approx(C[r, c].sum() / n, rel=1e-12)


def test_row_and_column_shifts_move_the_value_exactly(oracle_mod):
    rng = np.random.default_rng(11)
    t, s = 7, 5
    C = rng.uniform(0, 4, size=(t, s))
    p = rng.dirichlet(np.ones(t)); q = rng.dirichlet(np.ones(s))
    a = rng.normal(size=t); b = rng.normal(size=s)
    v0 = oracle_mod.emd_cost(C, p, q)[0]
    v1 = oracle_mod.emd_cost(C + a[:, None] + b[None, :], p, q)[0]
    assert v1 == pytest.approx(v0 + p @ a + q @ b, rel=1e-12, abs=1e-13)


def test_squared_distance_cost_matches_the_point_form(oracle_mod):
    rng = np.random.default_rng(12)
    x = rng.normal(size=(6, 3)); y = rng.normal(size=(9, 3))
    p = rng.dirichlet(np.ones(6)); q = rng.dirichlet(np.ones(9))
    C = ((x[:, None, :] - y[None, :, :]) ** 2).sum(-1)
    assert oracle_mod.emd_cost(C, p, q)[0] == pytest.approx(oracle_mod.emd_pair(x, p, y, q)[0],
                                                           rel=1e-12)


def test_non_finite_cost_is_rejected(oracle_mod):
    C = np.ones((3, 3)); C[1, 2] = np.inf
    with pytest.raises(ArithmeticError) as e:
        oracle_mod.emd_cost(C, np.ones(3), np.ones(3))
    assert e.value.status == 4


def test_mm_distance_one_atom_centroids_against_highs(oracle_mod):
    rng = np.random.default_rng(13)
    A = rng.normal(size=(6, 2)) * 3; B = rng.normal(size=(8, 2)) * 3
    Z1 = synth.from_bags([(a[None, :], [1.0]) for a in A])
    Z2 = synth.from_bags([(b[None, :], [1.0]) for b in B])
    p1 = rng.dirichlet(np.ones(6)); p2 = rng.dirichlet(np.ones(8))
    mm2, M, plan = oracle_mod.mm_distance(Z1, p1, Z2, p2)
    want_M = ((A[:, None, :] - B[None, :, :]) ** 2).sum(-1)
    np.testing.assert_allclose(M, want_M, rtol=1e-13, atol=1e-13)
    assert mm2 == pytest.approx(highs(want_M, p1, p2), rel=1e-8)


def test_mm_distance_metric_properties(oracle_mod):
    rng = np.random.default_rng(14)

    def cset(k):
        return synth.from_bags([(rng.normal(size=(t, 3)), rng.dirichlet(np.ones(t)))
                                for t in rng.integers(1, 6, size=k)]), rng.dirichlet(np.ones(k))

    (Za, pa), (Zb, pb), (Zc, pc) = cset(5), cset(4), cset(6)
    assert oracle_mod.mm_distance(Za, pa, Za, pa)[0] == 0.0
    ab = oracle_mod.mm_distance(Za, pa, Zb, pb)[0]
    ba = oracle_mod.mm_distance(Zb, pb, Za, pa)[0]
    assert ab == pytest.approx(ba, rel=1e-12)
    bc = oracle_mod.mm_distance(Zb, pb, Zc, pc)[0]
    ac = oracle_mod.mm_distance(Za, pa, Zc, pc)[0]
    assert np.sqrt(ac) <= np.sqrt(ab) + np.sqrt(bc) + 1e-12
    assert ab > 0.0
