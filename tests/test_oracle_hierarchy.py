"""Pins for the oracle's weighted update (Eq. (4)), labelling within segments
and hierarchical driver (Alg. 3), no GPU.

* integer object weights are the same as repeating each object that many
  times (Eq. (3)-(4) weight the objective and both sums of the mean);
* labelling within segments equals the nearest-centroid labelling of the
  oracle's own assign restricted to the segment's centroids;
* the hierarchy keeps every segment within tau, conserves the total weight
  (the number of original objects), ends with at most k centroids, and no
  final cluster mixes well-separated blobs;
* identical objects, where no split can separate anything, fall back to
  halving and still terminate.
"""
import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle


def test_integer_weights_equal_repetition(oracle_mod):
    rng = np.random.default_rng(41)
    bags = [(rng.normal(size=(t, 2)), rng.dirichlet(np.ones(t))) for t in rng.integers(1, 6, size=12)]
    Z = synth.from_bags([(rng.normal(size=(3, 2)), np.full(3, 1 / 3)) for _ in range(3)])
    labels = rng.integers(0, 3, size=12)
    w = rng.integers(1, 4, size=12)
    X = synth.from_bags(bags)
    Xr = synth.from_bags([b for b, c in zip(bags, w) for _ in range(c)])
    lr = np.repeat(labels, w)
    z, e1, e3, st = oracle_mod.centroid_update(X, Z, labels, weights=w.astype(float))
    zr, f1, f3, _ = oracle_mod.centroid_update(Xr, Z, lr)
    np.testing.assert_allclose(z, zr, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(e1, f1, rtol=1e-12)
    np.testing.assert_allclose(e3, f3, rtol=1e-12)
    bad = w.astype(float)
    bad[3] = -1.0
    st = oracle_mod.centroid_update(X, Z, labels, weights=bad)[3]
    assert st[3] == 1 and (np.delete(st, 3) == 0).all()


def test_segmented_labels_match_restricted_assign(oracle_mod):
    from oracle.hierarchy import assign_segmented
    X = synth.make_data(1)
    Z = synth.make_centroids(1)
    rng = np.random.default_rng(42)
    zoff = np.array([0, 3, 3, 7, 10])        # segment 1 has no centroids
    seg = rng.integers(-1, 4, size=X.n)       # -1: no segment
    lab, best, st = assign_segmented(X, Z, seg, zoff)
    for s in range(4):
        rows = np.flatnonzero(seg == s)
        if zoff[s] == zoff[s + 1]:
            assert (lab[rows] == -1).all() and (st[rows] == 5).all()
            continue
        sub = Z.subset(np.arange(zoff[s], zoff[s + 1]))
        o_lab, o_best, _, _, _ = oracle_mod.assign(X.subset(rows), sub)
        np.testing.assert_array_equal(lab[rows], o_lab + zoff[s])
        np.testing.assert_allclose(best[rows], o_best, rtol=1e-13)
    assert (lab[seg == -1] == -1).all()


def blobs(n_per, centres, rng, spread=0.05):
    bags = []
    for c in centres:
        for _ in range(n_per):
            t = int(rng.integers(1, 5))
            bags.append((c + spread * rng.normal(size=(t, len(c))), rng.dirichlet(np.ones(t))))
    return synth.from_bags(bags)


def test_hierarchy_invariants_and_separated_blobs(oracle_mod):
    from oracle.hierarchy import hierarchy
    rng = np.random.default_rng(43)
    centres = [np.array([0.0, 0.0]), np.array([50.0, 0.0]), np.array([0.0, 50.0]), np.array([50.0, 50.0])]
    X = blobs(60, centres, rng)
    order = rng.permutation(X.n)
    X = X.subset(order)
    truth = np.repeat(np.arange(4), 60)[order]
    U = np.random.default_rng(44).random(10000)
    # the hierarchy stops at the first level with at most k centroids; with
    # 240 objects, tau = 50 and e = 5 that is the second level's ~10
    (off, pts, w), lab, levels, omega = hierarchy(X, tau=50, e=5, k=12, uniforms=U)
    assert levels[-1]["centroids"] <= 12
    assert omega.sum() == X.n
    assert len(levels) >= 2
    assert levels[-1]["centroids"] >= 4
    assert all(lv["max_segment"] <= 50 for lv in levels)
    # no final cluster mixes blobs
    for c in range(lab.max() + 1):
        assert len(set(truth[lab == c])) == 1
    assert lab.min() >= 0 and lab.max() < off.size - 1


def test_identical_objects_fall_back_to_halving(oracle_mod):
    from oracle.hierarchy import hierarchy
    X = synth.from_bags([(np.array([[1.0, 2.0]]), [1.0])] * 130)
    U = np.random.default_rng(45).random(10000)
    (off, pts, w), lab, levels, omega = hierarchy(X, tau=50, e=5, k=3, uniforms=U)
    assert levels[0]["segments"] == 4           # 130 -> 65 + 65 -> 4 x 32/33
    assert omega.sum() == 130
    np.testing.assert_allclose(pts, 1.0 * np.array([[1.0, 2.0]] * pts.shape[0]))


# ---- hand-derived steps of Alg. 3 (tests/golden/hierarchy_steps.json)

import json as _json
import os

_STEPS = _json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hierarchy_steps.json")))


@pytest.mark.parametrize("case", _STEPS["split_positions"], ids=lambda c: f"n{c['n']}")
def test_split_positions_golden(case):
    from oracle import hierarchy as H
    U = H._Uniforms(case["u"])
    assert list(H.split_positions(case["n"], U)) == case["want"], case["derivation"]
    assert U.k == 2


@pytest.mark.parametrize("case", _STEPS["segment_positions"], ids=lambda c: f"n{c['n']}e{c['e']}")
def test_segment_positions_golden(case):
    from oracle import hierarchy as H
    U = H._Uniforms(case["u"])
    assert H.segment_positions(case["n"], case["e"], U) == case["want"], case["derivation"]
    assert U.k == len(case["want"])   # one uniform per group, ceil(n / e) groups


@pytest.mark.parametrize("case", _STEPS["split_sides"], ids=lambda c: str(c["first"]))
def test_split_sides_golden(case):
    from oracle import hierarchy as H
    labels = np.full(max(case["S"]) + 1, -1)
    for i, lab in case["labels"].items():
        labels[int(i)] = lab
    A, B = H.split_sides(np.array(case["S"]), labels, case["first"])
    assert [list(A), list(B)] == case["want"], case["derivation"]


@pytest.mark.parametrize("case", _STEPS["merge_level"], ids=lambda c: "two_segments")
def test_merge_level_golden(case):
    """Eq. (5) offsets, the drop of a cluster without members, member-sum
    weights and the inheritance of Eq. (6), against the written-out case."""
    from oracle import hierarchy as H
    keep, Ct, omega, C = H.merge_level([np.array(s) for s in case["segs"]], case["zoff"],
                                       np.array(case["labels"]), np.array(case["omega"], float),
                                       np.array(case["C"]))
    assert keep == case["want_keep"], case["derivation"]
    assert list(Ct) == case["want_Ct"], case["derivation"]
    assert list(omega) == case["want_omega"], case["derivation"]
    assert list(C) == case["want_C"], case["derivation"]
