"""Host-side helpers of bench.py: the seeded pivot samples and the work
arithmetic that the pivot-weighted roofline uses (no GPU)."""
import numpy as np
import pytest

import bench
import synth


@pytest.mark.parametrize("cfg", [1, 2, 3, 4, 5])
def test_pivot_sample_is_valid_and_seeded(cfg):
    A, B, pairs, d = bench.pivot_sample(cfg, count=512)
    assert pairs.ndim == 2 and pairs.shape[1] == 2 and pairs.shape[0] > 0
    assert pairs.min() >= 0 and pairs[:, 0].max() < A.n and pairs[:, 1].max() < B.n
    assert d == synth.CONFIGS[cfg]["d"] == A.points.shape[1] == B.points.shape[1]
    assert np.unique(pairs, axis=0).shape[0] == pairs.shape[0]
    if cfg == 4:
        assert np.all(pairs[:, 0] < pairs[:, 1])       # one orientation of each object pair
    _, _, again, _ = bench.pivot_sample(cfg, count=512)
    np.testing.assert_array_equal(pairs, again)


def test_work_factor_closed_forms():
    ts, ss = np.array([4, 16, 9]), np.array([16, 16, 2])
    # no pivots: only the certifying pass, which the lower bound already counts
    assert bench.pivot_work_factor(ts, ss, np.zeros(3), 8) == pytest.approx(1.0)
    # P pivots on every pair: (3d + 3(P + 1)) / (3d + 3), whatever the supports
    for d, p in ((8, 7), (128, 21), (3, 0)):
        want = (3 * d + 3 * (p + 1)) / (3 * d + 3)
        assert bench.pivot_work_factor(ts, ss, np.full(3, p), d) == pytest.approx(want)
    # pairs weigh by t s: one pivot on the 16 x 16 pair alone
    got = bench.pivot_work_factor(ts, ss, np.array([0, 1, 0]), 1)
    w = ts * ss
    assert got == pytest.approx((w.sum() * 6 + w[1] * 3) / (w.sum() * 6))


def test_pivot_summary():
    s = bench._pivot_summary(np.array([0, 0, 2, 4, 10]))
    assert s["mean"] == pytest.approx(3.2) and s["p50"] == 2.0 and s["max"] == 10
    assert s["zero_frac"] == pytest.approx(0.4)
    # bins 0 | 1-2 | 3-4 | 5-8 | 9-16 | 17-32 | 33-64 | 65-128 | 129-256 | >256
    assert s["hist"] == [2, 1, 1, 0, 1, 0, 0, 0, 0, 0]
    h = bench._pivot_summary(np.array([1, 2, 3, 8, 9, 16, 17, 64, 65, 128, 129, 256, 257, 9999]))["hist"]
    assert h == [0, 2, 1, 1, 2, 1, 1, 2, 2, 2]


def test_fast_pair_tolerance_equals_the_per_pair_one():
    """The moment form of the independent-coupling cost (used to check every
    pair of a pairwise matrix) against the direct double sum."""
    from tests.parity import pair_tolerance, pair_tolerance_fast
    X = synth.make_data(4, n=120)
    Z = synth.make_centroids(2)
    Y = synth.make_data(2, n=60)
    rng = np.random.default_rng(3)
    p = np.stack([rng.integers(0, 120, 800), rng.integers(0, 120, 800)], 1)
    np.testing.assert_allclose(pair_tolerance_fast(X, X, p), pair_tolerance(X, X, p), rtol=1e-12)
    q = np.stack([rng.integers(0, 60, 300), rng.integers(0, 512, 300)], 1)
    np.testing.assert_allclose(pair_tolerance_fast(Y, Z, q), pair_tolerance(Y, Z, q), rtol=1e-12)
