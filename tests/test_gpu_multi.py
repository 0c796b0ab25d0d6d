"""GPU parity of the labelling under the combined distance of Eq. (9)
(d2_assign_multi), through the C ABI, against the FP64 oracle on the same
seeded inputs: the summed matrix element by element at the pair rule's
tolerance (summed floors), labels equal up to near-ties, statuses equal.
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


def floors(Xs, Zs):
    n, K = Xs[0].n, Zs[0].n
    f = np.zeros((n, K))
    for X, Z in zip(Xs, Zs):
        f += np.array([[1e-14 * coupling_cost(*X.bag(i), *Z.bag(j)) for j in range(K)] for i in range(n)])
    return f


def check(d2, h, Xs, Zs, init=0):
    lab, best, allv, st = d2.d2_assign_multi(h, [d2.DeviceSet.from_ragged(X, DEV) for X in Xs],
                                             [d2.DeviceSet.from_ragged(Z, DEV) for Z in Zs],
                                             d2.Opts(init=init), want_all=True)
    torch.cuda.synchronize()
    lab, best, allv, st = (t.cpu().numpy() for t in (lab, best, allv, st))
    o_lab, o_best, o_all, o_st = oracle.assign_multi(Xs, Zs)
    np.testing.assert_array_equal(st, o_st)
    ok = o_st == 0
    fl = floors(Xs, Zs)
    bound = np.maximum(REL * np.abs(o_all), fl)
    assert np.all(np.abs(allv - o_all)[ok] <= bound[ok])
    for i in np.flatnonzero(ok):
        if lab[i] != o_lab[i]:
            assert o_all[i, lab[i]] - o_all[i, o_lab[i]] <= bound[i].max(), f"row {i}"
    assert np.all(lab[~ok] == -1)
    assert np.all(np.abs(best[ok] - o_best[ok]) <= np.max(bound, axis=1)[ok])
    return lab, allv


def random_types(rng, n, K, spec):
    Xs, Zs = [], []
    for tmax, s, d in spec:
        Xs.append(synth.from_bags([(rng.normal(size=(t, d)) * 2, rng.dirichlet(np.ones(t)))
                                   for t in rng.integers(1, tmax + 1, size=n)]))
        Zs.append(synth.from_bags([(rng.normal(size=(s, d)) * 2, rng.dirichlet(np.ones(s)))
                                   for _ in range(K)]))
    return Xs, Zs


@pytest.mark.parametrize("init", [0, 1, 2])
def test_colour_and_texture_types(d2, h, init):
    """Two types of different dimension and support, as an image's colour and
    texture bags."""
    rng = np.random.default_rng(31 + init)
    Xs, Zs = random_types(rng, 60, 9, [(8, 6, 3), (20, 12, 6)])
    check(d2, h, Xs, Zs, init)


def test_three_types_every_class(d2, h):
    rng = np.random.default_rng(34)
    Xs, Zs = random_types(rng, 40, 5, [(16, 16, 2), (32, 20, 4), (64, 40, 3)])
    check(d2, h, Xs, Zs)


def test_identical_types_double_the_single_type(d2, h):
    X = synth.make_data(1)
    Z = synth.make_centroids(1)
    Xd, Zd = d2.DeviceSet.from_ragged(X, DEV), d2.DeviceSet.from_ragged(Z, DEV)
    _, _, a1, _ = d2.d2_assign(h, Xd, Zd, want_all=True)
    lab, _, a2, _ = d2.d2_assign_multi(h, [Xd, Xd], [Zd, Zd], want_all=True)
    torch.cuda.synchronize()
    assert torch.equal(a2, 2.0 * a1)
    check(d2, h, [X, X], [Z, Z])


def test_failed_pair_in_one_type(d2, h):
    rng = np.random.default_rng(35)
    Xs, Zs = random_types(rng, 12, 4, [(6, 5, 2), (6, 5, 3)])
    w = Xs[1].weights.copy()
    w[int(Xs[1].offsets[5])] = np.nan
    Xs[1] = synth.RaggedSet(Xs[1].offsets, Xs[1].points, w)
    lab, _ = check(d2, h, Xs, Zs)
    assert lab[5] == -1


def test_single_type_equals_assign(d2, h):
    X = synth.make_data(2, n=3000)
    Z = synth.make_centroids(2)
    Xd, Zd = d2.DeviceSet.from_ragged(X, DEV), d2.DeviceSet.from_ragged(Z, DEV)
    l1, b1, _, _ = d2.d2_assign(h, Xd, Zd)
    l2, b2, _, _ = d2.d2_assign_multi(h, [Xd], [Zd])
    torch.cuda.synchronize()
    assert torch.equal(l1, l2) and torch.equal(b1, b2)


def test_bf16_mode_is_the_sum_of_the_types(d2, h):
    """The BF16-MFMA cost mode through the multi-type path equals the sum of
    the per-type BF16 matrices, bit for bit (each type runs the same launch;
    one FP64 addition per cell)."""
    rng = np.random.default_rng(36)
    Xs, Zs = random_types(rng, 50, 7, [(16, 16, 40), (24, 20, 33)])
    Xs = [X.astype(np.float32) for X in Xs]
    Zs = [Z.astype(np.float32) for Z in Zs]
    Xd = [d2.DeviceSet.from_ragged(X, DEV) for X in Xs]
    Zd = [d2.DeviceSet.from_ragged(Z, DEV) for Z in Zs]
    opts = d2.Opts(cost_mode=d2.D2_COST_BF16_MFMA)
    singles = [d2.d2_assign(h, x, z, opts, want_all=True)[2] for x, z in zip(Xd, Zd)]
    lab, best, allv, st = d2.d2_assign_multi(h, Xd, Zd, opts, want_all=True)
    torch.cuda.synchronize()
    assert int(st.max()) == 0
    assert torch.equal(allv, singles[0] + singles[1])
    assert torch.equal(best, allv.min(dim=1).values)
