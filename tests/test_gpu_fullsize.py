"""Parity at the full workload sizes, in the launch configuration bench.py
times (default schedule and start, graph capture), checked against the
FP64 oracle on seeded samples of the outputs.

* 100,000 x 512 (d=8): all labels and minima of 48 sampled rows.
* 50,000 x 256 (d=128): 24 sampled rows, FP64 cost; and the BF16-MFMA cost
  mode within its error bound.
* The 4,096-object pairwise matrix (8,386,560 pairs): 3,000 sampled pairs,
  plus the condensed index of every sampled pair.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.bf16 import cell_bound, input_rounding_bound, round_bf16
from tests.parity import assert_close, assert_labels, coupling_cost

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


def rows_floor(X, Z, rows, o_lab):
    return np.array([1e-14 * coupling_cost(*X.bag(int(i)), *Z.bag(int(o_lab[k])))
                     for k, i in enumerate(rows)])


@pytest.mark.parametrize("cfg,nrows", [(2, 2048), (3, 256)])
def test_full_assign_sampled_rows(d2, h, cfg, nrows):
    X = synth.make_data(cfg)
    Z = synth.make_centroids(cfg)
    lab, best, _, st = d2.d2_assign(h, d2.DeviceSet.from_ragged(X, DEV),
                                    d2.DeviceSet.from_ragged(Z, DEV), d2.Opts())
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    assert st.max() == 0
    lab = lab.cpu().numpy()
    best = best.cpu().numpy()
    assert lab.min() >= 0 and lab.max() < Z.n
    rows = synth.sample_rows(cfg, X.n, nrows, tag=7)
    sub = X.subset(rows)
    o_lab, o_best, o_all, o_st, _ = oracle.assign(sub, Z)
    assert o_st.max() == 0
    floor = rows_floor(X, Z, rows, o_lab)
    assert_close(best[rows], o_best, floor)
    assert_labels(lab[rows], o_lab, o_all, floor)


def test_full_assign_bf16_sampled_rows(d2, h):
    X = synth.make_data(3)
    Z = synth.make_centroids(3)
    lab, best, _, st = d2.d2_assign(h, d2.DeviceSet.from_ragged(X, DEV),
                                    d2.DeviceSet.from_ragged(Z, DEV), d2.Opts(cost_mode=1))
    torch.cuda.synchronize()
    assert st.cpu().numpy().max() == 0
    best = best.cpu().numpy()
    lab = lab.cpu().numpy()
    rows = synth.sample_rows(3, X.n, 96, tag=8)
    sub = X.subset(rows)
    _, _, o_all, _, _ = oracle.assign(sub, Z)
    for k, i in enumerate(rows):
        x, _ = X.bag(int(i))
        bounds = np.array([cell_bound(round_bf16(x), round_bf16(Z.bag(j)[0])).max()
                           + input_rounding_bound(x, Z.bag(j)[0]).max() for j in range(Z.n)])
        g = best[i]
        # the device's minimum is within the bound of the exact minimum, and
        # its label's exact distance is within twice the bound of it
        assert abs(g - o_all[k].min()) <= bounds.max()
        assert o_all[k, lab[i]] - o_all[k].min() <= 2 * bounds.max()


def test_full_pairwise_sampled_pairs(d2, h):
    X = synth.make_data(4)
    out, st = d2.d2_pairwise(h, d2.DeviceSet.from_ragged(X, DEV), d2.Opts())
    torch.cuda.synchronize()
    n = X.n
    assert out.numel() == n * (n - 1) // 2
    st = st.cpu().numpy()
    assert st.max() == 0
    g = out.cpu().numpy()
    p = synth.sample_pairs(4, n, n, 120000, tag=9)
    p = p[p[:, 0] < p[:, 1]][:60000]
    i, j = p[:, 0], p[:, 1]
    idx = i * n - i * (i + 1) // 2 + (j - i - 1)
    o, o_st, _ = oracle.emd_batch(X, X, p)
    assert o_st.max() == 0
    floor = np.array([1e-14 * coupling_cost(*X.bag(int(a)), *X.bag(int(b))) for a, b in p])
    assert_close(g[idx], o, floor)


@pytest.mark.parametrize("init", [1, 2, 3])
def test_identical_distributions_assign_every_class(d2, h, init):
    """Every object against itself as a centroid (supports 1..64, all four
    classes): D^2 = 0 exactly on the diagonal, under every start rule."""
    rng = np.random.default_rng(41)
    bags = []
    for t in [1, 2, 7, 16, 17, 31, 32, 33, 48, 63, 64]:
        bags.append((rng.normal(size=(t, 5)), rng.dirichlet(np.ones(t))))
    X = synth.from_bags(bags)
    Xd = d2.DeviceSet.from_ragged(X, DEV)
    lab, best, allv, st = d2.d2_assign(h, Xd, Xd, d2.Opts(init=init), want_all=True)
    torch.cuda.synchronize()
    assert st.cpu().numpy().max() == 0
    allv = allv.cpu().numpy()
    assert np.all(np.diag(allv) == 0.0)
    assert np.array_equal(lab.cpu().numpy(), np.arange(X.n))
    o_lab, o_best, o_all, _, _ = oracle.assign(X, X)
    floor = np.array([[1e-14 * coupling_cost(*X.bag(a), *X.bag(b)) for b in range(X.n)]
                      for a in range(X.n)])
    assert_close(allv, o_all, floor)
