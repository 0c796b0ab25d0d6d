"""GPU checks of the BF16-MFMA cost mode, through the C ABI.

The mode is approximate by design, so it is held to two bounds instead of
the FP64 tolerance (derivations in tests/bf16.py):
  * against the exact costs of the BF16-rounded points, every cost cell
    and every D^2 within the FP32 accumulation bound of its pair;
  * against the FP64 oracle on the original points, within that bound plus
    the input-rounding bound.
Integer-valued points make every step exact, which pins the MFMA operand
layout and the tile orientation bit for bit.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.bf16 import cell_bound, input_rounding_bound, round_bf16, rounded_set
from tests.parity import pair_tolerance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"
BF16 = 1


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


def dev(d2, S):
    return d2.DeviceSet.from_ragged(S, DEV)


def integer_set(seed, n, d, tmax=32, lo=-6, hi=6):
    rng = np.random.default_rng(seed)
    bags = []
    for _ in range(n):
        t = int(rng.integers(1, tmax + 1))
        bags.append((rng.integers(lo, hi + 1, size=(t, d)).astype(np.float64),
                     rng.dirichlet(np.ones(t))))
    return synth.from_bags(bags)


def pair_bound(A, B, pairs, rounding=False):
    out = np.empty(len(pairs))
    for k, (i, j) in enumerate(pairs):
        x, _ = A.bag(int(i)); y, _ = B.bag(int(j))
        xr, yr = round_bf16(x), round_bf16(y)
        b = cell_bound(xr, yr).max()
        if rounding:
            b += input_rounding_bound(x, y).max()
        out[k] = b
    return out


def tiles_of(d2, h, A, B, pairs):
    t, off = d2.d2_cost_tiles(h, dev(d2, A), dev(d2, B), torch.as_tensor(pairs), cost_mode=BF16)
    torch.cuda.synchronize()
    return t.cpu().numpy(), off.cpu().numpy()


def test_tiles_exact_on_integer_points(d2, h):
    # |coordinates| <= 6, d = 40: every product, norm and sum is exact in
    # FP32, so the MFMA tile must equal the exact cost bit for bit
    A = integer_set(1, 9, 40)
    B = integer_set(2, 7, 40)
    pairs = np.array([(i, j) for i in range(A.n) for j in range(B.n)])
    t, off = tiles_of(d2, h, A, B, pairs)
    for k, (i, j) in enumerate(pairs):
        x, _ = A.bag(i); y, _ = B.bag(j)
        C = ((x[:, None] - y[None]) ** 2).sum(-1)
        assert np.array_equal(t[off[k]:off[k + 1]].reshape(C.shape), C), (i, j)


@pytest.mark.parametrize("cfg,dt", [(3, "f32"), (2, "f64")])
def test_tiles_within_fp32_bound(d2, h, cfg, dt):
    A = synth.make_data(cfg, n=14)
    B = synth.make_centroids(cfg, k=9)
    if dt == "f64":
        A, B = A.astype(np.float64), B.astype(np.float64)
    pairs = np.array([(i, j) for i in range(A.n) for j in range(B.n)])
    t, off = tiles_of(d2, h, A, B, pairs)
    for k, (i, j) in enumerate(pairs):
        x, _ = A.bag(i); y, _ = B.bag(j)
        xr, yr = round_bf16(x), round_bf16(y)
        C = ((xr[:, None] - yr[None]) ** 2).sum(-1)
        g = t[off[k]:off[k + 1]].reshape(C.shape)
        assert np.all(g >= 0)
        assert np.all(np.abs(g - C) <= cell_bound(xr, yr)), (i, j)


def test_tiles_transpose_symmetric(d2, h):
    A = synth.make_data(3, n=10)
    pairs = np.array([(i, j) for i in range(A.n) for j in range(A.n)])
    t, off = tiles_of(d2, h, A, A, pairs)
    sz = np.diff(A.offsets)
    idx = {(int(i), int(j)): k for k, (i, j) in enumerate(pairs)}
    for (i, j), k in idx.items():
        a = t[off[k]:off[k + 1]].reshape(sz[i], sz[j])
        b = t[off[idx[(j, i)]]:off[idx[(j, i)] + 1]].reshape(sz[j], sz[i])
        assert np.array_equal(a, b.T)


def test_assign_exact_on_integer_points(d2, h):
    X = integer_set(3, 30, 24)
    Z = integer_set(4, 12, 24)
    lab, best, allv, st = d2.d2_assign(h, dev(d2, X), dev(d2, Z), d2.Opts(cost_mode=BF16),
                                       want_all=True)
    torch.cuda.synchronize()
    o_lab, o_best, o_all, o_st, _ = oracle.assign(X, Z)
    assert st.cpu().numpy().max() == 0
    pairs = np.array([(i, j) for i in range(X.n) for j in range(Z.n)])
    tol = pair_tolerance(X, Z, pairs).reshape(X.n, Z.n)
    g = allv.cpu().numpy()
    assert np.all(np.abs(g - o_all) <= np.maximum(1e-10 * np.abs(o_all), tol))


@pytest.mark.parametrize("init", [0, 2])
def test_assign_within_bound_of_rounded_oracle(d2, h, init):
    X = synth.make_data(3, n=24)
    Z = synth.make_centroids(3, k=20)
    lab, best, allv, st = d2.d2_assign(h, dev(d2, X), dev(d2, Z),
                                       d2.Opts(cost_mode=BF16, init=init), want_all=True)
    torch.cuda.synchronize()
    assert st.cpu().numpy().max() == 0
    Xr, Zr = rounded_set(X), rounded_set(Z)
    o_lab, o_best, o_all, o_st, _ = oracle.assign(Xr, Zr)
    pairs = np.array([(i, j) for i in range(X.n) for j in range(Z.n)])
    bnd = pair_bound(X, Z, pairs).reshape(X.n, Z.n)
    g = allv.cpu().numpy()
    assert np.all(np.abs(g - o_all) <= bnd)
    # labels: the device's pick is within the bound of the oracle's minimum
    glab = lab.cpu().numpy()
    for i in range(X.n):
        assert o_all[i, glab[i]] - o_all[i, o_lab[i]] <= 2 * bnd[i].max()
    assert np.array_equal(best.cpu().numpy(), g[np.arange(X.n), glab])


def test_assign_error_against_fp64_oracle(d2, h):
    X = synth.make_data(3, n=16)
    Z = synth.make_centroids(3, k=16)
    _, _, allv, st = d2.d2_assign(h, dev(d2, X), dev(d2, Z), d2.Opts(cost_mode=BF16),
                                  want_all=True)
    torch.cuda.synchronize()
    _, _, o_all, _, _ = oracle.assign(X, Z)
    pairs = np.array([(i, j) for i in range(X.n) for j in range(Z.n)])
    bnd = pair_bound(X, Z, pairs, rounding=True).reshape(X.n, Z.n)
    err = np.abs(allv.cpu().numpy() - o_all)
    assert np.all(err <= bnd)
    print(f"BF16 D^2 relative error vs FP64: max {np.max(err / o_all):.3e}, "
          f"median {np.median(err / o_all):.3e}")


def test_assign_row_blocks(d2, h):
    # K = 2048 centroids: 8 MiB of tiles per row, 128 rows per block, so 300
    # rows take three blocks; rows at the block edges go to the oracle
    rng = np.random.default_rng(8)
    Z = synth.from_bags([(rng.normal(size=(int(t), 6)), rng.dirichlet(np.ones(int(t))))
                         for t in rng.integers(1, 9, 2048)])
    X = synth.from_bags([(rng.normal(size=(int(t), 6)), rng.dirichlet(np.ones(int(t))))
                         for t in rng.integers(1, 9, 300)])
    lab, best, allv, st = d2.d2_assign(h, dev(d2, X), dev(d2, Z), d2.Opts(cost_mode=BF16),
                                       want_all=True)
    torch.cuda.synchronize()
    g = allv.cpu().numpy()
    glab = lab.cpu().numpy()
    assert st.cpu().numpy().max() == 0
    assert np.array_equal(glab, np.argmin(g, axis=1))
    assert np.array_equal(best.cpu().numpy(), g.min(axis=1))
    rows = [0, 127, 128, 255, 256, 299]
    Xs = rounded_set(X).subset(rows)
    _, _, o_all, _, _ = oracle.assign(Xs, rounded_set(Z))
    pairs = np.array([(i, j) for i in rows for j in range(Z.n)])
    bnd = pair_bound(X, Z, pairs).reshape(len(rows), Z.n)
    assert np.all(np.abs(g[rows] - o_all) <= bnd)


def test_assign_repeat_is_bitwise(d2, h):
    X = synth.make_data(3, n=20)
    Z = synth.make_centroids(3, k=12)
    Xd, Zd = dev(d2, X), dev(d2, Z)
    outs = []
    for flags in (0, 0, 1):   # graph capture, replay, eager
        _, _, allv, _ = d2.d2_assign(h, Xd, Zd, d2.Opts(cost_mode=BF16, flags=flags), want_all=True)
        torch.cuda.synchronize()
        outs.append(allv.cpu().numpy())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_bad_points_flagged(d2, h):
    X = synth.make_data(3, n=4).astype(np.float64)
    X.points[X.offsets[2]] = np.nan
    Z = synth.make_centroids(3, k=3).astype(np.float64)
    lab, best, _, st = d2.d2_assign(h, dev(d2, X), dev(d2, Z), d2.Opts(cost_mode=BF16))
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    assert st[2] == 4 and lab.cpu().numpy()[2] == -1
    assert np.all(st[[0, 1, 3]] == 0)


def test_unsupported_shapes_and_calls(d2, h):
    X = synth.make_data(3, n=4)
    Z = synth.make_centroids(3, k=3)
    Xd, Zd = dev(d2, X), dev(d2, Z)
    big = dev(d2, X)
    big.max_support = 33
    with pytest.raises(d2.D2Error) as e:
        d2.d2_assign(h, big, Zd, d2.Opts(cost_mode=BF16))
    assert e.value.code == 3
    with pytest.raises(d2.D2Error) as e:
        d2.d2_pairwise(h, Xd, d2.Opts(cost_mode=BF16))
    assert e.value.code == 3
    with pytest.raises(d2.D2Error) as e:
        d2.d2_emd_batch(h, Xd, Zd, torch.tensor([[0, 0]]), d2.Opts(cost_mode=BF16))
    assert e.value.code == 3
