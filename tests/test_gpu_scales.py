"""GPU: the lane-group solver at extreme scales, against exact invariants
and the oracle.

* Scaling every point by a power of two scales every squared cost, every
  potential and the tolerance by its square, exactly in binary, so the pivot
  path is the same and D^2 scales by exactly that factor (no overflow or
  subnormals at the factors used).
* Very uneven weights (Dirichlet(0.02): most weights many orders of
  magnitude below the largest) still give the oracle's values.
Pairs cover every lane-group class (supports up to 64 on both sides)."""
import numpy as np
import pytest

import oracle
import synth
from tests.parity import assert_close, pair_tolerance

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


def bags(rng, n, sizes, d, alpha, scale=1.0):
    out = []
    for k in range(n):
        t = int(sizes[k % len(sizes)])
        x = rng.normal(size=(t, d)) * scale + rng.uniform(-5, 5, size=d)
        w = rng.dirichlet(np.full(t, alpha))
        out.append((x, w))
    return out


def emd(d2, A, B, pairs, init):
    h = d2.Handle(0)
    dist, st, _, _, piv = d2.d2_emd_batch(h, d2.DeviceSet.from_ragged(A, DEV),
                                          d2.DeviceSet.from_ragged(B, DEV), torch.as_tensor(pairs),
                                          d2.Opts(init=init), want_pivots=True)
    torch.cuda.synchronize()
    return dist.cpu().numpy(), st.cpu().numpy(), piv.cpu().numpy()


def scaled(S, f):
    return synth.RaggedSet(S.offsets.copy(), S.points * f, S.weights.copy())


@pytest.mark.parametrize("init", [1, 3])     # north-west corner, least cost
def test_power_of_two_scaling_is_exact(d2, init):
    rng = np.random.default_rng(77)
    A = synth.from_bags(bags(rng, 24, [5, 16, 20, 32, 40, 64], 6, 0.7))
    B = synth.from_bags(bags(rng, 24, [8, 16, 30, 33, 64], 6, 0.7))
    pairs = np.stack(np.meshgrid(np.arange(A.n), np.arange(B.n)), -1).reshape(-1, 2).astype(np.int64)
    base, st, piv = emd(d2, A, B, pairs, init)
    assert np.all(st == 0)
    for k in (-20, 20):
        f = 2.0 ** k
        got, st2, piv2 = emd(d2, scaled(A, f), scaled(B, f), pairs, init)
        assert np.all(st2 == 0)
        np.testing.assert_array_equal(piv2, piv)
        np.testing.assert_array_equal(got, base * (f * f))


def test_very_uneven_weights_match_oracle(d2):
    rng = np.random.default_rng(78)
    A = synth.from_bags(bags(rng, 20, [7, 16, 25, 48, 64], 4, 0.02))
    B = synth.from_bags(bags(rng, 20, [9, 16, 32, 50, 64], 4, 0.02))
    assert A.weights.min() < 1e-30            # the law gives weights far below the largest
    pairs = np.stack(np.meshgrid(np.arange(A.n), np.arange(B.n)), -1).reshape(-1, 2).astype(np.int64)
    o_d, o_st, _ = oracle.emd_batch(A, B, pairs)
    assert np.all(o_st == 0)
    for init in (1, 2, 3):
        g, st, _ = emd(d2, A, B, pairs, init)
        assert np.all(st == 0), (init, np.unique(st))
        assert_close(g, o_d, pair_tolerance(A, B, pairs))


def test_workgroup_simplex_scaling_is_exact(d2):
    """Supports beyond 64 run on the workgroup simplex; its costs, pointer-
    jumped potentials and block pricing scale the same way."""
    rng = np.random.default_rng(79)
    A = synth.from_bags(bags(rng, 4, [96, 130], 5, 0.7))
    B = synth.from_bags(bags(rng, 4, [80, 160], 5, 0.7))
    pairs = np.stack(np.meshgrid(np.arange(A.n), np.arange(B.n)), -1).reshape(-1, 2).astype(np.int64)
    base, st, piv = emd(d2, A, B, pairs, 3)
    assert np.all(st == 0)
    for k in (-20, 20):
        f = 2.0 ** k
        got, st2, piv2 = emd(d2, scaled(A, f), scaled(B, f), pairs, 3)
        assert np.all(st2 == 0)
        np.testing.assert_array_equal(piv2, piv)
        np.testing.assert_array_equal(got, base * (f * f))


def test_bf16_mode_scaling_is_exact(d2):
    """BF16-MFMA cost mode: rounding to BF16 commutes with a power-of-two
    factor, and the FP32 products, norms and sums scale exactly, so every
    D^2 scales by the factor squared, bit for bit."""
    rng = np.random.default_rng(80)
    X = synth.from_bags(bags(rng, 40, [4, 11, 16, 23, 32], 64, 0.7), np.float32)
    Z = synth.from_bags(bags(rng, 24, [8, 16, 32], 64, 0.7), np.float32)
    h = d2.Handle(0)

    def run(f):
        Xs = synth.RaggedSet(X.offsets.copy(), (X.points * np.float32(f)).astype(np.float32), X.weights)
        Zs = synth.RaggedSet(Z.offsets.copy(), (Z.points * np.float32(f)).astype(np.float32), Z.weights)
        lab, best, allv, st = d2.d2_assign(h, d2.DeviceSet.from_ragged(Xs, DEV),
                                           d2.DeviceSet.from_ragged(Zs, DEV),
                                           d2.Opts(cost_mode=d2.D2_COST_BF16_MFMA), want_all=True)
        torch.cuda.synchronize()
        assert int(st.max().item()) == 0
        return lab.cpu().numpy(), allv.cpu().numpy()
    lab0, all0 = run(1.0)
    for k in (-16, 16):
        f = 2.0 ** k
        lab, allv = run(f)
        np.testing.assert_array_equal(lab, lab0)
        np.testing.assert_array_equal(allv, all0 * (f * f))


def test_bf16_mode_is_exact_on_small_integer_points(d2):
    """Integer coordinates in [-8, 8] are exact in BF16, and at d = 64 every
    product, norm and sum of the FP32 cost stays below 2^24, so the BF16-MFMA
    cost tile equals the FP64 direct one and the whole solve is the FP64
    path's, bit for bit."""
    rng = np.random.default_rng(81)

    def mk(n, sizes):
        return synth.from_bags([(rng.integers(-8, 9, size=(int(sizes[k % len(sizes)]), 64)).astype(np.float64),
                                 rng.dirichlet(np.ones(int(sizes[k % len(sizes)]))))
                                for k in range(n)], np.float32)
    X, Z = mk(36, [3, 9, 16, 21, 32]), mk(20, [8, 16, 32])
    h = d2.Handle(0)
    Xd, Zd = d2.DeviceSet.from_ragged(X, DEV), d2.DeviceSet.from_ragged(Z, DEV)
    outs = []
    for mode in (d2.D2_COST_F64_DIRECT, d2.D2_COST_BF16_MFMA):
        lab, best, allv, st = d2.d2_assign(h, Xd, Zd, d2.Opts(cost_mode=mode), want_all=True)
        torch.cuda.synchronize()
        assert int(st.max().item()) == 0
        outs.append((lab.cpu().numpy(), allv.cpu().numpy()))
    np.testing.assert_array_equal(outs[1][1], outs[0][1])
    np.testing.assert_array_equal(outs[1][0], outs[0][0])


def test_bf16_cost_tiles_are_exact_on_small_integer_points(d2):
    """The stand-alone cost-tile entry in its BF16-MFMA mode returns the FP64
    tiles exactly on inputs where its arithmetic is exact (as above)."""
    rng = np.random.default_rng(82)

    def mk(n, sizes):
        return synth.from_bags([(rng.integers(-8, 9, size=(int(sizes[k % len(sizes)]), 40)).astype(np.float64),
                                 rng.dirichlet(np.ones(int(sizes[k % len(sizes)]))))
                                for k in range(n)], np.float32)
    A, B = mk(10, [1, 7, 16, 32]), mk(9, [5, 16, 20, 32])      # the BF16 mode's supports (<= 32)
    pairs = np.stack(np.meshgrid(np.arange(A.n), np.arange(B.n)), -1).reshape(-1, 2).astype(np.int64)
    h = d2.Handle(0)
    Ad, Bd = d2.DeviceSet.from_ragged(A, DEV), d2.DeviceSet.from_ragged(B, DEV)
    f64, off64 = d2.d2_cost_tiles(h, Ad, Bd, torch.as_tensor(pairs), cost_mode=d2.D2_COST_F64_DIRECT)
    b16, off16 = d2.d2_cost_tiles(h, Ad, Bd, torch.as_tensor(pairs), cost_mode=d2.D2_COST_BF16_MFMA)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(off16.cpu().numpy(), off64.cpu().numpy())
    np.testing.assert_array_equal(b16.cpu().numpy().astype(np.float64), f64.cpu().numpy())
