"""GPU: the Bland anti-cycling branch of both device solvers, against the
oracle, through d2_emd_batch's per-pair pivot counts.

The paper leaves the LP solver, and so cycling, open; both sides switch from
Dantzig's rule to Bland's after a run of degenerate pivots (2(t+s) by
default, `bland_after` when given).  The family here is the degenerate one
of synth.make_degenerate: equal weights with power-of-two supports and
integer grid points, so every flow, cost, potential and objective is exact
in binary.  On it the lane-group solver started from the north-west corner
takes exactly the oracle's pivot path, so pivot and Bland counts must agree
pair by pair, as must the values, bit for bit.  The workgroup solver prices
in blocks, so only its values are compared, with its Bland count shown to
be non-zero.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.parity import assert_close, pair_tolerance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEV = "cuda:0"
NWC = 1


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


def run(d2, h, A, B, pairs, opts):
    dist, st, _, _, piv = d2.d2_emd_batch(h, d2.DeviceSet.from_ragged(A, DEV),
                                          d2.DeviceSet.from_ragged(B, DEV),
                                          torch.as_tensor(pairs), opts, want_pivots=True)
    torch.cuda.synchronize()
    return dist.cpu().numpy(), st.cpu().numpy(), piv.cpu().numpy()


# one shape per lane-group class: 16, 32, 64 x 32 and 64 x 64 lanes/columns
@pytest.mark.parametrize("t,s", [(16, 16), (32, 32), (64, 32), (64, 64)])
@pytest.mark.parametrize("bland_after", [1, 3])
def test_lane_group_bland_path_is_the_oracle_path(d2, h, t, s, bland_after):
    A, B, pairs = synth.make_degenerate(11, 12, t, s)
    o_d, o_st, o_piv, o_bl = oracle.emd_batch_stats(A, B, pairs, bland_after=bland_after)
    assert np.all(o_st == 0) and np.all(o_bl > 0)      # the family reaches Bland's rule
    g_d, g_st, g_piv = run(d2, h, A, B, pairs, d2.Opts(init=NWC, bland_after=bland_after))
    assert np.all(g_st == 0), g_st
    np.testing.assert_array_equal(g_d, o_d)
    np.testing.assert_array_equal(g_piv[:, 0], o_piv)
    np.testing.assert_array_equal(g_piv[:, 1], o_bl)


@pytest.mark.parametrize("t,s", [(16, 16), (64, 64)])
def test_default_threshold_counts_match(d2, h, t, s):
    """At the default threshold the family does not reach Bland's rule on
    either side, and the pivot counts still agree."""
    A, B, pairs = synth.make_degenerate(12, 8, t, s)
    o_d, o_st, o_piv, o_bl = oracle.emd_batch_stats(A, B, pairs)
    g_d, g_st, g_piv = run(d2, h, A, B, pairs, d2.Opts(init=NWC))
    assert np.all(g_st == 0)
    np.testing.assert_array_equal(g_d, o_d)
    np.testing.assert_array_equal(g_piv[:, 0], o_piv)
    assert np.all(g_piv[:, 1] == 0) and np.all(o_bl == 0)


def test_default_start_reports_pivots(d2, h):
    """Under the least-cost start the counts are the device's own: at most
    the cap, Bland's share at most the total."""
    A, B, pairs = synth.make_degenerate(13, 16, 32, 32)
    o_d, _, _, _ = oracle.emd_batch_stats(A, B, pairs)
    g_d, g_st, g_piv = run(d2, h, A, B, pairs, d2.Opts(bland_after=2))
    assert np.all(g_st == 0)
    np.testing.assert_array_equal(g_d, o_d)
    assert np.all(g_piv[:, 1] <= g_piv[:, 0]) and np.all(g_piv[:, 0] <= 50 * 32 * 32)


@pytest.mark.parametrize("bland_after", [1, 4])
def test_workgroup_bland_path_reaches_the_optimum(d2, h, bland_after):
    t = 128
    A, B, pairs = synth.make_degenerate(14, 8, t, t, identical_every=2)
    o_d, o_st, _, _ = oracle.emd_batch_stats(A, B, pairs)
    g_d, g_st, g_piv = run(d2, h, A, B, pairs, d2.Opts(init=NWC, bland_after=bland_after))
    assert np.all(g_st == 0), g_st
    np.testing.assert_array_equal(g_d, o_d)
    ident = np.arange(pairs.shape[0]) % 2 == 0
    assert np.all(g_piv[ident, 1] > 0), g_piv
    assert np.all(g_piv[:, 1] <= g_piv[:, 0])


def test_workgroup_tight_tolerance_never_enters_a_basic_cell(d2, h):
    """opt_tol far below the default: the workgroup solver's potentials come
    from pointer jumping, so a basic cell's reduced cost is a rounding
    residue; it must never enter.  Values and statuses against the oracle."""
    rng = np.random.default_rng(2024)
    bags_a, bags_b = [], []
    for _ in range(24):
        ta, tb = int(rng.integers(70, 131)), int(rng.integers(70, 131))
        bags_a.append((rng.normal(size=(ta, 3)), rng.gamma(1.0, size=ta)))
        bags_b.append((rng.normal(size=(tb, 3)), rng.gamma(1.0, size=tb)))
    A, B = synth.from_bags(bags_a), synth.from_bags(bags_b)
    pairs = np.stack([np.arange(24), np.arange(24)], axis=1).astype(np.int64)
    o_d, o_st, _ = oracle.emd_batch(A, B, pairs)
    for tol in (1e-16, 1e-18):
        g_d, g_st, g_piv = run(d2, h, A, B, pairs, d2.Opts(opt_tol=tol, max_pivots=200000))
        assert np.all(g_st == 0), (tol, g_st)
        assert_close(g_d, o_d, pair_tolerance(A, B, pairs))
