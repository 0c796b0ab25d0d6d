"""GPU: the device's Dantzig pivot path against the oracle's on generic data.

Started from the same north-west-corner basis, the device and the oracle
price with the same rule (most negative reduced cost, lowest cell on ties)
and the same ratio-test tie rule, so on every configuration's seeded pair
sample (the one `bench.py --op pivots` reports) each pair must take the same
number of pivots on both sides, none under Bland's rule, and reach the same
value within the FP64 tolerance."""
import numpy as np
import pytest

import bench
import oracle
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


@pytest.mark.parametrize("cfg", [1, 2, 3, 4, 5])
def test_north_west_corner_pivot_path_is_the_oracle_path(d2, cfg):
    A, B, pairs, _ = bench.pivot_sample(cfg)
    o_d, o_st, o_piv, o_bl = oracle.emd_batch_stats(A, B, pairs, init=oracle.INIT_NWC)
    assert np.all(o_st == 0)
    h = d2.Handle(0)
    dist, st, _, _, piv = d2.d2_emd_batch(h, d2.DeviceSet.from_ragged(A, DEV),
                                          d2.DeviceSet.from_ragged(B, DEV), torch.as_tensor(pairs),
                                          d2.Opts(init=d2.D2_INIT_NWC), want_pivots=True)
    torch.cuda.synchronize()
    st, piv, dist = st.cpu().numpy(), piv.cpu().numpy(), dist.cpu().numpy()
    assert np.all(st == 0), np.unique(st)
    np.testing.assert_array_equal(piv[:, 0], o_piv)
    assert np.all(piv[:, 1] == 0) and np.all(o_bl == 0)
    assert_close(dist, o_d, pair_tolerance(A, B, pairs))


@pytest.mark.parametrize("cfg", [2, 5])
def test_least_cost_start_values_and_counts(d2, cfg):
    """The default start takes its own path: values still match the oracle,
    and its pivot counts stay below the north-west corner's on average."""
    A, B, pairs, _ = bench.pivot_sample(cfg, count=1024)
    o_d, _, o_piv, _ = oracle.emd_batch_stats(A, B, pairs, init=oracle.INIT_NWC)
    h = d2.Handle(0)
    dist, st, _, _, piv = d2.d2_emd_batch(h, d2.DeviceSet.from_ragged(A, DEV),
                                          d2.DeviceSet.from_ragged(B, DEV), torch.as_tensor(pairs),
                                          d2.Opts(init=d2.D2_INIT_LCM), want_pivots=True)
    torch.cuda.synchronize()
    st, piv, dist = st.cpu().numpy(), piv.cpu().numpy(), dist.cpu().numpy()
    assert np.all(st == 0)
    assert_close(dist, o_d, pair_tolerance(A, B, pairs))
    assert piv[:, 0].mean() < o_piv.mean()
