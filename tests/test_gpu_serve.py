"""Serving on the GPU: a request's result is the same alone and in the mix
(bitwise), and matches the oracle."""
import numpy as np
import pytest

import oracle
import synth
from tests.parity import assert_close, coupling_cost

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("k,n_pool,n_req,max_batch,alone_every,oracle_every,budget", [
    (48, 90, 360, 48, 7, 9, 1 << 28),
    (1024, 24, 96, 16, 5, 8, 1 << 28),      # the serving workload's resident centroid count
    # a budget of a few requests: batches are cut by the buffer's free ranges,
    # which the completed batches' ranges return to
    (48, 90, 360, 48, 7, 9, 6 * (64 * 32 * 8 + 64 * 8 + 8 + 48 * 8 + 16) + 4096),
])
def test_serving_results_alone_equal_mix(k, n_pool, n_req, max_batch, alone_every, oracle_every,
                                         budget):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests selected but no GPU is visible")
    import paper_1302_0435_amd as d2
    from paper_1302_0435_amd import serve
    Z = synth.make_centroids(5, k=k)
    Zd = d2.DeviceSet.from_ragged(Z, "cuda:0")
    q = synth.make_data(5, n=n_pool)
    pool = serve.QueryPool(q.offsets, q.points.astype(np.float64), q.weights.astype(np.float64))
    arrivals = np.sort(np.random.default_rng(3).uniform(0.0, 0.05, n_req))
    req_idx = np.arange(n_req) % pool.n
    ex = serve.GpuExecutor(pool, req_idx, Zd, Z.n, slots=3, max_batch=max_batch, keep_results=True,
                           budget_bytes=budget)
    sch = serve.Scheduler(ex, pool.sizes()[req_idx], pool.d, Z.n, budget, max_batch, 3)
    st = sch.run(arrivals)
    assert np.all(~np.isnan(st.done_s))
    assert max(st.batch_sizes) > 1
    assert all(ex.results[r][3] == 0 for r in range(n_req))
    # the same pool entry served in different batches gives the same bits
    for r in range(pool.n, n_req):
        assert np.array_equal(ex.results[r][2], ex.results[r - pool.n][2])
    # alone: each pool entry as a one-request call
    h = d2.Handle(0)
    P = synth.RaggedSet(pool.offsets, pool.points, pool.weights)
    for q in range(0, pool.n, alone_every):
        one = P.subset([q])
        lab, best, allv, stt = d2.d2_assign(h, d2.DeviceSet.from_ragged(one, "cuda:0"), Zd,
                                            want_all=True)
        torch.cuda.synchronize()
        assert np.array_equal(allv.cpu().numpy()[0], ex.results[q][2])
        assert int(lab.cpu().numpy()[0]) == ex.results[q][0]
    # and the oracle agrees
    picked = list(range(0, pool.n, oracle_every))
    sub = P.subset(picked)
    o_lab, o_best, o_all, _, _ = oracle.assign(sub, Z)
    g_all = np.stack([ex.results[q][2] for q in picked])
    floor = np.array([[1e-14 * coupling_cost(*sub.bag(i), *Z.bag(j)) for j in range(Z.n)]
                      for i in range(sub.n)])
    assert_close(g_all, o_all, floor)
    g_lab = np.array([ex.results[q][0] for q in picked])
    assert np.array_equal(g_lab, o_lab) or all(
        o_all[i, g_lab[i]] - o_all[i, o_lab[i]] <= max(1e-10 * abs(o_all[i, o_lab[i]]), floor[i].min())
        for i in range(len(picked)))


def test_serving_at_the_serving_shape_matches_the_oracle():
    """The serving workload's shape: 1,024 resident centroids of support 32
    (d = 32) and 128 distinct queries of support 4..64 arriving as a Poisson
    stream at 10,000 per second; every served query's 1,024 distances and
    its label against the oracle."""
    if not torch.cuda.is_available():
        pytest.fail("GPU tests selected but no GPU is visible")
    import paper_1302_0435_amd as d2
    from paper_1302_0435_amd import serve
    Z = synth.make_centroids(5)
    assert Z.n == 1024
    Zd = d2.DeviceSet.from_ragged(Z, "cuda:0")
    n_req = 128
    q = synth.make_data(5, n=n_req)
    pool = serve.QueryPool(q.offsets, q.points.astype(np.float64), q.weights.astype(np.float64))
    arrivals = synth.arrivals(5, 10000.0, 0.05)[:n_req]
    assert arrivals.size == n_req
    req_idx = np.arange(n_req)                 # every request a distinct query
    ex = serve.GpuExecutor(pool, req_idx, Zd, Z.n, slots=4, max_batch=64, keep_results=True,
                           budget_bytes=64 << 20)
    st = serve.Scheduler(ex, pool.sizes(), pool.d, Z.n, 64 << 20, 64, 4).run(arrivals)
    assert np.all(~np.isnan(st.done_s))
    assert all(ex.results[r][3] == 0 for r in range(n_req))
    P = synth.RaggedSet(pool.offsets, pool.points, pool.weights)
    o_lab, o_best, o_all, o_st, _ = oracle.assign(P, Z)
    assert o_st.max() == 0
    g_all = np.stack([ex.results[r][2] for r in range(n_req)])
    g_lab = np.array([ex.results[r][0] for r in range(n_req)])
    floor = np.array([[1e-14 * coupling_cost(*P.bag(r), *Z.bag(j)) for j in range(Z.n)]
                      for r in range(n_req)])
    assert_close(g_all, o_all, floor)
    for r in range(n_req):
        if g_lab[r] != o_lab[r]:
            assert o_all[r, g_lab[r]] - o_all[r, o_lab[r]] <= max(1e-10 * abs(o_all[r, o_lab[r]]),
                                                                  floor[r].min())
