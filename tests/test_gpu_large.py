"""GPU parity of d2_emd_batch on supports beyond 64 atoms (the workgroup
simplex), through the C ABI, against the FP64 oracle on the same seeded
inputs: values at the pair rule, statuses equal, plans by their marginals
and value, duals by the LP certificate.  A 1,024 x 1,024 pair in one
dimension is checked against the quantile closed form of W2^2 (the
oracle would take minutes there).
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


def bags(rng, sizes, d, alpha=1.0):
    return synth.from_bags([(rng.normal(size=(t, d)) * 2, rng.dirichlet(np.full(t, alpha))) for t in sizes])


def run(d2, h, A, B, pairs, opts=None):
    dist, st, (plan, poff), (duals, doff) = d2.d2_emd_batch(
        h, d2.DeviceSet.from_ragged(A, DEV), d2.DeviceSet.from_ragged(B, DEV), torch.as_tensor(pairs),
        opts or d2.Opts(), want_plan=True, want_duals=True)
    torch.cuda.synchronize()
    return (dist.cpu().numpy(), st.cpu().numpy(), plan.cpu().numpy(), poff.cpu().numpy(),
            duals.cpu().numpy(), doff.cpu().numpy())


def check(A, B, pairs, got):
    dist, st, plan, poff, duals, doff = got
    o, o_st, _ = oracle.emd_batch(A, B, pairs)
    np.testing.assert_array_equal(st, o_st)
    for k, (i, j) in enumerate(pairs):
        if o_st[k] != 0:
            assert np.isnan(dist[k])
            continue
        x, p = A.bag(int(i)); y, q = B.bag(int(j))
        x = np.asarray(x, np.float64); y = np.asarray(y, np.float64)
        pn = np.asarray(p, np.float64); pn = pn / pn.sum()
        qn = np.asarray(q, np.float64); qn = qn / qn.sum()
        S = coupling_cost(x, p, y, q)
        assert abs(dist[k] - o[k]) <= max(REL * abs(o[k]), 1e-14 * S), (k, dist[k], o[k])
        P = plan[poff[k]:poff[k + 1]].reshape(len(pn), len(qn))
        C = ((x[:, None, :] - y[None, :, :]) ** 2).sum(-1)
        assert P.min() >= 0.0
        np.testing.assert_allclose(P.sum(1), pn, atol=1e-12)
        np.testing.assert_allclose(P.sum(0), qn, atol=1e-12)
        assert abs(float((P * C).sum()) - o[k]) <= max(REL * abs(o[k]), 1e-14 * S) + 1e-13 * C.max()
        u = duals[doff[k]:doff[k] + len(pn)]
        v = duals[doff[k] + len(pn):doff[k + 1]]
        R = C - u[:, None] - v[None, :]
        tol = 1e-12 * max(C.max(), 1e-300)
        assert R.min() >= -tol
        assert np.abs(R[P > 0]).max(initial=0.0) <= tol


@pytest.mark.parametrize("dtype,d,alpha", [(np.float64, 2, 1.0), (np.float32, 5, 0.3), (np.float64, 8, 1.0),
                                           (np.float64, 12, 0.5)])
def test_random_large_pairs(d2, h, dtype, d, alpha):
    rng = np.random.default_rng(71 + d)
    A = bags(rng, rng.integers(40, 161, size=24), d, alpha).astype(dtype)
    B = bags(rng, rng.integers(1, 131, size=20), d, alpha).astype(dtype)
    pairs = np.stack([rng.integers(0, A.n, 60), rng.integers(0, B.n, 60)], 1).astype(np.int64)
    check(A, B, pairs, run(d2, h, A, B, pairs))


@pytest.mark.parametrize("init", ["nwc", "vogel"])
def test_large_pairs_other_starts(d2, h, init):
    """The workgroup path starts from the north-west corner under
    D2_INIT_NWC and from the least-cost start under every other choice."""
    rng = np.random.default_rng(78)
    A = bags(rng, rng.integers(65, 121, size=10), 4)
    B = bags(rng, rng.integers(1, 101, size=8), 4)
    pairs = np.stack([rng.integers(0, A.n, 30), rng.integers(0, B.n, 30)], 1).astype(np.int64)
    code = d2.D2_INIT_NWC if init == "nwc" else d2.D2_INIT_VOGEL
    check(A, B, pairs, run(d2, h, A, B, pairs, d2.Opts(init=code)))


def test_more_pairs_than_workgroups(d2, h):
    """A batch of 2,600 pairs: the persistent workgroups take several pairs
    each, so later pairs start from a workgroup's leftover LDS state.
    Sampled pairs from every stretch of the list, including the last,
    against the oracle."""
    rng = np.random.default_rng(79)
    A = bags(rng, rng.integers(65, 91, size=40), 3, 0.5)
    B = bags(rng, rng.integers(1, 91, size=30), 3, 0.5)
    pairs = np.stack([rng.integers(0, A.n, 2600), rng.integers(0, B.n, 2600)], 1).astype(np.int64)
    dist, st, *_ = run(d2, h, A, B, pairs)
    sample = np.unique(np.concatenate([np.arange(0, 2600, 37), [1023, 1024, 2047, 2048, 2599]]))
    sub = pairs[sample]
    o, o_st, _ = oracle.emd_batch(A, B, sub)
    np.testing.assert_array_equal(st[sample], o_st)
    for k, (i, j) in zip(sample, sub):
        S = coupling_cost(*A.bag(int(i)), *B.bag(int(j)))
        ok = o[list(sample).index(k)]
        assert abs(dist[k] - ok) <= max(REL * abs(ok), 1e-14 * S), (k, dist[k], ok)


def test_edge_cases_large(d2, h):
    rng = np.random.default_rng(72)
    sizes = [100, 80, 120, 70, 90]
    A = bags(rng, sizes, 3)
    w = A.weights.copy()
    w[int(A.offsets[1]) + 3] = np.nan                        # object 1: bad weight
    w[int(A.offsets[2]):int(A.offsets[2]) + 60] = 0.0        # object 2: 60 zero-mass atoms
    A = synth.RaggedSet(A.offsets, A.points, w)
    B = synth.from_bags([A.bag(0), A.bag(4)] + [(rng.normal(size=(75, 3)), rng.dirichlet(np.ones(75)))])
    pairs = np.array([[0, 0], [1, 2], [2, 2], [3, 1], [4, 1], [0, 2]], dtype=np.int64)
    got = run(d2, h, A, B, pairs)
    assert got[1][1] == 1
    check(A, B, pairs, got)
    S0 = coupling_cost(*A.bag(0), *B.bag(0))
    assert abs(got[0][0]) <= 1e-14 * S0                      # identical distributions
    assert abs(got[0][4]) <= 1e-14 * coupling_cost(*A.bag(4), *B.bag(1))


def w2sq_1d(x, p, y, q):
    """Quantile coupling of two one-dimensional distributions."""
    ix, iy = np.argsort(x), np.argsort(y)
    x, p = x[ix], p[ix] / p.sum()
    y, q = y[iy], q[iy] / q.sum()
    a = b = 0
    ra, rb = p[0], q[0]
    tot = 0.0
    while True:
        m = min(ra, rb)
        tot += m * (x[a] - y[b]) ** 2
        ra -= m
        rb -= m
        if a == len(x) - 1 and b == len(y) - 1:
            return tot
        if (ra <= rb and a < len(x) - 1) or b == len(y) - 1:
            a += 1
            ra = p[a]
        else:
            b += 1
            rb = q[b]


def test_1024_atoms_per_side_closed_form(d2, h):
    rng = np.random.default_rng(73)
    x = rng.normal(size=1024); y = rng.normal(size=1024) * 1.5 + 0.3
    p = rng.dirichlet(np.ones(1024)); q = rng.dirichlet(np.ones(1024))
    A = synth.from_bags([(x[:, None], p)])
    B = synth.from_bags([(y[:, None], q)])
    pairs = np.array([[0, 0]], dtype=np.int64)
    dist, st, *_ = run(d2, h, A, B, pairs, d2.Opts(max_pivots=200000))
    assert st[0] == 0
    want = w2sq_1d(x, p, y, q)
    assert abs(dist[0] - want) <= 1e-10 * want


def test_middle_instance(d2, h):
    """Supports of 257..512 run the middle instance (two workgroups per CU):
    one-dimensional pairs against the quantile closed form, and 3-D pairs
    against the oracle."""
    rng = np.random.default_rng(80)
    sizes_a, sizes_b = rng.integers(257, 513, size=6), rng.integers(200, 513, size=6)
    one = [(rng.normal(size=(t, 1)), rng.dirichlet(np.ones(t))) for t in sizes_a]
    two = [(rng.normal(size=(s, 1)) * 1.3 + 0.2, rng.dirichlet(np.ones(s))) for s in sizes_b]
    A, B = synth.from_bags(one), synth.from_bags(two)
    pairs = np.array([[k, k] for k in range(6)] + [[0, 5], [5, 0]], dtype=np.int64)
    dist, st, *_ = run(d2, h, A, B, pairs)
    assert (st == 0).all()
    for k, (i, j) in enumerate(pairs):
        (x, p), (y, q) = one[i], two[j]
        want = w2sq_1d(x[:, 0], p, y[:, 0], q)
        assert abs(dist[k] - want) <= 1e-10 * want, (k, dist[k], want)
    A3 = bags(rng, [300, 270], 3)
    B3 = bags(rng, [260, 280], 3)
    check(A3, B3, np.array([[0, 0], [1, 1], [0, 1]], dtype=np.int64),
          run(d2, h, A3, B3, np.array([[0, 0], [1, 1], [0, 1]], dtype=np.int64)))


def test_declared_bounds(d2, h):
    import ctypes
    rng = np.random.default_rng(74)
    A = bags(rng, [1100], 2)
    Ad = d2.DeviceSet.from_ragged(A, DEV)
    a = Ad.c()
    o = d2.Opts().c()
    pairs = torch.zeros((1, 2), dtype=torch.int64, device=DEV)
    dist = torch.empty(1, dtype=torch.float64, device=DEV)
    rc = d2._ffi.lib().d2_emd_batch(h.ptr, ctypes.byref(a), ctypes.byref(a),
                                    ctypes.c_void_p(pairs.data_ptr()), 1, ctypes.byref(o),
                                    ctypes.c_void_p(dist.data_ptr()), None, None, None, None, None,
                                    None, None, 0, None)
    assert rc == 3                                           # above D2_MAX_SUPPORT_LARGE
    B = bags(rng, [100], 2)
    Bd = d2.DeviceSet.from_ragged(B, DEV)
    b = Bd.c()
    rc = d2._ffi.lib().d2_emd_batch(h.ptr, ctypes.byref(b), ctypes.byref(b),
                                    ctypes.c_void_p(pairs.data_ptr()), 1, ctypes.byref(o),
                                    ctypes.c_void_p(dist.data_ptr()), None, None, None, None, None,
                                    None, None, 0, None)
    assert rc == 2                                           # the workgroup path needs its workspace


def test_large_pairs_root_and_plain_schedule(d2, h):
    """want_sqrt returns D = sqrt(D^2) on the workgroup path, and the
    schedule option does not change its results."""
    rng = np.random.default_rng(75)
    A = bags(rng, [90, 70], 3)
    B = bags(rng, [80, 100], 3)
    pairs = np.array([[0, 0], [1, 1], [0, 1]], dtype=np.int64)
    d2sq = run(d2, h, A, B, pairs)[0]
    root = run(d2, h, A, B, pairs, d2.Opts(want_sqrt=1))[0]
    np.testing.assert_array_equal(root, np.sqrt(d2sq))
    plain = run(d2, h, A, B, pairs, d2.Opts(schedule=d2.D2_SCHED_PLAIN))[0]
    np.testing.assert_array_equal(plain, d2sq)


@pytest.mark.parametrize("want_all", [True, False])
def test_assign_large_supports(d2, h, want_all):
    rng = np.random.default_rng(76)
    X = bags(rng, rng.integers(20, 101, size=30), 3)
    Z = bags(rng, rng.integers(50, 91, size=6), 3)
    lab, best, allv, st = d2.d2_assign(h, d2.DeviceSet.from_ragged(X, DEV), d2.DeviceSet.from_ragged(Z, DEV),
                                       want_all=want_all)
    torch.cuda.synchronize()
    o_lab, o_best, o_all, o_st, _ = oracle.assign(X, Z)
    np.testing.assert_array_equal(st.cpu().numpy(), o_st)
    floor = np.array([[1e-14 * coupling_cost(*X.bag(i), *Z.bag(j)) for j in range(Z.n)] for i in range(X.n)])
    if want_all:
        g = allv.cpu().numpy()
        assert np.all(np.abs(g - o_all) <= np.maximum(REL * np.abs(o_all), floor))
    g_lab, g_best = lab.cpu().numpy(), best.cpu().numpy()
    for i in range(X.n):
        if g_lab[i] != o_lab[i]:
            assert o_all[i, g_lab[i]] - o_all[i, o_lab[i]] <= max(REL * o_best[i], floor[i].max())
        assert abs(g_best[i] - o_best[i]) <= max(REL * abs(o_best[i]), floor[i].max())


def test_pairwise_large_supports(d2, h):
    rng = np.random.default_rng(77)
    X = bags(rng, rng.integers(10, 91, size=14), 2)
    X = synth.from_bags([X.bag(i) for i in range(X.n)] + [X.bag(3)])   # one duplicate: D^2 = 0
    out, st = d2.d2_pairwise(h, d2.DeviceSet.from_ragged(X, DEV))
    torch.cuda.synchronize()
    o, o_st, _ = oracle.pairwise(X)
    np.testing.assert_array_equal(st.cpu().numpy(), o_st)
    g = out.cpu().numpy()
    n = X.n
    k = 0
    for i in range(n):
        for j in range(i + 1, n):
            S = coupling_cost(*X.bag(i), *X.bag(j))
            assert abs(g[k] - o[k]) <= max(REL * abs(o[k]), 1e-14 * S), (i, j, g[k], o[k])
            k += 1
    assert g[3 * n - 3 * 4 // 2 + (n - 1 - 3 - 1)] <= 1e-14 * coupling_cost(*X.bag(3), *X.bag(3))
