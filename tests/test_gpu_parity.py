"""GPU parity: the HIP path against the FP64 CPU oracle, through the C ABI.

Every comparison is element by element on the same seeded inputs, at the
tolerance of the FP64 path (see parity.py).  Sizes keep the oracle to
seconds while spanning several group widths, chunked and unchunked
launches, and ragged tails.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.parity import assert_close, assert_labels, coupling_cost, pair_tolerance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


DEV = "cuda:0"


def dev(d2, S, max_support=None):
    s = d2.DeviceSet.from_ragged(S, DEV)
    if max_support is not None:
        s.max_support = max_support
    return s


def row_floor(X, Z, rows=None):
    rows = range(X.n) if rows is None else rows
    return np.array([1e-14 * min(coupling_cost(*X.bag(i), *Z.bag(j)) for j in range(Z.n))
                     for i in rows])


def full_floor(X, Z):
    return np.array([[1e-14 * coupling_cost(*X.bag(i), *Z.bag(j)) for j in range(Z.n)]
                     for i in range(X.n)])


def run_assign(d2, h, X, Z, init=0, max_support=None, want_all=True):
    opts = d2.Opts(init=init)
    lab, best, allv, st = d2.d2_assign(h, dev(d2, X, max_support), dev(d2, Z, max_support), opts,
                                       want_all=want_all)
    torch.cuda.synchronize()
    return (lab.cpu().numpy(), best.cpu().numpy(),
            allv.cpu().numpy() if allv is not None else None, st.cpu().numpy())


@pytest.mark.parametrize("init", [1, 2, 3])
def test_config1_full_assign(d2, h, init):
    """All 2,000 pairs of the plain FP64 configuration, plus labels."""
    X = synth.make_data(1)
    Z = synth.make_centroids(1)
    lab, best, allv, st = run_assign(d2, h, X, Z, init=init)
    o_lab, o_best, o_all, o_st, _ = oracle.assign(X, Z)
    assert st.max() == 0
    assert_close(allv, o_all, full_floor(X, Z))
    assert_close(best, o_best, row_floor(X, Z))
    assert_labels(lab, o_lab, o_all, row_floor(X, Z))
    assert np.array_equal(best, allv[np.arange(X.n), lab])


@pytest.mark.parametrize("cfg,n,k", [(2, 120, 64), (3, 24, 20), (5, 20, 40)])
@pytest.mark.parametrize("init", [1, 2, 3])
def test_config_shapes_assign(d2, h, cfg, n, k, init):
    """Config-shaped subsets: FP32 inputs (2, 3), d=128 (3), supports to 64 (5)."""
    X = synth.make_data(cfg, n=n)
    Z = synth.make_centroids(cfg, k=k)
    lab, best, allv, st = run_assign(d2, h, X, Z, init=init)
    o_lab, o_best, o_all, o_st, _ = oracle.assign(X, Z)
    assert st.max() == 0 and o_st.max() == 0
    assert_close(allv, o_all, full_floor(X, Z))
    assert_labels(lab, o_lab, o_all, row_floor(X, Z))


@pytest.mark.parametrize("init", [1, 2, 3])
def test_group_widths_are_bitwise_identical(d2, h, init):
    """The same pair gives the same bits whichever group width runs it."""
    X = synth.make_data(2, n=60)
    Z = synth.make_centroids(2, k=24)
    ref = run_assign(d2, h, X, Z, init=init)
    for ms in (32, 64):
        got = run_assign(d2, h, X, Z, init=init, max_support=ms)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b)


def test_repeat_runs_are_bitwise_identical(d2, h):
    X = synth.make_data(2, n=200)
    Z = synth.make_centroids(2, k=32)
    a = run_assign(d2, h, X, Z)
    b = run_assign(d2, h, X, Z)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_chunked_assign_matches_unchunked(d2, h):
    """Few rows split the centroids over workgroups (workspace path)."""
    X = synth.make_data(5, n=3)
    Z = synth.make_centroids(5, k=300)
    lab, best, allv, st = run_assign(d2, h, X, Z)
    o_lab, o_best, o_all, _, _ = oracle.assign(X, Z)
    assert st.max() == 0
    assert_close(allv, o_all, full_floor(X, Z))
    assert_labels(lab, o_lab, o_all, row_floor(X, Z))


def random_sets(seed, n, tmax, d, alpha=0.7, dtype=np.float64):
    rng = np.random.default_rng(seed)
    bags = []
    for _ in range(n):
        t = int(rng.integers(1, tmax + 1))
        bags.append((rng.normal(size=(t, d)) * 2, rng.dirichlet(np.full(t, alpha))))
    return synth.from_bags(bags, dtype)


@pytest.mark.parametrize("tmax", [8, 16, 31, 64])
def test_emd_batch_certificates(d2, h, tmax):
    """Plan marginals, non-negativity, dual feasibility and duality gap."""
    A = random_sets(10 + tmax, 40, tmax, 4)
    B = random_sets(20 + tmax, 30, tmax, 4)
    rng = np.random.default_rng(tmax)
    pairs = np.stack([rng.integers(0, A.n, 150), rng.integers(0, B.n, 150)], 1)
    dist, st, (plan, poff), (duals, doff) = d2.d2_emd_batch(
        h, dev(d2, A), dev(d2, B), torch.as_tensor(pairs), want_plan=True, want_duals=True)
    torch.cuda.synchronize()
    dist = dist.cpu().numpy(); st = st.cpu().numpy()
    plan = plan.cpu().numpy(); poff = poff.cpu().numpy()
    duals = duals.cpu().numpy(); doff = doff.cpu().numpy()
    o, o_st, _ = oracle.emd_batch(A, B, pairs)
    assert st.max() == 0
    assert_close(dist, o, pair_tolerance(A, B, pairs))
    for k, (i, j) in enumerate(pairs):
        x, p = A.bag(i); y, q = B.bag(j)
        p = p / p.sum(); q = q / q.sum()
        t, s = len(p), len(q)
        w = plan[poff[k]:poff[k + 1]].reshape(t, s)
        u = duals[doff[k]:doff[k] + t]; v = duals[doff[k] + t:doff[k + 1]]
        C = ((x[:, None] - y[None]) ** 2).sum(-1)
        assert w.min() >= 0.0
        assert np.abs(w.sum(1) - p).max() <= 1e-12
        assert np.abs(w.sum(0) - q).max() <= 1e-12
        assert abs((w * C).sum() - dist[k]) <= 1e-12 * max(1.0, dist[k])
        assert np.all(u[:, None] + v[None, :] <= C + 1e-13 * C.max())
        assert abs(u @ p + v @ q - dist[k]) <= 1e-11 * max(1.0, C.max())


def test_pairwise_small_segment(d2, h):
    X = synth.make_data(4, n=72)
    out, st = d2.d2_pairwise(h, dev(d2, X))
    torch.cuda.synchronize()
    o, o_st, _ = oracle.pairwise(X)
    assert st.cpu().numpy().max() == 0
    n = X.n
    pairs = np.array([(i, j) for i in range(n) for j in range(i + 1, n)])
    assert_close(out.cpu().numpy(), o, pair_tolerance(X, X, pairs))


def test_pairwise_tiny_and_empty(d2, h):
    for n in (0, 1, 2, 3):
        X = random_sets(50 + n, n, 5, 2) if n else synth.from_bags([])
        if n == 0:
            X = synth.RaggedSet(np.zeros(1, np.int64), np.zeros((0, 2)), np.zeros(0))
            s = d2.DeviceSet(torch.zeros(1, dtype=torch.int64, device=DEV),
                             torch.zeros((0, 2), dtype=torch.float64, device=DEV),
                             torch.zeros(0, dtype=torch.float64, device=DEV), 1)
        else:
            s = dev(d2, X)
        out, st = d2.d2_pairwise(h, s)
        torch.cuda.synchronize()
        assert out.numel() == n * (n - 1) // 2
        if n > 1:
            o, _, _ = oracle.pairwise(X)
            assert_close(out.cpu().numpy(), o, np.zeros(len(o)) + 1e-300)


def test_identical_distributions_give_exact_zero(d2, h):
    X = synth.make_data(5, n=30)
    pairs = np.stack([np.arange(30), np.arange(30)], 1)
    for init in (1, 2, 3):
        dist, st, _, _ = d2.d2_emd_batch(h, dev(d2, X), dev(d2, X), torch.as_tensor(pairs),
                                         d2.Opts(init=init))
        torch.cuda.synchronize()
        assert st.cpu().numpy().max() == 0
        assert np.all(dist.cpu().numpy() == 0.0)


def test_one_dimensional_closed_form(d2, h):
    from tests.test_oracle_pins import w2sq_1d
    A = random_sets(71, 30, 40, 1)
    B = random_sets(72, 30, 40, 1)
    pairs = np.stack([np.arange(30), np.arange(30)[::-1]], 1)
    dist, st, _, _ = d2.d2_emd_batch(h, dev(d2, A), dev(d2, B), torch.as_tensor(pairs))
    torch.cuda.synchronize()
    ref = np.array([w2sq_1d(*A.bag(i), *B.bag(j)) for i, j in pairs])
    assert np.all(np.abs(dist.cpu().numpy() - ref) <= 1e-12 * ref)


def test_single_atom_and_degenerate_inputs(d2, h):
    rng = np.random.default_rng(5)
    bags = []
    bags.append((rng.normal(size=(1, 3)), np.array([2.0])))                 # single atom
    bags.append((np.zeros((5, 3)), np.ones(5)))                              # duplicate atoms
    bags.append((rng.normal(size=(6, 3)), np.array([0, 1, 0, 2, 0, 1.0])))   # zero mass
    bags.append((np.round(rng.normal(size=(12, 3))), np.ones(12)))           # ties, equal weights
    bags.append((rng.normal(size=(64, 3)) * 1e100, rng.dirichlet(np.ones(64))))   # huge scale
    bags.append((rng.normal(size=(7, 3)) * 1e-100, rng.dirichlet(np.ones(7))))    # tiny scale
    bags.append((rng.normal(size=(16, 3)), np.full(16, 1e-300)))            # tiny weights
    A = synth.from_bags(bags)
    pairs = np.array([(i, j) for i in range(A.n) for j in range(A.n)])
    dist, st, _, _ = d2.d2_emd_batch(h, dev(d2, A), dev(d2, A), torch.as_tensor(pairs))
    torch.cuda.synchronize()
    o, o_st, _ = oracle.emd_batch(A, A, pairs)
    assert st.cpu().numpy().max() == 0
    assert_close(dist.cpu().numpy(), o, pair_tolerance(A, A, pairs))


def test_bad_inputs_are_reported_per_pair(d2, h):
    X = synth.make_data(1, n=6)
    X.weights[X.offsets[1]] = -1.0
    X.weights[X.offsets[3]:X.offsets[4]] = 0.0
    X.points[X.offsets[4], 0] = np.nan
    Z = synth.make_centroids(1)
    lab, best, allv, st = run_assign(d2, h, X, Z)
    assert st[1] == d2.D2_PAIR_BAD_WEIGHTS and lab[1] == -1 and np.isnan(best[1])
    assert st[3] == d2.D2_PAIR_BAD_WEIGHTS and lab[3] == -1
    assert st[4] == d2.D2_PAIR_BAD_POINTS and lab[4] == -1
    ok = [0, 2, 5]
    o_lab, o_best, o_all, _, _ = oracle.assign(X.subset(ok), Z)
    assert np.array_equal(lab[ok], o_lab)
    assert np.all(st[ok] == 0)


def test_support_above_declared_bound_is_reported(d2, h):
    A = random_sets(81, 4, 40, 2)      # supports up to 40
    B = random_sets(82, 4, 8, 2)
    s = dev(d2, A, max_support=16)      # lies: kernel for 16 runs
    pairs = np.array([(i, j) for i in range(4) for j in range(4)])
    dist, st, _, _ = d2.d2_emd_batch(h, s, dev(d2, B, max_support=16), torch.as_tensor(pairs))
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    big = np.diff(A.offsets)[pairs[:, 0]] > 16
    assert np.all(st[big] == d2.D2_PAIR_TOO_LARGE)
    assert np.all(st[~big] == 0)
    assert np.all(np.isnan(dist.cpu().numpy()[big]))


def test_pivot_cap_is_reported(d2, h):
    X = synth.make_data(3, n=4)
    Z = synth.make_centroids(3, k=4)
    lab, best, allv, st = d2.d2_assign(h, dev(d2, X), dev(d2, Z), d2.Opts(init=1, max_pivots=1),
                                       want_all=True)
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == d2.D2_PAIR_PIVOT_CAP)
    assert np.all(lab.cpu().numpy() == -1)


def test_want_sqrt(d2, h):
    X = synth.make_data(1, n=20)
    Z = synth.make_centroids(1)
    a = run_assign(d2, h, X, Z)
    lab, best, allv, st = d2.d2_assign(h, dev(d2, X), dev(d2, Z), d2.Opts(want_sqrt=1),
                                       want_all=True)
    torch.cuda.synchronize()
    assert np.array_equal(lab.cpu().numpy(), a[0])
    assert np.allclose(allv.cpu().numpy(), np.sqrt(a[2]), rtol=1e-15, atol=0)


def test_host_validation_codes(d2, h):
    X = dev(d2, synth.make_data(1, n=4))
    Z = dev(d2, synth.make_centroids(1))
    with pytest.raises(d2.D2Error) as e:
        d2.d2_assign(h, X, Z, d2.Opts(init=7))
    assert e.value.code == 1
    big = dev(d2, synth.make_data(1, n=4), max_support=1025)
    with pytest.raises(d2.D2Error) as e:
        d2.d2_assign(h, big, Z)
    assert e.value.code == 3
    # a declared bound above 64 takes the workgroup simplex: same labels
    wide = dev(d2, synth.make_data(1, n=4), max_support=65)
    l1, b1, _, _ = d2.d2_assign(h, X, Z)
    l2, b2, _, s2 = d2.d2_assign(h, wide, Z)
    torch.cuda.synchronize()
    assert int(s2.max()) == 0
    assert torch.equal(l1, l2)
    assert torch.allclose(b1, b2, rtol=1e-12, atol=0)


def test_cost_tiles_match_direct_form(d2, h):
    A = synth.make_data(2, n=10)
    B = synth.make_centroids(2, k=5)
    pairs = np.array([(i, j) for i in range(10) for j in range(5)])
    tiles, off = d2.d2_cost_tiles(h, dev(d2, A), dev(d2, B), torch.as_tensor(pairs))
    torch.cuda.synchronize()
    tiles = tiles.cpu().numpy(); off = off.cpu().numpy()
    for k, (i, j) in enumerate(pairs):
        x, _ = A.bag(i); y, _ = B.bag(j)
        C = ((x.astype(np.float64)[:, None] - y.astype(np.float64)[None]) ** 2).sum(-1)
        assert np.allclose(tiles[off[k]:off[k + 1]].reshape(C.shape), C, rtol=1e-15, atol=0)


def mixed_support_set(seed, n, d=6):
    """Supports spread over every support class (1..64), log-uniform."""
    rng = np.random.default_rng(seed)
    bags = []
    for _ in range(n):
        t = int(min(64, np.floor(np.exp(rng.uniform(0, np.log(65))))))
        bags.append((rng.normal(size=(t, d)) * 2 + rng.normal(size=d), rng.dirichlet(np.full(t, 0.5))))
    return synth.from_bags(bags)


def test_pairwise_binned_all_classes(d2, h):
    X = mixed_support_set(91, 90)
    sizes = np.diff(X.offsets)
    assert (sizes <= 16).any() and ((sizes > 16) & (sizes <= 32)).any() and (sizes > 32).sum() >= 2
    out, st = d2.d2_pairwise(h, dev(d2, X))
    torch.cuda.synchronize()
    o, o_st, _ = oracle.pairwise(X)
    assert st.cpu().numpy().max() == 0
    n = X.n
    pairs = np.array([(i, j) for i in range(n) for j in range(i + 1, n)])
    assert_close(out.cpu().numpy(), o, pair_tolerance(X, X, pairs))


def test_schedules_and_graph_replays_are_bitwise_identical(d2, h):
    """Plain one-wavefront-per-pair, binned eager, and several graph replays
    (with other eager work and synchronisations in between) give the same
    bits."""
    X = mixed_support_set(92, 70)
    Xd = dev(d2, X)
    ref, st = d2.d2_pairwise(h, Xd, d2.Opts(schedule=d2.D2_SCHED_PLAIN, flags=d2.D2_FLAG_EAGER))
    torch.cuda.synchronize()
    ref = ref.cpu().numpy()
    eager, _ = d2.d2_pairwise(h, Xd, d2.Opts(flags=d2.D2_FLAG_EAGER))
    torch.cuda.synchronize()
    assert np.array_equal(eager.cpu().numpy(), ref)
    # graph path: same output buffers every call so the recorded graph replays
    m = X.n * (X.n - 1) // 2
    out = torch.full((m,), -1.0, dtype=torch.float64, device=DEV)
    status = torch.empty(m, dtype=torch.int32, device=DEV)
    nbytes = d2.d2_workspace_bytes(h, 3, Xd)
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=DEV)
    import ctypes
    from paper_1302_0435_amd import _ffi
    x = Xd.c()
    o = d2.Opts().c()
    for rep in range(4):
        out.fill_(-1.0)
        _ = torch.ones(1000, device=DEV).sum()      # unrelated eager work
        rc = _ffi.lib().d2_pairwise(h.ptr, ctypes.byref(x), ctypes.byref(o),
                                    ctypes.c_void_p(out.data_ptr()),
                                    ctypes.c_void_p(status.data_ptr()),
                                    ctypes.c_void_p(ws.data_ptr()), nbytes,
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert rc == 0
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref), f"replay {rep}"


def test_assign_plain_and_binned_agree(d2, h):
    X = mixed_support_set(93, 40, d=5)
    Z = mixed_support_set(94, 33, d=5)
    a = d2.d2_assign(h, dev(d2, X), dev(d2, Z), d2.Opts(schedule=d2.D2_SCHED_PLAIN), want_all=True)
    b = d2.d2_assign(h, dev(d2, X), dev(d2, Z), d2.Opts(), want_all=True)
    torch.cuda.synchronize()
    for u, v in zip(a, b):
        assert np.array_equal(u.cpu().numpy(), v.cpu().numpy())
    o_lab, o_best, o_all, _, _ = oracle.assign(X, Z)
    assert_close(b[2].cpu().numpy(), o_all, full_floor(X, Z))


def test_autotuned_pairwise_matches(d2, h):
    X = mixed_support_set(95, 60)
    Xd = dev(d2, X)
    out, st, best_ms = d2.d2_tune_pairwise(h, Xd)
    torch.cuda.synchronize()
    assert best_ms > 0.0
    again, _ = d2.d2_pairwise(h, Xd)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), again.cpu().numpy())
    o, _, _ = oracle.pairwise(X)
    n = X.n
    pairs = np.array([(i, j) for i in range(n) for j in range(i + 1, n)])
    assert_close(again.cpu().numpy(), o, pair_tolerance(X, X, pairs))


@pytest.mark.parametrize("n", [7, 300])
def test_duplicate_centroids_take_the_lowest_index(d2, h, n):
    """Exact ties: centroids repeated at later indices (within one chunk of
    centroids and across chunks) give bitwise-equal distances, and the label
    is the first of them, as in the oracle."""
    X = synth.make_data(1, n=n)
    Z0 = synth.make_centroids(1, k=20)
    order = list(range(20)) + [3, 0, 19, 7, 3, 12, 0, 5] * 3   # duplicates after their originals
    Z = Z0.subset(np.array(order))
    g_lab, g_best, g_all, g_st = run_assign(d2, h, X, Z)
    o_lab, o_best, o_all, o_st, _ = oracle.assign(X, Z)
    assert np.all(g_st == 0)
    np.testing.assert_array_equal(g_lab, o_lab)
    first = {j: order.index(j) for j in set(order)}
    for j, src in enumerate(order):
        np.testing.assert_array_equal(g_all[:, j], g_all[:, first[src]])
    assert np.all(g_lab < 20)
