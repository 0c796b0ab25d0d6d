"""GPU parity of the given-cost transport LP (d2_emd_cost_batch) and of the MM
distance of Eq. (10) built on it, through the C ABI, against the FP64
oracle on the same seeded inputs.

Tolerance: the pair rule with the cost's magnitude in place of the squared
distance, |g - o| <= 1e-10 * max(|o|, 1e-4 * S), S = sum_ab p_a q_b |C_ab|;
plans are checked by their marginals (1e-12) and their value (plans need not
be unique).
"""
import numpy as np
import pytest

import oracle
import synth
from tests.parity import REL

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


def batch(problems):
    """Ragged arrays of (C, p, q) problems."""
    roff = np.zeros(len(problems) + 1, np.int64)
    coff = np.zeros(len(problems) + 1, np.int64)
    moff = np.zeros(len(problems), np.int64)
    rw, cw, cs = [], [], []
    m = 0
    for k, (C, p, q) in enumerate(problems):
        roff[k + 1] = roff[k] + len(p)
        coff[k + 1] = coff[k] + len(q)
        moff[k] = m
        m += C.size
        rw.append(p); cw.append(q); cs.append(C.ravel())
    cat = lambda xs: np.concatenate(xs) if xs else np.zeros(0)   # noqa: E731
    return roff, cat(rw), coff, cat(cw), cat(cs), moff


def run(d2, h, problems, init=0, max_rows=None, max_cols=None, share=None):
    roff, rw, coff, cw, cs, moff = batch(problems)
    if share is not None:
        moff = share
    T = lambda a: torch.as_tensor(a, device=DEV)   # noqa: E731
    dist, st, (plan, poff) = d2.d2_emd_cost_batch(h, T(roff), T(rw), T(coff), T(cw), T(cs), T(moff),
                                                  max_rows, max_cols, d2.Opts(init=init),
                                                  want_plan=True)
    torch.cuda.synchronize()
    return dist.cpu().numpy(), st.cpu().numpy(), plan.cpu().numpy(), poff.cpu().numpy()


def check(problems, dist, st, plan, poff):
    for k, (C, p, q) in enumerate(problems):
        try:
            o = oracle.emd_cost(C, p, q)[0]
        except ArithmeticError as e:
            assert st[k] == e.status, f"problem {k}"
            continue
        assert st[k] == 0, f"problem {k}: status {st[k]}"
        pn, qn = p / p.sum(), q / q.sum()
        S = float(pn @ np.abs(C) @ qn)
        assert abs(dist[k] - o) <= REL * max(abs(o), 1e-4 * S), f"problem {k}: {dist[k]!r} vs {o!r}"
        P = plan[poff[k]:poff[k + 1]].reshape(C.shape)
        assert P.min() >= 0.0
        np.testing.assert_allclose(P.sum(axis=1), pn, atol=1e-12)
        np.testing.assert_allclose(P.sum(axis=0), qn, atol=1e-12)
        assert abs(float((P * C).sum()) - o) <= REL * max(abs(o), 1e-4 * S) + 1e-12 * np.abs(C).max()


@pytest.mark.parametrize("tmax,smax", [(8, 8), (30, 12), (64, 20), (40, 64), (64, 64)])
@pytest.mark.parametrize("init", [1, 2, 3])
def test_random_costs_both_signs(d2, h, tmax, smax, init):
    rng = np.random.default_rng(tmax * 100 + smax + init)
    problems = []
    for _ in range(120):
        t, s = int(rng.integers(1, tmax + 1)), int(rng.integers(1, smax + 1))
        C = rng.normal(size=(t, s)) * rng.choice([1e-3, 1.0, 1e3]) + rng.choice([0.0, 5.0])
        problems.append((C, rng.dirichlet(np.full(t, 0.7)), rng.dirichlet(np.full(s, 0.7))))
    got = run(d2, h, problems, init=init, max_rows=tmax, max_cols=smax)
    check(problems, *got)


def test_shared_matrix_zero_weights_and_failures(d2, h):
    rng = np.random.default_rng(5)
    C = rng.uniform(0, 3, size=(6, 5))
    good = (C, np.array([0.2, 0.0, 0.3, 0.1, 0.4, 0.0]), np.array([0.5, 0.0, 0.2, 0.3, 0.0]))
    Cinf = C.copy(); Cinf[2, 3] = np.inf
    problems = [good, good, (Cinf, good[1], good[2]), (C, -good[1], good[2]),
                (np.array([[2.5]]), np.array([1.0]), np.array([3.0]))]
    roff, rw, coff, cw, cs, moff = batch(problems)
    got = run(d2, h, problems, max_rows=6, max_cols=5)
    dist, st = got[0], got[1]
    np.testing.assert_array_equal(st, [0, 0, 4, 1, 0])
    assert dist[4] == 2.5
    check(problems, *got)
    # two problems reading one matrix
    got2 = run(d2, h, problems[:2], max_rows=6, max_cols=5, share=np.array([0, 0], np.int64))
    assert got2[0][0] == got2[0][1] == dist[0]


def test_squared_distance_costs_match_the_point_path(d2, h):
    X = synth.make_data(1)
    Z = synth.make_centroids(1)
    pairs = synth.sample_pairs(1, X.n, Z.n, 200, tag=3)
    problems = []
    for i, j in pairs:
        x, p = X.bag(int(i)); y, q = Z.bag(int(j))
        problems.append((((x[:, None, :] - y[None, :, :]) ** 2).sum(-1), p, q))
    dist = run(d2, h, problems, max_rows=8, max_cols=8)[0]
    ref, st, _, _ = d2.d2_emd_batch(h, d2.DeviceSet.from_ragged(X, DEV), d2.DeviceSet.from_ragged(Z, DEV),
                                    torch.as_tensor(pairs))
    torch.cuda.synchronize()
    np.testing.assert_allclose(dist, ref.cpu().numpy(), rtol=1e-12, atol=1e-14)


def test_rejects_bad_arguments(d2, h):
    import ctypes
    L = d2._ffi.lib()
    o = d2.Opts().c()
    assert L.d2_emd_cost_batch(h.ptr, 1, None, None, None, None, None, None, 8, 8, ctypes.byref(o),
                               None, None, None, None, None, 0, None) == 1
    assert L.d2_emd_cost_batch(h.ptr, 0, None, None, None, None, None, None, 65, 8, ctypes.byref(o),
                               None, None, None, None, None, 0, None) == 3
    ob = d2.Opts(cost_mode=d2.D2_COST_BF16_MFMA).c()
    assert L.d2_emd_cost_batch(h.ptr, 0, None, None, None, None, None, None, 8, 8, ctypes.byref(ob),
                               None, None, None, None, None, 0, None) == 3


@pytest.mark.parametrize("cfg,k1,k2", [(1, 10, 7), (2, 40, 64)])
def test_mm_distance_against_oracle(d2, h, cfg, k1, k2):
    Z = synth.make_centroids(cfg)
    Z1 = Z.subset(np.arange(k1))
    Z2 = Z.subset(np.arange(Z.n - k2, Z.n))
    rng = synth.rng_for(cfg, synth.STREAM_SAMPLE, 55)
    p1 = rng.dirichlet(np.ones(k1)); p2 = rng.dirichlet(np.ones(k2))
    mm2, M, plan = d2.d2_mm_distance(h, d2.DeviceSet.from_ragged(Z1, DEV), torch.as_tensor(p1),
                                     d2.DeviceSet.from_ragged(Z2, DEV), torch.as_tensor(p2))
    torch.cuda.synchronize()
    o_mm2, o_M, o_plan = oracle.mm_distance(Z1, p1, Z2, p2)
    g_M = M.cpu().numpy()
    assert np.all(np.abs(g_M - o_M) <= REL * np.maximum(np.abs(o_M), 1e-12))
    S = float((p1 / p1.sum()) @ o_M @ (p2 / p2.sum()))
    assert abs(float(mm2) - o_mm2) <= REL * max(abs(o_mm2), 1e-4 * S)
    P = plan.cpu().numpy()
    np.testing.assert_allclose(P.sum(axis=1), p1 / p1.sum(), atol=1e-12)
    np.testing.assert_allclose(P.sum(axis=0), p2 / p2.sum(), atol=1e-12)


def test_mm_distance_of_a_set_to_itself_is_zero(d2, h):
    Z = synth.make_centroids(1)
    p = synth.rng_for(1, synth.STREAM_SAMPLE, 56).dirichlet(np.ones(Z.n))
    Zd = d2.DeviceSet.from_ragged(Z, DEV)
    mm2, M, _ = d2.d2_mm_distance(h, Zd, torch.as_tensor(p), Zd, torch.as_tensor(p))
    torch.cuda.synchronize()
    assert float(mm2) == 0.0
    assert np.all(np.diag(M.cpu().numpy()) == 0.0)


def test_plain_schedule_within_tolerance(d2, h):
    rng = np.random.default_rng(9)
    problems = []
    for _ in range(50):
        t, s = int(rng.integers(1, 20)), int(rng.integers(1, 20))
        problems.append((rng.normal(size=(t, s)), rng.dirichlet(np.ones(t)), rng.dirichlet(np.ones(s))))
    a = run(d2, h, problems, max_rows=20, max_cols=20)
    roff, rw, coff, cw, cs, moff = batch(problems)
    T = lambda x: torch.as_tensor(x, device=DEV)   # noqa: E731
    dist, st, _ = d2.d2_emd_cost_batch(h, T(roff), T(rw), T(coff), T(cw), T(cs), T(moff), 20, 20,
                                       d2.Opts(schedule=d2.D2_SCHED_PLAIN))
    torch.cuda.synchronize()
    # the plain schedule runs the widest shape; values agree to the tolerance
    o = np.array([oracle.emd_cost(C, p, q)[0] for C, p, q in problems])
    g = dist.cpu().numpy()
    S = np.array([float((p / p.sum()) @ np.abs(C) @ (q / q.sum())) for C, p, q in problems])
    assert np.all(np.abs(g - o) <= np.maximum(REL * np.abs(o), 1e-14 * S))
    assert np.all(np.abs(a[0] - o) <= np.maximum(REL * np.abs(o), 1e-14 * S))
