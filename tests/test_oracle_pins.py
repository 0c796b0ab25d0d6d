"""Pins for the FP64 CPU oracle (no GPU).

The paper prints no worked example of a Mallows distance, so the oracle is
pinned by what the mathematics fixes about the LP of Eq. (1) (centroid fixed):
hand-derived fixtures (tests/golden), the one-dimensional quantile closed
form, brute force over permutations (Birkhoff) and over every spanning tree in
exact rationals, an independent LP solver (HiGHS through scipy), the
assignment solver for equal weights, LP duality certificates, and the metric
and geometric invariants.  Each check is written here independently of the
oracle's code, so that a dropped term, a wrong sign or index or a transposed
operand in the oracle fails at least one of them.
"""
import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")


def cost(x, y):
    x = np.asarray(x, float); y = np.asarray(y, float)
    return ((x[:, None, :] - y[None, :, :]) ** 2).sum(-1)


def norm(w):
    w = np.asarray(w, float)
    return w / w.sum()


def w2sq_1d(x, p, y, q):
    """One-dimensional closed form: integral over u in (0,1) of
    (F^-1(u) - G^-1(u))^2, evaluated on the merged breakpoints of the two
    cumulative weight sequences."""
    x = np.asarray(x, float).ravel(); y = np.asarray(y, float).ravel()
    p = norm(p); q = norm(q)
    ix = np.argsort(x, kind="stable"); iy = np.argsort(y, kind="stable")
    xs, ps, ys, qs = x[ix], p[ix], y[iy], q[iy]
    Fp = np.cumsum(ps); Fq = np.cumsum(qs)
    Fp[-1] = 1.0; Fq[-1] = 1.0
    cuts = np.unique(np.concatenate([[0.0], Fp, Fq]))
    total = 0.0
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        mid = 0.5 * (lo + hi)
        a = min(np.searchsorted(Fp, mid, side="right"), len(xs) - 1)
        b = min(np.searchsorted(Fq, mid, side="right"), len(ys) - 1)
        total += (hi - lo) * (xs[a] - ys[b]) ** 2
    return total


def lp_highs(x, p, y, q):
    from scipy.optimize import linprog
    C = cost(x, y)
    t, s = C.shape
    A = np.zeros((t + s, t * s))
    for a in range(t):
        A[a, a * s:(a + 1) * s] = 1
    for b in range(s):
        A[t + b, b::s] = 1
    res = linprog(C.ravel(), A_eq=A, b_eq=np.concatenate([norm(p), norm(q)]), bounds=(0, None),
                  method="highs", options={"primal_feasibility_tolerance": 1e-10,
                                           "dual_feasibility_tolerance": 1e-10})
    assert res.status == 0
    return res.fun


def tree_bruteforce(xi, pi, yi, qi):
    """Exact LP value over rational data: the optimum of a transportation LP
    sits at a vertex, every vertex is the flow of some spanning tree of the
    complete bipartite graph; enumerate all of them, solve each tree's flows by
    leaf elimination in Fractions, keep the non-negative ones, take the least
    cost."""
    t, s = len(pi), len(qi)
    P = [Fraction(v) / sum(Fraction(w) for w in pi) for v in pi]
    Q = [Fraction(v) / sum(Fraction(w) for w in qi) for v in qi]
    C = [[sum((Fraction(a) - Fraction(b)) ** 2 for a, b in zip(xi[i], yi[j])) for j in range(s)]
         for i in range(t)]
    cells = [(i, j) for i in range(t) for j in range(s)]
    best = None
    for tree in itertools.combinations(cells, t + s - 1):
        parent = list(range(t + s))

        def find(a):
            while parent[a] != a:
                parent[a] = parent[parent[a]]
                a = parent[a]
            return a
        ok = True
        for i, j in tree:
            ra, rb = find(i), find(t + j)
            if ra == rb:
                ok = False
                break
            parent[ra] = rb
        if not ok:
            continue
        mass = P + Q
        edges = set(tree)
        flow = {}
        while edges:
            deg = {}
            for i, j in edges:
                deg[i] = deg.get(i, 0) + 1
                deg[t + j] = deg.get(t + j, 0) + 1
            leaf = next(n for n, k in deg.items() if k == 1)
            e = next(e for e in edges if e[0] == leaf or t + e[1] == leaf)
            f = mass[leaf]
            flow[e] = f
            other = t + e[1] if leaf == e[0] else e[0]
            mass[other] -= f
            mass[leaf] = Fraction(0)
            edges.remove(e)
        if any(f < 0 for f in flow.values()):
            continue
        c = sum(f * C[i][j] for (i, j), f in flow.items())
        best = c if best is None or c < best else best
    return best


def d2(oracle_mod, x, p, y, q, init=0):
    return oracle_mod.emd_pair(x, p, y, q, init)[0]


# ------------------------------------------------------------------ fixtures

def test_golden_closed_forms(oracle_mod):
    cases = json.load(open(GOLDEN))["cases"]
    assert len(cases) >= 6
    for c in cases:
        for init in (oracle_mod.INIT_NWC, oracle_mod.INIT_VOGEL):
            got = d2(oracle_mod, c["x"], c["p"], c["y"], c["q"], init)
            assert abs(got - c["d2"]) <= 1e-13 * max(1.0, c["d2"]), (c["name"], init, got)


def test_golden_1d_cases_agree_with_quantile_formula():
    for c in json.load(open(GOLDEN))["cases"]:
        if len(c["x"][0]) == 1:
            assert abs(w2sq_1d(c["x"], c["p"], c["y"], c["q"]) - c["d2"]) < 1e-13, c["name"]


@pytest.mark.parametrize("seed", range(40))
def test_1d_quantile_closed_form(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    t, s = rng.integers(1, 20, size=2)
    x = rng.normal(size=(t, 1)) * 3; y = rng.normal(size=(s, 1)) * 3 + 1
    p = rng.dirichlet(np.full(t, 0.7)); q = rng.dirichlet(np.full(s, 0.7))
    ref = w2sq_1d(x, p, y, q)
    for init in (0, 1):
        got, plan, _, _, piv = oracle_mod.emd_pair(x, p, y, q, init)
        assert abs(got - ref) <= 1e-12 * max(ref, 1e-12), (got, ref)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_equal_weights_permutation_bruteforce(oracle_mod, n):
    rng = np.random.default_rng(100 + n)
    for _ in range(5):
        x = rng.normal(size=(n, 3)); y = rng.normal(size=(n, 3)) + 0.5
        C = cost(x, y)
        ref = min(sum(C[a, pi[a]] for a in range(n)) for pi in itertools.permutations(range(n))) / n
        w = np.ones(n)
        for init in (0, 1):
            got = d2(oracle_mod, x, w, y, w, init)
            assert abs(got - ref) <= 1e-12 * ref


@pytest.mark.parametrize("n", [8, 17, 33, 64])
def test_equal_weights_assignment_solver(oracle_mod, n):
    from scipy.optimize import linear_sum_assignment
    rng = np.random.default_rng(200 + n)
    x = rng.normal(size=(n, 4)); y = rng.normal(size=(n, 4))
    C = cost(x, y)
    r, c = linear_sum_assignment(C)
    ref = C[r, c].sum() / n
    w = np.full(n, 3.0)
    got = d2(oracle_mod, x, w, y, w, 1)
    assert abs(got - ref) <= 1e-11 * ref


@pytest.mark.parametrize("shape", [(1, 1), (2, 2), (2, 3), (3, 2), (3, 3), (3, 4), (4, 3)])
def test_exact_rational_spanning_tree_bruteforce(oracle_mod, shape):
    t, s = shape
    rng = np.random.default_rng(300 + 10 * t + s)
    for _ in range(3):
        xi = rng.integers(-4, 5, size=(t, 2)).tolist()
        yi = rng.integers(-4, 5, size=(s, 2)).tolist()
        pi = rng.integers(0, 4, size=t).tolist()
        qi = rng.integers(0, 4, size=s).tolist()
        pi[0] += 1; qi[-1] += 1   # keep positive sums; zeros stay (degenerate)
        ref = float(tree_bruteforce(xi, pi, yi, qi))
        for init in (0, 1):
            got = d2(oracle_mod, xi, pi, yi, qi, init)
            assert abs(got - ref) <= 1e-12 * max(ref, 1e-12), (xi, pi, yi, qi, got, ref)


def test_exact_rational_4x4_with_ties(oracle_mod):
    # Equal weights and integer grid points make many tied costs and a
    # degenerate LP.
    xi = [[0, 0], [1, 0], [0, 1], [1, 1]]
    yi = [[0, 0], [2, 0], [0, 2], [1, 1]]
    pi = [1, 1, 1, 1]
    qi = [1, 1, 1, 1]
    ref = float(tree_bruteforce(xi, pi, yi, qi))
    for init in (0, 1):
        assert abs(d2(oracle_mod, xi, pi, yi, qi, init) - ref) <= 1e-13 * ref


@pytest.mark.parametrize("seed", range(25))
def test_against_highs_lp(oracle_mod, seed):
    rng = np.random.default_rng(400 + seed)
    t, s = rng.integers(1, 17, size=2)
    d = int(rng.integers(1, 9))
    x = rng.normal(size=(t, d)) * 2; y = rng.normal(size=(s, d)) * 2 + 0.3
    p = rng.dirichlet(np.full(t, 0.5)); q = rng.dirichlet(np.full(s, 0.5))
    ref = lp_highs(x, p, y, q)
    for init in (0, 1):
        assert abs(d2(oracle_mod, x, p, y, q, init) - ref) <= 1e-9 * max(1.0, ref)


def certify(x, p, y, q, val, plan, u, v):
    C = cost(x, y)
    p = norm(p); q = norm(q)
    S = float(p @ C @ q)
    delta = 1e-14 * C.max()
    assert np.all(plan >= -1e-15)
    assert np.max(np.abs(plan.sum(1) - p)) <= 1e-12
    assert np.max(np.abs(plan.sum(0) - q)) <= 1e-12
    assert np.all(u[:, None] + v[None, :] <= C + delta + 1e-15 * C.max())
    assert abs(u @ p + v @ q - val) <= 1e-12 * max(1.0, S)
    assert abs(float((plan * C).sum()) - val) <= 1e-12 * max(1.0, S)


@pytest.mark.parametrize("cfg", [1, 2, 3, 4, 5])
def test_duality_certificate_on_config_samples(oracle_mod, cfg):
    X = synth.make_data(cfg, n=12).astype(np.float64)
    Z = synth.make_centroids(cfg, k=6).astype(np.float64) if cfg != 4 else X
    for i in range(X.n):
        for j in range(Z.n):
            x, p = X.bag(i); y, q = Z.bag(j)
            for init in (0, 1):
                val, plan, u, v, _ = oracle_mod.emd_pair(x, p, y, q, init)
                certify(x, p, y, q, val, plan, u, v)


def test_marginals_with_zero_mass_atoms(oracle_mod):
    rng = np.random.default_rng(7)
    for _ in range(20):
        t, s = rng.integers(2, 12, size=2)
        x = rng.normal(size=(t, 3)); y = rng.normal(size=(s, 3))
        p = rng.dirichlet(np.ones(t)); q = rng.dirichlet(np.ones(s))
        p[rng.integers(0, t)] = 0.0; q[rng.integers(0, s)] = 0.0
        p[0] += 0.1; q[0] += 0.1
        val, plan, u, v, _ = oracle_mod.emd_pair(x, p, y, q, 0)
        certify(x, p, y, q, val, plan, u, v)
        assert abs(val - lp_highs(x, p, y, q)) <= 1e-9 * max(1, val)


# ------------------------------------------------------------- invariants

def bags(seed, n, d=3, tmax=12):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        t = int(rng.integers(1, tmax + 1))
        out.append((rng.normal(size=(t, d)) * 2 + rng.normal(size=d), rng.dirichlet(np.ones(t))))
    return out


def test_identity_is_zero(oracle_mod):
    for x, p in bags(11, 30):
        for init in (0, 1):
            assert d2(oracle_mod, x, p, x, p, init) == 0.0


def test_symmetry(oracle_mod):
    B = bags(12, 12)
    for (x, p), (y, q) in itertools.combinations(B, 2):
        a = d2(oracle_mod, x, p, y, q); b = d2(oracle_mod, y, q, x, p)
        assert abs(a - b) <= 1e-12 * max(a, 1e-300)


def test_triangle_inequality_on_D(oracle_mod):
    B = bags(13, 9)
    D = np.zeros((9, 9))
    for i in range(9):
        for j in range(9):
            D[i, j] = np.sqrt(d2(oracle_mod, *B[i], *B[j]))
    for i, j, k in itertools.permutations(range(9), 3):
        assert D[i, k] <= (D[i, j] + D[j, k]) * (1 + 1e-10) + 1e-12


def test_mean_lower_bound_and_product_upper_bound(oracle_mod):
    B = bags(14, 12)
    for (x, p), (y, q) in itertools.combinations(B, 2):
        val = d2(oracle_mod, x, p, y, q)
        mp = norm(p) @ x; mq = norm(q) @ y
        S = float(norm(p) @ cost(x, y) @ norm(q))
        assert np.sum((mp - mq) ** 2) <= val * (1 + 1e-12) + 1e-14
        assert val <= S * (1 + 1e-12)


def test_translation_identity(oracle_mod):
    rng = np.random.default_rng(15)
    B = bags(15, 10)
    for (x, p), (y, q) in itertools.combinations(B, 2):
        c = rng.normal(size=3)
        base = d2(oracle_mod, x, p, y, q)
        moved = d2(oracle_mod, x + c, p, y, q)
        mp = norm(p) @ x; mq = norm(q) @ y
        ref = base + 2 * c @ (mp - mq) + c @ c
        assert abs(moved - ref) <= 1e-10 * max(1.0, moved)
        assert abs(d2(oracle_mod, x, p, x + c, p) - c @ c) <= 1e-12 * max(1.0, c @ c)


def test_power_of_two_scaling_is_exact(oracle_mod):
    for (x, p), (y, q) in itertools.combinations(bags(16, 8), 2):
        base = d2(oracle_mod, x, p, y, q)
        assert d2(oracle_mod, 2 * x, p, 2 * y, q) == 4 * base
        assert d2(oracle_mod, x, 2 * p, y, 8 * q) == base


def test_atom_permutation_and_rotation(oracle_mod):
    rng = np.random.default_rng(17)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    for (x, p), (y, q) in itertools.combinations(bags(17, 8), 2):
        base = d2(oracle_mod, x, p, y, q)
        ix = rng.permutation(len(p)); iy = rng.permutation(len(q))
        assert abs(d2(oracle_mod, x[ix], p[ix], y[iy], q[iy]) - base) <= 1e-12 * max(base, 1e-300)
        assert abs(d2(oracle_mod, x @ Q, p, y @ Q, q) - base) <= 1e-10 * max(base, 1e-12)


def test_single_atom_closed_form(oracle_mod):
    for (x, p), (y, q) in itertools.combinations(bags(18, 10), 2):
        ref = float(norm(q) @ ((y - x[0]) ** 2).sum(1))
        assert abs(d2(oracle_mod, x[:1], [1.0], y, q) - ref) <= 1e-13 * ref
        assert abs(d2(oracle_mod, y, q, x[:1], [2.0]) - ref) <= 1e-13 * ref


def test_bad_weights_status(oracle_mod):
    x = np.zeros((2, 2)); y = np.ones((3, 2))
    for p in ([1.0, -0.5], [np.nan, 1.0], [0.0, 0.0], [np.inf, 1.0]):
        with pytest.raises(ArithmeticError):
            oracle_mod.emd_pair(x, p, y, [1, 1, 1])


# ----------------------------------------------------- batch entry points

def test_assign_matches_highs_on_small_config(oracle_mod):
    X = synth.make_data(1, n=40)
    Z = synth.make_centroids(1)
    labels, best, allv, status, piv = oracle_mod.assign(X, Z)
    assert status.max() == 0
    ref = np.zeros((X.n, Z.n))
    for i in range(X.n):
        for j in range(Z.n):
            ref[i, j] = lp_highs(*X.bag(i), *Z.bag(j))
    assert np.all(np.abs(allv - ref) <= 1e-9 * np.maximum(1.0, ref))
    gap = ref[np.arange(X.n), labels] - ref.min(1)
    assert np.all(gap <= 1e-9 * np.maximum(1.0, ref.min(1)))
    assert np.array_equal(best, allv[np.arange(X.n), labels])


def test_assign_tie_goes_to_lowest_index(oracle_mod):
    X = synth.make_data(1, n=10)
    Z = synth.make_centroids(1)
    bags_ = [Z.bag(j) for j in range(Z.n)]
    labels, best, allv, _, _ = oracle_mod.assign(X, Z)
    # append duplicates of every centroid after the originals
    Z2 = synth.from_bags(bags_ + bags_)
    l2, b2, a2, _, _ = oracle_mod.assign(X, Z2)
    assert np.array_equal(l2, labels)
    assert np.array_equal(b2, best)
    assert np.array_equal(a2[:, :Z.n], a2[:, Z.n:])


def test_assign_bad_row_gets_minus_one(oracle_mod):
    X = synth.make_data(1, n=5)
    X.weights[X.offsets[2]] = -1.0
    labels, best, _, status, _ = oracle_mod.assign(X, synth.make_centroids(1))
    assert labels[2] == -1 and status[2] == 1 and np.isnan(best[2])
    assert np.all(labels[[0, 1, 3, 4]] >= 0)


def test_pairwise_condensed_order_matches_squareform(oracle_mod):
    from scipy.spatial.distance import squareform
    X = synth.make_data(4, n=14)
    cond, status, _ = oracle_mod.pairwise(X)
    assert status.max() == 0
    n = X.n
    pairs = np.array([(i, j) for i in range(n) for j in range(n)])
    full, st, _ = oracle_mod.emd_batch(X, X, pairs)
    full = full.reshape(n, n)
    assert np.all(np.diag(full) == 0.0)
    assert np.allclose(full, full.T, rtol=1e-12, atol=0)
    upper = np.triu(full, 1)
    sym = upper + upper.T
    assert np.array_equal(squareform(sym, checks=False), cond)


def test_nwc_and_vogel_agree(oracle_mod):
    X = synth.make_data(2, n=60).astype(np.float64)
    Z = synth.make_centroids(2, k=16).astype(np.float64)
    pairs = np.array([(i, j) for i in range(X.n) for j in range(Z.n)])
    a, sa, pa = oracle_mod.emd_batch(X, Z, pairs, init=0)
    b, sb, pb = oracle_mod.emd_batch(X, Z, pairs, init=1)
    assert sa.max() == 0 and sb.max() == 0
    assert np.all(np.abs(a - b) <= 1e-12 * np.maximum(a, 1e-300))
    assert pb.mean() < pa.mean()


def test_threads_do_not_change_results(oracle_mod):
    X = synth.make_data(1, n=50)
    Z = synth.make_centroids(1)
    r1 = oracle_mod.assign(X, Z, threads=1)
    r8 = oracle_mod.assign(X, Z, threads=8)
    for a, b in zip(r1, r8):
        assert np.array_equal(a, b)


# ---- the Bland anti-cycling branch (a reading: the paper leaves cycling open)

@pytest.mark.parametrize("t", [16, 32, 64])
@pytest.mark.parametrize("bland_after", [1, 3])
def test_bland_branch_reaches_the_assignment_optimum(oracle_mod, t, bland_after):
    """Equal weights on integer grids: the LP optimum is the assignment
    optimum over C / t (Birkhoff), and the values are exact in binary.  With
    a short degenerate run before Bland's rule, every pair of the family
    pivots under it, and still reaches that optimum."""
    from scipy.optimize import linear_sum_assignment
    A, B, pairs = synth.make_degenerate(1, 6, t, t)
    for k in range(pairs.shape[0]):
        x, p = A.bag(k)
        y, q = B.bag(k)
        C = cost(x, y)
        r, c = linear_sum_assignment(C)
        want = C[r, c].sum() / t
        got, _, _, _, piv, bl = oracle_mod.emd_pair(x, p, y, q, stats=True, bland_after=bland_after)
        assert abs(got - want) <= 1e-12 * max(1.0, want), (k, got, want)
        assert bl > 0 and piv >= bl, (k, piv, bl)
        default = oracle_mod.emd_pair(x, p, y, q)
        assert default[0] == got   # same optimum (exact arithmetic), another pivot path


def test_bland_counts_in_the_batch_entry(oracle_mod):
    """The batch entry reports the same per-pair pivot and Bland counts as
    single solves, and the default run (2(t+s) degenerate pivots) does not
    reach Bland's rule on this family."""
    A, B, pairs = synth.make_degenerate(2, 8, 32, 32)
    dist, st, piv, bl = oracle_mod.emd_batch_stats(A, B, pairs, bland_after=2)
    assert np.all(st == 0)
    for k in range(pairs.shape[0]):
        x, p = A.bag(k)
        y, q = B.bag(k)
        one = oracle_mod.emd_pair(x, p, y, q, stats=True, bland_after=2)
        assert (one[0], one[4], one[5]) == (dist[k], piv[k], bl[k])
    assert np.all(bl > 0)
    _, _, _, bl0 = oracle_mod.emd_batch_stats(A, B, pairs)
    assert np.all(bl0 == 0)


def test_identical_pairs_under_bland_rule_from_the_first_degenerate_pivot(oracle_mod):
    """With bland_after = 1 on a bag against itself, every pivot from the
    north-west corner is degenerate (the corner plan is the identity, already
    optimal at 0), so the first pivot is Dantzig's and every later one is
    Bland's.  The run ends at exactly 0 with a dual-feasible basis."""
    for t in (8, 16, 64):
        A, B, pairs = synth.make_degenerate(3, 1, t, t, identical_every=1)
        x, p = A.bag(0)
        got, plan, u, v, piv, bl = oracle_mod.emd_pair(x, p, x, p, stats=True, bland_after=1)
        assert got == 0.0
        assert piv >= 1 and bl == piv - 1, (t, piv, bl)
        C = cost(x, x)
        assert np.all(C - u[:, None] - v[None, :] >= -1e-14 * C.max())
