"""GPU: Alg. 1's passes never increase the clustering objective.

Within a pass, Step 2 moves each atom to the weighted mean of what its
plans send it, which minimises the objective for those plans, so the Step 3
value is at most the Step 1 value.  Across passes, the previous plans (and,
with free weights, the previous centroid weights) stay feasible for the next
Step 1, whose optimum is therefore at most the previous Step 3 value.  So
per cluster Step1[0] >= Step3[0] >= Step1[1] >= Step3[1] >= ..., checked on
the device's own outputs for the constrained update (centroid weights held)
and the update with free centroid weights."""
import numpy as np
import pytest

import synth

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


def case(seed, K=8, per=6, tlo=2, thi=14, s=6, d=3):
    rng = np.random.default_rng([8800, seed])
    centres = rng.normal(size=(K, d)) * 4.0
    bags, labels = [], []
    for j in range(K):
        for _ in range(per):
            t = int(rng.integers(tlo, thi + 1))
            bags.append((centres[j] + rng.normal(size=(t, d)), rng.dirichlet(np.ones(t))))
            labels.append(j)
    zb = [(centres[j] + rng.normal(size=(s, d)) * 1.5, np.full(s, 1.0 / s)) for j in range(K)]
    return synth.from_bags(bags), synth.from_bags(zb), np.asarray(labels, np.int32)


@pytest.mark.parametrize("free", [False, True])
@pytest.mark.parametrize("seed", [0, 1])
def test_passes_never_increase_the_objective(d2, free, seed):
    X, Z, labels = case(seed)
    h = d2.Handle(0)
    Xd = d2.DeviceSet.from_ragged(X, DEV)
    lab = torch.as_tensor(labels, device=DEV)
    cur = Z
    chain = []
    for _ in range(5):
        Zd = d2.DeviceSet.from_ragged(cur, DEV)
        if free:
            z, w, e1, e3, cnt, ost, cst = d2.d2_centroid_update_free(h, Xd, Zd, lab)
            torch.cuda.synchronize()
            assert int(cst.max().item()) == 0 and int(ost.max().item()) == 0
            cur = synth.RaggedSet(Z.offsets.copy(), z.cpu().numpy(), w.cpu().numpy())
        else:
            z, e1, e3, cnt, st = d2.d2_centroid_update(h, Xd, Zd, lab)
            torch.cuda.synchronize()
            assert int(st.max().item()) == 0
            cur = synth.RaggedSet(Z.offsets.copy(), z.cpu().numpy(), Z.weights.copy())
        chain += [e1.cpu().numpy(), e3.cpu().numpy()]
    chain = np.array(chain)                        # [step, cluster]
    assert np.all(np.isfinite(chain)) and np.all(chain >= 0)
    tol = 1e-12 * np.abs(chain).max(axis=0) + 1e-14
    assert np.all(np.diff(chain, axis=0) <= tol), np.diff(chain, axis=0).max(axis=0)
    assert np.all(chain[-1] < chain[0])            # and the passes did move the atoms
