"""d2_assign_noalloc, the labelling entry point that allocates nothing: its
workspace is the library's fixed per-GPU scratch array.  Checked through the
C ABI against d2_assign (same kernels, so bitwise) on two calls in a row,
the second smaller, with inputs that use the scratch for both the
support-class sort and split centroid ranges; and its size limit."""
import ctypes

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


@pytest.fixture(scope="module")
def h(d2):
    return d2.Handle(0)


def bags(rng, n, tmax, d):
    sizes = rng.integers(1, tmax + 1, size=n)
    return synth.from_bags([(rng.normal(size=(t, d)), rng.gamma(0.5, size=t) + 1e-3)
                            for t in sizes])


def noalloc(d2, h, Xd, Zd, opts, want_all=True):
    n, K = Xd.n, Zd.n
    lab = torch.full((n,), -7, dtype=torch.int32, device=DEV)
    best = torch.full((n,), -7.0, dtype=torch.float64, device=DEV)
    allv = torch.full((n, K), -7.0, dtype=torch.float64, device=DEV) if want_all else None
    st = torch.full((n,), -7, dtype=torch.int32, device=DEV)
    x, z, o = Xd.c(), Zd.c(), opts.c()
    p = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())   # noqa: E731
    rc = d2._ffi.lib().d2_assign_noalloc(h.ptr, ctypes.byref(x), ctypes.byref(z), ctypes.byref(o),
                                         p(lab), p(best), p(allv), p(st),
                                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return rc, lab.cpu().numpy(), best.cpu().numpy(), \
        (allv.cpu().numpy() if allv is not None else None), st.cpu().numpy()


def reference(d2, h, Xd, Zd, opts):
    lab, best, allv, st = d2.d2_assign(h, Xd, Zd, opts, want_all=True)
    torch.cuda.synchronize()
    return lab.cpu().numpy(), best.cpu().numpy(), allv.cpu().numpy(), st.cpu().numpy()


def test_noalloc_matches_assign_on_two_calls(d2, h):
    rng = np.random.default_rng(4242)
    Z = bags(rng, 64, 16, 5)
    Zd = d2.DeviceSet.from_ragged(Z, DEV)
    opts = d2.Opts(flags=1)
    for n in (240, 50):   # the second call is smaller
        X = bags(rng, n, 40, 5)          # supports 1..40 against 16: three classes, sorted
        Xd = d2.DeviceSet.from_ragged(X, DEV)
        need = d2.d2_workspace_bytes(h, 2, Xd, Zd, 0, opts)
        assert 0 < need <= d2._ffi.D2_NOALLOC_SCRATCH_BYTES
        rc, lab, best, allv, st = noalloc(d2, h, Xd, Zd, opts)
        assert rc == 0
        r_lab, r_best, r_all, r_st = reference(d2, h, Xd, Zd, opts)
        assert np.all(r_st == 0)
        np.testing.assert_array_equal(lab, r_lab)
        np.testing.assert_array_equal(best, r_best)
        np.testing.assert_array_equal(allv, r_all)
        np.testing.assert_array_equal(st, r_st)
        # without the full matrix as well
        rc, lab2, best2, _, st2 = noalloc(d2, h, Xd, Zd, opts, want_all=False)
        assert rc == 0
        np.testing.assert_array_equal(lab2, r_lab)
        np.testing.assert_array_equal(best2, r_best)


def test_noalloc_rejects_calls_beyond_the_scratch(d2, h):
    # 300,000 one-atom rows against centroids large enough (2 MiB of points)
    # to be split into 8 ranges by XCD: the partial minima (16 B per row and
    # range, 38.4 MB) exceed the scratch, so the call is refused and nothing
    # is enqueued
    rng = np.random.default_rng(4243)
    n = 300_000
    X = synth.RaggedSet(np.arange(n + 1, dtype=np.int64), rng.normal(size=(n, 16)), np.ones(n))
    Z = synth.RaggedSet(np.arange(0, 16 * 1024 + 1, 16, dtype=np.int64), rng.normal(size=(16 * 1024, 16)),
                        np.ones(16 * 1024))
    Xd, Zd = d2.DeviceSet.from_ragged(X, DEV), d2.DeviceSet.from_ragged(Z, DEV)
    opts = d2.Opts()
    assert d2.d2_workspace_bytes(h, 2, Xd, Zd, 0, opts) > d2._ffi.D2_NOALLOC_SCRATCH_BYTES
    rc, lab, _, _, _ = noalloc(d2, h, Xd, Zd, opts, want_all=False)
    assert rc == d2._ffi.D2_ESCRATCH
    assert np.all(lab == -7)
