"""Allocation failures, forced from the host (include/igdebug.h): for every
entry point that allocates device memory, the k-th allocation is made to
fail for k = 1, 2, ... until the call needs fewer; each failing call must
return IG_ERR_OUT_OF_MEMORY, and once the call's own handles are destroyed
and the library's caches released, the live-allocation count must be back
where it started (nothing leaked on the error path).  The call that finally
succeeds must give the right answer.  No kernel runs on a failed allocation's
path, so nothing here can fault the GPU."""
import ctypes

import numpy as np
import pytest

import igsynth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1609_03782_amd as ig
    ig.lib()
    return torch.device("cuda:0")


def _walk(call, max_k=80):
    """call() -> (status, value); it must release whatever handles it makes.
    Returns (allocations the call makes, the successful call's value)."""
    import torch
    import paper_1609_03782_amd as ig
    L = ig.lib()
    torch.cuda.synchronize()
    L.ig_debug_release_caches()
    base = L.ig_debug_live_allocations()
    for k in range(1, max_k):
        L.ig_debug_fail_alloc(k)
        rc, val = call()
        L.ig_debug_fail_alloc(0)
        torch.cuda.synchronize()
        L.ig_debug_release_caches()
        assert L.ig_debug_live_allocations() == base, f"leak with allocation {k} failing (status {rc})"
        if rc == ig.IG_OK:
            return k - 1, val
        assert rc == ig.IG_ERR_OUT_OF_MEMORY, (k, rc, L.ig_last_error())
    raise AssertionError("the call kept failing")


def test_filter_create_run_destroy(dev):
    import torch
    import paper_1609_03782_amd as ig
    L = ig.lib()
    x = torch.from_numpy(igsynth.random_cube((20, 30, 70), seed=1)).to(dev)
    ref = ig.Filter(tuple(x.shape), n_iter=5).run(x)
    out = torch.empty_like(x)
    p = ig.make_params(tuple(x.shape), n_iter=5)

    def call():
        h = ctypes.c_void_p()
        rc = L.ig_filter_create(ctypes.byref(p), 0, ctypes.byref(h))
        if rc != ig.IG_OK:
            assert not h.value
            return rc, None
        rc = L.ig_filter_run(h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), ig._stream_ptr(x), None)
        torch.cuda.synchronize()
        L.ig_filter_destroy(h)
        return rc, None

    n, _ = _walk(call)
    assert n == 6          # scratch cube, constants, partials, results; piece tables of depth 2 and 1
    assert torch.equal(out, ref)


def test_batch_plan(dev):
    import torch
    import paper_1609_03782_amd as ig
    L = ig.lib()
    cubes = [igsynth.random_cube(s, seed=10 + k) for k, s in enumerate([(8, 9, 10), (30, 40, 50), (12, 100, 90)])]
    xs = [torch.from_numpy(c).to(dev) for c in cubes]
    outs = [torch.empty_like(x) for x in xs]
    kw = dict(K=2.0, tau=1 / 16, n_iter=7)
    refs = [ig.Filter(tuple(x.shape), **kw).run(x) for x in xs]
    arr = ig._batch_array([(x, o, kw) for x, o in zip(xs, outs)])
    n, _ = _walk(lambda: (L.ig_filter_batch(arr, len(xs), 0, ig._stream_ptr(xs[0]), None, None), None))
    assert n >= 10
    for o, r in zip(outs, refs):
        assert torch.equal(o, r)


def test_reduce_quality_sweep(dev):
    import torch
    import paper_1609_03782_amd as ig
    L = ig.lib()
    x = torch.from_numpy(igsynth.cube_field(48, seed=3, nz=24)).to(dev)
    y = ig.Filter(tuple(x.shape), n_iter=5).run(x)
    torch.cuda.synchronize()
    nz, ny, nx = x.shape
    s = ctypes.c_double()
    n, _ = _walk(lambda: (L.ig_reduce(ctypes.c_void_p(x.data_ptr()), 0, x.numel(), 0, ig._stream_ptr(x),
                                      ctypes.byref(s), None, None), None))
    assert n == 2 and s.value == pytest.approx(float(x.double().sum()), rel=1e-12)
    q = ig._quality_params(None, (3.0,), 3.0, 0.0, 0.0, 1.0)
    res = ig.IgQualityResult()
    want = ig.quality(x, y)
    n, _ = _walk(lambda: (L.ig_quality(ctypes.byref(q), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                       None, nx, ny, nz, 0, ig._stream_ptr(x), ctypes.byref(res)), None))
    assert n == 5 and res.F[0] == want["F"][0]       # reduction scratch (2) and quality scratch (3)
    pts = [dict(K=1.5, tau=0.03, n_iter=3, C=(1, 1, 1)), dict(K=2.0, tau=0.05, n_iter=4, C=(2, 2, 2))]
    results, best, _ = ig.sweep(x, pts)
    base = ig.make_params(tuple(x.shape), cond="intensity")
    P = (ig.IgSweepPoint * 2)()
    for i, pt in enumerate(pts):
        P[i].K, P[i].tau, P[i].n_iter = pt["K"], pt["tau"], pt["n_iter"]
        for a in range(3):
            P[i].C[a] = pt["C"][a]
    R = (ig.IgQualityResult * 2)()
    b = ctypes.c_int32()
    n, _ = _walk(lambda: (L.ig_filter_sweep(ctypes.byref(base), P, 2, ctypes.c_void_p(x.data_ptr()), None,
                                            ctypes.byref(q), 0, ig._stream_ptr(x), R, ctypes.byref(b), None), None))
    assert n >= 10
    assert b.value == best and R[best].F[0] == results[best]["F"][0]


def test_surrogate_create_train_infer(dev):
    import torch
    import paper_1609_03782_amd as ig
    from paper_1609_03782_amd import surrogate as sg
    L = sg.slib()
    c = igsynth.random_cube((12, 14, 40), seed=5)
    x = torch.from_numpy(c).to(dev)
    t = ig.Filter(c.shape, n_iter=4).run(x)
    ref_net = sg.Surrogate(depth=3, seed=7, lr=1e-3)
    ref_net.train_step([x], [t])
    w_ref = ref_net.get_weights()
    y_ref = ref_net.infer(x)
    torch.cuda.synchronize()
    ref_net.close()
    prm = sg.IgSurrogateParams(ctypes.sizeof(sg.IgSurrogateParams), 3, 32, 0, 1e-3, 0.9, 0.999, 1e-8, 7)
    X = (ctypes.c_void_p * 1)(x.data_ptr())
    T = (ctypes.c_void_p * 1)(t.data_ptr())
    nz, ny, nx = x.shape
    y = torch.empty_like(x)
    w = np.empty(w_ref.size, np.float32)

    def call():
        h = ctypes.c_void_p()
        rc = L.ig_surrogate_create(ctypes.byref(prm), 0, ctypes.byref(h))
        if rc != ig.IG_OK:
            return rc, None
        rc = L.ig_surrogate_train_step(h, X, T, 1, nx, ny, nz, ig._stream_ptr(x), None)
        if rc == ig.IG_OK:
            rc = L.ig_surrogate_infer(h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), nx, ny, nz, 0,
                                      ig._stream_ptr(x))
        if rc == ig.IG_OK:
            rc = L.ig_surrogate_get_weights(h, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), w.size)
        torch.cuda.synchronize()
        L.ig_surrogate_destroy(h)
        return rc, None

    n, _ = _walk(call)
    assert n >= 10
    assert np.array_equal(w, w_ref)
    assert torch.equal(y, y_ref)
