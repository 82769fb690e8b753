"""ig_filter_run_static: the filter without a handle and without device
allocation in the library (its workspace is a static device array).  Checked
through the C ABI against ig_filter_run on the same inputs, bit for bit (every
schedule gives the same bits), over consecutive calls that share the array."""
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
    return torch.device("cuda:0")


def _static(x, out, stats=True, **kw):
    import torch
    import paper_1609_03782_amd as ig
    p = ig.make_params(tuple(x.shape), dtype=ig._torch_dtype_name(x), **kw)
    st = ig.IgStats()
    st.struct_size = ctypes.sizeof(ig.IgStats)
    rc = ig.lib().ig_filter_run_static(ctypes.byref(p), 0, ctypes.c_void_p(x.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                       ctypes.byref(st) if stats else None)
    return rc, st


def _handle(x, **kw):
    import paper_1609_03782_amd as ig
    f = ig.Filter(tuple(x.shape), dtype=ig._torch_dtype_name(x), **kw)
    y, st = f.run(x, stats=True)
    f.close()
    return y, st


@pytest.mark.parametrize("cond", ["pm_exp", "intensity", "pm_rational"])
def test_two_calls_match_handle_run(dev, cond):
    import torch
    import paper_1609_03782_amd as ig
    kw = dict(K=2.0, tau=1.0 / 16, n_iter=9, cond=cond)
    # a cube of several tiles and a ragged tail, then a smaller one: the
    # second call reuses the array the first one left behind
    for shape, seed in (((40, 70, 131), 21), ((9, 13, 17), 22)):
        cube = igsynth.random_cube(shape, seed=seed) * 3.0
        x = torch.from_numpy(cube).to(dev)
        out = torch.full_like(x, 5.0)
        rc, st = _static(x, out, **kw)
        assert rc == ig.IG_OK, ig.lib().ig_last_error()
        ref, rst = _handle(x, **kw)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (shape, float((out - ref).abs().max()))
        assert st.rms_used == rst.rms_used and st.sum_in == rst.sum_in and st.sum_out == rst.sum_out
        assert st.passes >= 1


def test_in_place_no_stats_and_16bit(dev):
    import torch
    import paper_1609_03782_amd as ig
    cube = igsynth.random_cube((24, 33, 64), seed=23)
    for tdt in (torch.float32, torch.bfloat16):
        x = torch.from_numpy(cube).to(dev).to(tdt)
        ref, _ = _handle(x, n_iter=7, rms=1.1)
        y = x.clone()
        rc, _ = _static(y, y, stats=False, n_iter=7, rms=1.1)   # in place, no wait
        assert rc == ig.IG_OK, ig.lib().ig_last_error()
        torch.cuda.synchronize()
        assert torch.equal(y, ref), tdt


def test_largest_cube_and_limit(dev):
    import torch
    import paper_1609_03782_amd as ig
    cap = ig.static_max_bytes()
    assert cap == 64 << 20
    # 256^3 FP32 fills the workspace exactly
    shape = (256, 256, 256)
    rng = np.random.default_rng(24)
    x = torch.from_numpy(rng.standard_normal(shape, dtype=np.float32)).to(dev)
    out = torch.empty_like(x)
    rc, st = _static(x, out, n_iter=4)
    assert rc == ig.IG_OK, ig.lib().ig_last_error()
    ref, rst = _handle(x, n_iter=4)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    # one plane more is refused before any work; out is left as it was
    big = torch.zeros((257, 256, 256), device=dev)
    marker = torch.full_like(big, 2.0)
    rc, _ = _static(big, marker, n_iter=2)
    assert rc == ig.IG_ERR_INVALID_ARG
    assert "static workspace" in ig.lib().ig_last_error().decode()
    torch.cuda.synchronize()
    assert bool((marker == 2.0).all())


def test_nonfinite_input_sets_nan(dev):
    import torch
    import paper_1609_03782_amd as ig
    cube = igsynth.random_cube((8, 9, 10), seed=25)
    cube[3, 4, 5] = np.nan
    x = torch.from_numpy(cube).to(dev)
    out = torch.zeros_like(x)
    rc, st = _static(x, out, n_iter=3)
    assert rc == ig.IG_ERR_NONFINITE and st.nonfinite == 1
    torch.cuda.synchronize()
    assert bool(torch.isnan(out).all())
    # the next call on the same array is unaffected
    good = torch.from_numpy(igsynth.random_cube((8, 9, 10), seed=26)).to(dev)
    out2 = torch.empty_like(good)
    rc, _ = _static(good, out2, n_iter=3)
    assert rc == ig.IG_OK
    ref, _ = _handle(good, n_iter=3)
    torch.cuda.synchronize()
    assert torch.equal(out2, ref)
