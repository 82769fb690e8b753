"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point declared in include/*.h, the ctypes layouts match the C
structs, and argument validation rejects bad input before any device work."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_1609_03782_amd as ig

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(ig_[a-z0-9_]*)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    L = ig.lib()
    names = _declared()
    assert {"ig_filter_create", "ig_filter_run", "ig_filter_batch", "ig_filter_destroy",
            "ig_surrogate_train_step", "ig_surrogate_infer", "ig_conv3d_forward"} <= names
    for n in names:
        assert hasattr(L, n), n
    from paper_1609_03782_amd import surrogate
    bound = set(ig.SIGNATURES) | set(surrogate.SIGNATURES)
    assert names <= bound, names - bound


def test_struct_layouts_match_c(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "igfilter.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(ig_params), '
                   'sizeof(ig_schedule), sizeof(ig_stats), sizeof(ig_batch_item), sizeof(ig_compare_result), '
                   'offsetof(ig_params, rms), offsetof(ig_stats, schedule));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(ig.IgParams), ctypes.sizeof(ig.IgSchedule), ctypes.sizeof(ig.IgStats),
            ctypes.sizeof(ig.IgBatchItem), ctypes.sizeof(ig.IgCompareResult),
            ig.IgParams.rms.offset, ig.IgStats.schedule.offset]
    assert got == want


def _create(p):
    h = ctypes.c_void_p()
    rc = ig.lib().ig_filter_create(ctypes.byref(p), 0, ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("field,value", [
    ("nx", 0), ("ny", -1), ("nz", 0), ("n_iter", -1), ("K", 0.0), ("K", float("inf")),
    ("K", float("nan")), ("tau", -0.1), ("tau", float("nan")), ("dtype", 7), ("cond", 3),
    ("struct_size", 8), ("rms", float("nan")), ("reserved0", 1.0),
])
def test_create_rejects_invalid_params(field, value):
    p = ig.make_params((8, 8, 8))
    setattr(p, field, value)
    rc, h = _create(p)
    assert rc == ig.IG_ERR_INVALID_ARG
    assert not h.value
    assert ig.lib().ig_last_error()


def test_create_rejects_negative_C_and_huge_cube():
    p = ig.make_params((8, 8, 8))
    p.C[1] = -1.0
    assert _create(p)[0] == ig.IG_ERR_INVALID_ARG
    p = ig.make_params((2048, 1024, 1024))
    assert _create(p)[0] == ig.IG_ERR_INVALID_ARG


def test_null_arguments():
    L = ig.lib()
    assert L.ig_filter_create(None, 0, None) == ig.IG_ERR_INVALID_ARG
    assert L.ig_filter_run(None, None, None, None, None) == ig.IG_ERR_INVALID_ARG
    L.ig_filter_destroy(None)
    assert L.ig_status_string(ig.IG_ERR_NONFINITE) == b"non-finite input"
    assert L.ig_version().count(b".") == 2


def test_static_entry_point_validates_before_device_work():
    """ig_filter_run_static checks its arguments on the host: bad parameters,
    NULL buffers and cubes beyond the static workspace never reach a device."""
    L = ig.lib()
    assert L.ig_filter_static_max_bytes() == 64 << 20
    fake = ctypes.c_void_p(0x1000)
    assert L.ig_filter_run_static(None, 0, fake, fake, None, None) == ig.IG_ERR_INVALID_ARG
    p = ig.make_params((8, 8, 8))
    p.K = -1.0
    assert L.ig_filter_run_static(ctypes.byref(p), 0, fake, fake, None, None) == ig.IG_ERR_INVALID_ARG
    p = ig.make_params((8, 8, 8))
    assert L.ig_filter_run_static(ctypes.byref(p), 0, None, fake, None, None) == ig.IG_ERR_INVALID_ARG
    p = ig.make_params((257, 256, 256))                       # 1 plane past 64 MiB of FP32
    assert L.ig_filter_run_static(ctypes.byref(p), 0, fake, fake, None, None) == ig.IG_ERR_INVALID_ARG
    assert b"static workspace" in L.ig_last_error()
    p = ig.make_params((513, 256, 256), dtype="bf16")         # the same limit in bytes for 16-bit storage
    assert L.ig_filter_run_static(ctypes.byref(p), 0, fake, fake, None, None) == ig.IG_ERR_INVALID_ARG
    st = ig.IgStats()
    st.struct_size = 3
    p = ig.make_params((8, 8, 8))
    assert L.ig_filter_run_static(ctypes.byref(p), 0, fake, fake, None, ctypes.byref(st)) == ig.IG_ERR_INVALID_ARG


def test_valid_params_reach_the_device_check():
    # With valid parameters the only failure left on a GPU-less host is the device lookup.
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc, h = _create(ig.make_params((8, 8, 8)))
    assert rc == ig.IG_ERR_DEVICE and not h.value


def test_gpu_test_schedules_are_valid():
    """Every explicit schedule the GPU tests use must serve its shapes (host-only check)."""
    import test_gpu_parity as g
    for shape in g.SCHED_SHAPES:
        for s in g.SCHEDS[1:]:
            assert ig.schedule_check(shape, s, n_iter=7) is None, (shape, s)
    for s in g.INPLACE_SCHEDS:
        assert ig.schedule_check(g.INPLACE_SHAPE, s, n_iter=5) is None, s
    for shape in g.ROWS_SHAPES:
        for s in g.ROWS_SCHEDS:
            if 64 // s["rows"] * 4 >= shape[2]:
                assert ig.schedule_check(shape, s, n_iter=7) is None, (shape, s)
    assert ig.schedule_check((17, 33, 66), dict(kind="blocked", t_block=4, waves=8, vec=2)) is not None
    # automatic layout for nx = 66: 4 voxels per lane, 2 rows per wavefront -> 16 rows, enough for t_block 4
    assert ig.schedule_check((17, 33, 66), dict(kind="blocked", t_block=4, waves=8)) is None
    assert ig.schedule_check((17, 33, 66), dict(kind="blocked", t_block=2, waves=8, vec=8, rows=2)) is not None
    assert ig.schedule_check((17, 33, 100), dict(kind="blocked", t_block=2, waves=8, vec=4, rows=4)) is not None
    assert ig.schedule_check((17, 33, 64), dict(kind="blocked", t_block=2, waves=8, vec=4, rows=4)) is None
    assert ig.schedule_check((17, 33, 64), dict(kind="blocked", t_block=2, waves=8, vec=4, rows=3)) is not None
    assert ig.schedule_check((17, 33, 600), dict(kind="blocked", t_block=4, waves=16, vec=8)) is not None


def test_quality_struct_layouts_match_c(tmp_path):
    src = tmp_path / "q.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "igquality.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu\\n", sizeof(ig_quality_params), '
                   'sizeof(ig_quality_result), offsetof(ig_quality_params, indep), '
                   'offsetof(ig_quality_result, N_f), offsetof(ig_quality_result, sigma_FM));return 0;}\n')
    exe = tmp_path / "q"
    subprocess.check_call(["gcc", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(ig.IgQualityParams), ctypes.sizeof(ig.IgQualityResult), ig.IgQualityParams.indep.offset,
            ig.IgQualityResult.N_f.offset, ig.IgQualityResult.sigma_FM.offset]
    assert got == want


def _qparams(**kw):
    q = ig.IgQualityParams()
    q.struct_size = ctypes.sizeof(ig.IgQualityParams)
    q.n_thr = 1
    q.thr_f[0] = 3.0
    q.thr_o = 3.0
    q.indep = 1.0
    for k, v in kw.items():
        if k == "roi":
            for j, x in enumerate(v):
                q.roi[j] = x
        else:
            setattr(q, k, v)
    return q


@pytest.mark.parametrize("kw", [dict(n_thr=0), dict(n_thr=64), dict(indep=0.0), dict(thr_o=float("nan")),
                                dict(struct_size=16), dict(roi=(0, 9, 0, 4, 0, 4)), dict(roi=(3, 3, 0, 4, 0, 4)),
                                dict(roi=(-1, 2, 0, 4, 0, 4)), dict(rms_f=float("inf"))])
def test_quality_rejects_invalid_arguments(kw):
    q = _qparams(**kw)
    r = ig.IgQualityResult()
    fake = ctypes.c_void_p(4096)   # never dereferenced: validation fails first
    rc = ig.lib().ig_quality(ctypes.byref(q), fake, fake, None, 8, 4, 4, 0, None, ctypes.byref(r))
    assert rc == ig.IG_ERR_INVALID_ARG, kw
    rc = ig.lib().ig_quality(ctypes.byref(_qparams()), None, fake, None, 8, 4, 4, 0, None, ctypes.byref(r))
    assert rc == ig.IG_ERR_INVALID_ARG


@pytest.mark.parametrize("kind,size,theta", [("box", (3, 5, 7), (0, 0, 0)), ("gauss", (3.0, 3.0, 3.0), (0, 0, 0)),
                                             ("gauss", (1.5, 4.0, 2.5), (0, 0, 0)),
                                             ("gauss", (2.0, 3.0, 3.0), (10.0, 20.0, 30.0)),
                                             ("gauss", (2.0, 5.0, 3.0), (0.0, 0.0, 30.0))])
def test_smooth_geometry_matches_oracle_kernel(kind, size, theta):
    from oracle import smooth as Sm
    r, sep = ig.smooth_geometry(kind, size, theta)
    k = Sm.box_kernel(size) if kind == "box" else Sm.gauss_kernel(size, theta)
    assert (2 * r[2] + 1, 2 * r[1] + 1, 2 * r[0] + 1) == k.shape
    assert sep == (kind == "box" or not any(theta))


@pytest.mark.parametrize("kind,size,theta", [("box", (2, 3, 3), (0, 0, 0)), ("box", (3, 3, 3), (0, 0, 5)),
                                             ("box", (3.5, 3, 3), (0, 0, 0)), ("gauss", (0.0, 3, 3), (0, 0, 0)),
                                             ("gauss", (3, float("nan"), 3), (0, 0, 0))])
def test_smooth_rejects_invalid(kind, size, theta):
    p = ig.smooth_params(kind, size, theta)
    assert ig.lib().ig_smooth_geometry(ctypes.byref(p), None, None) == ig.IG_ERR_INVALID_ARG


@pytest.mark.parametrize("kw,shape", [(dict(levels=0), (8, 8, 8)), (dict(levels=9), (8, 8, 8)), (dict(kind=2), (8, 8, 8)),
                                      (dict(reserved=1), (8, 8, 8)), ({}, (0, 8, 8)), ({}, (8, 8, 10241)),
                                      ({}, (2561, 8, 8))])
def test_wavelet_rejects_invalid(kw, shape):
    p = ig.wavelet_params()
    for k, v in kw.items():
        setattr(p, k, v)
    fake = ctypes.c_void_p(4096)   # never dereferenced: validation fails first
    nz, ny, nx = shape
    rc = ig.lib().ig_wavelet_forward(ctypes.byref(p), fake, fake, nx, ny, nz, None)
    assert rc in (ig.IG_ERR_INVALID_ARG, ig.IG_ERR_UNSUPPORTED), (kw, shape)
    if shape[2] > 10240 or shape[0] > 2560:
        assert rc == ig.IG_ERR_UNSUPPORTED


def test_batch_resident_limit_validation():
    """ig_batch_set_resident takes 0..32768 voxels and rejects the rest;
    ig_batch_get_resident reads it back (host only, no GPU)."""
    import ctypes
    import paper_1609_03782_amd as ig
    L = ig.lib()
    v = ctypes.c_int32()
    assert L.ig_batch_get_resident(ctypes.byref(v)) == ig.IG_OK
    old = v.value
    try:
        for bad in (-1, 32769, 1 << 30):
            assert L.ig_batch_set_resident(bad) == ig.IG_ERR_INVALID_ARG
        for good in (0, 1, 32768):
            assert L.ig_batch_set_resident(good) == ig.IG_OK
            assert L.ig_batch_get_resident(ctypes.byref(v)) == ig.IG_OK and v.value == good
        assert L.ig_batch_get_resident(None) == ig.IG_ERR_INVALID_ARG
    finally:
        L.ig_batch_set_resident(old)


def test_smooth_set_path_validation():
    assert ig.lib().ig_smooth_set_path(2) == ig.IG_ERR_INVALID_ARG
    assert ig.lib().ig_smooth_set_path(-1) == ig.IG_ERR_INVALID_ARG
    assert ig.lib().ig_smooth_set_path(1) == ig.IG_OK
    assert ig.lib().ig_smooth_set_path(0) == ig.IG_OK


def test_single_layer_conv_rejects_cubes_past_32bit_offsets():
    """The single-layer surrogate entry points run one kernel over the whole
    cube; a cube of 2^31 / 32 voxels or more is refused on the host, before
    any device work."""
    from paper_1609_03782_amd import surrogate as sg
    L = sg.slib()
    fake = ctypes.c_void_p(0x1000)
    n = (1 << 26)                         # 2^26 voxels x 32 channels = 2^31
    assert L.ig_conv3d_forward(fake, 32, fake, fake, 32, 1, None, fake, 1 << 10, 1 << 8, n >> 18, None) \
        == ig.IG_ERR_INVALID_ARG
    assert b"too large" in ig.lib().ig_last_error()
    assert L.ig_conv3d_input_grad(fake, 32, fake, 32, None, fake, 1 << 10, 1 << 8, n >> 18, None) == ig.IG_ERR_INVALID_ARG
    assert L.ig_conv3d_weight_grad(fake, 32, fake, 32, fake, fake, 1 << 10, 1 << 8, n >> 18, None) == ig.IG_ERR_INVALID_ARG


def test_infer_piece_limit_hook():
    """The test hook that lowers the surrogate's inference piece limit returns
    the previous limit; 0 restores the default of 2^28 voxels."""
    L = ig.lib()
    default = 1 << 28
    assert L.ig_debug_set_infer_piece_limit(12345) == default
    assert L.ig_debug_set_infer_piece_limit(0) == 12345
    assert L.ig_debug_set_infer_piece_limit(-5) == default
    assert L.ig_debug_set_infer_piece_limit(0) == default
