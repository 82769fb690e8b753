"""GPU parity of the HIP filter against the FP64 oracle, through the C ABI.

Tolerance: max |GPU - oracle| <= 1e-5 * rho for FP32 storage (rho = the rms
noise level used).  Integer-like facts (fixed points, identity, schedule
invariance, composition) are checked bitwise.
"""
import numpy as np
import pytest

import igsynth

pytestmark = pytest.mark.gpu

TOL = 1e-5
CONDS = ["intensity", "pm_exp", "pm_rational"]


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1609_03782_amd as ig
    ig.lib()
    return torch.device("cuda:0")


def _gpu(cube, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(cube)).to(dev)


def _run(cube, dev, sched=None, stats=False, **kw):
    import torch
    import paper_1609_03782_amd as ig
    f = ig.Filter(cube.shape, **kw)
    if sched is not None:
        f.set_schedule(**sched)
    x = _gpu(cube, dev)
    r = f.run(x, stats=stats)
    torch.cuda.synchronize()
    if stats:
        y, st = r
        return y.cpu().numpy(), st
    return r.cpu().numpy()


def _err(y, ref):
    return float(np.abs(y.astype(np.float64) - ref).max())


def test_small_config_parity(dev, oracle_lib):
    # 64x64x32 galaxy + tail cube, exponential conductance K=2, tau=1/16, 10 steps
    cube = igsynth.cube_small(seed=1)
    y, st = _run(cube, dev, stats=True, K=2.0, tau=1 / 16, n_iter=10, cond="pm_exp")
    ref, rho = oracle_lib.run(cube, "pm_exp", K=2.0, tau=1 / 16, n_iter=10)
    assert st.rms_used == pytest.approx(rho, rel=1e-13)
    e = _err(y, ref)
    print(f"64x64x32 pm_exp n=10: max-abs {e:.3e} = {e / rho:.3e} rms")
    assert e <= TOL * rho
    assert st.sum_in == pytest.approx(float(cube.astype(np.float64).sum()), rel=1e-12, abs=1e-9)
    assert abs(st.sum_out - st.sum_in) <= 1e-6 * rho * cube.size ** 0.5


@pytest.mark.parametrize("cond", CONDS)
def test_paper_defaults_parity(dev, oracle_lib, cond):
    # the paper's default parameters (K=1.5, tau=0.0325, n=20, C=5) on a ragged cube
    cube = igsynth.cube_field(72, seed=3, nz=37)[:, :61, :]
    cube = np.ascontiguousarray(cube)
    y = _run(cube, dev, K=1.5, tau=0.0325, n_iter=20, C=(5, 5, 5), cond=cond)
    ref, rho = oracle_lib.run(cube, cond, K=1.5, tau=0.0325, n_iter=20, C=(5, 5, 5))
    e = _err(y, ref)
    print(f"{cond} defaults 72x61x37: {e / rho:.3e} rms")
    assert e <= TOL * rho


SCHEDS = [
    dict(kind="naive"),
    dict(kind="blocked", t_block=1, waves=3, zchunk=3, vec=1),
    dict(kind="blocked", t_block=2, waves=5, zchunk=5, vec=1),
    dict(kind="blocked", t_block=3, waves=8, zchunk=7, vec=2),
    dict(kind="blocked", t_block=4, waves=9, zchunk=0, vec=4),
    dict(kind="blocked", t_block=2, waves=6, zchunk=4, vec=4),
    dict(kind="blocked", t_block=3, waves=10, zchunk=9, vec=8),
    dict(kind="blocked", t_block=2, waves=16, zchunk=0, vec=0, rounds=3),
    dict(kind="blocked", t_block=1, waves=16, zchunk=0, vec=0),
]


SCHED_SHAPES = [(13, 37, 70), (9, 20, 133), (21, 67, 45), (5, 3, 300)]


@pytest.mark.parametrize("cond", CONDS)
@pytest.mark.parametrize("shape", SCHED_SHAPES)
def test_schedules_bitwise_and_parity(dev, oracle_lib, cond, shape):
    cube = igsynth.random_cube(shape, seed=sum(shape), scale=2.0)
    cube[shape[0] // 2, shape[1] // 3, shape[2] // 4] = 12.0   # a bright source
    kw = dict(K=1.7, tau=0.05, n_iter=7, C=(1.0, 0.8, 1.3), cond=cond)
    ref, rho = oracle_lib.run(cube, cond, K=1.7, tau=0.05, n_iter=7, C=(1.0, 0.8, 1.3))
    outs = []
    for s in SCHEDS:
        y = _run(cube, dev, sched=s, **kw)
        e = _err(y, ref)
        assert e <= TOL * rho, (s, e / rho)
        outs.append(y)
    for s, y in zip(SCHEDS[1:], outs[1:]):
        assert np.array_equal(y, outs[0]), s


def test_edge_shapes(dev, oracle_lib):
    for shape in [(1, 1, 1), (1, 1, 9), (1, 7, 1), (6, 1, 1), (2, 2, 2), (3, 1, 65), (40, 2, 3)]:
        cube = igsynth.random_cube(shape, seed=7)
        for cond in CONDS:
            y = _run(cube, dev, K=1.2, tau=0.06, n_iter=5, C=(1, 2, 3), cond=cond)
            ref, rho = oracle_lib.run(cube, cond, K=1.2, tau=0.06, n_iter=5, C=(1, 2, 3))
            assert _err(y, ref) <= TOL * rho, (shape, cond)


def test_identity_cases_bitwise(dev):
    cube = igsynth.random_cube((11, 19, 29), seed=8)
    for kw in (dict(n_iter=0), dict(tau=0.0, n_iter=5), dict(C=(0, 0, 0), n_iter=5)):
        for cond in CONDS:
            y = _run(cube, dev, cond=cond, **kw)
            assert np.array_equal(y, cube), (kw, cond)
    const = np.full((9, 10, 11), 2.5, np.float32)
    for cond in CONDS:
        assert np.array_equal(_run(const, dev, cond=cond, n_iter=6), const)
    zero = np.zeros((4, 5, 6), np.float32)
    assert np.array_equal(_run(zero, dev, n_iter=3), zero)


# several rows per wavefront (narrow cubes): explicit layouts against the naive schedule
ROWS_SHAPES = [(11, 29, 40), (6, 50, 64), (9, 23, 100), (4, 70, 17)]
ROWS_SCHEDS = [dict(kind="blocked", t_block=1, waves=2, vec=4, rows=4),
               dict(kind="blocked", t_block=3, waves=4, vec=4, rows=2, zchunk=3),
               dict(kind="blocked", t_block=2, waves=3, vec=4, rows=2, rounds=2),
               dict(kind="blocked", t_block=4, waves=16, vec=4, rows=2)]


@pytest.mark.parametrize("cond", CONDS)
@pytest.mark.parametrize("shape", ROWS_SHAPES)
def test_rows_per_wavefront_bitwise(dev, oracle_lib, cond, shape):
    cube = igsynth.random_cube(shape, seed=3 * sum(shape), scale=2.0)
    kw = dict(K=1.3, tau=0.05, n_iter=7, C=(1.0, 0.7, 1.3), cond=cond)
    ref, rho = oracle_lib.run(cube, cond, K=1.3, tau=0.05, n_iter=7, C=(1.0, 0.7, 1.3))
    y0 = _run(cube, dev, sched=dict(kind="naive"), **kw)
    assert _err(y0, ref) <= TOL * rho
    for sc in ROWS_SCHEDS:
        if 64 // sc["rows"] * 4 < shape[2]:
            continue
        y = _run(cube, dev, sched=sc, **kw)
        assert np.array_equal(y, y0), (shape, sc)


INPLACE_SHAPE = (17, 33, 66)
INPLACE_SCHEDS = [dict(kind="naive"), dict(kind="blocked", t_block=1, waves=4, zchunk=8),
                  dict(kind="blocked", t_block=2, waves=8, zchunk=8),
                  dict(kind="blocked", t_block=4, waves=9, zchunk=0, vec=4)]


def test_in_place_and_odd_passes(dev, oracle_lib):
    import torch
    import paper_1609_03782_amd as ig
    cube = igsynth.random_cube(INPLACE_SHAPE, seed=9)
    ref, rho = oracle_lib.run(cube, "pm_exp", n_iter=5)
    for sched in INPLACE_SCHEDS:
        f = ig.Filter(cube.shape, n_iter=5)
        f.set_schedule(**sched)
        x = _gpu(cube, dev)
        y = f.run(x, out=x)
        torch.cuda.synchronize()
        assert y.data_ptr() == x.data_ptr()
        assert _err(x.cpu().numpy(), ref) <= TOL * rho, sched


def test_composition_bitwise(dev):
    import torch
    import paper_1609_03782_amd as ig
    cube = igsynth.random_cube((12, 40, 50), seed=10)
    x = _gpu(cube, dev)
    a = ig.Filter(cube.shape, n_iter=9, rms=1.25).run(x)
    b = ig.Filter(cube.shape, n_iter=4, rms=1.25).run(x)
    b = ig.Filter(cube.shape, n_iter=5, rms=1.25).run(b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_nonfinite_input_rejected(dev):
    import torch
    import paper_1609_03782_amd as ig
    cube = igsynth.random_cube((8, 9, 10), seed=11)
    cube[3, 4, 5] = np.nan
    cube[1, 1, 1] = np.inf
    x = _gpu(cube, dev)
    out = torch.full_like(x, 7.0)
    f = ig.Filter(cube.shape, n_iter=3)
    with pytest.raises(ig.IgError) as ei:
        f.run(x, out=out, stats=True)
    assert ei.value.status == ig.IG_ERR_NONFINITE
    torch.cuda.synchronize()
    assert bool(torch.isnan(out).all())   # no step ran; the output says so


@pytest.mark.parametrize("in_place", [False, True])
def test_nonfinite_input_visible_without_stats(dev, in_place):
    """With rho estimated and no statistics the call returns at once, so the
    failure shows in the output: every voxel NaN, out of place or in place."""
    import torch
    import paper_1609_03782_amd as ig
    cube = igsynth.random_cube((12, 17, 70), seed=14)
    cube[5, 6, 7] = np.inf
    x = _gpu(cube, dev)
    out = x if in_place else torch.zeros_like(x)
    y = ig.Filter(cube.shape, n_iter=4 if in_place else 3).run(x, out=out)
    torch.cuda.synchronize()
    assert bool(torch.isnan(y).all())
    if not in_place:
        assert bool(torch.isinf(x).any())   # the input is left as it was


def test_stats_and_monotone_flag(dev):
    cube = igsynth.random_cube((8, 16, 16), seed=12)
    _, st = _run(cube, dev, stats=True, tau=0.0625, C=(5, 5, 5), n_iter=2, cond="intensity")
    assert not st.monotone
    _, st = _run(cube, dev, stats=True, tau=1 / 16, C=(1, 1, 1), n_iter=2)
    assert st.monotone and st.nonfinite == 0 and st.passes >= 1


def test_reduce_and_compare(dev):
    import torch
    import paper_1609_03782_amd as ig
    cube = igsynth.random_cube((10, 20, 30), seed=13)
    x = _gpu(cube, dev)
    s, q, bad = ig.reduce(x)
    d = cube.astype(np.float64)
    assert s == pytest.approx(d.sum(), rel=1e-12, abs=1e-9) and q == pytest.approx((d * d).sum(), rel=1e-12)
    assert bad == 0
    ref = torch.from_numpy(d + 1e-3).to(dev)
    r = ig.compare(x, ref, tol=5e-4)
    assert r["max_abs"] == pytest.approx(1e-3, rel=1e-4) and r["n_over"] == cube.size


# Cubes wider than one x tile (64 V voxels): tiles start at multiples of V,
# so with nx a multiple of V the vector path serves them (1040, 600), else
# the scalar one (1037).  Bitwise against the naive schedule, in FP32 and in
# bfloat16 storage (buffer loads and stores), and FP32 against the oracle.
WIDE_SHAPES = [(4, 5, 1040), (3, 4, 1037), (6, 9, 600), (5, 6, 991)]


@pytest.mark.parametrize("cond", CONDS)
@pytest.mark.parametrize("shape", WIDE_SHAPES)
def test_wide_cubes_bitwise(dev, oracle_lib, cond, shape):
    import torch
    import paper_1609_03782_amd as ig
    cube = igsynth.random_cube(shape, seed=sum(shape) + 3, scale=2.0)
    cube[shape[0] // 2, shape[1] // 2, shape[2] - 3] = 10.0
    kw = dict(K=1.7, tau=0.05, n_iter=6, C=(1.0, 0.8, 1.3), cond=cond)
    ref, rho = oracle_lib.run(cube, cond, K=1.7, tau=0.05, n_iter=6, C=(1.0, 0.8, 1.3))
    for dtype in ("f32", "bf16"):
        x = torch.from_numpy(cube).to(dev)
        if dtype == "bf16":
            x = x.to(torch.bfloat16)
        outs = []
        for s in (dict(kind="naive"), None, dict(kind="blocked", t_block=3, waves=10, vec=8),
                  dict(kind="blocked", t_block=2, waves=12, vec=4)):
            f = ig.Filter(shape, dtype=dtype, **kw)
            if s is not None:
                f.set_schedule(**s)
            y = f.run(x)
            torch.cuda.synchronize()
            if s is None:
                sc = f.schedule()
                assert sc["kind"] == "blocked"
            outs.append(y.float().cpu().numpy())
            f.close()
        for k, y in enumerate(outs[1:], 1):
            assert np.array_equal(y, outs[0]), (dtype, k)
        if dtype == "f32":
            assert _err(outs[0], ref) <= TOL * rho


GROUPED_CASES = [((64, 512, 512), dict(kind="blocked", t_block=2, waves=16, vec=8)),
                 ((20, 130, 520), dict(kind="blocked", t_block=1, waves=16)),
                 ((24, 100, 300), dict(kind="blocked", t_block=2, waves=16, rounds=2))]


@pytest.mark.parametrize("cond", CONDS)
@pytest.mark.parametrize("shape,sched", GROUPED_CASES)
def test_grouped_workgroups_bitwise(dev, oracle_lib, cond, shape, sched):
    """Plans in which a workgroup runs a share of the pieces in turn (one or
    two pieces; the tile count does not divide the workgroups) give bitwise
    the naive schedule's result, and the oracle's within the parity bar."""
    import torch
    import paper_1609_03782_amd as ig
    grouped = ig.schedule_plan_groups(shape, sched, sched["t_block"])
    cube = igsynth.random_cube(shape, seed=sum(shape) + 11, scale=2.0)
    cube[shape[0] // 2, shape[1] // 2, shape[2] // 3] = 11.0
    x = torch.from_numpy(cube).to(dev)
    n = 5
    f0 = ig.Filter(shape, K=2.0, tau=1 / 16, n_iter=n, cond=cond)
    f0.set_schedule("naive")
    y0 = f0.run(x)
    f = ig.Filter(shape, K=2.0, tau=1 / 16, n_iter=n, cond=cond)
    f.set_schedule(**sched)
    y = f.run(x)
    torch.cuda.synchronize()
    assert torch.equal(y, y0), (shape, sched, grouped is not None)
    ref, rho = oracle_lib.run(cube, cond, K=2.0, tau=1 / 16, n_iter=n)
    assert _err(y.cpu().numpy(), ref) <= TOL * rho


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_grouped_workgroups_16bit_bitwise(dev, dtype):
    """The grouped 16-wave plan with 16-bit storage (not the default there,
    but reachable through an explicit schedule) gives bitwise the naive
    schedule's result in the same storage type."""
    import torch
    import paper_1609_03782_amd as ig
    shape, sched = (64, 512, 512), dict(kind="blocked", t_block=2, waves=16, vec=8)
    assert ig.schedule_plan_groups(shape, sched, 2) is not None
    tdt = {"bf16": torch.bfloat16, "f16": torch.float16}[dtype]
    cube = igsynth.random_cube(shape, seed=77, scale=2.0)
    x = torch.from_numpy(cube).to(dev).to(tdt)
    f0 = ig.Filter(shape, K=2.0, tau=1 / 16, n_iter=6, dtype=dtype)
    f0.set_schedule("naive")
    y0 = f0.run(x)
    f = ig.Filter(shape, K=2.0, tau=1 / 16, n_iter=6, dtype=dtype)
    f.set_schedule(**sched)
    y = f.run(x)
    torch.cuda.synchronize()
    assert torch.equal(y, y0)
