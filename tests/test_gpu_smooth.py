"""GPU machine / Gaussian smoothing (ig_smooth) against the FP64 oracle: ragged
cubes, kernels larger than the cube, axis-aligned (separable: the fused pass and three passes) and
rotated (dense) Gaussians, and sampled voxels of the 512^3 cube."""
import numpy as np
import pytest

import igsynth
from oracle import smooth as Sm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1609_03782_amd as ig
    ig.lib()
    return torch.device("cuda:0")


def _kernel(kind, size, theta=(0.0, 0.0, 0.0)):
    return Sm.box_kernel(size) if kind == "box" else Sm.gauss_kernel(size, theta)


def _tol(cube, kind, theta):
    # FP32 sums: three passes of <= 2r+1 taps, or one dense pass of up to ~10^3 taps
    rel = 2e-5 if (kind == "gauss" and any(theta)) else 5e-6
    return rel * float(np.abs(cube).max())


CASES = [("box", (3, 3, 3), (0, 0, 0)), ("box", (3, 5, 5), (0, 0, 0)), ("box", (1, 1, 1), (0, 0, 0)),
         ("box", (7, 3, 1), (0, 0, 0)), ("gauss", (3.0, 3.0, 3.0), (0, 0, 0)), ("gauss", (2.0, 3.0, 3.0), (0, 0, 0)),
         ("gauss", (1.5, 4.0, 2.5), (0, 0, 0)), ("gauss", (2.0, 3.0, 3.0), (10.0, 20.0, 30.0)),
         ("gauss", (3.0, 3.0, 3.0), (0.0, 45.0, 0.0)), ("gauss", (2.0, 4.0, 2.0), (0.0, 0.0, 90.0))]


@pytest.mark.parametrize("kind,size,theta", CASES)
def test_smooth_matches_oracle(dev, kind, size, theta):
    import torch
    import paper_1609_03782_amd as ig
    cube = igsynth.random_cube((23, 29, 71), seed=3)
    y = ig.smooth(torch.from_numpy(cube).to(dev), kind, size, theta)
    torch.cuda.synchronize()
    ref = Sm.smooth(cube, _kernel(kind, size, theta))
    err = np.abs(y.cpu().numpy() - ref).max()
    assert err <= _tol(cube, kind, theta), err
    r, sep = ig.smooth_geometry(kind, size, theta)
    k = _kernel(kind, size, theta)
    assert (2 * r[2] + 1, 2 * r[1] + 1, 2 * r[0] + 1) == k.shape
    assert sep == (kind == "box" or not any(theta))


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 3, 1), (1, 1, 300), (3, 70, 2), (9, 1, 65)])
def test_smooth_thin_cubes(dev, shape):
    import torch
    import paper_1609_03782_amd as ig
    cube = igsynth.random_cube(shape, seed=11)
    for kind, size, theta in [("box", (5, 5, 5), (0, 0, 0)), ("gauss", (4.0, 3.0, 5.0), (0, 0, 0)),
                              ("gauss", (3.0, 2.0, 2.0), (5.0, 15.0, 25.0))]:
        y = ig.smooth(torch.from_numpy(cube).to(dev), kind, size, theta)
        ref = Sm.smooth(cube, _kernel(kind, size, theta))
        assert np.abs(y.cpu().numpy() - ref).max() <= _tol(cube, kind, theta), (shape, kind)


def test_rotation_by_90_degrees_equals_swapped_widths(dev):
    import torch
    import paper_1609_03782_amd as ig
    x = torch.from_numpy(igsynth.random_cube((20, 33, 40), seed=5)).to(dev)
    a = ig.smooth(x, "gauss", (2.0, 4.0, 3.0), (0.0, 0.0, 90.0))     # dense path
    b = ig.smooth(x, "gauss", (4.0, 2.0, 3.0))                        # separable path
    assert float((a - b).abs().max()) <= 2e-5 * float(x.abs().max())


def test_smooth_fullsize_sampled(dev):
    """512^3: the value at a voxel depends only on its kernel window, so the
    oracle on the window (clipped to the cube) gives it exactly."""
    import torch
    import paper_1609_03782_amd as ig
    cube = igsynth.cube_field(512, seed=2)
    x = torch.from_numpy(cube).to(dev)
    rng = np.random.default_rng(4)
    pts = [(0, 0, 0), (511, 511, 511), (0, 255, 511), (300, 0, 17)] + \
          [tuple(int(v) for v in rng.integers(0, 512, 3)) for _ in range(8)]
    for kind, size, theta in [("gauss", (3.0, 3.0, 3.0), (0, 0, 0)), ("gauss", (2.0, 3.0, 3.0), (10.0, 20.0, 30.0)),
                              ("box", (3, 5, 5), (0, 0, 0))]:
        y = ig.smooth(x, kind, size, theta).cpu().numpy()
        k = _kernel(kind, size, theta)
        rz, ry, rx = (s // 2 for s in k.shape)
        for (z, yy, xx) in pts:
            z0, z1 = max(0, z - rz), min(512, z + rz + 1)
            y0, y1 = max(0, yy - ry), min(512, yy + ry + 1)
            x0, x1 = max(0, xx - rx), min(512, xx + rx + 1)
            ref = Sm.smooth(cube[z0:z1, y0:y1, x0:x1], k)[z - z0, yy - y0, xx - x0]
            assert abs(y[z, yy, xx] - ref) <= _tol(cube, kind, theta), (kind, (z, yy, xx))


FUSED_CASES = [("box", (1, 1, 1)), ("box", (3, 3, 3)), ("box", (3, 5, 5)), ("box", (7, 3, 1)), ("box", (17, 3, 9)),
               ("gauss", (3.0, 3.0, 3.0)), ("gauss", (2.0, 3.0, 3.0)), ("gauss", (1.5, 4.0, 2.5)),
               ("gauss", (5.0, 2.0, 6.5)), ("gauss", (7.0, 3.0, 3.0))]


@pytest.mark.parametrize("shape", [(150, 70, 130), (23, 29, 71), (9, 1, 65), (1, 1, 300), (17, 40, 1)])
def test_fused_pass_equals_three_passes(dev, shape):
    """The fused separable pass (half-widths up to 8) computes the three
    passes' sums term by term: the same values, on cubes of several tiles and
    z chunks with ragged edges (FWHM 7 has half-width 9: three passes both times)."""
    import torch
    import paper_1609_03782_amd as ig
    x = torch.from_numpy(igsynth.random_cube(shape, seed=21)).to(dev)
    for kind, size in FUSED_CASES:
        try:
            ig.smooth_set_path(1)
            a = ig.smooth(x, kind, size)
        finally:
            ig.smooth_set_path(0)
        b = ig.smooth(x, kind, size)
        torch.cuda.synchronize()
        assert torch.equal(a, b), (shape, kind, size, float((a - b).abs().max()))


def test_fused_pass_matches_oracle_across_chunks(dev):
    """A cube of 3 x 2 tiles in x, y and 9 z chunks of 8 planes against the
    FP64 oracle."""
    import torch
    import paper_1609_03782_amd as ig
    cube = igsynth.random_cube((70, 45, 130), seed=8)
    x = torch.from_numpy(cube).to(dev)
    for kind, size in [("box", (3, 5, 5)), ("gauss", (2.0, 3.0, 3.0)), ("gauss", (5.0, 2.0, 6.5))]:
        y = ig.smooth(x, kind, size).cpu().numpy()
        ref = Sm.smooth(cube, _kernel(kind, size))
        assert np.abs(y - ref).max() <= _tol(cube, kind, (0, 0, 0)), (kind, size)



def test_long_rows_take_the_three_pass_route(dev):
    """Rows up to 5,592,405 voxels run the fused pass, longer ones the three
    passes (a tile's rows must stay below 2^30 bytes); both sides of the limit
    against the oracle's renormalised moving mean along x, and the fused pass
    at the limit against the three passes."""
    import torch
    import paper_1609_03782_amd as ig
    for nx in (5_592_405, 5_592_406):
        cube = igsynth.random_cube((1, 1, nx), seed=nx % 97)
        x = torch.from_numpy(cube).to(dev)
        y = ig.smooth(x, "box", (3, 1, 1)).cpu().numpy()
        ref = Sm.smooth(cube, _kernel("box", (3, 1, 1)))
        assert np.abs(y - ref).max() <= _tol(cube, "box", (0, 0, 0)), nx
        if nx == 5_592_405:
            try:
                ig.smooth_set_path(1)
                a = ig.smooth(x, "gauss", (2.0, 1.0, 1.0))
            finally:
                ig.smooth_set_path(0)
            b = ig.smooth(x, "gauss", (2.0, 1.0, 1.0))
            assert torch.equal(a, b)
