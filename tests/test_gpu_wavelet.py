"""GPU wavelet lifting (Haar, Le Gall 5/3) and the thresholding denoiser
against the oracle: the FP32 oracle follows the same operation order, so
coefficients, thresholds and reconstructions match bit for bit; the FP64
oracle bounds the rounding."""
import numpy as np
import pytest

import igsynth
from oracle import wavelet as Wv

pytestmark = pytest.mark.gpu
SHAPES = [(8, 8, 8), (5, 7, 9), (1, 6, 11), (3, 1, 2), (1, 1, 1), (33, 47, 130), (2, 3, 700), (70, 20, 3)]
KINDS = [("haar", Wv.HAAR), ("legall53", Wv.LEGALL)]


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1609_03782_amd as ig
    ig.lib()
    return torch.device("cuda:0")


@pytest.mark.parametrize("name,kind", KINDS)
@pytest.mark.parametrize("shape", SHAPES)
def test_transform_bitwise_vs_fp32_oracle(dev, name, kind, shape):
    import torch
    import paper_1609_03782_amd as ig
    x = igsynth.random_cube(shape, seed=sum(shape))
    xt = torch.from_numpy(x).to(dev)
    for levels in (1, 2, 3):
        c = ig.wavelet_forward(xt, name, levels)
        ref = Wv.forward(x, kind, levels, np.float32)
        assert np.array_equal(c.cpu().numpy(), ref), (shape, levels)
        r = ig.wavelet_inverse(c, name, levels)
        assert np.array_equal(r.cpu().numpy(), Wv.inverse(ref, kind, levels, np.float32))
        assert np.abs(r.cpu().numpy() - x).max() <= 1e-5 * np.abs(x).max()
        c64 = Wv.forward(x, kind, levels)
        assert np.abs(c.cpu().numpy() - c64).max() <= 1e-5 * np.abs(x).max() * 2 ** levels


@pytest.mark.parametrize("name,kind,t", [("haar", Wv.HAAR, (0.5, 0.8, 1.1)), ("legall53", Wv.LEGALL, (1.0, 1.4, 1.7))])
def test_denoise_bitwise_vs_fp32_oracle(dev, name, kind, t):
    """The paper's level thresholds (Section 3.4) on a synthetic galaxy cube,
    rms given to both sides (the threshold test then sees identical numbers)."""
    import torch
    import paper_1609_03782_amd as ig
    cube = igsynth.cube_small(seed=1)
    rms = Wv.plain_rms(cube)
    y, used = ig.wavelet_denoise(torch.from_numpy(cube).to(dev), name, 3, t, rms=rms)
    assert used == rms
    ref = Wv.denoise(cube, kind, 3, t, rms=rms, dtype=np.float32)
    assert np.array_equal(y.cpu().numpy(), ref)
    # in place, and with the noise level estimated on the GPU
    xt = torch.from_numpy(cube).to(dev)
    y2, used2 = ig.wavelet_denoise(xt, name, 3, t, out=xt)
    assert used2 == pytest.approx(rms, rel=1e-12)
    assert np.array_equal(y2.cpu().numpy(), Wv.denoise(cube, kind, 3, t, rms=used2, dtype=np.float32))


def test_denoise_larger_cube_bitwise(dev):
    import torch
    import paper_1609_03782_amd as ig
    cube = igsynth.cube_field(256, seed=9, nz=96)
    for name, kind in KINDS:
        y, rms = ig.wavelet_denoise(torch.from_numpy(cube).to(dev), name, 3, (0.7, 1.0, 1.3))
        ref = Wv.denoise(cube, kind, 3, (0.7, 1.0, 1.3), rms=rms, dtype=np.float32)
        assert np.array_equal(y.cpu().numpy(), ref), name


def test_fullsize_round_trip_and_paper_pipeline(dev):
    """512^3: inverse(forward(x)) reproduces x to rounding; the paper's pipeline
    (Gaussian FWHM 5 pre-smoothing, 3 levels, the Haar level thresholds)
    equals forward -> the oracle's threshold rule -> inverse bit for bit, and
    removes most of the (noise-dominated) cube."""
    import torch
    import paper_1609_03782_amd as ig
    cube = igsynth.cube_field(512, seed=2)
    x = torch.from_numpy(cube).to(dev)
    for name, _ in KINDS:
        c = ig.wavelet_forward(x, name, 3)
        r = ig.wavelet_inverse(c, name, 3)
        assert float((r - x).abs().max()) <= 1e-5 * float(x.abs().max())
    s = ig.smooth(x, "gauss", (5.0, 5.0, 5.0))
    rms = Wv.plain_rms(cube)
    t = (0.5, 0.8, 1.1)
    y, _ = ig.wavelet_denoise(s, "haar", 3, t, rms=rms)
    c = ig.wavelet_forward(s, "haar", 3).cpu().numpy()
    ct = torch.from_numpy(Wv.threshold(c, t, rms, 3)).to(dev)
    y_ref = ig.wavelet_inverse(ct, "haar", 3)
    torch.cuda.synchronize()
    assert torch.equal(y, y_ref)
    assert float((y == 0).float().mean()) >= 0.5


@pytest.mark.parametrize("shape", [(13, 9, 21), (1, 37, 50), (1, 1, 77), (6, 1, 5), (2, 2, 2)])
@pytest.mark.parametrize("levels", [1, 2, 3])
def test_denoise_levels_and_thin_cubes_bitwise(dev, shape, levels):
    """Odd sizes and axes of length 1 (the first level-1 inverse pass then runs
    along y or x), 1-3 levels: every threshold decision and reconstruction as
    the FP32 oracle's."""
    import torch
    import paper_1609_03782_amd as ig
    cube = igsynth.random_cube(shape, seed=sum(shape) + levels)
    t = (0.4, 0.9, 1.2)[:levels]
    for name, kind in KINDS:
        rms = Wv.plain_rms(cube)
        y, _ = ig.wavelet_denoise(torch.from_numpy(cube).to(dev), name, levels, t, rms=rms)
        ref = Wv.denoise(cube, kind, levels, t, rms=rms, dtype=np.float32)
        assert np.array_equal(y.cpu().numpy(), ref), (name, shape, levels)
