"""Pins of the box / Gaussian smoothing oracle: SciPy's separable filters (the
renormalised face rule is the ratio of two zero-padded filters), brute-force
loops, closed-form impulse responses, rotation identities and invariants."""
import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import smooth as Sm


def _cube(shape=(9, 10, 11), seed=0):
    return np.random.default_rng(seed).standard_normal(shape) * 2 + 1


@pytest.mark.parametrize("size", [(3, 3, 3), (3, 5, 5), (1, 3, 7), (5, 1, 1)])
def test_box_is_scipy_uniform_filter_renormalised(size):
    a = _cube()
    got = Sm.smooth(a, Sm.box_kernel(size))
    sz = (size[2], size[1], size[0])
    num = ndimage.uniform_filter(a, size=sz, mode="constant", cval=0.0)
    den = ndimage.uniform_filter(np.ones_like(a), size=sz, mode="constant", cval=0.0)
    assert np.allclose(got, num / den, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("fwhm", [(3, 3, 3), (2, 3, 3), (1.5, 4.0, 2.5)])
def test_axis_aligned_gauss_is_scipy_gaussian_filter_renormalised(fwhm):
    a = _cube((12, 13, 14), seed=1)
    got = Sm.smooth(a, Sm.gauss_kernel(fwhm))
    sig = tuple(f * Sm.FWHM_TO_SIGMA for f in (fwhm[2], fwhm[1], fwhm[0]))
    num = ndimage.gaussian_filter(a, sigma=sig, mode="constant", cval=0.0, truncate=3.0)
    den = ndimage.gaussian_filter(np.ones_like(a), sigma=sig, mode="constant", cval=0.0, truncate=3.0)
    assert np.allclose(got, num / den, rtol=1e-12, atol=1e-12)


def test_brute_force_loops():
    a = _cube((5, 6, 7), seed=2)
    for k in [Sm.box_kernel((3, 1, 5)), Sm.gauss_kernel((2.0, 3.0, 1.5), (10.0, 20.0, 30.0))]:
        assert np.allclose(Sm.smooth(a, k), Sm.smooth_loops(a, k), rtol=1e-13, atol=1e-13)


def test_box_interior_impulse_and_identity():
    # every voxel the impulse reaches has its whole window inside the cube
    a = np.zeros((15, 15, 15))
    a[7, 7, 7] = 1.0
    out = Sm.smooth(a, Sm.box_kernel((3, 5, 7)))
    want = np.zeros_like(a)
    want[4:11, 5:10, 6:9] = 1.0 / (3 * 5 * 7)
    assert np.allclose(out, want, rtol=0, atol=1e-16)
    b = _cube()
    assert np.array_equal(Sm.smooth(b, Sm.box_kernel((1, 1, 1))), b)


def test_gauss_interior_impulse_closed_form():
    a = np.zeros((21, 21, 21))
    a[10, 10, 10] = 1.0
    fwhm = (2.0, 3.0, 2.5)
    out = Sm.smooth(a, Sm.gauss_kernel(fwhm))
    s = [f / (2 * math.sqrt(2 * math.log(2))) for f in fwhm]
    r = [int(math.floor(3 * v + 0.5)) for v in s]
    num = lambda dx, dy, dz: math.exp(-dx * dx / (2 * s[0] ** 2) - dy * dy / (2 * s[1] ** 2) - dz * dz / (2 * s[2] ** 2))
    tot = sum(num(dx, dy, dz) for dx in range(-r[0], r[0] + 1) for dy in range(-r[1], r[1] + 1)
              for dz in range(-r[2], r[2] + 1))
    for (dz, dy, dx) in [(0, 0, 0), (1, -2, 1), (-r[2], r[1], -r[0])]:
        assert out[10 + dz, 10 + dy, 10 + dx] == pytest.approx(num(dx, dy, dz) / tot, rel=1e-13)
    assert out[10, 10, 10 + r[0] + 1] == 0.0
    assert out.sum() == pytest.approx(1.0, rel=1e-13)


def test_rotation_by_90_degrees_swaps_the_widths():
    a = _cube((11, 12, 13), seed=4)
    k1 = Sm.gauss_kernel((2.0, 4.0, 3.0), theta=(0.0, 0.0, 90.0))
    k2 = Sm.gauss_kernel((4.0, 2.0, 3.0))
    assert k1.shape == k2.shape
    assert np.allclose(Sm.smooth(a, k1), Sm.smooth(a, k2), rtol=1e-12, atol=1e-12)
    k3 = Sm.gauss_kernel((2.0, 3.0, 4.0), theta=(90.0, 0.0, 0.0))   # about x: y and z swap
    k4 = Sm.gauss_kernel((2.0, 4.0, 3.0))
    assert np.allclose(Sm.smooth(a, k3), Sm.smooth(a, k4), rtol=1e-12, atol=1e-12)


def test_isotropic_kernel_ignores_rotation():
    a = _cube((10, 10, 10), seed=5)
    k0 = Sm.gauss_kernel((3.0, 3.0, 3.0))
    k1 = Sm.gauss_kernel((3.0, 3.0, 3.0), theta=(17.0, -40.0, 33.0))
    assert k0.shape == k1.shape
    assert np.allclose(Sm.smooth(a, k0), Sm.smooth(a, k1), rtol=1e-12, atol=1e-12)


def test_rotated_kernel_is_symmetric_and_rotates_the_impulse():
    k = Sm.gauss_kernel((2.0, 5.0, 3.0), theta=(0.0, 0.0, 30.0))
    assert np.allclose(k, k[::-1, ::-1, ::-1], rtol=0, atol=1e-15)   # even function
    kz, ky, kx = k.shape
    # the long axis (y) turned by +30 degrees about z: weight at (x, y) = (-sin 30, cos 30) * 2
    # exceeds the weight at the mirrored (+sin 30, cos 30) * 2 position
    cz, cy, cx = kz // 2, ky // 2, kx // 2
    assert k[cz, cy + 2, cx - 1] > k[cz, cy + 2, cx + 1]


def test_constant_cube_and_linearity():
    c = np.full((6, 7, 8), 3.25)
    for k in [Sm.box_kernel((3, 3, 5)), Sm.gauss_kernel((3, 2, 2), (5, 10, 15))]:
        assert np.allclose(Sm.smooth(c, k), c, rtol=1e-14, atol=0)
        a, b = _cube((6, 7, 8), 7), _cube((6, 7, 8), 8)
        assert np.allclose(Sm.smooth(2 * a - 3 * b, k), 2 * Sm.smooth(a, k) - 3 * Sm.smooth(b, k), atol=1e-12)
