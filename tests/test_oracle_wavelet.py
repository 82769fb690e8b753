"""Pins of the wavelet-lifting oracle (Section 3.4): a Haar example by hand,
the published CDF 5/3 analysis filters, vanishing moments, perfect
reconstruction on odd sizes, separability, the level map, and the identity
and annihilating thresholds."""
import numpy as np
import pytest

from oracle import wavelet as Wv

SHAPES = [(8, 8, 8), (5, 7, 9), (1, 6, 11), (3, 1, 2), (16, 12, 10)]


def test_haar_line_by_hand():
    x = np.array([4.0, 6.0, 10.0, 12.0, 7.0])
    # even 4 10 7, odd 6 12: d = 2 2, c = 4+1 10+1 7 (7 has no partner)
    assert np.array_equal(Wv._fwd_line(x, Wv.HAAR, np.float64), [5.0, 11.0, 7.0, 2.0, 2.0])


def test_legall_interior_is_the_cdf53_analysis_filter_pair():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(32)
    y = Wv._fwd_line(x, Wv.LEGALL, np.float64)
    c, d = y[:16], y[16:]
    lo = np.array([-1 / 8, 1 / 4, 3 / 4, 1 / 4, -1 / 8])   # analysis low-pass, centred on x_2i
    hi = np.array([-1 / 2, 1.0, -1 / 2])                    # analysis high-pass, centred on x_2i+1
    for i in range(2, 14):
        assert c[i] == pytest.approx(float(np.dot(lo, x[2 * i - 2:2 * i + 3])), abs=1e-14)
        assert d[i] == pytest.approx(float(np.dot(hi, x[2 * i:2 * i + 3])), abs=1e-14)


def test_vanishing_moments_and_constants():
    ramp = np.arange(20, dtype=np.float64) * 0.75 + 2.0
    d = Wv._fwd_line(ramp, Wv.LEGALL, np.float64)[10:]
    assert np.allclose(d[:-1], 0.0, atol=1e-14)        # linear signals predicted exactly (interior)
    for kind in (Wv.HAAR, Wv.LEGALL):
        for n in (7, 8):
            y = Wv._fwd_line(np.full(n, 3.5), kind, np.float64)
            ne = (n + 1) // 2
            assert np.all(y[:ne] == 3.5) and np.all(y[ne:] == 0.0)


@pytest.mark.parametrize("kind", [Wv.HAAR, Wv.LEGALL])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("levels", [1, 2, 3])
def test_perfect_reconstruction(kind, shape, levels):
    x = np.random.default_rng(sum(shape)).standard_normal(shape)
    c = Wv.forward(x, kind, levels)
    assert np.allclose(Wv.inverse(c, kind, levels), x, rtol=0, atol=1e-13)
    c32 = Wv.forward(x.astype(np.float32), kind, levels, np.float32)
    assert c32.dtype == np.float32
    assert np.allclose(c32, c, rtol=0, atol=2e-5 * np.abs(x).max() * 4)


def test_one_level_is_separable():
    rng = np.random.default_rng(3)
    f, g, h = rng.standard_normal(6), rng.standard_normal(5), rng.standard_normal(7)
    cube = np.einsum("z,y,x->zyx", h, g, f)
    for kind in (Wv.HAAR, Wv.LEGALL):
        want = np.einsum("z,y,x->zyx", Wv._fwd_line(h, kind, np.float64), Wv._fwd_line(g, kind, np.float64),
                         Wv._fwd_line(f, kind, np.float64))
        assert np.allclose(Wv.forward(cube, kind, 1), want, atol=1e-13)


def test_constant_cube_has_no_details():
    c = Wv.forward(np.full((9, 8, 7), 2.25), Wv.LEGALL, 3)
    lv = Wv.level_map(c.shape, 3)
    assert np.all(c[lv == 4] == 2.25) and np.all(c[lv <= 3] == 0.0)


def test_level_map_counts():
    lv = Wv.level_map((16, 16, 16), 3)
    for l, n in [(1, 16), (2, 8), (3, 4)]:
        assert np.sum(lv == l) == n ** 3 - (n // 2) ** 3
    assert np.sum(lv == 4) == 2 ** 3


def test_threshold_extremes():
    x = np.random.default_rng(6).standard_normal((6, 7, 8)) + 1.0
    for kind in (Wv.HAAR, Wv.LEGALL):
        assert np.allclose(Wv.denoise(x, kind, 2, t=(0.0, 0.0)), x, atol=1e-13)
        assert np.all(Wv.denoise(x, kind, 2, t=(1e9, 1e9)) == 0.0)


def test_threshold_uses_level_thresholds():
    coef = np.full((4, 4, 4), 1.0)
    out = Wv.threshold(coef, (0.5, 2.0), 1.0, 2)
    lv = Wv.level_map(coef.shape, 2)
    assert np.all(out[lv == 1] == 1.0)                 # 1 >= 0.5: kept
    assert np.all(out[lv >= 2] == 0.0)                 # level-2 details and approximation: 1 < 2
