"""Pins of the quality-diagnostics oracle (Section 6: F, sigma_F, F_M) against
hand-computed values, closed forms, the definition of first-order error
propagation, region-of-interest consistency and brute-force loops."""
import math

import numpy as np
import pytest

from oracle import quality as Q


def _worked():
    orig = np.array([[[1.0, 5.0, 2.0], [4.0, 0.5, 6.0]]])
    filt = np.array([[[3.0, 4.0, 1.0], [5.0, 2.0, 7.0]]])
    model = np.array([[[0.0, 2.0, 0.0], [1.0, 0.0, 3.0]]])
    return orig, filt, model


def test_worked_example_by_hand():
    orig, filt, model = _worked()
    r = Q.quality(orig, filt, model, thr_f=(3.0,), thr_o=3.0, rms_o=1.0, rms_f=1.0)
    # M_o: original >= 3 -> {5, 4, 6}; M_f: filtered >= 3 -> voxels whose originals are {1, 5, 4, 6}
    assert r["S_oo"] == 15.0 and r["N_o"] == 3
    assert r["S_of"] == [16.0] and r["N_f"] == [4]
    assert r["F"][0] == pytest.approx(16.0 / 15.0, rel=1e-15)
    # sigma_F^2 = 4/15^2 + 16^2 * 3 / 15^4 = (900 + 768) / 50625
    assert r["sigma_F"][0] == pytest.approx(math.sqrt(1668.0) / 225.0, rel=1e-14)
    # model under M_f: 0 + 2 + 1 + 3 = 6 = all of the model
    assert r["S_m"] == 6.0 and r["S_mf"] == [6.0]
    assert r["F_M"] == [1.0]
    assert r["sigma_FM"][0] == pytest.approx(2.0 / 6.0, rel=1e-15)


def test_identity_gives_one_and_closed_form_sigma():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((6, 7, 8)) * 2 + 0.5
    rms = Q.plain_rms(a)
    r = Q.quality(a, a, thr_f=(3.0,), thr_o=3.0)
    assert r["F"] == [1.0]
    S, N = r["S_oo"], r["N_o"]
    assert N > 0
    # sigma_F^2 = N rms^2 / S^2 + S^2 N rms^2 / S^4 = 2 N rms^2 / S^2
    assert r["sigma_F"][0] == pytest.approx(math.sqrt(2 * N) * rms / abs(S), rel=1e-13)


def test_sigma_is_first_order_error_propagation():
    """sigma_F^2 = (dF/dS_of)^2 sigma_of^2 + (dF/dS_oo)^2 sigma_oo^2, with the
    partial derivatives taken numerically from F = |S_of| / |S_oo|."""
    rng = np.random.default_rng(5)
    orig = rng.standard_normal((10, 12, 14)) + np.linspace(0, 6, 14)[None, None, :]
    filt = orig + 0.3 * rng.standard_normal(orig.shape)
    r = Q.quality(orig, filt, thr_f=(2.0, 3.0), thr_o=3.0, rms_o=1.1, rms_f=0.9)
    for k in range(2):
        a, b = r["S_of"][k], r["S_oo"]
        h = 1e-4 * abs(b)
        F = lambda u, v: abs(u) / abs(v)
        ga = (F(a + h, b) - F(a - h, b)) / (2 * h)
        gb = (F(a, b + h) - F(a, b - h)) / (2 * h)
        sa = math.sqrt(r["N_f"][k]) * 0.9
        sb = math.sqrt(r["N_o"]) * 1.1
        assert r["sigma_F"][k] == pytest.approx(math.sqrt(ga ** 2 * sa ** 2 + gb ** 2 * sb ** 2), rel=1e-6)


def test_roi_equals_cropped_cube():
    rng = np.random.default_rng(8)
    orig = rng.standard_normal((9, 11, 13)) * 3
    filt = orig * 0.7 + 1.0
    model = np.abs(orig)
    roi = (2, 9, 1, 10, 3, 7)          # x0, x1, y0, y1, z0, z1
    crop = lambda a: a[3:7, 1:10, 2:9]
    r1 = Q.quality(orig, filt, model, roi=roi, thr_f=(0.5, 1.5, 3.0), rms_o=2.0, rms_f=1.5)
    r2 = Q.quality(crop(orig), crop(filt), crop(model), thr_f=(0.5, 1.5, 3.0), rms_o=2.0, rms_f=1.5)
    for key in ["S_oo", "N_o", "S_m", "S_of", "N_f", "S_mf", "F", "F_M"]:
        assert r1[key] == r2[key], key


def test_brute_force_loops_with_ties():
    """Integer-valued cubes put voxels exactly on thresholds (>= includes them)."""
    rng = np.random.default_rng(11)
    orig = rng.integers(-4, 9, size=(5, 6, 7)).astype(np.float64)
    filt = rng.integers(-3, 10, size=(5, 6, 7)).astype(np.float64)
    model = rng.integers(0, 4, size=(5, 6, 7)).astype(np.float64)
    roi = (1, 6, 0, 5, 1, 4)
    thr = (0.0, 1.0, 2.5, 3.0, 4.5)
    r = Q.quality(orig, filt, model, roi=roi, thr_f=thr, thr_o=3.0, rms_o=1.0, rms_f=2.0)
    b = Q.quality_loops(orig, filt, model, roi, thr, 3.0, 1.0, 2.0)
    for key in ["S_oo", "N_o", "S_m", "S_of", "N_f", "S_mf"]:
        assert r[key] == b[key], key


def test_threshold_sweep_limits_and_monotonicity():
    rng = np.random.default_rng(2)
    orig = rng.standard_normal((8, 8, 8))
    filt = orig + 0.2
    thr = tuple(np.linspace(-50, 4.5, 30))
    r = Q.quality(orig, filt, thr_f=thr)
    assert all(a >= b for a, b in zip(r["N_f"], r["N_f"][1:]))
    assert r["N_f"][0] == orig.size                      # every voxel passes a very low threshold
    assert r["S_of"][0] == pytest.approx(orig.sum(), abs=1e-12)


def test_default_noise_level_is_plain_rms():
    rng = np.random.default_rng(4)
    a = rng.standard_normal((4, 5, 6)) * 1.7
    r = Q.quality(a, a * 2)
    assert r["rms_o"] == pytest.approx(math.sqrt(np.mean(a ** 2)), rel=1e-14)
    assert r["rms_f"] == pytest.approx(2 * math.sqrt(np.mean(a ** 2)), rel=1e-14)
    # scaling a cube scales its rms: the masks, hence N and F, are unchanged
    r2 = Q.quality(a, a * 5)
    assert r2["N_f"] == r["N_f"] and r2["F"] == r["F"]
