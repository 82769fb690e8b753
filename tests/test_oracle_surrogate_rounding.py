"""Pins of the surrogate oracle's rounding-point model (oracle/surrogate.py):
bf16 rounding against a brute-force nearest-neighbour definition and torch's
conversion, the GELU constants against the functions they bound, the
per-layer tolerances against an independent binary32 implementation of the
layers (which must land inside them, and equal the reference wherever the
tolerance is zero), and a planted mistake that they must catch."""
import numpy as np
import pytest
import torch

from oracle import surrogate as S


def _bf16_brute(v):
    """Nearest bf16 by enumeration of the two neighbours (ties: even last bit)."""
    out = np.empty_like(v)
    for i, x in enumerate(v):
        if x == 0.0:
            out[i] = 0.0
            continue
        e = np.floor(np.log2(abs(x)))
        step = 2.0 ** (e - 7)
        lo = np.floor(x / step) * step
        hi = lo + step
        if abs(x - lo) < abs(hi - x):
            out[i] = lo
        elif abs(x - lo) > abs(hi - x):
            out[i] = hi
        else:
            out[i] = lo if int(round(lo / step)) % 2 == 0 else hi
    return out


def test_round_bf16_definition():
    rng = np.random.default_rng(1)
    v = rng.standard_normal(4000) * np.exp(rng.uniform(-30, 30, 4000))
    ties = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 3.0 * 2.0 ** -9 + 1.0])
    v = np.concatenate([v, ties, [0.0, 1.0, -2.5]])
    np.testing.assert_array_equal(S.round_bf16(v), _bf16_brute(v))
    assert S.round_bf16(1.0 + 2.0 ** -8) == 1.0                     # tie to even
    assert S.round_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6     # tie to even (up)


def test_round_bf16_matches_torch_on_binary32():
    rng = np.random.default_rng(2)
    u = rng.integers(0, 2 ** 32, 200000, dtype=np.uint64).astype(np.uint32).view(np.float32)
    u = u[np.isfinite(u) & (np.abs(u) < 1e37) & (np.abs(u) > 1e-37)]
    ref = torch.from_numpy(u).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(S.round_bf16(u.astype(np.float64)), ref)


def test_gelu_constants():
    z = np.linspace(-12, 12, 2_400_001)
    assert np.abs(S.gelu_grad(z)).max() <= S.GELU_SLOPE_MAX
    assert np.abs(S.gelu_grad(z)).max() > S.GELU_SLOPE_MAX - 1e-4


def _erf_as32(x):
    """Abramowitz & Stegun 7.1.26 in binary32, the form the GPU's 32-channel
    layers evaluate (reciprocal, exp2, four fused multiply-adds)."""
    f = np.float32
    x = np.asarray(x, np.float32)
    ax = np.abs(x)
    t = (f(1) / (f(0.3275911) * ax + f(1))).astype(f)
    ex = np.exp2(-(ax * ax) * f(1.4426950408889634)).astype(f)
    pl = (f(1.061405429) * t + f(-1.453152027)).astype(f)
    for c in (1.421413741, -0.284496736, 0.254829592):
        pl = (pl * t + f(c)).astype(f)
    y = (f(1) - (pl * t) * ex).astype(f)
    return np.where(x < 0, -y, y).astype(f)


def _gelu32(z):
    """GELU in binary32 in the form the GPU's forward kernels evaluate:
    gelu(z) = max(z, 0) - |z|/2 erfc(|z|/sqrt2), erfc from the same formula
    (fused multiply-adds rounded once, as the hardware's are)."""
    f = np.float32
    z = np.asarray(z, f)
    az = np.abs(z)
    fma = lambda a, b, c: (np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64)).astype(f)
    t = (f(1) / fma(f(0.3275911) * f(0.70710678118654752), az, f(1))).astype(f)
    ex = np.exp2(((z * f(-0.72134752044448170)).astype(f) * z).astype(f)).astype(f)
    pl = fma(f(1.061405429), t, f(-1.453152027))
    for c in (1.421413741, -0.284496736, 0.254829592):
        pl = fma(pl, t, f(c))
    c = ((pl * t).astype(f) * ex).astype(f)
    return fma((f(-0.5) * az).astype(f), c, np.maximum(z, f(0)))


def _gelu32_erf(z):
    """GELU in binary32 through erf, 0.5 z (1 + erf(z / sqrt2))."""
    f = np.float32
    z = np.asarray(z, f)
    return (f(0.5) * z * (f(1) + _erf_as32(z * f(0.70710678118654752)))).astype(f)


def _gelu_grad32(z):
    f = np.float32
    z = np.asarray(z, f)
    e = np.exp(-f(0.5) * z * z).astype(f)
    return (f(0.5) * (f(1) + _erf_as32(z * f(0.70710678118654752))) + z * (f(0.39894228040143268) * e)).astype(f)


def test_gelu_error_constants_cover_binary32_forms():
    """GELU_ERR_REL and GELU_GRAD_ERR cover the approximated erf evaluated
    in binary32 (and leave room for the hardware's reciprocal and exp2,
    each within a few ulps)."""
    z = np.concatenate([np.linspace(-10, 10, 400001), np.geomspace(1e-6, 10, 20000), -np.geomspace(1e-6, 10, 20000)])
    z = z.astype(np.float32).astype(np.float64)
    for form in (_gelu32, _gelu32_erf):
        e1 = np.abs(form(z).astype(np.float64) - S.gelu(z))
        assert (e1 <= 0.5 * S.GELU_ERR_REL * np.abs(z)).all(), (form.__name__, float((e1 / np.abs(z)).max()))
    e2 = np.abs(_gelu_grad32(z).astype(np.float64) - S.gelu_grad(z))
    assert e2.max() <= 0.5 * S.GELU_GRAD_ERR, float(e2.max())


def _conv32(a, W, b=None, order=1):
    """A binary32 convolution with its own summation order (taps forward
    or backward, products of the bf16 inputs exact)."""
    Z, Y, X, C = a.shape
    P = np.pad(a.astype(np.float32), ((1, 1), (1, 1), (1, 1), (0, 0)))
    z = np.zeros((Z, Y, X, W.shape[2]), np.float32)
    for t in list(range(27))[::order]:
        dz, dy, dx = S.TAPS[t]
        sh = P[1 + dz:1 + dz + Z, 1 + dy:1 + dy + Y, 1 + dx:1 + dx + X, :]
        z = (z + sh @ W[t].astype(np.float32)).astype(np.float32)
    if b is not None:
        z = (z + np.asarray(b, np.float32)).astype(np.float32)
    return z


def _net(depth, seed):
    rng = np.random.default_rng(seed)
    Ws, bs = S.init_params(rng, widths=(1,) + (32,) * (depth - 1) + (1,))
    Ws[-1] = rng.standard_normal(Ws[-1].shape) * 0.05
    Ws = [S.round_bf16(W) for W in Ws]
    bs = [(rng.standard_normal(b.shape) * 0.05).astype(np.float32).astype(np.float64) for b in bs]
    return Ws, bs


@pytest.mark.parametrize("order", [1, -1])
def test_layer_tolerances_hold_for_binary32_layers(order):
    """Every layer of an independent binary32 implementation, fed its own
    previous layer, lands within the per-layer tolerances: bitwise equal
    where the tolerance is zero."""
    Ws, bs = _net(4, seed=3)
    x = (np.random.default_rng(9).standard_normal((9, 11, 20)) * 2).astype(np.float32)
    a = S.round_bf16(x[..., None].astype(np.float64))
    for l in range(3):
        act, act_tol, pre, pre_tol = S.conv_gelu_ref(a, Ws[l], bs[l])
        z32 = _conv32(a, Ws[l], bs[l], order)
        got_pre = S.round_bf16(z32.astype(np.float64))
        got = S.round_bf16(_gelu32(z32).astype(np.float64))
        assert (np.abs(got - act) <= act_tol).all() and (np.abs(got_pre - pre) <= pre_tol).all(), l
        # the check has teeth: most activations must match bit for bit
        assert (act_tol == 0).mean() > 0.5 and (pre_tol == 0).mean() > 0.5, l
        a = got
    y, ytol = S.residual_ref(a, Ws[3], bs[3], x)
    y32 = (x + _conv32(a, Ws[3], bs[3], order)[..., 0]).astype(np.float32)
    assert (np.abs(y32 - y) <= ytol).all()


def test_layer_tolerances_catch_a_planted_mistake():
    """A layer that drops the bias of one channel (or evaluates gelu with
    the wrong scale) falls outside the tolerances."""
    Ws, bs = _net(2, seed=4)
    x = (np.random.default_rng(5).standard_normal((6, 7, 12)) * 2).astype(np.float32)
    a = S.round_bf16(x[..., None].astype(np.float64))
    act, act_tol, _, _ = S.conv_gelu_ref(a, Ws[0], bs[0])
    b2 = bs[0].copy()
    b2[5] = 0.0
    bad = S.round_bf16(_gelu32(_conv32(a, Ws[0], b2)).astype(np.float64))
    assert (np.abs(bad - act) > act_tol).any()
    z = _conv32(a, Ws[0], bs[0])
    bad2 = S.round_bf16((0.5 * z * (1 + _erf_as32(z * np.float32(0.7)))).astype(np.float64))
    assert (np.abs(bad2 - act) > act_tol).any()


def test_gradient_tolerances_hold_for_binary32_layers():
    Ws, bs = _net(3, seed=6)
    rng = np.random.default_rng(8)
    a = S.round_bf16(rng.standard_normal((6, 8, 15, 32)))
    dz = S.round_bf16(rng.standard_normal((6, 8, 15, 32)) * 1e-3)
    zpre = S.round_bf16(rng.standard_normal((6, 8, 15, 32)))
    # weight gradient in binary32, voxels summed in reverse order
    dW, dWb, db, dbb = S.weight_grad_ref(a, dz)
    P = np.pad(a.astype(np.float32), ((1, 1), (1, 1), (1, 1), (0, 0)))
    A32 = np.stack([P[1 + tz:7 + tz, 1 + ty:9 + ty, 1 + tx:16 + tx, :].reshape(-1, 32) for tz, ty, tx in S.TAPS])
    D32 = dz.reshape(-1, 32).astype(np.float32)
    acc = np.zeros((27, 32, 32), np.float32)
    for v in range(D32.shape[0] - 1, -1, -1):
        acc = (acc + A32[:, v, :, None] * D32[v][None, None, :]).astype(np.float32)
    assert (np.abs(acc - dW) <= dWb).all()
    # input gradient with gelu' of the bf16 pre-activation, binary32
    ref, tol = S.input_grad_ref(dz, Ws[1], zpre)
    da32 = np.zeros(dz.shape[:3] + (32,), np.float32)
    Pd = np.pad(dz.astype(np.float32), ((1, 1), (1, 1), (1, 1), (0, 0)))
    for t, (tz, ty, tx) in enumerate(S.TAPS):
        sh = Pd[1 - tz:7 - tz, 1 - ty:9 - ty, 1 - tx:16 - tx, :]
        da32 = (da32 + sh @ Ws[1][t].T.astype(np.float32)).astype(np.float32)
    got = S.round_bf16((da32 * _gelu_grad32(zpre)).astype(np.float64))
    assert (np.abs(got - ref) <= tol).all()


def test_bf16_model_gradient_tracks_the_exact_gradient():
    """Training at bf16 rounding points approximates the FP64 gradient: on a
    small network the two agree in direction (cosine > 0.999 per layer)."""
    Ws, bs = _net(3, seed=7)
    rng = np.random.default_rng(10)
    x = S.round_bf16(rng.standard_normal((6, 8, 17))).astype(np.float32)
    t = (x + 0.5 * rng.standard_normal(x.shape)).astype(np.float32)
    _, gW, gb, _ = S.loss_and_grads(x.astype(np.float64), t.astype(np.float64), Ws, bs)
    _, hW, hb, _ = S.loss_and_grads_bf16(x, t, Ws, bs)
    for l in range(3):
        c = float((gW[l] * hW[l]).sum() / np.linalg.norm(gW[l]) / np.linalg.norm(hW[l]))
        assert c > 0.999, (l, c)
