"""FP64 NumPy oracle of the learned surrogate (a small 3-D CNN).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain definitions,
written for checking the GPU kernels, not for speed.

Network (not in the paper; it learns the paper's filter F_n):
    a_0 = x                           (1 channel)
    z_l = conv(a_{l-1}, W_l) + b_l    (3x3x3, zero outside the cube)
    a_l = gelu(z_l)                   l = 1..L-1
    y   = x + z_L                     (residual to the input; z_L has 1 channel)
with gelu(z) = z/2 (1 + erf(z / sqrt 2)).

Layouts: activations are channels-last arrays (Z, Y, X, C); a weight is
(27, C_in, C_out) with tap index t = (dz+1)*9 + (dy+1)*3 + (dx+1), i.e. the
output at v reads the input at v + (dz, dy, dx).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def conv3d(a, W, b=None):
    """z[v, o] = sum_t sum_c a[v + tap_t, c] W[t, c, o] (+ b[o]); a is zero outside the cube."""
    Z, Y, X, C = a.shape
    assert W.shape[0] == 27 and W.shape[1] == C
    P = np.pad(a, ((1, 1), (1, 1), (1, 1), (0, 0)))
    z = np.zeros((Z, Y, X, W.shape[2]))
    for t, (dz, dy, dx) in enumerate(TAPS):
        sh = P[1 + dz:1 + dz + Z, 1 + dy:1 + dy + Y, 1 + dx:1 + dx + X, :]
        z += sh @ W[t]
    if b is not None:
        z += b
    return z


def conv3d_input_grad(dz, W):
    """Gradient of conv3d w.r.t. its input: da[u, c] = sum_t dz[u - tap_t, o] W[t, c, o]."""
    Z, Y, X, O = dz.shape
    P = np.pad(dz, ((1, 1), (1, 1), (1, 1), (0, 0)))
    da = np.zeros((Z, Y, X, W.shape[1]))
    for t, (tz, ty, tx) in enumerate(TAPS):
        sh = P[1 - tz:1 - tz + Z, 1 - ty:1 - ty + Y, 1 - tx:1 - tx + X, :]
        da += sh @ W[t].T
    return da


def conv3d_weight_grad(a, dz):
    """dW[t, c, o] = sum_v a[v + tap_t, c] dz[v, o]; db[o] = sum_v dz[v, o]."""
    Z, Y, X, C = a.shape
    P = np.pad(a, ((1, 1), (1, 1), (1, 1), (0, 0)))
    dW = np.zeros((27, C, dz.shape[3]))
    for t, (tz, ty, tx) in enumerate(TAPS):
        sh = P[1 + tz:1 + tz + Z, 1 + ty:1 + ty + Y, 1 + tx:1 + tx + X, :]
        dW[t] = sh.reshape(-1, C).T @ dz.reshape(-1, dz.shape[3])
    return dW, dz.reshape(-1, dz.shape[3]).sum(axis=0)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(x, Ws, bs):
    """x: (Z, Y, X) cube.  Returns (y, cache) with cache = (activations, pre-activations)."""
    a = x[..., None].astype(np.float64)
    acts, pres = [a], []
    L = len(Ws)
    for l in range(L):
        z = conv3d(a, Ws[l], bs[l])
        pres.append(z)
        if l < L - 1:
            a = gelu(z)
            acts.append(a)
    y = x.astype(np.float64) + pres[-1][..., 0]
    return y, (acts, pres)


def loss_and_grads(x, t, Ws, bs):
    """Mean squared error of the network on one cube and its gradients."""
    y, (acts, pres) = forward(x, Ws, bs)
    n = y.size
    r = y - t
    loss = float((r * r).sum() / n)
    dz = (2.0 / n) * r[..., None]
    gW, gb = [None] * len(Ws), [None] * len(Ws)
    for l in range(len(Ws) - 1, -1, -1):
        gW[l], gb[l] = conv3d_weight_grad(acts[l], dz)
        if l > 0:
            da = conv3d_input_grad(dz, Ws[l])
            dz = da * gelu_grad(pres[l - 1])
    return loss, gW, gb, y


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), returning new (p, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(rng, widths=(1, 32, 32, 32, 32, 32, 32, 32, 1)):
    """He-style initialisation; the last layer starts at zero (identity network)."""
    Ws, bs = [], []
    for l in range(len(widths) - 1):
        cin, cout = widths[l], widths[l + 1]
        std = math.sqrt(2.0 / (27 * cin))
        W = rng.standard_normal((27, cin, cout)) * std
        if l == len(widths) - 2:
            W *= 0.0
        Ws.append(W)
        bs.append(np.zeros(cout))
    return Ws, bs


# ----------------------------------------------------------------------------
# The network at the GPU path's rounding points, and per-layer references with
# the deviation any implementation that rounds at those points may show.
# Rounding points (the HIP kernels' data types):
#   forward   a_0 = bf16(x); z_l = sum of exact bf16 x bf16 products + b_l,
#             accumulated in FP32; a_l = bf16(gelu(z_l)); the pre-activation
#             is also kept as bf16(z_l); y = x + z_L in FP32.
#   backward  dy = bf16(2 (y - t) / N); weight and bias gradients are FP32
#             sums of exact bf16 x bf16 products; dz_{l-1} =
#             bf16(conv^T(dz_l, W_l) * gelu'(bf16(z_{l-1}))).
# The reference below computes every step in FP64 and rounds to bf16 where
# the GPU stores bf16 (round to nearest, ties to even).

U32 = 2.0 ** -24                # binary32 unit roundoff
GELU_SLOPE_MAX = 1.1290         # max |gelu'(z)| = gelu'(sqrt 2), 1.12897...
CONV_DEPTH = 64                 # additions a conv output term can pass through
GELU_ERR_REL = 1e-6             # |gelu_impl(z) - gelu(z)| <= 1e-6 |z|
GELU_GRAD_ERR = 2e-6            # |gelu'_impl(z) - gelu'(z)| <= 2e-6


def gamma(n):
    """Higham's gamma_n = n u / (1 - n u) for binary32: a sum whose terms
    each pass through at most n roundings is off by at most gamma_n times
    the sum of the terms' magnitudes."""
    return n * U32 / (1.0 - n * U32)


def round_bf16(v):
    """Round float64 values to the nearest bfloat16 (8 significant bits),
    ties to even; returned as float64.  Exact: frexp's mantissa times 2^8 is
    an exact float64, and rint rounds half to even."""
    v = np.asarray(v, dtype=np.float64)
    m, e = np.frexp(v)
    return np.ldexp(np.rint(m * 256.0), e - 8)


def _bf16_spread(v, d):
    """Largest |bf16(w) - bf16(v)| over |w - v| <= d (rounding is monotone,
    so the extremes sit at the ends): zero unless a rounding boundary lies
    within d of v."""
    r = round_bf16(v)
    return np.maximum(round_bf16(v + d) - r, r - round_bf16(v - d))


def forward_bf16(x, Ws, bs):
    """The network at the GPU's rounding points, in FP64 between them.
    Returns (y, acts, pres): acts[l] = a_l (bf16 values), pres[l] = z_{l+1}
    (FP64, before rounding)."""
    a = round_bf16(np.asarray(x, np.float64)[..., None])
    acts, pres = [a], []
    for l in range(len(Ws)):
        z = conv3d(a, Ws[l], bs[l])
        pres.append(z)
        if l < len(Ws) - 1:
            a = round_bf16(gelu(z))
            acts.append(a)
    return np.asarray(x, np.float64) + pres[-1][..., 0], acts, pres


def loss_and_grads_bf16(x, t, Ws, bs):
    """Loss and gradients at the GPU's rounding points (see above); loss =
    mean of (y - t)^2 over the cube."""
    y, acts, pres = forward_bf16(x, Ws, bs)
    n = y.size
    r = y - np.asarray(t, np.float64)
    loss = float((r * r).sum() / n)
    dz = loss_grad_bf16(y, t, n)[..., None]
    gW, gb = [None] * len(Ws), [None] * len(Ws)
    for l in range(len(Ws) - 1, -1, -1):
        gW[l], gb[l] = conv3d_weight_grad(acts[l], dz)
        if l > 0:
            da = conv3d_input_grad(dz, Ws[l])
            dz = round_bf16(da * gelu_grad(round_bf16(pres[l - 1])))
    return loss, gW, gb, y


# Per-layer references.  Each takes the layer's inputs as the implementation
# stored them (bf16 values) and returns the FP64 result with the largest
# deviation an implementation may show: FP32 sums off by at most
# gamma(depth) times the sum of the terms' magnitudes, and a bf16 output
# equal to the reference's rounding except where a rounding boundary lies
# within that error (then at most the distance to the other neighbour).  A
# worst-case bound carried through several layers is useless for bf16
# networks (once a neighbour differs by one bf16 step, the next layer's
# error radius covers a boundary almost everywhere), so whole networks are
# checked layer by layer on the implementation's own intermediate values.

def conv_ref(a, W, b=None):
    """Raw conv output (FP32 on the GPU): (z, |z_impl - z| bound)."""
    z = conv3d(a, W, b)
    return z, gamma(CONV_DEPTH) * conv3d(np.abs(a), np.abs(W), None if b is None else np.abs(b))


def conv_gelu_ref(a, W, b):
    """A hidden layer: (act, act_tol, pre, pre_tol) for the bf16 activation
    bf16(gelu(z)) and the bf16 pre-activation bf16(z); the tolerances are
    zero wherever no rounding boundary lies within the FP32 error of z
    (and of gelu, within GELU_ERR_REL |z|)."""
    z, ez = conv_ref(a, W, b)
    v = gelu(z)
    act_tol = _bf16_spread(v, GELU_SLOPE_MAX * ez + GELU_ERR_REL * (np.abs(z) + ez))
    return round_bf16(v), act_tol, round_bf16(z), _bf16_spread(z, ez)


def residual_ref(a, W, b, x):
    """Last layer: y = x + z (FP32 sum, then FP32 add): (y, bound)."""
    z, ez = conv_ref(a, W, b)
    x64 = np.asarray(x, np.float64)
    y = x64 + z[..., 0]
    return y, ez[..., 0] + U32 * (np.abs(x64) + np.abs(z[..., 0]) + ez[..., 0])


def input_grad_ref(dz, W, zpre=None):
    """Gradient of a conv's input (FP32), or with zpre (the bf16
    pre-activation of the layer below) the bf16 product with gelu'(zpre):
    (value, tolerance)."""
    da = conv3d_input_grad(dz, W)
    eda = gamma(CONV_DEPTH) * conv3d_input_grad(np.abs(dz), np.abs(W))
    if zpre is None:
        return da, eda
    gp = gelu_grad(zpre)
    w = da * gp
    ew = np.abs(da) * GELU_GRAD_ERR + eda * (np.abs(gp) + GELU_GRAD_ERR)
    return round_bf16(w), _bf16_spread(w, ew + U32 * (np.abs(w) + ew))


def weight_grad_ref(a, dz):
    """Weight and bias gradients (FP32 sums over the N voxels, each term
    through at most N + 4096 roundings): (dW, dW_bound, db, db_bound)."""
    dW, db = conv3d_weight_grad(a, dz)
    sW, sb = conv3d_weight_grad(np.abs(a), np.abs(dz))
    g = gamma(a.shape[0] * a.shape[1] * a.shape[2] + 4096)
    return dW, g * sW, db, g * sb


def loss_grad_bf16(y, t, n_total):
    """dy as the GPU forms it from its FP32 output: bf16(fp32(2 (y - t) / N))
    with the difference and scaling in FP64."""
    r = np.asarray(y, np.float64) - np.asarray(t, np.float64)
    v = (2.0 * (1.0 / n_total)) * r
    return round_bf16(v.astype(np.float32).astype(np.float64))
