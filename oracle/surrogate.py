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
