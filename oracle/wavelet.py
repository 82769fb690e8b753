"""Oracle of the wavelet-lifting denoiser of Section 3.4 (Haar and Le Gall
5/3), TEST INFRASTRUCTURE ONLY: imported by tests/ and nothing else.

Lifting of one line x of length n (split, predict, update):
  even_i = x_{2i} (ceil(n/2) of them), odd_i = x_{2i+1} (floor(n/2));
  Haar:       d_i = odd_i - even_i,                   c_i = even_i + d_i / 2;
  Le Gall 5/3: d_i = odd_i - (even_i + even_{i+1}) / 2, c_i = even_i + (d_{i-1} + d_i) / 4.
The line is stored back as [c_0 .. c_{ne-1}, d_0 .. d_{no-1}] (approximation
first).  The inverse undoes the steps in reverse order.

3-D, level by level: the current approximation box (the whole cube at level
1) is lifted along x, then y, then z; level l+1 works on the box of the
first ceil(n/2) entries of each axis.  Denoising: the detail coefficients of
level l are zeroed where |w| < t_l * rms and the final approximation box
where |w| < t_L * rms (the paper thresholds both), then the cube is
reconstructed.

Readings (the paper gives the Haar operators only): Le Gall 5/3 is the
standard linear CDF 5/3 lifting; both wavelets extend a line symmetrically at
its ends (even_{ne} := even_{ne-1} where odd_{ne-1} exists without a right
even neighbour, d_{-1} := d_0, and d_{no} := d_{no-1} for an even without a
detail partner); for Haar a trailing even without partner keeps c = even; an
axis of length 1 is not lifted; hard thresholding on |w|; rms is the plain rms
of the input cube unless given.

``dtype`` selects the arithmetic: float64 (the definition) or float32 with
the operations in the order written above and no fused multiply-adds, which is
how the GPU library computes; the constants 1/2 and 1/4 are exact in both.

Pins: tests/test_oracle_wavelet.py.
"""
from __future__ import annotations

import math

import numpy as np

HAAR, LEGALL = "haar", "legall53"


def _fwd_line(x, kind, dt):
    """Forward lifting along the last axis of x (any leading shape)."""
    n = x.shape[-1]
    if n < 2:
        return x.copy()
    ev = x[..., 0::2].astype(dt, copy=True)
    od = x[..., 1::2].astype(dt, copy=True)
    ne, no = ev.shape[-1], od.shape[-1]
    h, q = dt(0.5), dt(0.25)
    if kind == HAAR:
        d = od - ev[..., :no]
        c = ev.copy()
        c[..., :no] = ev[..., :no] + d * h
    else:
        right = np.concatenate([ev[..., 1:], ev[..., -1:]], axis=-1)[..., :no]   # even_{i+1}, mirrored at the end
        d = od - (ev[..., :no] + right) * h
        dl = np.concatenate([d[..., :1], d], axis=-1)[..., :ne]                 # d_{i-1}, d_{-1} = d_0
        dr = np.concatenate([d, d[..., -1:]], axis=-1)[..., :ne]                # d_i, d_{no} = d_{no-1}
        c = ev + (dl + dr) * q
    return np.concatenate([c, d], axis=-1)


def _inv_line(y, kind, dt):
    n = y.shape[-1]
    if n < 2:
        return y.copy()
    ne = (n + 1) // 2
    no = n // 2
    c = y[..., :ne].astype(dt, copy=True)
    d = y[..., ne:].astype(dt, copy=True)
    h, q = dt(0.5), dt(0.25)
    if kind == HAAR:
        ev = c.copy()
        ev[..., :no] = c[..., :no] - d * h
        od = d + ev[..., :no]
    else:
        dl = np.concatenate([d[..., :1], d], axis=-1)[..., :ne]
        dr = np.concatenate([d, d[..., -1:]], axis=-1)[..., :ne]
        ev = c - (dl + dr) * q
        right = np.concatenate([ev[..., 1:], ev[..., -1:]], axis=-1)[..., :no]
        od = d + (ev[..., :no] + right) * h
    out = np.empty(y.shape, dtype=dt)
    out[..., 0::2] = ev
    out[..., 1::2] = od
    return out


def _sizes(shape, levels):
    """Approximation-box sizes (nz, ny, nx) before each level, and after the last."""
    s = [tuple(shape)]
    for _ in range(levels):
        s.append(tuple((v + 1) // 2 for v in s[-1]))
    return s


def _along(a, axis, fn):
    moved = np.moveaxis(a, axis, -1)
    return np.moveaxis(fn(moved), -1, axis)


def forward(cube, kind=HAAR, levels=3, dtype=np.float64):
    a = np.array(cube, dtype=dtype, copy=True)
    sz = _sizes(a.shape, levels)
    for l in range(levels):
        nz, ny, nx = sz[l]
        box = a[:nz, :ny, :nx]
        for axis in (2, 1, 0):                      # x, then y, then z
            box = _along(box, axis, lambda v: _fwd_line(v, kind, dtype))
        a[:nz, :ny, :nx] = box
    return a


def inverse(coef, kind=HAAR, levels=3, dtype=np.float64):
    a = np.array(coef, dtype=dtype, copy=True)
    sz = _sizes(a.shape, levels)
    for l in reversed(range(levels)):
        nz, ny, nx = sz[l]
        box = a[:nz, :ny, :nx]
        for axis in (0, 1, 2):                      # z, then y, then x
            box = _along(box, axis, lambda v: _inv_line(v, kind, dtype))
        a[:nz, :ny, :nx] = box
    return a


def level_map(shape, levels):
    """Level of every coefficient: l in 1..levels for detail coefficients,
    levels + 1 for the final approximation box."""
    sz = _sizes(shape, levels)
    lv = np.full(shape, levels + 1, dtype=np.int32)
    for l in range(levels, 0, -1):
        nz, ny, nx = sz[l - 1]
        mz, my, mx = sz[l]
        box = lv[:nz, :ny, :nx]
        outside = np.ones((nz, ny, nx), dtype=bool)
        outside[:mz, :my, :mx] = False
        box[outside] = l
    return lv


def threshold(coef, t, rms, levels):
    """Hard thresholding: level-l details below t[l-1] * rms and the final
    approximation below t[levels-1] * rms (absolute values) are zeroed.  The
    comparison is |w| >= t * rms in FP64 with the product rounded to FP64."""
    lv = level_map(coef.shape, levels)
    thr = np.array([float(t[min(l, levels) - 1]) * float(rms) for l in range(1, levels + 2)])
    keep = np.abs(coef.astype(np.float64)) >= thr[lv - 1]
    return np.where(keep, coef, coef.dtype.type(0))


def plain_rms(cube):
    a = np.asarray(cube, dtype=np.float64).ravel()
    return math.sqrt(float(np.dot(a, a)) / a.size) if a.size else 0.0


def denoise(cube, kind=HAAR, levels=3, t=(0.5, 0.8, 1.1), rms=None, dtype=np.float64):
    rho = plain_rms(cube) if rms is None or rms <= 0 else float(rms)
    c = forward(cube, kind, levels, dtype)
    c = threshold(c, t, rho, levels)
    return inverse(c, kind, levels, dtype)
