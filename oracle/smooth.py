"""FP64 oracle of the box and Gaussian smoothing filters of Section 3 (the
paper's comparison set for the gradient filter).

TEST INFRASTRUCTURE ONLY: imported by tests/ and nothing else; shares no code
with the GPU library.

Definitions written out (out[v] = sum_d w(d) I(v + d) over the kernel box):
  * box: the mean over an N_x x N_y x N_z neighbourhood (odd N) centred on v,
    v included;
  * Gaussian: w(d) = exp(-sum_j u_j^2 / (2 sigma_j^2)) with u = R^T d, i.e.
    the Gaussian of the equation in Section 3.2 with its principal axes
    rotated by R = R_z(theta_z) R_y(theta_y) R_x(theta_x) (right-handed
    Euler matrices, angles in degrees), and sigma_j = FWHM_j / (2 sqrt(2 ln 2));
    the amplitude A makes the weights sum to one.

Readings (the paper is silent): the kernel box has half-width
r_i = floor(truncate * s_i + 0.5) with truncate = 3, where s_i is sigma_i for
an axis-aligned kernel and sqrt(sum_j R_ij^2 sigma_j^2) (the extent of the
rotated kernel along axis i) otherwise; at the cube faces the weighted mean
runs over the neighbours inside the cube (the weights are renormalised over
them), which for the box is the plain mean of the existing neighbours.

Pins: tests/test_oracle_smooth.py.
"""
from __future__ import annotations

import math

import numpy as np

FWHM_TO_SIGMA = 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)))


def half_width(s: float, truncate: float = 3.0) -> int:
    return int(math.floor(truncate * s + 0.5))


def rotation(theta_deg):
    """R = R_z R_y R_x for Euler angles (theta_x, theta_y, theta_z) in degrees."""
    tx, ty, tz = (math.radians(float(t)) for t in theta_deg)
    cx, sx, cy, sy, cz, sz = math.cos(tx), math.sin(tx), math.cos(ty), math.sin(ty), math.cos(tz), math.sin(tz)
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]], dtype=np.float64)
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]], dtype=np.float64)
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]], dtype=np.float64)
    return Rz @ Ry @ Rx


def box_kernel(size):
    """Weights (z, y, x) of the N_x x N_y x N_z box (size = (N_x, N_y, N_z), odd)."""
    nx, ny, nz = (int(v) for v in size)
    if min(nx, ny, nz) < 1 or not (nx % 2 and ny % 2 and nz % 2):
        raise ValueError("box sizes must be odd and >= 1")
    return np.ones((nz, ny, nx), dtype=np.float64)


def gauss_kernel(fwhm, theta=(0.0, 0.0, 0.0), truncate=3.0):
    """Weights (z, y, x) of the (rotated) Gaussian with the given FWHM (x, y, z)."""
    sig = np.array([float(f) * FWHM_TO_SIGMA for f in fwhm])
    if np.any(sig <= 0):
        raise ValueError("FWHM must be > 0")
    R = rotation(theta)
    if all(float(t) == 0.0 for t in theta):
        ext = sig
    else:
        ext = np.sqrt((R ** 2) @ (sig ** 2))
    rx, ry, rz = (half_width(e, truncate) for e in ext)
    w = np.empty((2 * rz + 1, 2 * ry + 1, 2 * rx + 1))
    for iz, dz in enumerate(range(-rz, rz + 1)):
        for iy, dy in enumerate(range(-ry, ry + 1)):
            for ix, dx in enumerate(range(-rx, rx + 1)):
                u = R.T @ np.array([dx, dy, dz], dtype=np.float64)
                w[iz, iy, ix] = math.exp(-float(np.sum(u * u / (2.0 * sig * sig))))
    return w


def smooth(cube, kernel):
    """Weighted mean of every voxel's kernel-box neighbourhood inside the cube,
    FP64.  kernel: (2rz+1, 2ry+1, 2rx+1) weights."""
    a = np.asarray(cube, dtype=np.float64)
    kz, ky, kx = kernel.shape
    rz, ry, rx = kz // 2, ky // 2, kx // 2
    nz, ny, nx = a.shape
    pad = np.zeros((nz + 2 * rz, ny + 2 * ry, nx + 2 * rx))
    msk = np.zeros_like(pad)
    pad[rz:rz + nz, ry:ry + ny, rx:rx + nx] = a
    msk[rz:rz + nz, ry:ry + ny, rx:rx + nx] = 1.0
    num = np.zeros_like(a)
    den = np.zeros_like(a)
    for iz in range(kz):
        for iy in range(ky):
            for ix in range(kx):
                w = kernel[iz, iy, ix]
                num += w * pad[iz:iz + nz, iy:iy + ny, ix:ix + nx]
                den += w * msk[iz:iz + nz, iy:iy + ny, ix:ix + nx]
    return num / den


def smooth_loops(cube, kernel):
    """The same weighted mean as plain loops over voxels (tiny cubes only)."""
    a = np.asarray(cube, dtype=np.float64)
    nz, ny, nx = a.shape
    kz, ky, kx = kernel.shape
    rz, ry, rx = kz // 2, ky // 2, kx // 2
    out = np.empty_like(a)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                s = 0.0
                ws = 0.0
                for dz in range(-rz, rz + 1):
                    for dy in range(-ry, ry + 1):
                        for dx in range(-rx, rx + 1):
                            if 0 <= z + dz < nz and 0 <= y + dy < ny and 0 <= x + dx < nx:
                                w = kernel[dz + rz, dy + ry, dx + rx]
                                s += w * a[z + dz, y + dy, x + dx]
                                ws += w
                out[z, y, x] = s / ws
    return out
