"""FP64 CPU oracle for the intensity-driven gradient filter.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU library
never imports, links or calls it, and it shares no code with the GPU library:
the only module both sides use is the seeded input generator ``igsynth``.

Contents
  * ``run`` / ``rms`` / ``round_bf16`` / ``round_f16``: ctypes front end to
    ``oracle.c`` (plain C, FP64, OpenMP over z-planes), the definition of the
    filter written out (Section 3.3, Eqs. 5-7).
  * ``error_bound``: the exact result with a per-voxel first-order running
    error bound for binary32 computations of the same steps (oracle.c).
  * ``brute``: an independent NumPy pad-and-shift form of the same step, for
    tiny cubes.
  * ``surrogate``: FP64 NumPy forms of the learned surrogate's layers.
  * ``quality``: the filtering-quality diagnostics of Section 6 (F, sigma_F,
    F_M) over a region of interest and a sweep of mask thresholds.
  * ``sweep``: the parameter sweep scored by F, and the paper's tuning grid.
  * ``smooth``: the box and (rotated) Gaussian smoothing filters of Section 3.
  * ``wavelet``: Haar / Le Gall 5/3 lifting and the thresholding denoiser of
    Section 3.4, in FP64 or in FP32 in the GPU's operation order.

Pins (tests/test_oracle_pins.py): constant cube is a fixed point, zero
conductance is the identity, flux conservation of the per-edge forms under
reflecting faces, a weighted conservation identity of the intensity form,
closed-form impulse responses, the linear limit diagonalised by the
orthonormal DCT-II, the maximum principle, symmetries, composition, the
brute-force cross-check, and the storage rounding against IEEE casts.
Quality pins (tests/test_oracle_quality.py): a hand-computed example, the
identity case in closed form, sigma_F against numerical error propagation,
region-of-interest consistency, brute-force loops with threshold ties.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

COND = {"intensity": 0, "pm_exp": 1, "pm_rational": 2}
ROUND = {None: 0, "bf16": 1, "f16": 2, "f32": 3}


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (no fast-math, no FMA)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
                               "-shared", "-fPIC", src, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int
        p = ctypes.c_void_p
        lib.oracle_run.argtypes = [p, p, i64, i64, i64, i32, d, d, i32, d, d, d, d, i32,
                                   ctypes.POINTER(d)]
        lib.oracle_run.restype = i32
        lib.oracle_error_bound.argtypes = [p, p, p, i64, i64, i64, i32, d, d, i32, d, d, d, d, ctypes.POINTER(d)]
        lib.oracle_error_bound.restype = i32
        lib.oracle_rms.argtypes = [p, i64, ctypes.POINTER(d), ctypes.POINTER(i64)]
        lib.oracle_rms.restype = d
        lib.oracle_round_bf16.argtypes = [d]
        lib.oracle_round_bf16.restype = d
        lib.oracle_round_f16.argtypes = [d]
        lib.oracle_round_f16.restype = d
        lib.oracle_round_n.argtypes = [p, p, p, p, i64, i32]
        lib.oracle_round_n.restype = None
        lib.oracle_threads.argtypes = []
        lib.oracle_threads.restype = i32
        lib.oracle_set_threads.argtypes = [i32]
        lib.oracle_set_threads.restype = None
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    pass


def run(cube, cond: str = "pm_exp", K: float = 2.0, tau: float = 1.0 / 16, n_iter: int = 1,
        C=(1.0, 1.0, 1.0), rms: float | None = None, round_to: str | None = None):
    """Filter `cube` (nz, ny, nx) in FP64.  Returns (result FP64 array, rho used)."""
    lib = _load()
    a = np.ascontiguousarray(cube, dtype=np.float64)
    if a.ndim != 3:
        raise ValueError("cube must be 3-D (nz, ny, nx)")
    out = np.empty_like(a)
    nz, ny, nx = a.shape
    used = ctypes.c_double(0.0)
    rc = lib.oracle_run(a.ctypes.data, out.ctypes.data, nx, ny, nz, COND[cond], float(K),
                        float(tau), int(n_iter), float(C[0]), float(C[1]), float(C[2]),
                        float(rms) if rms is not None else 0.0, ROUND[round_to], ctypes.byref(used))
    if rc != 0:
        raise OracleError({-1: "invalid argument", -2: "out of memory",
                           -3: "non-finite input"}.get(rc, str(rc)))
    return out, used.value


def error_bound(cube, cond: str = "pm_exp", K: float = 2.0, tau: float = 1.0 / 16, n_iter: int = 1,
                C=(1.0, 1.0, 1.0), rms: float | None = None):
    """(exact FP64 result, per-voxel first-order bound on the error of any
    binary32 computation of the same steps, rho used); see oracle.c."""
    lib = _load()
    a = np.ascontiguousarray(cube, dtype=np.float64)
    if a.ndim != 3:
        raise ValueError("cube must be 3-D (nz, ny, nx)")
    out = np.empty_like(a)
    bnd = np.empty_like(a)
    nz, ny, nx = a.shape
    used = ctypes.c_double(0.0)
    rc = lib.oracle_error_bound(a.ctypes.data, out.ctypes.data, bnd.ctypes.data, nx, ny, nz, COND[cond], float(K),
                                float(tau), int(n_iter), float(C[0]), float(C[1]), float(C[2]),
                                float(rms) if rms is not None else 0.0, ctypes.byref(used))
    if rc != 0:
        raise OracleError({-1: "invalid argument", -2: "out of memory",
                           -3: "non-finite input"}.get(rc, str(rc)))
    return out, bnd, used.value


def rms(cube):
    """(rho, sum, nonfinite count) with rho = sqrt(sum I^2 / N) in FP64."""
    lib = _load()
    a = np.ascontiguousarray(cube, dtype=np.float64).ravel()
    s = ctypes.c_double(0.0)
    bad = ctypes.c_int64(0)
    r = lib.oracle_rms(a.ctypes.data, a.size, ctypes.byref(s), ctypes.byref(bad))
    return r, s.value, bad.value


def threads() -> int:
    """OpenMP threads the oracle uses."""
    return int(_load().oracle_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's later parallel loops (this Python thread)."""
    _load().oracle_set_threads(int(n))


def round_bf16(x):
    lib = _load()
    return np.vectorize(lib.oracle_round_bf16, otypes=[np.float64])(np.asarray(x, np.float64))


def round_f16(x):
    lib = _load()
    return np.vectorize(lib.oracle_round_f16, otypes=[np.float64])(np.asarray(x, np.float64))


def round_storage(x, name: str, d=None):
    """Round values to the storage type `name` ("bf16", "f16", "f32"),
    nearest with ties to even.  With d (same shape, >= 0) also return the
    largest change of that rounding over [x - d, x + d]: zero wherever no
    rounding boundary lies within d of x.  Returns y or (y, spread)."""
    lib = _load()
    a = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(a)
    if d is None:
        lib.oracle_round_n(a.ctypes.data, None, y.ctypes.data, None, a.size, ROUND[name])
        return y
    dd = np.ascontiguousarray(np.broadcast_to(d, a.shape), dtype=np.float64)
    sp = np.empty_like(a)
    lib.oracle_round_n(a.ctypes.data, dd.ctypes.data, y.ctypes.data, sp.ctypes.data, a.size, ROUND[name])
    return y, sp


def step_points(cube, points, cond="pm_exp", K=2.0, tau=1.0 / 16, C=(1.0, 1.0, 1.0), rms: float = 1.0):
    """One step at selected voxels of a large cube: (exact FP64 values,
    first-order binary32 error bounds), each from the voxel's neighbourhood
    (its sub-box of half-width 1, clipped to the cube, whose real faces keep
    their boundary: after one step a voxel depends only on its six
    neighbours).  `rms` must be the whole cube's value."""
    a = np.asarray(cube)
    nz, ny, nx = a.shape
    vals, bnds = [], []
    for (z, y, x) in points:
        lo = [max(0, c - 1) for c in (z, y, x)]
        hi = [min(e, c + 2) for c, e in zip((z, y, x), (nz, ny, nx))]
        sub = a[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
        ex, bd, _ = error_bound(sub, cond, K, tau, 1, C, rms=rms)
        vals.append(ex[z - lo[0], y - lo[1], x - lo[2]])
        bnds.append(bd[z - lo[0], y - lo[1], x - lo[2]])
    return np.array(vals), np.array(bnds)


def run_points(cube, points, cond="pm_exp", K=2.0, tau=1.0 / 16, n_iter=1, C=(1.0, 1.0, 1.0),
               rms: float = 1.0, round_to=None):
    """Oracle values at selected voxels of a large cube, each from its own sub-box.

    After n steps a voxel depends only on voxels within n steps along each
    axis, so running the same oracle on the sub-box of half-width n around the
    voxel (clipped to the cube, whose real faces keep their boundary) gives
    that voxel's exact value.  `rms` must be given (the whole cube's value).
    `points` is an iterable of (z, y, x).  Returns FP64 values.
    """
    a = np.asarray(cube)
    nz, ny, nx = a.shape
    vals = []
    for (z, y, x) in points:
        lo = [max(0, c - n_iter) for c in (z, y, x)]
        hi = [min(e, c + n_iter + 1) for c, e in zip((z, y, x), (nz, ny, nx))]
        sub = a[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
        res, _ = run(sub, cond, K, tau, n_iter, C, rms=rms, round_to=round_to)
        vals.append(res[z - lo[0], y - lo[1], x - lo[2]])
    return np.array(vals)
