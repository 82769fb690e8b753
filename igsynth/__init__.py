"""Seeded synthetic H I data cubes (inputs only).

This module builds the input cubes that both the FP64 oracle and the GPU
library are run on.  It holds none of the filter's arithmetic: it only draws
noise and paints galaxy-like emission, so either side may import it without
sharing any part of the method.

Layout: a cube is a C-contiguous ``float32`` array of shape ``(nz, ny, nx)``,
x (right ascension) fastest, then y (declination), then z (velocity channel),
the axis order the paper gives for its cubes (Section 2, data description).

Emission model (a stand-in for the paper's data cubes, which are not
available): i.i.d. Gaussian noise of rms 1, exponential disks with a
sinusoidal rotation curve whose line-of-sight velocity follows from the disk
inclination and position angle, and faint 1-px-wide tails that follow
quadratic Bezier curves through (x, y, v).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FWHM_TO_SIGMA = 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)))


@dataclass
class Galaxy:
    xc: float
    yc: float
    v0: float
    h: float            # disk scale length [px]
    amp: float = 10.0   # peak S/N at the centre (noise rms = 1)
    incl_deg: float = 60.0
    pa_deg: float = 0.0
    sigma_v: float = 1.0  # line width [channels]


@dataclass
class Tail:
    p0: tuple
    p1: tuple
    p2: tuple            # quadratic Bezier control points in (x, y, v)
    amp: float = 1.0
    fwhm: float = 1.0    # cross-section FWHM [px]


@dataclass
class CubeSpec:
    nx: int
    ny: int
    nz: int
    galaxies: list = field(default_factory=list)
    tails: list = field(default_factory=list)
    noise_rms: float = 1.0


def _paint_galaxy(model: np.ndarray, g: Galaxy) -> None:
    nz, ny, nx = model.shape
    rmax = 7.0 * g.h
    x_lo, x_hi = max(0, int(g.xc - rmax)), min(nx, int(g.xc + rmax) + 2)
    y_lo, y_hi = max(0, int(g.yc - rmax)), min(ny, int(g.yc + rmax) + 2)
    if x_lo >= x_hi or y_lo >= y_hi:
        return
    xs = np.arange(x_lo, x_hi, dtype=np.float64)
    ys = np.arange(y_lo, y_hi, dtype=np.float64)
    X, Y = np.meshgrid(xs - g.xc, ys - g.yc)  # (ny', nx')
    pa, inc = math.radians(g.pa_deg), math.radians(g.incl_deg)
    xmaj = X * math.cos(pa) + Y * math.sin(pa)
    ymin = -X * math.sin(pa) + Y * math.cos(pa)
    xd, yd = xmaj, ymin / math.cos(inc)
    R = np.hypot(xd, yd)
    cos_th = np.where(R > 0, xd / np.where(R > 0, R, 1.0), 0.0)
    vmax = 0.25 * nz / math.sin(inc)
    vrot = vmax * np.sin(0.5 * math.pi * np.minimum(R / (2.0 * g.h), 1.0))
    vlos = g.v0 + vrot * math.sin(inc) * cos_th
    surf = g.amp * np.exp(-R / g.h)
    keep = surf > 1e-4
    if not keep.any():
        return
    yy, xx = np.nonzero(keep)
    vl, s = vlos[keep], surf[keep]
    xx = xx + x_lo
    yy = yy + y_lo
    half = int(math.ceil(6.0 * g.sigma_v))
    vc = np.rint(vl).astype(np.int64)
    for off in range(-half, half + 1):
        z = vc + off
        ok = (z >= 0) & (z < nz)
        if not ok.any():
            continue
        val = s[ok] * np.exp(-((z[ok] - vl[ok]) ** 2) / (2.0 * g.sigma_v ** 2))
        model[z[ok], yy[ok], xx[ok]] += val


def _paint_tail(model: np.ndarray, t: Tail) -> None:
    nz, ny, nx = model.shape
    p0, p1, p2 = (np.asarray(p, dtype=np.float64) for p in (t.p0, t.p1, t.p2))
    length = np.linalg.norm(p1 - p0) + np.linalg.norm(p2 - p1)
    ns = max(8, int(length * 4.0))
    u = np.linspace(0.0, 1.0, ns)[:, None]
    pts = (1 - u) ** 2 * p0 + 2 * (1 - u) * u * p1 + u ** 2 * p2  # (ns, 3) as (x, y, v)
    sig = t.fwhm * FWHM_TO_SIGMA
    rad = 2
    offs = np.arange(-rad, rad + 1)
    OX, OY, OZ = np.meshgrid(offs, offs, offs, indexing="ij")
    OX, OY, OZ = OX.ravel(), OY.ravel(), OZ.ravel()
    base = np.rint(pts).astype(np.int64)
    xs = base[:, 0:1] + OX[None, :]
    ys = base[:, 1:2] + OY[None, :]
    zs = base[:, 2:3] + OZ[None, :]
    d2 = (xs - pts[:, 0:1]) ** 2 + (ys - pts[:, 1:2]) ** 2 + (zs - pts[:, 2:3]) ** 2
    val = t.amp * np.exp(-d2 / (2.0 * sig * sig))
    ok = (xs >= 0) & (xs < nx) & (ys >= 0) & (ys < ny) & (zs >= 0) & (zs < nz)
    flat = (zs[ok] * ny + ys[ok]) * nx + xs[ok]
    tube = np.zeros(model.size, dtype=np.float64)
    np.maximum.at(tube, flat, val[ok])
    model += tube.reshape(model.shape)


def render(spec: CubeSpec, rng: np.random.Generator, with_model: bool = False):
    """Noise + emission, FP64 internally, returned as float32 (nz, ny, nx)."""
    model = np.zeros((spec.nz, spec.ny, spec.nx), dtype=np.float64)
    for g in spec.galaxies:
        _paint_galaxy(model, g)
    for t in spec.tails:
        _paint_tail(model, t)
    cube = rng.standard_normal(model.shape, dtype=np.float64) * spec.noise_rms
    cube += model
    out = cube.astype(np.float32)
    if with_model:
        return out, model.astype(np.float32)
    return out


def _rand_galaxy(rng, nx, ny, nz, h, amp=10.0, centre=None):
    if centre is None:
        xc, yc = rng.uniform(0.1 * nx, 0.9 * nx), rng.uniform(0.1 * ny, 0.9 * ny)
        v0 = rng.uniform(0.3 * nz, 0.7 * nz)
    else:
        xc, yc, v0 = centre
    return Galaxy(xc=xc, yc=yc, v0=v0, h=h, amp=amp,
                  incl_deg=rng.uniform(30.0, 75.0), pa_deg=rng.uniform(0.0, 360.0))


def _attached_tail(rng, g: Galaxy, nx, ny, nz, amp):
    ang = rng.uniform(0, 2 * math.pi)
    r0 = 3.0 * g.h
    p0 = (g.xc + r0 * math.cos(ang), g.yc + r0 * math.sin(ang), g.v0 + rng.uniform(-3, 3))
    L = rng.uniform(4.0, 8.0) * g.h
    bend = rng.uniform(-0.6, 0.6)
    p1 = (p0[0] + 0.5 * L * math.cos(ang + bend), p0[1] + 0.5 * L * math.sin(ang + bend),
          p0[2] + rng.uniform(-0.1, 0.1) * nz)
    p2 = (p0[0] + L * math.cos(ang + 2 * bend), p0[1] + L * math.sin(ang + 2 * bend),
          p0[2] + rng.uniform(-0.15, 0.15) * nz)
    return Tail(p0, p1, p2, amp=amp)


def _bridge(rng, a: Galaxy, b: Galaxy, amp):
    dx, dy = b.xc - a.xc, b.yc - a.yc
    d = math.hypot(dx, dy) or 1.0
    p0 = (a.xc + 3 * a.h * dx / d, a.yc + 3 * a.h * dy / d, a.v0)
    p2 = (b.xc - 3 * b.h * dx / d, b.yc - 3 * b.h * dy / d, b.v0)
    mid = ((p0[0] + p2[0]) / 2 - 0.2 * dy, (p0[1] + p2[1]) / 2 + 0.2 * dx, (p0[2] + p2[2]) / 2)
    return Tail(p0, mid, p2, amp=amp)


# ---------------------------------------------------------------- workloads
def spec_single(rng, nx, ny, nz, h, tail_amp=1.0, with_tail=True, centred=True) -> CubeSpec:
    """One galaxy (peak S/N 10) plus optionally one attached tail."""
    centre = (nx / 2.0 + rng.uniform(-1, 1), ny / 2.0 + rng.uniform(-1, 1),
              nz / 2.0 + rng.uniform(-1, 1)) if centred else None
    g = _rand_galaxy(rng, nx, ny, nz, h, centre=centre)
    tails = [_attached_tail(rng, g, nx, ny, nz, tail_amp)] if with_tail else []
    return CubeSpec(nx, ny, nz, [g], tails)


def spec_field(rng, nx, ny, nz, n_gal=16, h_range=(6.0, 40.0), n_attached=4, n_bridge=4,
               tail_amp=(0.5, 1.5)) -> CubeSpec:
    """Many galaxies at random positions plus attached tails and bridges."""
    gals = [_rand_galaxy(rng, nx, ny, nz, rng.uniform(*h_range)) for _ in range(n_gal)]
    tails = []
    for k in range(n_attached):
        tails.append(_attached_tail(rng, gals[k % n_gal], nx, ny, nz, rng.uniform(*tail_amp)))
    for _ in range(n_bridge):
        i, j = rng.choice(n_gal, size=2, replace=False)
        tails.append(_bridge(rng, gals[i], gals[j], rng.uniform(*tail_amp)))
    return CubeSpec(nx, ny, nz, gals, tails)


def cube_small(seed: int = 1, with_model: bool = False):
    """64x64x32 (x, y, v): one galaxy h = 8 px at the centre, one tail at S/N 1."""
    rng = np.random.default_rng(seed)
    spec = spec_single(rng, 64, 64, 32, h=8.0, tail_amp=1.0)
    return render(spec, rng, with_model)


def cube_field(n: int = 512, seed: int = 2, with_model: bool = False, nz: int | None = None):
    """n x n x nz field: 16 galaxies (h in 6..40 px), 4 attached tails, 4 bridges."""
    nz = n if nz is None else nz
    rng = np.random.default_rng(seed)
    spec = spec_field(rng, n, n, nz)
    return render(spec, rng, with_model)


@dataclass
class BatchItem:
    shape: tuple   # (nz, ny, nx)
    K: float
    n_iter: int
    seed: int


def batch_plan(count: int = 96, seed: int = 4, lo=(32, 32, 32), hi=(256, 256, 160)):
    """Uneven batch: nx, ny log-uniform in [32, 256], nz in [32, 160]; K in [1.5, 3];
    20..80 iterations."""
    rng = np.random.default_rng(seed)
    items = []
    for k in range(count):
        nx = int(round(math.exp(rng.uniform(math.log(lo[0]), math.log(hi[0])))))
        ny = int(round(math.exp(rng.uniform(math.log(lo[1]), math.log(hi[1])))))
        nz = int(round(math.exp(rng.uniform(math.log(lo[2]), math.log(hi[2])))))
        K = float(rng.uniform(1.5, 3.0))
        n_iter = int(rng.integers(20, 81))
        items.append(BatchItem((nz, ny, nx), K, n_iter, seed * 100000 + k))
    return items


def batch_cube(item: BatchItem):
    nz, ny, nx = item.shape
    rng = np.random.default_rng(item.seed)
    h = rng.uniform(4.0, max(4.0, min(nx, ny) / 8.0))
    spec = spec_single(rng, nx, ny, nz, h=h, tail_amp=rng.uniform(0.5, 1.5),
                       with_tail=bool(rng.uniform() < 0.5), centred=False)
    return render(spec, rng)


def random_cube(shape, seed, scale=1.0, offset=0.0):
    """Plain Gaussian random cube (nz, ny, nx) for small parity cases."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(shape) * scale + offset).astype(np.float32)


def train_cube(seed: int, n: int = 96):
    """n^3 cube: one galaxy (h in 4 .. n/8 px, peak S/N 10) plus, with probability
    0.5, a tail at S/N 0.5-1.5; noise rms 1.  Used for surrogate training."""
    return batch_cube(BatchItem((n, n, n), 2.0, 50, seed))


def _train_cube_args(a):
    return train_cube(*a)


def train_set(seeds, n: int = 96, workers: int = 8):
    """Stack of train_cube(seed, n) for each seed, generated in worker processes."""
    import multiprocessing as mp
    seeds = list(seeds)
    if workers <= 1 or len(seeds) < 8:
        return np.stack([train_cube(s, n) for s in seeds])
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        cubes = pool.map(_train_cube_args, [(s, n) for s in seeds], chunksize=16)
    return np.stack(cubes)
