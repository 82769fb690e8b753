"""FP64 oracle of the filtering-quality diagnostics (Section 6: the F parameter,
its propagated error sigma_F, and the recovered-signal fraction F_M of the
model-cube study).

TEST INFRASTRUCTURE ONLY: imported by tests/ and nothing else; shares no code
with the GPU library.

Definitions (all sums run over a region of interest, a half-open sub-box
[x0, x1) x [y0, y1) x [z0, z1) of the cube, the whole cube by default):

  M_i(v)  = 1 if I_i(v) >= t * rms_i else 0           (i = o original, f filtered)
  S_oo    = sum I_o M_o,   S_of = sum I_o M_f        (both on the ORIGINAL values)
  F       = |S_of| / |S_oo|
  sigma_S = sqrt(N_i) rms_i for S_o,i, N_i the number of independent voxels in M_i
  sigma_F = sqrt(sigma_Sof^2 / S_oo^2 + S_of^2 sigma_Soo^2 / S_oo^4)
  S_mf    = sum I_m M_f,  S_m = sum I_m               (I_m: the noiseless model cube)
  F_M     = |S_mf| / |S_m|

Readings (where the paper is silent):
  * rms_i is the plain root mean square of the whole cube i (the same reading
    as the filter's noise level), unless given;
  * the threshold comparison is made in FP64: float(I) >= t * rms, the product
    rounded to FP64;
  * N_i = (mask voxel count) / indep, where indep is the number of voxels per
    independent element (1 for the i.i.d. noise of the synthetic cubes; the
    beam area for correlated noise);
  * sigma of F_M (printed in the paper's table without a formula) is taken as
    sigma_Smf / |S_m| with sigma_Smf = sqrt(N_f) rms_f, S_m being noise-free;
  * the threshold sweep varies the M_f threshold only; M_o keeps its own.

Pins: tests/test_oracle_quality.py.
"""
from __future__ import annotations

import math

import numpy as np


def plain_rms(cube) -> float:
    a = np.asarray(cube, dtype=np.float64).ravel()
    return float(math.sqrt(float(np.dot(a, a)) / a.size)) if a.size else 0.0


def _roi(a, roi):
    nz, ny, nx = a.shape
    if roi is None:
        return np.asarray(a, dtype=np.float64)
    x0, x1, y0, y1, z0, z1 = roi
    return np.asarray(a[z0:z1, y0:y1, x0:x1], dtype=np.float64)


def quality(orig, filt, model=None, roi=None, thr_f=(3.0,), thr_o=3.0, rms_o=None, rms_f=None, indep=1.0):
    """Returns a dict with rms_o, rms_f, S_oo, N_o, S_m (None without a model)
    and per-threshold lists S_of, N_f, S_mf, F, sigma_F, F_M, sigma_FM."""
    rms_o = plain_rms(orig) if not rms_o or rms_o <= 0 else float(rms_o)
    rms_f = plain_rms(filt) if not rms_f or rms_f <= 0 else float(rms_f)
    Io, If = _roi(orig, roi), _roi(filt, roi)
    Im = _roi(model, roi) if model is not None else None

    Mo = Io >= float(thr_o) * rms_o
    S_oo = float(Io[Mo].sum())
    N_o = int(Mo.sum())
    S_m = float(Im.sum()) if Im is not None else None
    sig_oo = math.sqrt(N_o / indep) * rms_o

    out = {"rms_o": rms_o, "rms_f": rms_f, "S_oo": S_oo, "N_o": N_o, "S_m": S_m,
           "S_of": [], "N_f": [], "S_mf": [], "F": [], "sigma_F": [], "F_M": [], "sigma_FM": []}
    for t in thr_f:
        Mf = If >= float(t) * rms_f
        S_of = float(Io[Mf].sum())
        N_f = int(Mf.sum())
        sig_of = math.sqrt(N_f / indep) * rms_f
        if S_oo != 0.0:
            F = abs(S_of) / abs(S_oo)
            sF = math.sqrt(sig_of ** 2 / S_oo ** 2 + S_of ** 2 * sig_oo ** 2 / S_oo ** 4)
        else:
            F = sF = math.nan
        out["S_of"].append(S_of)
        out["N_f"].append(N_f)
        out["F"].append(F)
        out["sigma_F"].append(sF)
        if Im is not None:
            S_mf = float(Im[Mf].sum())
            out["S_mf"].append(S_mf)
            out["F_M"].append(abs(S_mf) / abs(S_m) if S_m != 0.0 else math.nan)
            out["sigma_FM"].append(sig_of / abs(S_m) if S_m != 0.0 else math.nan)
    return out


def quality_loops(orig, filt, model, roi, thr_f, thr_o, rms_o, rms_f):
    """The same sums as pure-Python loops over voxels (tiny cubes only): the
    brute-force form the vectorised one is checked against."""
    nz, ny, nx = np.shape(orig)
    x0, x1, y0, y1, z0, z1 = roi if roi is not None else (0, nx, 0, ny, 0, nz)
    S_oo = 0.0
    N_o = 0
    S_m = 0.0
    S_of = [0.0] * len(thr_f)
    N_f = [0] * len(thr_f)
    S_mf = [0.0] * len(thr_f)
    for z in range(z0, z1):
        for y in range(y0, y1):
            for x in range(x0, x1):
                o = float(orig[z][y][x])
                f = float(filt[z][y][x])
                m = float(model[z][y][x]) if model is not None else 0.0
                S_m += m
                if o >= thr_o * rms_o:
                    S_oo += o
                    N_o += 1
                for k, t in enumerate(thr_f):
                    if f >= t * rms_f:
                        S_of[k] += o
                        N_f[k] += 1
                        S_mf[k] += m
    return {"S_oo": S_oo, "N_o": N_o, "S_m": S_m, "S_of": S_of, "N_f": N_f, "S_mf": S_mf}
