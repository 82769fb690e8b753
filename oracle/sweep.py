"""Oracle of the parameter sweep (Section 6's tuning: the gradient filter run
over a grid of (K, tau, n, C) and scored by F on the same cube).

TEST INFRASTRUCTURE ONLY: imported by tests/ and nothing else.

For each grid point the FP64 filter (oracle.run) is applied to the cube and
the result scored with oracle.quality.quality; the best point is the one with
the largest F at the first M_f threshold (the lowest index among equal F).
"""
from __future__ import annotations

import itertools
import math

from . import quality as Q
from . import rms as _rms
from . import run


def paper_grid():
    """The intensity-driven filter's grid of the paper's tuning (Section 6):
    K in {0.5, 1, 1.5, 2}, n in {20, 30}, tau in {0.0325, 0.0625},
    C_x, C_y, C_z in {4, 5, 6}: 432 points, in that nesting order (C_z fastest)."""
    pts = []
    for K, n, tau, cx, cy, cz in itertools.product((0.5, 1.0, 1.5, 2.0), (20, 30), (0.0325, 0.0625),
                                                   (4.0, 5.0, 6.0), (4.0, 5.0, 6.0), (4.0, 5.0, 6.0)):
        pts.append({"K": K, "tau": tau, "n_iter": n, "C": (cx, cy, cz)})
    return pts


def sweep(cube, points, cond="intensity", model=None, roi=None, thr_f=(3.0,), thr_o=3.0, rms=None, indep=1.0):
    """Returns (list of quality dicts, best index).  rms: the input's noise
    level used by both the filter and the M_o mask (None: the filter's plain
    rms of the input)."""
    rho = _rms(cube)[0] if rms is None else float(rms)   # the filter's own estimate
    results = []
    for p in points:
        out, _ = run(cube, cond, K=p["K"], tau=p["tau"], n_iter=p["n_iter"], C=p["C"], rms=rho)
        results.append(Q.quality(cube, out, model, roi=roi, thr_f=thr_f, thr_o=thr_o, rms_o=rho, indep=indep))
    best, bestF = 0, -math.inf
    for i, r in enumerate(results):
        F = r["F"][0]
        if F == F and F > bestF:
            best, bestF = i, F
    return results, best
