"""Pins of the parameter-sweep oracle: the paper's tuning grid against the
values it prints, a one-point sweep against a direct run, the identity point,
and the choice of the best point."""
import os

import igsynth
import oracle
from oracle import quality as Q
from oracle import sweep as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_tuning_grid.txt")


def _golden():
    vals = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            k, *v = line.split()
            vals[k] = [float(x) for x in v]
    return vals


def test_paper_grid_matches_the_printed_lists():
    g = _golden()
    pts = S.paper_grid()
    assert len(pts) == 432
    assert len({(p["K"], p["tau"], p["n_iter"], p["C"]) for p in pts}) == 432
    assert sorted({p["K"] for p in pts}) == g["K"]
    assert sorted({p["n_iter"] for p in pts}) == g["n"]
    assert sorted({p["tau"] for p in pts}) == g["tau"]
    for a in range(3):
        assert sorted({p["C"][a] for p in pts}) == g["C"]
    # nesting order: C_z fastest, K slowest
    assert pts[0]["C"] == (4.0, 4.0, 4.0) and pts[1]["C"] == (4.0, 4.0, 5.0)
    assert pts[0]["K"] == 0.5 and pts[-1]["K"] == 2.0 and pts[108]["K"] == 1.0


def test_one_point_sweep_is_run_then_quality():
    cube = igsynth.cube_small(seed=1)[:, :24, :24].copy()
    p = {"K": 1.5, "tau": 0.0325, "n_iter": 4, "C": (5.0, 4.0, 6.0)}
    res, best = S.sweep(cube, [p], thr_f=(3.0, 1.0))
    out, rho = oracle.run(cube, "intensity", K=1.5, tau=0.0325, n_iter=4, C=(5.0, 4.0, 6.0))
    ref = Q.quality(cube, out, thr_f=(3.0, 1.0), rms_o=rho)
    assert best == 0
    assert res[0] == ref


def test_identity_point_scores_one():
    cube = igsynth.cube_small(seed=1)[:, :20, :20].copy()
    res, _ = S.sweep(cube, [{"K": 1.0, "tau": 0.0, "n_iter": 3, "C": (5.0, 5.0, 5.0)}])
    assert res[0]["F"] == [1.0]


def test_best_is_the_largest_F_and_follows_a_permutation():
    cube = igsynth.cube_small(seed=1)[:, :24, :24].copy()
    pts = [{"K": K, "tau": 0.0325, "n_iter": n, "C": (5.0, 5.0, 5.0)} for K in (0.5, 2.0) for n in (2, 6)]
    res, best = S.sweep(cube, pts)
    Fs = [r["F"][0] for r in res]
    assert Fs[best] == max(Fs)
    perm = [2, 0, 3, 1]
    res2, best2 = S.sweep(cube, [pts[i] for i in perm])
    assert perm[best2] == best
