"""GPU parameter sweep (ig_filter_sweep) and in-place re-parameterisation
(ig_filter_set_params): each point's score equals the FP64 oracle's scoring of
that point's GPU output (mask counts bit-exact), the scores track the oracle
sweep, the best output is returned bitwise, and set_params equals a fresh
handle bitwise."""
import math

import numpy as np
import pytest

import igsynth
from oracle import quality as Q
from oracle import sweep as S

pytestmark = pytest.mark.gpu
THR = (3.0, 2.0, 1.0, 0.0)


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1609_03782_amd as ig
    ig.lib()
    return torch.device("cuda:0")


def _points():
    pts = [{"K": K, "tau": tau, "n_iter": n, "C": C}
           for K, tau, n, C in [(0.5, 0.0325, 6, (4.0, 5.0, 6.0)), (1.5, 0.0325, 4, (5.0, 5.0, 5.0)),
                                (2.0, 0.0625, 3, (6.0, 4.0, 4.0)), (1.0, 0.0, 5, (5.0, 5.0, 5.0)),
                                (1.0, 0.0325, 7, (4.0, 4.0, 4.0))]]
    return pts


def test_set_params_equals_a_fresh_handle(dev):
    import torch
    import paper_1609_03782_amd as ig
    cube = igsynth.cube_small(seed=1)
    x = torch.from_numpy(cube).to(dev)
    f = ig.Filter(cube.shape, K=2.0, tau=1 / 16, n_iter=10, cond="pm_exp")
    y0 = f.run(x)
    for kw in [dict(K=1.5, tau=0.0325, n_iter=7, C=(5, 4, 6), cond="intensity"),
               dict(K=3.0, tau=0.05, n_iter=3, C=(1, 2, 1), cond="pm_rational", rms=2.5),
               dict(K=2.0, tau=1 / 16, n_iter=10, C=(1, 1, 1), cond="pm_exp", rms=0.0)]:
        f.set_params(**kw)
        g = ig.Filter(cube.shape, **{k: v for k, v in kw.items() if k != "rms"},
                      rms=kw.get("rms") or None)
        assert torch.equal(f.run(x), g.run(x)), kw
        g.close()
    assert torch.equal(f.run(x), y0)
    bad = ig.make_params((32, 64, 65))
    assert ig.lib().ig_filter_set_params(f._h, __import__("ctypes").byref(bad)) == ig.IG_ERR_INVALID_ARG


def test_sweep_scores_each_point_like_the_oracle(dev):
    import torch
    import paper_1609_03782_amd as ig
    cube = igsynth.cube_small(seed=1)
    x = torch.from_numpy(cube).to(dev)
    model = np.clip(cube, 0, None).astype(np.float32)
    xm = torch.from_numpy(model).to(dev)
    roi = (8, 56, 4, 60, 2, 30)
    pts = _points()
    res, best, yb = ig.sweep(x, pts, cond="intensity", model=xm, roi=roi, thr_f=THR, want_best=True)
    torch.cuda.synchronize()
    rho = res[0]["rms_o"]
    assert rho == pytest.approx(Q.plain_rms(cube), rel=1e-12)
    outs = []
    for p, r in zip(pts, res):
        f = ig.Filter(cube.shape, K=p["K"], tau=p["tau"], n_iter=p["n_iter"], C=p["C"], cond="intensity", rms=rho)
        y = f.run(x).cpu().numpy()
        f.close()
        outs.append(y)
        ref = Q.quality(cube, y, model, roi=roi, thr_f=THR, rms_o=rho, rms_f=r["rms_f"])
        assert r["rms_f"] == pytest.approx(Q.plain_rms(y), rel=1e-12)
        assert r["N_o"] == ref["N_o"] and r["N_f"] == ref["N_f"]
        for a, b in zip(r["F"] + r["F_M"], ref["F"] + ref["F_M"]):
            assert (math.isnan(a) and math.isnan(b)) or a == pytest.approx(b, rel=1e-12)
    # the tau = 0 point leaves the cube unchanged: F = 1 at the shared 3-rms threshold
    assert res[3]["F"][0] == 1.0
    Fs = [r["F"][0] for r in res]
    assert best == int(np.argmax(Fs)) and Fs[best] == max(Fs)
    assert np.array_equal(yb.cpu().numpy(), outs[best])
    # against the FP64 oracle sweep (its filter differs from the GPU's by ~1e-5 rms,
    # which can move a voxel across a mask threshold): scores agree closely
    ores, obest = S.sweep(cube, pts, cond="intensity", model=model, roi=roi, thr_f=THR)
    for r, o in zip(res, ores):
        for a, b in zip(r["F"], o["F"]):
            assert a == pytest.approx(b, rel=1e-2)
    assert Fs[obest] >= max(Fs) * (1 - 1e-2)


def test_sweep_paper_grid_on_a_small_cube(dev):
    """All 432 points of the paper's tuning grid (n = 20 and 30) on a 48^3 cube:
    every point scored, the best one returned, scores finite."""
    import torch
    import paper_1609_03782_amd as ig
    cube = igsynth.cube_small(seed=1)[:, 8:56, 8:56].copy()
    x = torch.from_numpy(cube).to(dev)
    pts = S.paper_grid()
    res, best, yb = ig.sweep(x, pts, cond="intensity", thr_f=(3.0,), want_best=True)
    Fs = [r["F"][0] for r in res]
    assert len(Fs) == 432 and all(math.isfinite(v) for v in Fs)
    assert best == int(np.argmax(Fs))
    p = pts[best]
    f = ig.Filter(cube.shape, K=p["K"], tau=p["tau"], n_iter=p["n_iter"], C=p["C"], cond="intensity",
                  rms=res[0]["rms_o"])
    assert torch.equal(f.run(x), yb)


def test_sweep_rejects_a_bad_point_before_any_work(dev):
    import torch
    import paper_1609_03782_amd as ig
    x = torch.zeros((8, 8, 8), device=dev)
    pts = _points() + [{"K": -1.0, "tau": 0.03, "n_iter": 2, "C": (1, 1, 1)}]
    with pytest.raises(ig.IgError):
        ig.sweep(x, pts)
