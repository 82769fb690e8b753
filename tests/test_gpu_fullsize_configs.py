"""Parity at the benchmark sizes, in the launch configurations bench.py times,
on sampled outputs the oracle computes one by one:

  * 16-bit storage of the 512^3 cube, 50 steps (the rounding oracle on each
    sample's 50-neighbourhood);
  * the 96-cube batch after its autotuner (each sampled cube's oracle run on
    the sample's neighbourhood, with the batch's own noise level);
  * surrogate inference on the 512^3 cube with library-chosen tiles (the FP64
    network on each sample's receptive field, bf16 rounding points as on the
    GPU).
"""
import numpy as np
import pytest

import igsynth
from oracle import surrogate as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1609_03782_amd as ig
    ig.lib()
    return torch.device("cuda:0")


def _points(shape, rng, k=10):
    nz, ny, nx = shape
    pts = [(0, 0, 0), (nz - 1, ny - 1, nx - 1), (0, ny - 1, nx // 2), (nz // 2, 0, nx - 1)]
    pts += [tuple(int(rng.integers(0, e)) for e in shape) for _ in range(k)]
    return pts


@pytest.mark.parametrize("name", ["bf16", "f16"])
def test_16bit_storage_fullsize_sampled(dev, oracle_lib, name):
    import torch
    import paper_1609_03782_amd as ig
    dt = {"bf16": torch.bfloat16, "f16": torch.float16}[name]
    cube = igsynth.cube_field(512, seed=2)
    xq = torch.from_numpy(cube).to(dev).to(dt)
    q = xq.double().cpu().numpy()
    f = ig.Filter(q.shape, K=2.0, tau=1 / 16, n_iter=50, dtype=name)
    y, st = f.run(xq, stats=True)
    g = y.double().cpu().numpy()
    pts = _points(q.shape, np.random.default_rng(7))
    ref = oracle_lib.run_points(q, pts, "pm_exp", K=2.0, tau=1 / 16, n_iter=50, rms=st.rms_used, round_to=name)
    got = np.array([g[p] for p in pts])
    bits = 7 if name == "bf16" else 10
    unit = 2.0 ** (np.floor(np.log2(np.abs(g).max())) - bits)
    d = np.abs(got - ref)
    print(f"{name} 512^3 n=50: {np.mean(d == 0):.2f} of samples bitwise equal, max diff {d.max():.3e} "
          f"(= {d.max() / unit:.2f} storage units at the cube's largest value)")
    assert d.max() <= 2.0 * unit
    assert np.mean(d == 0) >= 0.75


def test_batch_fullsize_sampled(dev, oracle_lib):
    import torch
    import paper_1609_03782_amd as ig
    plan = igsynth.batch_plan(96, seed=4)
    cubes, items = [], []
    for it in plan:
        c = igsynth.batch_cube(it)
        x = torch.from_numpy(c).to(dev)
        cubes.append(c)
        items.append((x, torch.empty_like(x), dict(K=it.K, tau=1 / 16, n_iter=it.n_iter, cond="pm_exp")))
    ig.batch_autotune(items)
    res = ig.batch(items, want_stats=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    for k in range(0, 96, 12):
        it, c = plan[k], cubes[k]
        rho = res["stats"][k].rms_used
        out = items[k][1].cpu().numpy()
        pts = _points(c.shape, rng, k=3)
        ref = oracle_lib.run_points(c, pts, "pm_exp", K=it.K, tau=1 / 16, n_iter=it.n_iter, rms=rho)
        got = np.array([out[p] for p in pts], dtype=np.float64)
        err = np.abs(got - ref).max()
        assert err <= 1e-5 * rho, (k, c.shape, it.n_iter, err / rho)
    ig.batch_cache_clear()


def _bf(a):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16)
    return t.to(torch.float64).numpy()


def test_surrogate_inference_fullsize_sampled(dev):
    import torch
    from paper_1609_03782_amd import surrogate as sg
    depth = 8
    rng = np.random.default_rng(21)
    Ws, bs = S.init_params(rng, widths=(1,) + (32,) * (depth - 1) + (1,))
    Ws[-1] = rng.standard_normal(Ws[-1].shape) * 0.05
    bs = [rng.standard_normal(b.shape) * 0.05 for b in bs]
    Ws = [_bf(W) for W in Ws]
    net = sg.Surrogate(depth=depth, seed=1)
    net.set_weights(sg.join_params([W.astype(np.float32) for W in Ws], [b.astype(np.float32) for b in bs]))
    cube = igsynth.cube_field(512, seed=2)
    y = net.infer(torch.from_numpy(cube).to(dev)).cpu().numpy()
    pts = _points(cube.shape, np.random.default_rng(5), k=6)
    errs, scale = [], 0.0
    for (z, yy, x) in pts:
        z0, z1 = max(0, z - depth), min(512, z + depth + 1)
        y0, y1 = max(0, yy - depth), min(512, yy + depth + 1)
        x0, x1 = max(0, x - depth), min(512, x + depth + 1)
        sub = cube[z0:z1, y0:y1, x0:x1]
        a = _bf(sub[..., None])
        for l in range(depth - 1):
            a = _bf(S.gelu(S.conv3d(a, Ws[l], bs[l])))
        ref = float(sub[z - z0, yy - y0, x - x0]) + float(S.conv3d(a, Ws[-1], bs[-1])[z - z0, yy - y0, x - x0, 0])
        errs.append(abs(float(y[z, yy, x]) - ref))
        scale = max(scale, abs(ref - float(sub[z - z0, yy - y0, x - x0])))
    print(f"surrogate 512^3: max sampled diff {max(errs):.3e}, largest correction {scale:.3e}")
    assert max(errs) <= 2e-2 * scale + 1e-6
