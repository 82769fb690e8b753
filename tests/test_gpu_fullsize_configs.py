"""Parity at the benchmark sizes, in the launch configurations bench.py times,
on sampled outputs the oracle computes one by one:

  * 16-bit storage of the 512^3 cube, 50 steps (the rounding oracle on each
    sample's 50-neighbourhood);
  * the 96-cube batch after its autotuner (each sampled cube's oracle run on
    the sample's neighbourhood, with the batch's own noise level);
  * surrogate inference on the 512^3 cube with library-chosen tiles (each
    sample's receptive field as single-layer GPU calls, every layer against
    the oracle's per-layer reference, and the network equal to that chain).
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
    """The 512^3 cube, 50 steps, 16-bit storage (the bench's schedule).  The
    50-step run equals the chain of single steps bit for bit; at each step,
    sampled voxels (random, faces and corners, and the 200 brightest, where
    backward diffusion amplifies differences) of the GPU's next state equal
    the storage rounding of the exact FP64 step from the GPU's own state,
    except where a rounding boundary lies within the oracle's binary32 error
    bound of that step (reading R15)."""
    import torch
    import paper_1609_03782_amd as ig
    dt = {"bf16": torch.bfloat16, "f16": torch.float16}[name]
    cube = igsynth.cube_field(512, seed=2)
    xq = torch.from_numpy(cube).to(dev).to(dt)
    n = 50
    y, st = ig.Filter(cube.shape, K=2.0, tau=1 / 16, n_iter=n, dtype=name).run(xq, stats=True)
    rho = st.rms_used
    one = ig.Filter(cube.shape, K=2.0, tau=1 / 16, n_iter=1, rms=rho, dtype=name)
    bright = np.argsort(cube.ravel())[-200:]
    pts = _points(cube.shape, np.random.default_rng(7), k=300) + [tuple(int(c) for c in np.unravel_index(b, cube.shape))
                                                                   for b in bright]
    s, amb, diff = xq, 0, 0
    for k in range(n):
        s1 = one.run(s)
        prev = s.float().cpu().numpy()
        got = s1.float().cpu().numpy()
        ex, bd = oracle_lib.step_points(prev, pts, "pm_exp", K=2.0, tau=1 / 16, rms=rho)
        ref, tol = oracle_lib.round_storage(ex, name, bd)
        g = np.array([got[p] for p in pts], dtype=np.float64)
        d = np.abs(g - ref)
        assert (d <= tol).all(), (k, int((d > tol).sum()))
        amb, diff = amb + int((tol > 0).sum()), diff + int((d > 0).sum())
        s = s1
    assert torch.equal(s, y)
    print(f"{name} 512^3 n=50: {len(pts)} samples per step; {diff} sample-steps differ from the rounded FP64 "
          f"step, {amb} may")


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
    try:
        ig.batch_autotune(items)
        res = ig.batch(items, want_stats=True)
        torch.cuda.synchronize()
        print(f"batch autotuner: {'persistent launch' if ig.batch_get_launch() else 'launch per round'}")
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
    finally:
        ig.batch_set_launch(False)
        ig.batch_set_schedule(0, 16, 32)
        ig.batch_cache_clear()


def test_surrogate_inference_fullsize_sampled(dev):
    """The 8-layer network on the 512^3 cube (library-chosen slabs).  At each
    sample, the receptive field (radius 8) is run as single-layer GPU calls,
    every layer checked against the oracle's per-layer reference on the GPU's
    own input to it (FP32 sums within gamma(64) of their terms' magnitudes,
    bf16 outputs equal to the FP64 rounding except where a rounding boundary
    lies within that error); the network's output at the sample must equal
    that chain's bit for bit."""
    import torch
    from paper_1609_03782_amd import surrogate as sg
    depth = 8
    rng = np.random.default_rng(21)
    Ws, bs = S.init_params(rng, widths=(1,) + (32,) * (depth - 1) + (1,))
    Ws[-1] = rng.standard_normal(Ws[-1].shape) * 0.05
    bs = [(rng.standard_normal(b.shape) * 0.05).astype(np.float32).astype(np.float64) for b in bs]
    Ws = [S.round_bf16(W) for W in Ws]
    net = sg.Surrogate(depth=depth, seed=1)
    net.set_weights(sg.join_params([W.astype(np.float32) for W in Ws], [b.astype(np.float32) for b in bs]))
    dW = [torch.from_numpy(W.astype(np.float32)).to(dev) for W in Ws]
    db = [torch.from_numpy(b.astype(np.float32)).to(dev) for b in bs]
    cube = igsynth.cube_field(512, seed=2)
    y = net.infer(torch.from_numpy(cube).to(dev)).cpu().numpy()
    pts = _points(cube.shape, np.random.default_rng(5), k=6) + [(511, 300, 7)]
    amb = diff = total = 0
    for (z, yy, x) in pts:
        z0, y0, x0 = max(0, z - depth), max(0, yy - depth), max(0, x - depth)
        sub = np.ascontiguousarray(cube[z0:z + depth + 1, y0:yy + depth + 1, x0:x + depth + 1])
        tx = torch.from_numpy(sub).to(dev)
        a = tx[..., None].to(torch.bfloat16)
        for l in range(depth - 1):
            out = sg.conv3d_forward(a, a.shape[-1], dW[l], db[l], 32, epilogue=1)
            torch.cuda.synchronize()
            act, act_tol, _, _ = S.conv_gelu_ref(a.double().cpu().numpy(), Ws[l], bs[l])
            m, d = _within(out.double().cpu().numpy(), act, act_tol, f"sample {(z, yy, x)} layer {l}")
            amb, diff, total = amb + m, diff + d, total + act.size
            a = out
        yc = sg.conv3d_forward(a, 32, dW[-1], db[-1], 1, epilogue=3, aux=tx)
        torch.cuda.synchronize()
        ref, tol = S.residual_ref(a.double().cpu().numpy(), Ws[-1], bs[-1], sub)
        yc = yc.cpu().numpy()
        _within(yc, ref, tol, f"sample {(z, yy, x)} output layer")
        assert yc[z - z0, yy - y0, x - x0] == y[z, yy, x], (z, yy, x)
    print(f"surrogate 512^3: {len(pts)} samples; hidden activations {diff} differ from the FP64 rounding, "
          f"{amb} may, of {total}")


def _within(got, ref, tol, what):
    d = np.abs(np.asarray(got, np.float64) - ref)
    bad = d > tol
    assert not bad.any(), f"{what}: {int(bad.sum())} of {bad.size} outside the bound (largest excess {(d - tol).max():.3e})"
    return int((tol > 0).sum()), int((d > 0).sum())
