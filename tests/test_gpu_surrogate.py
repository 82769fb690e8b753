"""GPU checks of the surrogate's HIP kernels against the FP64 oracle.

Inputs and weights are rounded to bfloat16 before both sides see them, so a
bf16 x bf16 product is exact in FP32 and the remaining differences are the
ones the oracle's per-layer references bound (oracle/surrogate.py): FP32
sums within gamma(depth) of the sum of their terms' magnitudes, and bf16
outputs equal to the FP64 result's rounding except where a rounding
boundary lies within that error (there, within the distance to the other
neighbour).  Whole networks are checked layer by layer on the GPU's own
intermediate values, and the fused network must equal that chain of
single-layer calls bit for bit.
"""
import zlib

import numpy as np
import pytest

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


def _bf(a):
    """Round to bfloat16 (torch RNE) and return (fp64 numpy, torch bf16 cpu)."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16)
    return t.to(torch.float64).numpy(), t


def _within(got, ref, tol, what):
    """Elementwise |got - ref| <= tol; returns (outputs with a nonzero
    tolerance, outputs that differ) for the record."""
    d = np.abs(np.asarray(got, np.float64) - ref)
    bad = d > tol
    assert not bad.any(), f"{what}: {int(bad.sum())} of {bad.size} outside the bound (largest excess {(d - tol).max():.3e})"
    return int((tol > 0).sum()), int((d > 0).sum())


SHAPES = [(5, 6, 40), (3, 9, 33), (7, 4, 70)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("cin,cout", [(32, 32), (1, 32), (32, 1)])
def test_conv_forward_raw(dev, shape, cin, cout):
    import torch
    from paper_1609_03782_amd import surrogate as sg
    rng = np.random.default_rng(zlib.crc32(repr((shape, cin, cout)).encode()))
    a, ta = _bf(rng.standard_normal(shape + (cin,)))
    W, _ = _bf(rng.standard_normal((27, cin, cout)) * 0.2)
    b = rng.standard_normal(cout).astype(np.float32)
    out = sg.conv3d_forward(ta.to(dev), cin, torch.from_numpy(W.astype(np.float32)).to(dev),
                            torch.from_numpy(b).to(dev), cout, epilogue=0)
    torch.cuda.synchronize()
    got = out.cpu().numpy()[..., :cout].astype(np.float64)
    ref, tol = S.conv_ref(a, W, b.astype(np.float64))
    _within(got, ref, tol, "raw conv")


def test_conv_forward_gelu_and_residual(dev):
    import torch
    from paper_1609_03782_amd import surrogate as sg
    rng = np.random.default_rng(7)
    shape = (4, 8, 37)
    a, ta = _bf(rng.standard_normal(shape + (32,)))
    W, _ = _bf(rng.standard_normal((27, 32, 32)) * 0.1)
    b = rng.standard_normal(32).astype(np.float32) * 0.1
    pre = torch.empty(shape + (32,), dtype=torch.bfloat16, device=dev)
    out = sg.conv3d_forward(ta.to(dev), 32, torch.from_numpy(W.astype(np.float32)).to(dev),
                            torch.from_numpy(b).to(dev), 32, epilogue=1, aux=pre)
    torch.cuda.synchronize()
    act, act_tol, zb, zb_tol = S.conv_gelu_ref(a, W, b.astype(np.float64))
    amb, diff = _within(out.double().cpu().numpy(), act, act_tol, "gelu activation")
    _within(pre.double().cpu().numpy(), zb, zb_tol, "bf16 pre-activation")
    print(f"gelu layer: {diff} of {act.size} activations differ from the FP64 rounding, {amb} may")
    # residual epilogue: y = x + conv(a) + b with one output channel
    W1, _ = _bf(rng.standard_normal((27, 32, 1)) * 0.1)
    x = rng.standard_normal(shape).astype(np.float32)
    y = sg.conv3d_forward(ta.to(dev), 32, torch.from_numpy(W1.astype(np.float32)).to(dev),
                          torch.from_numpy(b[:1].copy()).to(dev), 1, epilogue=3, aux=torch.from_numpy(x).to(dev))
    torch.cuda.synchronize()
    ref, tol = S.residual_ref(a, W1, b[:1].astype(np.float64), x)
    _within(y.cpu().numpy(), ref, tol, "residual")


@pytest.mark.parametrize("cin,cout", [(32, 32), (32, 1)])
def test_conv_input_grad(dev, cin, cout):
    import torch
    from paper_1609_03782_amd import surrogate as sg
    rng = np.random.default_rng(cin + cout)
    shape = (5, 7, 45)
    dz, tdz = _bf(rng.standard_normal(shape + (cout,)))
    W, _ = _bf(rng.standard_normal((27, cin, cout)) * 0.2)
    got = sg.conv3d_input_grad(tdz.to(dev), cout, torch.from_numpy(W.astype(np.float32)).to(dev), cin)
    torch.cuda.synchronize()
    ref, tol = S.input_grad_ref(dz, W)
    _within(got.cpu().numpy()[..., :cin], ref, tol, "input gradient")
    # with the gelu' epilogue of the layer below
    if cin == 32:
        z, tz = _bf(rng.standard_normal(shape + (32,)))
        got2 = sg.conv3d_input_grad(tdz.to(dev), cout, torch.from_numpy(W.astype(np.float32)).to(dev), cin,
                                    aux=tz.to(dev))
        torch.cuda.synchronize()
        ref2, tol2 = S.input_grad_ref(dz, W, z)
        _within(got2.double().cpu().numpy(), ref2, tol2, "input gradient times gelu'")


@pytest.mark.parametrize("cin,cout", [(32, 32), (1, 32), (32, 1)])
def test_conv_weight_grad(dev, cin, cout):
    import torch
    from paper_1609_03782_amd import surrogate as sg
    rng = np.random.default_rng(100 + cin + cout)
    shape = (11, 6, 39)          # 11 planes: two z-chunks of the split-K
    a, ta = _bf(rng.standard_normal(shape + (cin,)))
    dz, tdz = _bf(rng.standard_normal(shape + (cout,)))
    dW, db = sg.conv3d_weight_grad(ta.to(dev), cin, tdz.to(dev), cout)
    torch.cuda.synchronize()
    rW, tW, rb, tb = S.weight_grad_ref(a, dz)
    _within(dW.cpu().numpy(), rW, tW, "weight gradient")
    _within(db.cpu().numpy(), rb, tb, "bias gradient")


def _net(depth=4, seed=3):
    """Weights exact in bf16 and biases exact in FP32, so both sides start
    from the same numbers."""
    rng = np.random.default_rng(seed)
    Ws, bs = S.init_params(rng, widths=(1,) + (32,) * (depth - 1) + (1,))
    Ws[-1] = rng.standard_normal(Ws[-1].shape) * 0.05
    bs = [(rng.standard_normal(b.shape) * 0.05).astype(np.float32).astype(np.float64) for b in bs]
    Ws = [_bf(W)[0] for W in Ws]
    return Ws, bs


def _dev_params(dev, Ws, bs):
    import torch
    return ([torch.from_numpy(W.astype(np.float32)).to(dev) for W in Ws],
            [torch.from_numpy(b.astype(np.float32)).to(dev) for b in bs])


def _chain_forward(dev, x, Ws, bs, check=True):
    """The network as single-layer GPU calls; with check, every layer is
    compared with the oracle's reference evaluated on the GPU's own input to
    that layer.  Returns (y, acts, pres) as device tensors."""
    import torch
    from paper_1609_03782_amd import surrogate as sg
    dW, db = _dev_params(dev, Ws, bs)
    tx = torch.from_numpy(x).to(dev)
    a = tx[..., None].to(torch.bfloat16)            # round to nearest even, as the GPU's input rounding
    acts, pres, amb, diff = [a], [], 0, 0
    for l in range(len(Ws) - 1):
        pre = torch.empty(x.shape + (32,), dtype=torch.bfloat16, device=dev)
        out = sg.conv3d_forward(a, a.shape[-1], dW[l], db[l], 32, epilogue=1, aux=pre)
        torch.cuda.synchronize()
        if check:
            act, act_tol, zb, zb_tol = S.conv_gelu_ref(a.double().cpu().numpy(), Ws[l], bs[l])
            m, d = _within(out.double().cpu().numpy(), act, act_tol, f"layer {l} activation")
            _within(pre.double().cpu().numpy(), zb, zb_tol, f"layer {l} pre-activation")
            amb, diff = amb + m, diff + d
        acts.append(out)
        pres.append(pre)
        a = out
    y = sg.conv3d_forward(a, 32, dW[-1], db[-1], 1, epilogue=3, aux=tx)
    torch.cuda.synchronize()
    if check:
        ref, tol = S.residual_ref(a.double().cpu().numpy(), Ws[-1], bs[-1], x)
        _within(y.cpu().numpy(), ref, tol, "output layer")
        print(f"hidden activations: {diff} differ from the FP64 rounding, {amb} may "
              f"(of {sum(t.numel() for t in acts[1:])})")
    return y, acts, pres


def test_network_forward_and_tiling(dev):
    import torch
    from paper_1609_03782_amd import surrogate as sg
    depth = 4
    Ws, bs = _net(depth)
    net = sg.Surrogate(depth=depth, seed=1)
    net.set_weights(sg.join_params([W.astype(np.float32) for W in Ws], [b.astype(np.float32) for b in bs]))
    rng = np.random.default_rng(9)
    x = (rng.standard_normal((19, 21, 40)) * 2).astype(np.float32)
    tx = torch.from_numpy(x).to(dev)
    y = net.infer(tx)
    yt = net.infer(tx, tile=8)
    torch.cuda.synchronize()
    assert torch.equal(y, yt)                    # halo of `depth` voxels makes tiles exact
    yc, _, _ = _chain_forward(dev, x, Ws, bs)    # each layer within its derived bound ...
    assert torch.equal(y, yc)                    # ... and the fused network is that chain
    # end to end against the oracle run from scratch (for the record: layers
    # that differ by a bf16 step move later layers' inputs)
    ref, _, _ = S.forward_bf16(x, Ws, bs)
    err = np.abs(y.cpu().numpy() - ref)
    print(f"end to end: max |y - oracle| {err.max():.3e}, largest correction {np.abs(ref - x).max():.3e}")


def test_large_cube_auto_tiles(dev):
    """A cube above the library's piece limit is cut into slabs when tile == 0;
    tiling is exact, so the result equals an explicit tiling and the whole-cube
    pass bit for bit.  The limit (2^28 voxels by default) is lowered through
    the test hook so that a small cube takes the tiled path."""
    import torch
    import paper_1609_03782_amd as ig
    from paper_1609_03782_amd import surrogate as sg
    net = sg.Surrogate(depth=8, seed=5)
    # random weights in every layer (the initial last layer is zero, which
    # would make y = x whatever the tiling)
    rng = np.random.default_rng(15)
    Ws, bs = sg.split_params(net.get_weights(), 8)
    Ws = [(rng.standard_normal(W.shape) * np.sqrt(1.0 / (27 * W.shape[1]))).astype(np.float32) for W in Ws]
    bs = [(0.1 * rng.standard_normal(b.shape)).astype(np.float32) for b in bs]
    net.set_weights(sg.join_params(Ws, bs))
    x = torch.randn(40, 256, 512, device=dev)        # 5.2e6 voxels
    yw = net.infer(x)                                # one piece under the default limit
    L = ig.lib()
    L.ig_debug_set_infer_piece_limit(1 << 22)        # 4.2e6 voxels: slabs of 14 planes + halo
    try:
        y0 = net.infer(x)                            # library-picked slabs
        y1 = net.infer(x, tile=200)                  # cubes of 200^3
        torch.cuda.synchronize()
        with pytest.raises(Exception):
            net.infer(x, tile=500)                   # 512 x 256 x 40 voxels with the halo >= the limit
    finally:
        L.ig_debug_set_infer_piece_limit(0)
    assert torch.equal(y0, yw)
    assert torch.equal(y1, yw)
    assert bool(torch.isfinite(yw).all())
    assert float((yw - x).abs().max()) > 1e-2       # the network changes its input
    # a piece of the interior equals the network on that piece with its halo
    sub = x[10:34, 100:160, 300:380].contiguous()
    ys = net.infer(sub)
    torch.cuda.synchronize()
    assert torch.equal(ys[8:-8, 8:-8, 8:-8], yw[18:26, 108:152, 308:372])


def test_training_gradient_matches_oracle(dev):
    """One training step's loss and gradients: the backward pass as
    single-layer GPU calls, each compared with the oracle's reference on the
    GPU's own inputs, and the fused training step equal to that chain bit
    for bit."""
    import torch
    from paper_1609_03782_amd import surrogate as sg
    depth = 3
    Ws, bs = _net(depth, seed=4)
    net = sg.Surrogate(depth=depth, seed=2, lr=1e-12)
    net.set_weights(sg.join_params([W.astype(np.float32) for W in Ws], [b.astype(np.float32) for b in bs]))
    rng = np.random.default_rng(11)
    x = _bf(rng.standard_normal((8, 10, 33)))[0].astype(np.float32)
    t = (x + 0.5 * rng.standard_normal(x.shape)).astype(np.float32)
    loss = net.train_step([torch.from_numpy(x).to(dev)], [torch.from_numpy(t).to(dev)])
    gW, gb = sg.split_params(net.get_grads(), depth)

    y, acts, pres = _chain_forward(dev, x, Ws, bs)
    dWt, _ = _dev_params(dev, Ws, bs)
    yh = y.cpu().numpy()
    n = yh.size
    r = yh.astype(np.float64) - t
    assert loss == pytest.approx(float((r * r).sum() / n), rel=1e-12, abs=0)   # FP64 sums of the same terms
    dz = torch.from_numpy(S.loss_grad_bf16(yh, t, n)[..., None].astype(np.float32)).to(torch.bfloat16).to(dev)
    cW, cb = [None] * depth, [None] * depth
    for l in range(depth - 1, -1, -1):
        a = acts[l]
        w_gpu, b_gpu = sg.conv3d_weight_grad(a, a.shape[-1], dz, dz.shape[-1])
        torch.cuda.synchronize()
        cW[l], cb[l] = w_gpu.cpu().numpy(), b_gpu.cpu().numpy()
        rW, tW, rb, tb = S.weight_grad_ref(a.double().cpu().numpy(), dz.double().cpu().numpy())
        _within(cW[l], rW, tW, f"layer {l} weight gradient")
        _within(cb[l], rb, tb, f"layer {l} bias gradient")
        if l > 0:
            nxt = sg.conv3d_input_grad(dz, dz.shape[-1], dWt[l], 32, aux=pres[l - 1])
            torch.cuda.synchronize()
            ref, tol = S.input_grad_ref(dz.double().cpu().numpy(), Ws[l], pres[l - 1].double().cpu().numpy())
            _within(nxt.double().cpu().numpy(), ref, tol, f"layer {l} input gradient")
            dz = nxt
    for l in range(depth):
        assert np.array_equal(gW[l], cW[l]) and np.array_equal(gb[l], cb[l]), l


def test_training_lowers_the_loss(dev):
    import torch
    import paper_1609_03782_amd as ig
    from paper_1609_03782_amd import surrogate as sg
    import igsynth
    xs, ts = [], []
    for k in range(4):
        c = igsynth.batch_cube(igsynth.BatchItem((24, 24, 24), 2.0, 20, 500 + k))
        x = torch.from_numpy(c).to(dev)
        xs.append(x)
        ts.append(ig.Filter(c.shape, K=2.0, tau=1 / 16, n_iter=20).run(x))
    torch.cuda.synchronize()
    net = sg.Surrogate(depth=4, seed=5, lr=2e-3)
    first = net.train_step(xs, ts)
    for _ in range(40):
        last = net.train_step(xs, ts)
    assert last < 0.5 * first, (first, last)


def test_checkpoint_resume_is_bitwise(dev, tmp_path):
    """Save after 3 steps, load into a fresh handle (other seed), take 2 more
    steps on both: the losses and the weights of the resumed run equal the
    uninterrupted run's bit for bit (weights, Adam m and v, and the step count
    are restored; every kernel sums in a fixed order)."""
    import torch
    import paper_1609_03782_amd as ig
    from paper_1609_03782_amd import surrogate as sg
    import igsynth
    xs, ts = [], []
    for k in range(4):
        c = igsynth.batch_cube(igsynth.BatchItem((20, 22, 24), 2.0, 10, 800 + k))
        x = torch.from_numpy(c).to(dev)
        xs.append(x)
        ts.append(ig.Filter(c.shape, K=2.0, tau=1 / 16, n_iter=10).run(x))
    torch.cuda.synchronize()
    a = sg.Surrogate(depth=3, seed=11, lr=2e-3)
    for k in range(3):
        a.train_step(xs[k % 2 * 2:k % 2 * 2 + 2], ts[k % 2 * 2:k % 2 * 2 + 2])
    path = tmp_path / "s.ckpt"
    a.save(path)
    info = sg.checkpoint_info(path)
    assert info["step"] == 3 and info["seed"] == 11 and info["depth"] == 3 and info["nparam"] == a.param_count
    b = sg.Surrogate(depth=3, seed=12, lr=2e-3)
    assert not np.array_equal(a.get_weights(), b.get_weights())
    b.load(path)
    assert b.step == 3 and np.array_equal(a.get_weights(), b.get_weights())
    for k in range(3, 5):
        la = a.train_step(xs[k % 2 * 2:k % 2 * 2 + 2], ts[k % 2 * 2:k % 2 * 2 + 2])
        lb = b.train_step(xs[k % 2 * 2:k % 2 * 2 + 2], ts[k % 2 * 2:k % 2 * 2 + 2])
        assert la == lb, (k, la, lb)
    assert np.array_equal(a.get_weights(), b.get_weights())
    ya, yb = a.infer(xs[0]), b.infer(xs[0])
    torch.cuda.synchronize()
    assert torch.equal(ya, yb)
    # a checkpoint of another depth is refused and leaves the handle as it was
    c = sg.Surrogate(depth=4, seed=13)
    w0 = c.get_weights()
    with pytest.raises(ig.IgError):
        c.load(path)
    assert np.array_equal(w0, c.get_weights()) and c.step == 0


def test_gradient_clipping(dev):
    """The reported gradient norm is the FP64 norm of the step's gradient; a
    limit above it changes nothing (bitwise), a limit below it changes the
    later steps (Adam's first step is scale-invariant, its later ones are not)."""
    import torch
    import paper_1609_03782_amd as ig
    from paper_1609_03782_amd import surrogate as sg
    import igsynth
    c = igsynth.batch_cube(igsynth.BatchItem((16, 18, 20), 2.0, 8, 900))
    x = torch.from_numpy(c).to(dev)
    t = ig.Filter(c.shape, K=2.0, tau=1 / 16, n_iter=8).run(x)
    torch.cuda.synchronize()
    nets = [sg.Surrogate(depth=3, seed=21, lr=1e-3) for _ in range(3)]
    nets[1].set_clip(1e30)
    for k in range(3):
        for n in nets:
            n.train_step([x], [t], want_loss=False)
        g = nets[0].get_grads().astype(np.float64)
        assert nets[0].last_grad_norm() == pytest.approx(float(np.sqrt((g * g).sum())), rel=1e-6)
        if k == 0:
            nets[2].set_clip(0.01 * nets[0].last_grad_norm())
    assert np.array_equal(nets[0].get_weights(), nets[1].get_weights())
    assert not np.array_equal(nets[0].get_weights(), nets[2].get_weights())
    with pytest.raises(ig.IgError):
        nets[0].set_clip(-1.0)


def test_checked_inference_and_fallback(dev):
    import torch
    import paper_1609_03782_amd as ig
    from paper_1609_03782_amd import surrogate as sg
    import igsynth
    c = igsynth.random_cube((20, 24, 28), seed=3)
    x = torch.from_numpy(c).to(dev)
    params = dict(K=2.0, tau=1 / 16, n_iter=12, cond="pm_exp")
    net = sg.Surrogate(depth=4, seed=6)          # untrained: y = x
    y, rep = net.infer_checked(x, params, slope=1.0, threshold=0.0)
    plain = ig.Filter(c.shape, **params).run(x)
    torch.cuda.synchronize()
    assert rep["fell_back"] and torch.equal(y, plain)
    y2, rep2 = net.infer_checked(x, params, slope=1.0, threshold=1e9)
    torch.cuda.synchronize()
    assert not rep2["fell_back"] and torch.equal(y2, x)
    assert rep2["residual"] > 0


def test_trained_network_gain(dev):
    """What the trained network gains over the method without it: on held-out
    cubes its prediction of the n-step filter is much closer than the
    untrained network's (which returns its input), and the test reports the
    error of the plain filter given the same time budget as one inference."""
    import time

    import torch
    import paper_1609_03782_amd as ig
    from paper_1609_03782_amd import surrogate as sg
    import igsynth
    n = 20
    cubes = [igsynth.batch_cube(igsynth.BatchItem((24, 24, 24), 2.0, n, 700 + k)) for k in range(20)]
    xs = [torch.from_numpy(c).to(dev) for c in cubes]
    f = ig.Filter(cubes[0].shape, K=2.0, tau=1 / 16, n_iter=n)
    ts = [f.run(x) for x in xs]
    torch.cuda.synchronize()
    train_x, train_t, test_x, test_t = xs[:16], ts[:16], xs[16:], ts[16:]
    net = sg.Surrogate(depth=4, seed=9, lr=2e-3)

    def rmse(net_):
        e = [float(torch.sqrt(torch.mean((net_.infer(x).double() - t.double()) ** 2))) for x, t in zip(test_x, test_t)]
        return float(np.mean(e))

    before = rmse(net)                                   # untrained: the identity
    for k in range(300):
        i = (4 * k) % 16
        net.train_step(train_x[i:i + 4], train_t[i:i + 4])
    after = rmse(net)
    # the plain filter given one inference's time: as many steps as fit
    x, t = test_x[0], test_t[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        net.infer(x)
    torch.cuda.synchronize()
    t_inf = (time.perf_counter() - t0) / 5
    f1 = ig.Filter(cubes[0].shape, K=2.0, tau=1 / 16, n_iter=1)
    t0 = time.perf_counter()
    for _ in range(5):
        f1.run(x)
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / 5
    k_eq = max(0, min(n, int(t_inf / t_step)))
    fk = ig.Filter(cubes[0].shape, K=2.0, tau=1 / 16, n_iter=k_eq)
    rm_k = float(torch.sqrt(torch.mean((fk.run(x).double() - t.double()) ** 2)))
    print(f"held-out RMSE to the {n}-step filter: untrained {before:.4f}, trained {after:.4f}; "
          f"plain filter in one inference's time ({k_eq} steps): {rm_k:.4f}")
    assert after < 0.5 * before
