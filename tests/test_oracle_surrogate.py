"""Pins of the FP64 surrogate oracle: convolution and its two gradients against
torch's CPU conv3d and autograd (a library implementation of the same
definitions), the whole network's gradient against central finite
differences, GELU against torch's erf GELU, and Adam against torch.optim."""
import numpy as np
import pytest
import torch

from oracle import surrogate as S


def _torch_w(W):
    # (27, Cin, Cout) -> torch (Cout, Cin, 3, 3, 3), tap t = (dz+1)*9 + (dy+1)*3 + (dx+1)
    cin, cout = W.shape[1], W.shape[2]
    return torch.from_numpy(W.reshape(3, 3, 3, cin, cout).transpose(4, 3, 0, 1, 2).copy())


def _ncdhw(a):
    return torch.from_numpy(np.ascontiguousarray(a.transpose(3, 0, 1, 2))[None])


@pytest.mark.parametrize("cin,cout", [(1, 4), (3, 5), (4, 1)])
def test_conv3d_matches_torch(cin, cout):
    rng = np.random.default_rng(cin * 10 + cout)
    a = rng.standard_normal((5, 6, 7, cin))
    W = rng.standard_normal((27, cin, cout))
    b = rng.standard_normal(cout)
    ref = torch.nn.functional.conv3d(_ncdhw(a), _torch_w(W), torch.from_numpy(b), padding=1)
    got = S.conv3d(a, W, b)
    np.testing.assert_allclose(got, ref[0].numpy().transpose(1, 2, 3, 0), rtol=0, atol=1e-12)


def test_conv3d_gradients_match_autograd():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((4, 5, 6, 3))
    W = rng.standard_normal((27, 3, 2))
    dz = rng.standard_normal((4, 5, 6, 2))
    ta = _ncdhw(a).requires_grad_()
    tw = _torch_w(W).requires_grad_()
    tb = torch.zeros(2, dtype=torch.float64, requires_grad=True)
    out = torch.nn.functional.conv3d(ta, tw, tb, padding=1)
    out.backward(_ncdhw(dz))
    da = S.conv3d_input_grad(dz, W)
    dW, db = S.conv3d_weight_grad(a, dz)
    np.testing.assert_allclose(da, ta.grad[0].numpy().transpose(1, 2, 3, 0), atol=1e-11)
    np.testing.assert_allclose(dW, tw.grad.numpy().transpose(2, 3, 4, 1, 0).reshape(27, 3, 2), atol=1e-11)
    np.testing.assert_allclose(db, tb.grad.numpy(), atol=1e-11)


def test_gelu_and_its_derivative():
    z = np.linspace(-6, 6, 1001)
    ref = torch.nn.functional.gelu(torch.from_numpy(z), approximate="none").numpy()
    np.testing.assert_allclose(S.gelu(z), ref, atol=1e-15)
    h = 1e-6
    np.testing.assert_allclose(S.gelu_grad(z), (S.gelu(z + h) - S.gelu(z - h)) / (2 * h), atol=1e-8)


def test_network_gradient_finite_differences():
    rng = np.random.default_rng(4)
    Ws, bs = S.init_params(rng, widths=(1, 3, 2, 1))
    Ws[-1] = rng.standard_normal(Ws[-1].shape) * 0.2   # non-zero last layer
    bs = [rng.standard_normal(b.shape) * 0.1 for b in bs]
    x = rng.standard_normal((4, 4, 5))
    t = x + 0.3 * rng.standard_normal(x.shape)
    loss, gW, gb, _ = S.loss_and_grads(x, t, Ws, bs)
    h = 1e-6
    for l in range(3):
        for idx in [(0, 0, 0), (13, 0, 0), (26, Ws[l].shape[1] - 1, Ws[l].shape[2] - 1)]:
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[l][idx] += h
            Wm[l][idx] -= h
            fd = (S.loss_and_grads(x, t, Wp, bs)[0] - S.loss_and_grads(x, t, Wm, bs)[0]) / (2 * h)
            assert gW[l][idx] == pytest.approx(fd, rel=1e-6, abs=1e-9)
        bp = [b.copy() for b in bs]
        bm = [b.copy() for b in bs]
        bp[l][0] += h
        bm[l][0] -= h
        fd = (S.loss_and_grads(x, t, Ws, bp)[0] - S.loss_and_grads(x, t, Ws, bm)[0]) / (2 * h)
        assert gb[l][0] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_identity_network_at_init():
    rng = np.random.default_rng(5)
    Ws, bs = S.init_params(rng)
    x = rng.standard_normal((3, 4, 5))
    y, _ = S.forward(x, Ws, bs)
    np.testing.assert_array_equal(y, x)


def test_adam_matches_torch():
    rng = np.random.default_rng(6)
    p0 = rng.standard_normal(10)
    tp = torch.from_numpy(p0.copy()).requires_grad_()
    opt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(10), np.zeros(10)
    for step in range(1, 4):
        g = rng.standard_normal(10)
        tp.grad = torch.from_numpy(g.copy())
        opt.step()
        p, m, v = S.adam_step(p, g, m, v, step, 1e-3)
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=0, atol=1e-12)
