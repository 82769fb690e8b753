"""Python binding of the learned surrogate (include/igsurrogate.h).

Argument marshalling only; every layer, gradient and optimiser step runs in
the library's HIP kernels.  Tensors are torch CUDA tensors: cubes FP32
(nz, ny, nx); activations bfloat16 channels-last (nz, ny, nx, C).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import IgParams, _check, _stream_ptr, lib, make_params


class IgSurrogateParams(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("depth", ctypes.c_int32), ("width", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("lr", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("seed", ctypes.c_uint64)]


class IgSurrogateReport(ctypes.Structure):
    _fields_ = [("residual", ctypes.c_double), ("predicted_rmse", ctypes.c_double), ("rho", ctypes.c_double),
                ("fell_back", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_P = ctypes.c_void_p
_F = ctypes.POINTER(ctypes.c_float)
_I64 = ctypes.c_int64
SIGNATURES = {
    "ig_surrogate_create": (ctypes.c_int, [ctypes.POINTER(IgSurrogateParams), ctypes.c_int, ctypes.POINTER(_P)]),
    "ig_surrogate_destroy": (None, [_P]),
    "ig_surrogate_param_count": (_I64, [_P]),
    "ig_surrogate_set_weights": (ctypes.c_int, [_P, _F, _I64]),
    "ig_surrogate_get_weights": (ctypes.c_int, [_P, _F, _I64]),
    "ig_surrogate_get_grads": (ctypes.c_int, [_P, _F, _I64]),
    "ig_surrogate_train_step": (ctypes.c_int, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.c_int32, _I64, _I64,
                                               _I64, _P, ctypes.POINTER(ctypes.c_double)]),
    "ig_surrogate_infer": (ctypes.c_int, [_P, _P, _P, _I64, _I64, _I64, ctypes.c_int32, _P]),
    "ig_surrogate_infer_checked": (ctypes.c_int, [_P, ctypes.POINTER(IgParams), _P, _P, ctypes.c_int32,
                                                  ctypes.c_double, ctypes.c_double, _P,
                                                  ctypes.POINTER(IgSurrogateReport)]),
    "ig_surrogate_save": (ctypes.c_int, [_P, ctypes.c_char_p]),
    "ig_surrogate_load": (ctypes.c_int, [_P, ctypes.c_char_p]),
    "ig_surrogate_checkpoint_info": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32),
                                                    ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_I64),
                                                    ctypes.POINTER(_I64), ctypes.POINTER(ctypes.c_uint64)]),
    "ig_surrogate_set_lr": (ctypes.c_int, [_P, ctypes.c_float]),
    "ig_surrogate_get_step": (_I64, [_P]),
    "ig_surrogate_set_clip": (ctypes.c_int, [_P, ctypes.c_float]),
    "ig_surrogate_last_grad_norm": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double)]),
    "ig_conv3d_forward": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, ctypes.c_int32, ctypes.c_int32, _P, _P, _I64,
                                         _I64, _I64, _P]),
    "ig_conv3d_input_grad": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int32, _P, _P, _I64, _I64, _I64, _P]),
    "ig_conv3d_weight_grad": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int32, _P, _P, _I64, _I64, _I64, _P]),
}
_bound = False


def slib():
    global _bound
    L = lib()
    if not _bound:
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _bound = True
    return L


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Surrogate:
    """3-D CNN surrogate of the n-step filter (ig_surrogate_*)."""

    def __init__(self, depth=8, width=32, lr=1e-3, betas=(0.9, 0.999), eps=1e-8, seed=0, device=0):
        p = IgSurrogateParams(ctypes.sizeof(IgSurrogateParams), depth, width, 0, lr, betas[0], betas[1], eps, seed)
        h = ctypes.c_void_p()
        _check(slib().ig_surrogate_create(ctypes.byref(p), device, ctypes.byref(h)), "ig_surrogate_create")
        self._h = h
        self.depth = depth
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            slib().ig_surrogate_destroy(self._h)
            self._h = None

    __del__ = close

    @property
    def param_count(self):
        return int(slib().ig_surrogate_param_count(self._h))

    def get_weights(self) -> np.ndarray:
        a = np.empty(self.param_count, np.float32)
        _check(slib().ig_surrogate_get_weights(self._h, a.ctypes.data_as(_F), a.size), "ig_surrogate_get_weights")
        return a

    def get_grads(self) -> np.ndarray:
        a = np.empty(self.param_count, np.float32)
        _check(slib().ig_surrogate_get_grads(self._h, a.ctypes.data_as(_F), a.size), "ig_surrogate_get_grads")
        return a

    def set_weights(self, w):
        a = np.ascontiguousarray(w, np.float32)
        _check(slib().ig_surrogate_set_weights(self._h, a.ctypes.data_as(_F), a.size), "ig_surrogate_set_weights")

    def save(self, path):
        """Checkpoint weights, Adam state, step and seed (ig_surrogate_save)."""
        _check(slib().ig_surrogate_save(self._h, str(path).encode()), "ig_surrogate_save")

    def load(self, path):
        """Restore a checkpoint of a network of the same depth (ig_surrogate_load)."""
        _check(slib().ig_surrogate_load(self._h, str(path).encode()), "ig_surrogate_load")

    def set_lr(self, lr):
        _check(slib().ig_surrogate_set_lr(self._h, float(lr)), "ig_surrogate_set_lr")

    def set_clip(self, max_norm):
        """Clip later steps by the global gradient norm (0: off)."""
        _check(slib().ig_surrogate_set_clip(self._h, float(max_norm)), "ig_surrogate_set_clip")

    def last_grad_norm(self):
        v = ctypes.c_double()
        _check(slib().ig_surrogate_last_grad_norm(self._h, ctypes.byref(v)), "ig_surrogate_last_grad_norm")
        return v.value

    @property
    def step(self):
        return int(slib().ig_surrogate_get_step(self._h))

    def train_step(self, xs, ts, want_loss=True):
        n = len(xs)
        shape = tuple(xs[0].shape)
        X = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        T = (ctypes.c_void_p * n)(*[t.data_ptr() for t in ts])
        loss = ctypes.c_double()
        nz, ny, nx = shape
        _check(slib().ig_surrogate_train_step(self._h, X, T, n, nx, ny, nz, _stream_ptr(xs[0]),
                                              ctypes.byref(loss) if want_loss else None), "ig_surrogate_train_step")
        return loss.value if want_loss else None

    def infer(self, x, out=None, tile=0):
        import torch
        out = torch.empty_like(x) if out is None else out
        nz, ny, nx = x.shape
        _check(slib().ig_surrogate_infer(self._h, _ptr(x), _ptr(out), nx, ny, nz, int(tile), _stream_ptr(x)),
               "ig_surrogate_infer")
        return out

    def infer_checked(self, x, params: dict, slope, threshold, out=None, tile=0):
        import torch
        out = torch.empty_like(x) if out is None else out
        p = make_params(tuple(x.shape), **params)
        rep = IgSurrogateReport()
        _check(slib().ig_surrogate_infer_checked(self._h, ctypes.byref(p), _ptr(x), _ptr(out), int(tile),
                                                 float(slope), float(threshold), _stream_ptr(x), ctypes.byref(rep)),
               "ig_surrogate_infer_checked")
        return out, {"residual": rep.residual, "predicted_rmse": rep.predicted_rmse, "rho": rep.rho,
                     "fell_back": bool(rep.fell_back)}


def checkpoint_info(path):
    """Header of a checkpoint file, checked on the host (no GPU needed):
    dict with depth, width, nparam, step, seed."""
    d, w = ctypes.c_int32(), ctypes.c_int32()
    n, st, sd = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_uint64()
    _check(slib().ig_surrogate_checkpoint_info(str(path).encode(), ctypes.byref(d), ctypes.byref(w), ctypes.byref(n),
                                               ctypes.byref(st), ctypes.byref(sd)), "ig_surrogate_checkpoint_info")
    return {"depth": d.value, "width": w.value, "nparam": n.value, "step": st.value, "seed": sd.value}


def param_layout(depth=8, width=32):
    """[(W shape, b shape)] per layer in the flat parameter vector."""
    out = []
    for l in range(depth):
        cin = 1 if l == 0 else width
        cout = 1 if l == depth - 1 else width
        out.append(((27, cin, cout), (cout,)))
    return out


def split_params(flat, depth=8, width=32):
    Ws, bs, k = [], [], 0
    for ws, bsh in param_layout(depth, width):
        n = int(np.prod(ws))
        Ws.append(flat[k:k + n].reshape(ws))
        k += n
        bs.append(flat[k:k + bsh[0]].copy())
        k += bsh[0]
    return Ws, bs


def join_params(Ws, bs):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in zip(Ws, bs)]).astype(np.float32)


def conv3d_forward(a, cin, W, b, cout, epilogue=0, aux=None, out=None):
    """a: bf16 (nz, ny, nx, cin); W, b: FP32 device tensors."""
    import torch
    nz, ny, nx = a.shape[:3]
    if out is None:
        if epilogue == 0:
            out = torch.empty((nz, ny, nx, 16 * ((cout + 15) // 16)), dtype=torch.float32, device=a.device)
        elif epilogue == 1:
            out = torch.empty((nz, ny, nx, 32), dtype=torch.bfloat16, device=a.device)
        else:
            out = torch.empty((nz, ny, nx), dtype=torch.float32, device=a.device)
    _check(slib().ig_conv3d_forward(_ptr(a), cin, _ptr(W), _ptr(b), cout, epilogue, _ptr(aux), _ptr(out), nx, ny,
                                    nz, _stream_ptr(a)), "ig_conv3d_forward")
    return out


def conv3d_input_grad(dz, cout, W, cin, aux=None):
    import torch
    nz, ny, nx = dz.shape[:3]
    if aux is None:
        out = torch.empty((nz, ny, nx, 16 * ((cin + 15) // 16)), dtype=torch.float32, device=dz.device)
    else:
        out = torch.empty((nz, ny, nx, 32), dtype=torch.bfloat16, device=dz.device)
    _check(slib().ig_conv3d_input_grad(_ptr(dz), cout, _ptr(W), cin, _ptr(aux), _ptr(out), nx, ny, nz,
                                       _stream_ptr(dz)), "ig_conv3d_input_grad")
    return out


def conv3d_weight_grad(a, cin, dz, cout):
    import torch
    nz, ny, nx = a.shape[:3]
    dW = torch.empty((27, cin, cout), dtype=torch.float32, device=a.device)
    db = torch.empty((cout,), dtype=torch.float32, device=a.device)
    _check(slib().ig_conv3d_weight_grad(_ptr(a), cin, _ptr(dz), cout, _ptr(dW), _ptr(db), nx, ny, nz,
                                        _stream_ptr(a)), "ig_conv3d_weight_grad")
    return dW, db


# ---------------------------------------------------------------- driver
def filter_targets(xs, n_iter=50, K=2.0, tau=1.0 / 16, C=(1.0, 1.0, 1.0), cond="pm_exp"):
    """n-step filtered copies of the cubes in xs (one shape), computed by the
    library's filter on the GPU (the training targets)."""
    import torch
    from . import Filter
    f = Filter(tuple(xs[0].shape), K=K, tau=tau, n_iter=n_iter, C=C, cond=cond)
    return [f.run(x) for x in xs]


def train(net, xs, ts, epochs=1, batch=4, seed=0, log=None):
    """Plain minibatch Adam over the (x, t) pairs; returns the per-step losses."""
    rng = np.random.default_rng(seed)
    losses = []
    for ep in range(epochs):
        order = rng.permutation(len(xs))
        for k in range(0, len(order) - batch + 1, batch):
            idx = order[k:k + batch]
            losses.append(net.train_step([xs[i] for i in idx], [ts[i] for i in idx]))
            if log and len(losses) % 50 == 0:
                log(f"epoch {ep} step {len(losses)} loss {np.mean(losses[-50:]):.5f}")
    return losses


def calibrate(net, xs, ts, params, tile=0, quantile=1.0):
    """Residual-check calibration on validation pairs: slope = the given
    quantile of true_rmse / residual (both in units of rho).  Returns
    (slope, list of (residual, true_rmse))."""
    import torch
    pairs = []
    for x, t in zip(xs, ts):
        y, rep = net.infer_checked(x, params, slope=1.0, threshold=float("inf"), tile=tile)
        e = float(torch.sqrt(torch.mean((y.double() - t.double()) ** 2)).item()) / rep["rho"]
        pairs.append((rep["residual"], e))
    ratios = np.array([e / max(r, 1e-30) for r, e in pairs])
    return float(np.quantile(ratios, quantile)), pairs
