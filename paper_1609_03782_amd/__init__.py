"""Python binding of libigfilter (the MI355X intensity-driven gradient filter).

Argument marshalling only: every step of the filter runs in the library's HIP
kernels, reached through the C ABI declared in include/igfilter.h.  PyTorch
supplies device memory (tensor data pointers) and the current HIP stream.
There is no fallback: if the built library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libigfilter.so")

IG_OK, IG_ERR_INVALID_ARG, IG_ERR_OUT_OF_MEMORY, IG_ERR_DEVICE, IG_ERR_NONFINITE, IG_ERR_UNSUPPORTED = range(6)
DTYPES = {"f32": 0, "bf16": 1, "f16": 2}
CONDS = {"intensity": 0, "pm_exp": 1, "pm_rational": 2}
SCHED = {"auto": 0, "naive": 1, "blocked": 2}


class IgParams(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("dtype", ctypes.c_int32), ("cond", ctypes.c_int32),
                ("n_iter", ctypes.c_int32), ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("nz", ctypes.c_int64), ("K", ctypes.c_float), ("tau", ctypes.c_float),
                ("C", ctypes.c_float * 3), ("reserved0", ctypes.c_float), ("rms", ctypes.c_double)]


class IgSchedule(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("t_block", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("zchunk", ctypes.c_int32), ("vec", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("rows", ctypes.c_int32)]


class IgStats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("passes", ctypes.c_int32), ("rms_used", ctypes.c_double),
                ("sum_in", ctypes.c_double), ("sum_out", ctypes.c_double), ("nonfinite", ctypes.c_int64),
                ("monotone", ctypes.c_int32), ("reserved", ctypes.c_int32), ("schedule", IgSchedule)]


class IgBatchItem(ctypes.Structure):
    _fields_ = [("p", IgParams), ("d_in", ctypes.c_void_p), ("d_out", ctypes.c_void_p)]


class IgCompareResult(ctypes.Structure):
    _fields_ = [("max_abs", ctypes.c_double), ("rms", ctypes.c_double), ("max_ref", ctypes.c_double),
                ("sum_x", ctypes.c_double), ("sum_ref", ctypes.c_double), ("n_over", ctypes.c_int64)]


QMAX = 63   # IG_QUALITY_MAX_THR


class IgQualityParams(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("n_thr", ctypes.c_int32), ("roi", ctypes.c_int64 * 6),
                ("thr_f", ctypes.c_double * QMAX), ("thr_o", ctypes.c_double), ("rms_o", ctypes.c_double),
                ("rms_f", ctypes.c_double), ("indep", ctypes.c_double)]


class IgQualityResult(ctypes.Structure):
    _fields_ = [("rms_o", ctypes.c_double), ("rms_f", ctypes.c_double), ("S_oo", ctypes.c_double),
                ("S_m", ctypes.c_double), ("N_o", ctypes.c_int64), ("n_roi", ctypes.c_int64),
                ("S_of", ctypes.c_double * QMAX), ("S_mf", ctypes.c_double * QMAX), ("N_f", ctypes.c_int64 * QMAX),
                ("F", ctypes.c_double * QMAX), ("sigma_F", ctypes.c_double * QMAX), ("F_M", ctypes.c_double * QMAX),
                ("sigma_FM", ctypes.c_double * QMAX)]


class IgSweepPoint(ctypes.Structure):
    _fields_ = [("K", ctypes.c_float), ("tau", ctypes.c_float), ("n_iter", ctypes.c_int32), ("C", ctypes.c_float * 3)]


class IgSmoothParams(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("kind", ctypes.c_int32), ("size", ctypes.c_float * 3),
                ("theta", ctypes.c_float * 3), ("truncate", ctypes.c_float), ("reserved", ctypes.c_int32)]


SMOOTH_KINDS = {"box": 0, "gauss": 1}
WAVELETS = {"haar": 0, "legall53": 1}
WMAX = 8   # IG_WAVELET_MAX_LEVELS


class IgWaveletParams(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("kind", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("t", ctypes.c_double * WMAX), ("rms", ctypes.c_double)]


# name -> (restype, argtypes); the exported C ABI
_P = ctypes.c_void_p
SIGNATURES = {
    "ig_filter_create": (ctypes.c_int, [ctypes.POINTER(IgParams), ctypes.c_int, ctypes.POINTER(_P)]),
    "ig_filter_run": (ctypes.c_int, [_P, _P, _P, _P, ctypes.POINTER(IgStats)]),
    "ig_filter_run_static": (ctypes.c_int, [ctypes.POINTER(IgParams), ctypes.c_int, _P, _P, _P,
                                            ctypes.POINTER(IgStats)]),
    "ig_filter_static_max_bytes": (ctypes.c_int64, []),
    "ig_filter_set_schedule": (ctypes.c_int, [_P, ctypes.POINTER(IgSchedule)]),
    "ig_filter_get_schedule": (ctypes.c_int, [_P, ctypes.POINTER(IgSchedule)]),
    "ig_filter_destroy": (None, [_P]),
    "ig_filter_autotune": (ctypes.c_int, [_P, _P, _P, _P, ctypes.POINTER(IgSchedule), ctypes.POINTER(ctypes.c_double)]),
    "ig_batch_autotune": (ctypes.c_int, [ctypes.POINTER(IgBatchItem), ctypes.c_int32, ctypes.c_int, _P,
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    "ig_filter_set_timing": (ctypes.c_int, [_P, ctypes.c_int]),
    "ig_filter_get_timing": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                            ctypes.c_int]),
    "ig_schedule_plan": (ctypes.c_int, [ctypes.POINTER(IgParams), ctypes.POINTER(IgSchedule), ctypes.c_int32,
                                        ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                        ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    "ig_schedule_check": (ctypes.c_int, [ctypes.POINTER(IgParams), ctypes.POINTER(IgSchedule)]),
    "ig_schedule_auto": (ctypes.c_int, [ctypes.POINTER(IgParams), ctypes.POINTER(IgSchedule)]),
    "ig_schedule_plan_groups": (ctypes.c_int, [ctypes.POINTER(IgParams), ctypes.POINTER(IgSchedule), ctypes.c_int32,
                                               ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.c_int64,
                                               ctypes.POINTER(ctypes.c_int64)]),
    "ig_filter_batch": (ctypes.c_int, [ctypes.POINTER(IgBatchItem), ctypes.c_int32, ctypes.c_int, _P,
                                       ctypes.POINTER(IgStats), ctypes.POINTER(ctypes.c_double)]),
    "ig_batch_cache_clear": (None, []),
    "ig_batch_cache_size": (ctypes.c_int32, []),
    "ig_batch_set_schedule": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "ig_batch_set_launch": (ctypes.c_int, [ctypes.c_int32]),
    "ig_batch_get_launch": (ctypes.c_int32, []),
    "ig_batch_set_resident": (ctypes.c_int, [ctypes.c_int32]),
    "ig_batch_get_resident": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int32)]),
    "ig_compare": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int64, ctypes.c_double, ctypes.c_int, _P,
                                  ctypes.POINTER(IgCompareResult)]),
    "ig_reduce": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int, _P,
                                 ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_int64)]),
    "ig_quality": (ctypes.c_int, [ctypes.POINTER(IgQualityParams), _P, _P, _P, ctypes.c_int64, ctypes.c_int64,
                                  ctypes.c_int64, ctypes.c_int, _P, ctypes.POINTER(IgQualityResult)]),
    "ig_filter_set_params": (ctypes.c_int, [_P, ctypes.POINTER(IgParams)]),
    "ig_filter_sweep": (ctypes.c_int, [ctypes.POINTER(IgParams), ctypes.POINTER(IgSweepPoint), ctypes.c_int32, _P, _P,
                                       ctypes.POINTER(IgQualityParams), ctypes.c_int, _P,
                                       ctypes.POINTER(IgQualityResult), ctypes.POINTER(ctypes.c_int32), _P]),
    "ig_smooth_geometry": (ctypes.c_int, [ctypes.POINTER(IgSmoothParams), ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_int32)]),
    "ig_smooth": (ctypes.c_int, [ctypes.POINTER(IgSmoothParams), _P, _P, _P, ctypes.c_int64, ctypes.c_int64,
                                 ctypes.c_int64, _P]),
    "ig_smooth_set_path": (ctypes.c_int, [ctypes.c_int32]),
    "ig_wavelet_forward": (ctypes.c_int, [ctypes.POINTER(IgWaveletParams), _P, _P, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_int64, _P]),
    "ig_wavelet_inverse": (ctypes.c_int, [ctypes.POINTER(IgWaveletParams), _P, _P, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_int64, _P]),
    "ig_wavelet_denoise": (ctypes.c_int, [ctypes.POINTER(IgWaveletParams), _P, _P, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_int64, _P, ctypes.POINTER(ctypes.c_double)]),
    "ig_debug_fail_alloc": (None, [ctypes.c_int64]),
    "ig_debug_live_allocations": (ctypes.c_int64, []),
    "ig_debug_release_caches": (None, []),
    "ig_debug_set_infer_piece_limit": (ctypes.c_int64, [ctypes.c_int64]),
    "ig_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "ig_last_error": (ctypes.c_char_p, []),
    "ig_version": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libigfilter.so (built by build.py); raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1609_03782_amd.build` "
                               "(or __graft_entry__.build()) first; there is no fallback")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class IgError(RuntimeError):
    def __init__(self, status, where):
        L = lib()
        msg = L.ig_last_error().decode(errors="replace")
        super().__init__(f"{where}: {L.ig_status_string(status).decode()} ({msg})")
        self.status = status


def _check(status, where):
    if status != IG_OK:
        raise IgError(status, where)


def make_params(shape, K=2.0, tau=1.0 / 16, n_iter=50, C=(1.0, 1.0, 1.0), rms=None, cond="pm_exp",
                dtype="f32") -> IgParams:
    nz, ny, nx = shape
    p = IgParams()
    p.struct_size = ctypes.sizeof(IgParams)
    p.dtype = DTYPES[dtype]
    p.cond = CONDS[cond]
    p.n_iter = int(n_iter)
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    p.K, p.tau = float(K), float(tau)
    for a in range(3):
        p.C[a] = float(C[a])
    p.reserved0 = 0.0
    p.rms = float(rms) if rms is not None else 0.0
    return p


def schedule_check(shape, sched: dict, **params) -> str | None:
    """None if `sched` can serve cubes of `shape`, else the reason (host only)."""
    p = make_params(shape, **params)
    s = IgSchedule(SCHED[sched.get("kind", "blocked")], sched.get("t_block", 2), sched.get("waves", 16),
                   sched.get("zchunk", 0), sched.get("vec", 0), sched.get("rounds", 0), sched.get("rows", 0))
    rc = lib().ig_schedule_check(ctypes.byref(p), ctypes.byref(s))
    return None if rc == IG_OK else lib().ig_last_error().decode()


def schedule_plan(shape, sched: dict, t_block: int, ncu: int = 256, **params):
    """Host-only work split of one pass: (geometry dict, pieces array (k, 4))."""
    import numpy as np
    p = make_params(shape, **params)
    s = IgSchedule(SCHED[sched.get("kind", "blocked")], sched.get("t_block", 2), sched.get("waves", 16),
                   sched.get("zchunk", 0), sched.get("vec", 0), sched.get("rounds", 0), sched.get("rows", 0))
    geom = (ctypes.c_int32 * 9)()
    cnt = ctypes.c_int64()
    _check(lib().ig_schedule_plan(ctypes.byref(p), ctypes.byref(s), t_block, ncu, geom, None, 0,
                                  ctypes.byref(cnt)), "ig_schedule_plan")
    arr = np.zeros((cnt.value, 4), np.int32)
    _check(lib().ig_schedule_plan(ctypes.byref(p), ctypes.byref(s), t_block, ncu, geom,
                                  arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), cnt.value,
                                  ctypes.byref(cnt)), "ig_schedule_plan")
    keys = ["ntx", "nty", "ox", "oy", "waves", "vec_io", "V", "pieces", "rows"]
    return dict(zip(keys, list(geom))), arr


def schedule_auto(shape, **params) -> dict:
    """Host-only: the schedule a Filter of this shape and parameters runs by default."""
    p = make_params(shape, **params)
    s = IgSchedule()
    _check(lib().ig_schedule_auto(ctypes.byref(p), ctypes.byref(s)), "ig_schedule_auto")
    return _sched_dict(s)


def schedule_plan_groups(shape, sched: dict, t_block: int, ncu: int = 256, **params):
    """Host-only: each workgroup's first piece (array of nwg + 1 entries) when
    the pass runs several pieces per workgroup, else None."""
    import numpy as np
    p = make_params(shape, **params)
    s = IgSchedule(SCHED[sched.get("kind", "blocked")], sched.get("t_block", 2), sched.get("waves", 16),
                   sched.get("zchunk", 0), sched.get("vec", 0), sched.get("rounds", 0), sched.get("rows", 0))
    n = ctypes.c_int64()
    _check(lib().ig_schedule_plan_groups(ctypes.byref(p), ctypes.byref(s), t_block, ncu, None, 0, ctypes.byref(n)),
           "ig_schedule_plan_groups")
    if n.value == 0:
        return None
    first = np.zeros(n.value + 1, np.int32)
    _check(lib().ig_schedule_plan_groups(ctypes.byref(p), ctypes.byref(s), t_block, ncu,
                                         first.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), n.value + 1,
                                         ctypes.byref(n)), "ig_schedule_plan_groups")
    return first


def _torch_dtype_name(t):
    import torch
    return {torch.float32: "f32", torch.bfloat16: "bf16", torch.float16: "f16"}[t.dtype]


def _stream_ptr(t):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


@dataclass
class Stats:
    passes: int
    rms_used: float
    sum_in: float
    sum_out: float
    nonfinite: int
    monotone: bool
    schedule: dict


def _sched_dict(s: IgSchedule):
    return {"kind": {v: k for k, v in SCHED.items()}[s.kind], "t_block": s.t_block, "waves": s.waves,
            "zchunk": s.zchunk, "vec": s.vec, "rounds": s.rounds, "rows": s.rows}


class Filter:
    """Handle for cubes of one shape and parameter set (ig_filter_create).

    shape is (nz, ny, nx), x fastest.  `run(x, out)` filters a CUDA tensor of
    that shape (float32 / bfloat16 / float16 matching `dtype`).
    """

    def __init__(self, shape, K=2.0, tau=1.0 / 16, n_iter=50, C=(1.0, 1.0, 1.0), rms=None, cond="pm_exp",
                 dtype="f32", device=0):
        self.shape = tuple(int(s) for s in shape)
        self.params = make_params(self.shape, K, tau, n_iter, C, rms, cond, dtype)
        self.dtype = dtype
        self.device = int(device)
        h = ctypes.c_void_p()
        _check(lib().ig_filter_create(ctypes.byref(self.params), self.device, ctypes.byref(h)),
               "ig_filter_create")
        self._h = h

    def set_params(self, K=None, tau=None, n_iter=None, C=None, rms=None, cond=None):
        """Change the filter parameters in place (ig_filter_set_params); shape
        and storage type stay.  Arguments left None keep their value."""
        p = IgParams.from_buffer_copy(self.params)
        if K is not None:
            p.K = float(K)
        if tau is not None:
            p.tau = float(tau)
        if n_iter is not None:
            p.n_iter = int(n_iter)
        if C is not None:
            for a in range(3):
                p.C[a] = float(C[a])
        if rms is not None:
            p.rms = float(rms)
        if cond is not None:
            p.cond = CONDS[cond]
        _check(lib().ig_filter_set_params(self._h, ctypes.byref(p)), "ig_filter_set_params")
        self.params = p

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            try:
                lib().ig_filter_destroy(h)
            except TypeError:   # interpreter shutdown: module globals are already gone
                pass

    __del__ = close

    def set_schedule(self, kind="blocked", t_block=2, waves=16, zchunk=0, vec=0, rounds=0, rows=0):
        if kind == "auto":
            _check(lib().ig_filter_set_schedule(self._h, None), "ig_filter_set_schedule")
            return
        s = IgSchedule(SCHED[kind], t_block, waves, zchunk, vec, rounds, rows)
        _check(lib().ig_filter_set_schedule(self._h, ctypes.byref(s)), "ig_filter_set_schedule")

    def autotune(self, x, work=None):
        """Time candidate schedules on x (into `work`), keep the fastest; returns (schedule, ms)."""
        import torch
        self._check_tensor(x, "x")
        work = torch.empty_like(x) if work is None else work
        best = IgSchedule()
        ms = ctypes.c_double()
        _check(lib().ig_filter_autotune(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(work.data_ptr()),
                                        _stream_ptr(x), ctypes.byref(best), ctypes.byref(ms)), "ig_filter_autotune")
        return _sched_dict(best), ms.value

    def set_timing(self, enable=True):
        _check(lib().ig_filter_set_timing(self._h, int(bool(enable))), "ig_filter_set_timing")

    def timing(self, reset=True):
        """(summed device ms, launches) of the step-loop kernels since the last reset."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(lib().ig_filter_get_timing(self._h, ctypes.byref(ms), ctypes.byref(n), int(reset)),
               "ig_filter_get_timing")
        return ms.value, n.value

    def schedule(self):
        s = IgSchedule()
        _check(lib().ig_filter_get_schedule(self._h, ctypes.byref(s)), "ig_filter_get_schedule")
        return _sched_dict(s)

    def _check_tensor(self, t, name):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA (HIP) tensor")
        if tuple(t.shape) != self.shape or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {self.shape}")
        if _torch_dtype_name(t) != self.dtype:
            raise TypeError(f"{name} dtype {t.dtype} does not match the handle's {self.dtype}")

    def run(self, x, out=None, stats=False):
        import torch
        self._check_tensor(x, "x")
        if out is None:
            out = torch.empty_like(x)
        self._check_tensor(out, "out")
        st = None
        if stats:
            st = IgStats()
            st.struct_size = ctypes.sizeof(IgStats)
        rc = lib().ig_filter_run(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                 _stream_ptr(x), ctypes.byref(st) if st is not None else None)
        _check(rc, "ig_filter_run")
        if stats:
            return out, Stats(st.passes, st.rms_used, st.sum_in, st.sum_out, st.nonfinite, bool(st.monotone),
                              _sched_dict(st.schedule))
        return out


def run_static(x, out=None, stats=False, K=2.0, tau=1.0 / 16, n_iter=50, C=(1.0, 1.0, 1.0), rms=None,
               cond="pm_exp"):
    """The filter without a handle and without device allocation in the
    library (ig_filter_run_static): cubes of at most
    ig_filter_static_max_bytes() bytes.  `out` defaults to a new tensor
    (allocated by torch here, not by the library)."""
    import torch
    if not isinstance(x, torch.Tensor) or not x.is_cuda or not x.is_contiguous() or x.dim() != 3:
        raise TypeError("x must be a contiguous 3-D CUDA (HIP) tensor")
    if out is None:
        out = torch.empty_like(x)
    if out.shape != x.shape or out.dtype != x.dtype or not out.is_contiguous() or out.device != x.device:
        raise ValueError("out must match x in shape, dtype and device")
    p = make_params(tuple(x.shape), K, tau, n_iter, C, rms, cond, _torch_dtype_name(x))
    st = None
    if stats:
        st = IgStats()
        st.struct_size = ctypes.sizeof(IgStats)
    _check(lib().ig_filter_run_static(ctypes.byref(p), x.device.index or 0, ctypes.c_void_p(x.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()), _stream_ptr(x),
                                      ctypes.byref(st) if st is not None else None), "ig_filter_run_static")
    if stats:
        return out, Stats(st.passes, st.rms_used, st.sum_in, st.sum_out, st.nonfinite, bool(st.monotone),
                          _sched_dict(st.schedule))
    return out


def static_max_bytes():
    return int(lib().ig_filter_static_max_bytes())


class PreparedBatch:
    """The marshalled item array of a batch, for repeated ig_filter_batch calls
    on the same tensors without rebuilding it (thousands of items take
    milliseconds to marshal).  Keeps the tensors alive."""

    def __init__(self, items):
        self.items = list(items)
        self.arr = _batch_array(self.items)

    def __len__(self):
        return len(self.items)


def batch_prepare(items):
    return PreparedBatch(items)


def batch(items, device=0, want_stats=False, want_latency=False):
    """items: list of (x, out, params-dict), or a PreparedBatch of one.  One
    graph launch (ig_filter_batch)."""
    import torch
    n = len(items)
    arr = items.arr if isinstance(items, PreparedBatch) else _batch_array(items)
    st = (IgStats * n)() if want_stats else None
    if st is not None:
        for k in range(n):
            st[k].struct_size = ctypes.sizeof(IgStats)
    lat = (ctypes.c_double * n)() if want_latency else None
    stream = ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)
    _check(lib().ig_filter_batch(arr, n, device, stream, st, lat), "ig_filter_batch")
    res = {}
    if st is not None:
        res["stats"] = [Stats(s.passes, s.rms_used, s.sum_in, s.sum_out, s.nonfinite, bool(s.monotone),
                              _sched_dict(s.schedule)) for s in st]
    if lat is not None:
        res["latency_ms"] = list(lat)
    return res


def _batch_array(items):
    n = len(items)
    arr = (IgBatchItem * n)()
    for k, (x, out, kw) in enumerate(items):
        arr[k].p = make_params(tuple(x.shape), dtype=_torch_dtype_name(x), **kw)
        arr[k].d_in = x.data_ptr()
        arr[k].d_out = out.data_ptr()
    return arr


def batch_autotune(items, device=0):
    """Time the batch under candidate schedules; keep the fastest.  Returns
    (t_block, waves, zchunk, ms)."""
    import torch
    arr = _batch_array(items)
    T, W, Z, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    stream = ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)
    _check(lib().ig_batch_autotune(arr, len(items), device, stream, ctypes.byref(T), ctypes.byref(W),
                                   ctypes.byref(Z), ctypes.byref(ms)), "ig_batch_autotune")
    return T.value, W.value, Z.value, ms.value


def batch_cache_clear():
    lib().ig_batch_cache_clear()


def batch_cache_size():
    return int(lib().ig_batch_cache_size())


def batch_set_schedule(t_block=0, waves=16, zchunk=32):
    _check(lib().ig_batch_set_schedule(int(t_block), int(waves), int(zchunk)), "ig_batch_set_schedule")


def batch_set_launch(persistent=False):
    """Later batches: one persistent launch (True) or one launch per pass round (False)."""
    _check(lib().ig_batch_set_launch(int(bool(persistent))), "ig_batch_set_launch")


def batch_get_launch():
    return bool(lib().ig_batch_get_launch())


def batch_set_resident(max_voxels=32768):
    """Cubes of at most max_voxels voxels run LDS-resident in later batches (0: none)."""
    _check(lib().ig_batch_set_resident(int(max_voxels)), "ig_batch_set_resident")


def batch_get_resident():
    v = ctypes.c_int32()
    _check(lib().ig_batch_get_resident(ctypes.byref(v)), "ig_batch_get_resident")
    return v.value


def compare(x, ref, tol=0.0):
    """FP64 error norms of device tensor x against FP64 device tensor ref (ig_compare)."""
    import torch
    assert ref.dtype == torch.float64 and ref.is_contiguous() and x.is_contiguous()
    assert x.numel() == ref.numel()
    r = IgCompareResult()
    _check(lib().ig_compare(ctypes.c_void_p(x.data_ptr()), DTYPES[_torch_dtype_name(x)],
                            ctypes.c_void_p(ref.data_ptr()), x.numel(), float(tol), x.device.index or 0,
                            _stream_ptr(x), ctypes.byref(r)), "ig_compare")
    return {"max_abs": r.max_abs, "rms": r.rms, "max_ref": r.max_ref, "sum_x": r.sum_x,
            "sum_ref": r.sum_ref, "n_over": r.n_over}


def reduce(x):
    """(sum, sum of squares, non-finite count) of a device tensor, FP64 (ig_reduce)."""
    s, q, b = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    _check(lib().ig_reduce(ctypes.c_void_p(x.data_ptr()), DTYPES[_torch_dtype_name(x)], x.numel(),
                           x.device.index or 0, _stream_ptr(x), ctypes.byref(s), ctypes.byref(q),
                           ctypes.byref(b)), "ig_reduce")
    return s.value, q.value, b.value


def _quality_params(roi, thr_f, thr_o, rms_o, rms_f, indep):
    thr_f = list(thr_f)
    if not 1 <= len(thr_f) <= QMAX:
        raise ValueError(f"1 to {QMAX} thresholds")
    q = IgQualityParams()
    q.struct_size = ctypes.sizeof(IgQualityParams)
    q.n_thr = len(thr_f)
    for j, t in enumerate(thr_f):
        q.thr_f[j] = float(t)
    for j, v in enumerate(roi if roi is not None else (0,) * 6):
        q.roi[j] = int(v)
    q.thr_o, q.rms_o, q.rms_f, q.indep = float(thr_o), float(rms_o), float(rms_f), float(indep)
    return q


def _quality_dict(r, k, has_model):
    return {"rms_o": r.rms_o, "rms_f": r.rms_f, "S_oo": r.S_oo, "N_o": r.N_o,
            "S_m": r.S_m if has_model else None, "n_roi": r.n_roi,
            "S_of": list(r.S_of[:k]), "N_f": list(r.N_f[:k]), "S_mf": list(r.S_mf[:k]) if has_model else [],
            "F": list(r.F[:k]), "sigma_F": list(r.sigma_F[:k]),
            "F_M": list(r.F_M[:k]) if has_model else [],
            "sigma_FM": list(r.sigma_FM[:k]) if has_model else []}


def quality(orig, filt, model=None, roi=None, thr_f=(3.0,), thr_o=3.0, rms_o=0.0, rms_f=0.0, indep=1.0):
    """Section 6 diagnostics (F, sigma_F, F_M, sigma_FM per M_f threshold) of
    FP32 device cubes (ig_quality).  roi = (x0, x1, y0, y1, z0, z1) or None."""
    import torch
    for t in (orig, filt) + ((model,) if model is not None else ()):
        assert t.dtype == torch.float32 and t.is_contiguous() and t.shape == orig.shape
    q = _quality_params(roi, thr_f, thr_o, rms_o, rms_f, indep)
    r = IgQualityResult()
    nz, ny, nx = orig.shape
    _check(lib().ig_quality(ctypes.byref(q), ctypes.c_void_p(orig.data_ptr()), ctypes.c_void_p(filt.data_ptr()),
                            ctypes.c_void_p(model.data_ptr()) if model is not None else None, nx, ny, nz,
                            orig.device.index or 0, _stream_ptr(orig), ctypes.byref(r)), "ig_quality")
    return _quality_dict(r, q.n_thr, model is not None)


def sweep(x, points, cond="intensity", model=None, roi=None, thr_f=(3.0,), thr_o=3.0, rms=0.0, rms_f=0.0,
          indep=1.0, want_best=False):
    """Parameter sweep scored by F (ig_filter_sweep).  points: dicts with K,
    tau, n_iter, C.  Returns (list of quality dicts, best index, best output
    or None)."""
    import torch
    assert x.dtype == torch.float32 and x.is_contiguous()
    if model is not None:
        assert model.dtype == torch.float32 and model.is_contiguous() and model.shape == x.shape
    base = make_params(tuple(x.shape), cond=cond, rms=rms if rms > 0 else None)
    pts = (IgSweepPoint * len(points))()
    for i, p in enumerate(points):
        pts[i].K, pts[i].tau, pts[i].n_iter = float(p["K"]), float(p["tau"]), int(p["n_iter"])
        for a in range(3):
            pts[i].C[a] = float(p["C"][a])
    q = _quality_params(roi, thr_f, thr_o, 0.0, rms_f, indep)
    res = (IgQualityResult * len(points))()
    best = ctypes.c_int32(-1)
    out = torch.empty_like(x) if want_best else None
    _check(lib().ig_filter_sweep(ctypes.byref(base), pts, len(points), ctypes.c_void_p(x.data_ptr()),
                                 ctypes.c_void_p(model.data_ptr()) if model is not None else None, ctypes.byref(q),
                                 x.device.index or 0, _stream_ptr(x), res, ctypes.byref(best),
                                 ctypes.c_void_p(out.data_ptr()) if out is not None else None), "ig_filter_sweep")
    return [_quality_dict(r, q.n_thr, model is not None) for r in res], best.value, out


def smooth_params(kind="gauss", size=(3.0, 3.0, 3.0), theta=(0.0, 0.0, 0.0), truncate=0.0):
    p = IgSmoothParams()
    p.struct_size = ctypes.sizeof(IgSmoothParams)
    p.kind = SMOOTH_KINDS[kind]
    for a in range(3):
        p.size[a] = float(size[a])
        p.theta[a] = float(theta[a])
    p.truncate = float(truncate)
    p.reserved = 0
    return p


def smooth_geometry(kind="gauss", size=(3.0, 3.0, 3.0), theta=(0.0, 0.0, 0.0), truncate=0.0):
    """((r_x, r_y, r_z), separable) of a box / Gaussian kernel (host only)."""
    p = smooth_params(kind, size, theta, truncate)
    r = (ctypes.c_int32 * 3)()
    sep = ctypes.c_int32()
    _check(lib().ig_smooth_geometry(ctypes.byref(p), r, ctypes.byref(sep)), "ig_smooth_geometry")
    return tuple(r), bool(sep.value)


def smooth(x, kind="gauss", size=(3.0, 3.0, 3.0), theta=(0.0, 0.0, 0.0), truncate=0.0, out=None, work=None):
    """Box (size = odd N_x, N_y, N_z) or Gaussian (size = FWHM_x, y, z; Euler
    angles theta in degrees) smoothing of an FP32 device cube (ig_smooth)."""
    import torch
    assert x.dtype == torch.float32 and x.is_contiguous()
    p = smooth_params(kind, size, theta, truncate)
    out = torch.empty_like(x) if out is None else out
    _, sep = smooth_geometry(kind, size, theta, truncate)
    if sep and work is None:
        work = torch.empty_like(x)
    nz, ny, nx = x.shape
    _check(lib().ig_smooth(ctypes.byref(p), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                           ctypes.c_void_p(work.data_ptr()) if work is not None else None, nx, ny, nz,
                           _stream_ptr(x)), "ig_smooth")
    return out


def smooth_set_path(path):
    """Route of the box and axis-aligned Gaussian smoothing, process-wide
    (ig_smooth_set_path): 0 the fused pass where it applies, 1 three passes."""
    _check(lib().ig_smooth_set_path(int(path)), "ig_smooth_set_path")


def wavelet_params(kind="haar", levels=3, t=(0.5, 0.8, 1.1), rms=0.0):
    p = IgWaveletParams()
    p.struct_size = ctypes.sizeof(IgWaveletParams)
    p.kind = WAVELETS[kind]
    p.levels = int(levels)
    p.reserved = 0
    for l, v in enumerate(t):
        p.t[l] = float(v)
    p.rms = float(rms)
    return p


def _wcall(fn, p, x, out):
    nz, ny, nx = x.shape
    _check(getattr(lib(), fn)(ctypes.byref(p), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), nx, ny,
                              nz, _stream_ptr(x)), fn)
    return out


def wavelet_forward(x, kind="haar", levels=3, out=None):
    """Multi-level lifting transform of an FP32 device cube (ig_wavelet_forward)."""
    import torch
    assert x.dtype == torch.float32 and x.is_contiguous()
    return _wcall("ig_wavelet_forward", wavelet_params(kind, levels), x, torch.empty_like(x) if out is None else out)


def wavelet_inverse(c, kind="haar", levels=3, out=None):
    import torch
    assert c.dtype == torch.float32 and c.is_contiguous()
    return _wcall("ig_wavelet_inverse", wavelet_params(kind, levels), c, torch.empty_like(c) if out is None else out)


def wavelet_denoise(x, kind="haar", levels=3, t=(0.5, 0.8, 1.1), rms=0.0, out=None):
    """Threshold denoiser (ig_wavelet_denoise); returns (output, rms used)."""
    import torch
    assert x.dtype == torch.float32 and x.is_contiguous()
    out = torch.empty_like(x) if out is None else out
    p = wavelet_params(kind, levels, t, rms)
    used = ctypes.c_double()
    nz, ny, nx = x.shape
    _check(lib().ig_wavelet_denoise(ctypes.byref(p), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                    nx, ny, nz, _stream_ptr(x), ctypes.byref(used)), "ig_wavelet_denoise")
    return out, used.value
