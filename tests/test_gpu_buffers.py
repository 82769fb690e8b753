"""Entry points reject buffers that are not device memory of the call's device
(here: host memory, plain and pinned) with IG_ERR_INVALID_ARG before any
kernel runs, and leave the runtime's error state clean for the next call."""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1609_03782_amd as ig
    ig.lib()
    return torch.device("cuda:0")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_run_rejects_host_buffers(dev):
    import torch
    import paper_1609_03782_amd as ig
    L = ig.lib()
    shape = (8, 9, 10)
    f = ig.Filter(shape, K=2.0, tau=1 / 16, n_iter=3)
    x = torch.randn(shape, device=dev)
    y = torch.empty_like(x)
    host = np.zeros(shape, np.float32)
    pinned = torch.zeros(shape, pin_memory=True)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for name, a, b in [("host input", host.ctypes.data, y.data_ptr()),
                       ("host output", x.data_ptr(), host.ctypes.data),
                       ("pinned input", pinned.data_ptr(), y.data_ptr())]:
        _say(f"ig_filter_run with {name}")
        rc = L.ig_filter_run(f._h, ctypes.c_void_p(a), ctypes.c_void_p(b), stream, None)
        assert rc == ig.IG_ERR_INVALID_ARG, name
        assert b"device memory" in L.ig_last_error() or b"runtime knows" in L.ig_last_error()
    # the handle and the runtime still work
    ref = f.run(x)
    torch.cuda.synchronize()
    assert torch.isfinite(ref).all()
    f.close()


def test_smooth_quality_wavelet_reject_host_buffers(dev):
    import torch
    import paper_1609_03782_amd as ig
    shape = (6, 7, 8)
    x = torch.randn(shape, device=dev)
    host = torch.zeros(shape)            # CPU tensor: host memory
    _say("smooth with a host output")
    with pytest.raises(ig.IgError) as ei:
        ig.smooth(x, "box", (3, 3, 3), out=host)
    assert ei.value.status == ig.IG_ERR_INVALID_ARG
    _say("quality with a host filtered cube")
    with pytest.raises(ig.IgError) as ei:
        ig.quality(x, host, thr_f=[0.5])
    assert ei.value.status == ig.IG_ERR_INVALID_ARG
    _say("wavelet forward with a host output")
    with pytest.raises(ig.IgError) as ei:
        ig.wavelet_forward(x, "haar", 1, out=host)
    assert ei.value.status == ig.IG_ERR_INVALID_ARG
    y = ig.smooth(x, "box", (3, 3, 3))
    torch.cuda.synchronize()
    assert torch.isfinite(y).all()
