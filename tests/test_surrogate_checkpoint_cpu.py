"""Host-only checks of the surrogate checkpoint format (no GPU): files written
here by the layout that include/igsurrogate.h documents are read back by
ig_surrogate_checkpoint_info, and every corruption of header, size or body is
refused.  The GPU round trip (save, load, resume bit for bit) is in
tests/test_gpu_surrogate.py."""
import ctypes
import struct

import numpy as np
import pytest

from paper_1609_03782_amd import surrogate as sg

FNV_BASIS, FNV_PRIME = 14695981039346656037, 1099511628211


def _fnv1a(data: bytes) -> int:
    h = FNV_BASIS
    for b in data:
        h = ((h ^ b) * FNV_PRIME) & 0xFFFFFFFFFFFFFFFF
    return h


def _file(path, depth=8, width=32, nparam=None, step=17, seed=5, magic=b"IGSURR\0\1", version=1, body=None,
          hash_fix=True):
    if nparam is None:
        nparam = sum(27 * ci * co + co for (ci, co) in
                     [(1 if l == 0 else width, 1 if l == depth - 1 else width) for l in range(depth)])
    hdr = magic + struct.pack("<IIiiqqQffff", 64, version, depth, width, nparam, step, seed, 1e-3, 0.9, 0.999, 1e-8)
    assert len(hdr) == 64
    if body is None:
        body = np.arange(3 * nparam, dtype=np.float32).tobytes()
    data = hdr + body
    h = _fnv1a(data) if hash_fix else 0
    path.write_bytes(data + struct.pack("<Q", h))
    return nparam


def test_fnv1a_reference_vector():
    # published FNV-1a 64 test vectors: "" and "a"
    assert _fnv1a(b"") == 0xcbf29ce484222325
    assert _fnv1a(b"a") == 0xaf63dc4c8601ec8c


def test_info_reads_a_valid_file(tmp_path):
    p = tmp_path / "net.ckpt"
    n = _file(p, depth=3, step=123, seed=99)
    assert n == 27 * 1 * 32 + 32 + 27 * 32 * 32 + 32 + 27 * 32 * 1 + 1
    info = sg.checkpoint_info(p)
    assert info == {"depth": 3, "width": 32, "nparam": n, "step": 123, "seed": 99}


@pytest.mark.parametrize("case", ["magic", "version", "truncated", "flipped", "depth", "width", "size"])
def test_info_rejects_corruption(tmp_path, case):
    import paper_1609_03782_amd as ig
    p = tmp_path / "bad.ckpt"
    if case == "magic":
        _file(p, magic=b"IGSURR\0\2")
    elif case == "version":
        _file(p, version=2)
    elif case == "depth":
        _file(p, depth=1, nparam=100)
    elif case == "width":
        _file(p, width=16, nparam=100)
    elif case == "size":      # header promises more parameters than the body holds
        _file(p, depth=2, nparam=2000, body=np.zeros(3 * 1000, np.float32).tobytes())
    else:
        _file(p, depth=2)
        raw = bytearray(p.read_bytes())
        if case == "truncated":
            raw = raw[:-9]
        else:
            raw[100] ^= 0x10   # one bit of the body
        p.write_bytes(bytes(raw))
    with pytest.raises(ig.IgError) as ei:
        sg.checkpoint_info(p)
    assert ei.value.status == ig.IG_ERR_INVALID_ARG


def test_missing_file_and_null_arguments(tmp_path):
    import paper_1609_03782_amd as ig
    L = sg.slib()
    assert L.ig_surrogate_checkpoint_info(str(tmp_path / "none").encode(), None, None, None, None,
                                          None) == ig.IG_ERR_INVALID_ARG
    assert L.ig_surrogate_checkpoint_info(None, None, None, None, None, None) == ig.IG_ERR_INVALID_ARG
    assert L.ig_surrogate_save(None, b"x") == ig.IG_ERR_INVALID_ARG
    assert L.ig_surrogate_load(None, b"x") == ig.IG_ERR_INVALID_ARG
    assert L.ig_surrogate_set_lr(None, ctypes.c_float(1e-3)) == ig.IG_ERR_INVALID_ARG
    assert L.ig_surrogate_get_step(None) == -1
    assert L.ig_surrogate_set_clip(None, ctypes.c_float(1.0)) == ig.IG_ERR_INVALID_ARG
    assert L.ig_surrogate_last_grad_norm(None, None) == ig.IG_ERR_INVALID_ARG
