"""Helpers for the GPU tests: device buffers from numpy, and the library."""
import numpy as np
import pytest


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def gpu_library():
    torch_cuda()
    import paper_1806_04211_amd as gf
    lib = gf.library()
    assert lib.backend_name() == "hip-gfx950"
    return lib


def dev(torch, a, pad=0):
    """numpy -> cuda uint8/int32 tensor (optionally with `pad` extra trailing elements)."""
    a = np.ascontiguousarray(a)
    flat = np.concatenate([a.ravel(), np.zeros(pad, a.dtype)]) if pad else a.ravel()
    return torch.from_numpy(flat.copy()).to("cuda:0")


def say(msg):
    print(msg, flush=True)
