"""MI355X-native blocked Gaussian elimination over GF(p) (Linton, Nebe,
Niemeyer, Parker and Thackray, arXiv 1806.04211).

The work runs in ``libgfech.so`` (HIP kernels for gfx950 + the C++ planner);
this package only loads it and marshals arguments.  There is no fallback: if
the library is missing or no gfx950 device is present, calls fail loudly.
"""
from __future__ import annotations

import ctypes
import os

from .api import GfechError, Library, Outputs, Result

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgfech.so")
_library = None


def library() -> Library:
    """The built HIP library (raises if it has not been built)."""
    global _library
    if _library is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "or python paper_1806_04211_amd/build.py")
        _library = Library(ctypes.CDLL(LIB_PATH))
    return _library


def echelonise(A, p: int, **kw) -> Result:
    """Echelonise a host numpy matrix over GF(p) on the GPU."""
    return library().echelonise(A, p, **kw)


def echelonise_tensor(t, p: int, stream=None, **kw) -> Result:
    """Echelonise a uint8 torch tensor resident on the GPU (row-major, stride(1) == 1)."""
    import torch
    if t.device.type != "cuda" or t.dtype != torch.uint8 or t.dim() != 2 or (t.numel() and t.stride(1) != 1):
        raise ValueError("expected a 2-D row-major uint8 tensor on the GPU")
    s = stream if stream is not None else torch.cuda.current_stream(t.device)
    m, n = t.shape
    return library().echelonise_dev(t.data_ptr(), m, n, max(t.stride(0), n, 1), p, stream=s.cuda_stream, **kw)


__all__ = ["GfechError", "Library", "Outputs", "Result", "library", "echelonise", "echelonise_tensor", "LIB_PATH"]
