"""The C ABI library loads and exports every symbol include/gfech.h declares
(no compute is run here), and the product path has no CPU fallback."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gfech.h")
LIB = os.path.join(ROOT, "paper_1806_04211_amd", "libgfech.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(gfech_[A-Za-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared()
    for must in ("gfech_echelonise_u8", "gfech_echelonise_u8_dev", "gfech_echelonise_batch", "gfech_rank",
                 "gfech_pivots", "gfech_get_R", "gfech_get_M", "gfech_get_K", "gfech_expand_rref",
                 "gfech_expand_transform", "gfech_result_free", "gfech_mad_dev", "gfech_ech_dev",
                 "gfech_echelonise_gf2", "gfech_echelonise_gf2_dev"):
        assert must in names


@pytest.fixture(scope="module")
def built():
    if not os.path.exists(LIB):
        from paper_1806_04211_amd import build
        build.build()
    return LIB


def test_library_exports_every_declared_symbol(built):
    out = subprocess.check_output(["nm", "-D", "--defined-only", built], text=True)
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


def test_library_loads_and_binds(built):
    from paper_1806_04211_amd import _abi
    lib = _abi.declare(ctypes.CDLL(built))
    assert lib.gfech_strerror(3) == b"input entry >= p"
    assert set(_abi.SIGNATURES) <= set(declared())


def test_emulator_exports_the_same_symbols():
    from tests import emu
    out = subprocess.check_output(["nm", "-D", "--defined-only", emu.build()], text=True)
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    assert not [n for n in declared() if n not in exported]


def test_product_fails_loudly_without_gpu(built):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_1806_04211_amd as gf
    with pytest.raises(gf.GfechError) as ex:
        gf.echelonise(np.eye(4, dtype=np.uint8), 5)
    assert ex.value.status == 6          # GFECH_E_DEVICE, never a CPU answer
    assert gf.library().backend_name() == "unavailable"
