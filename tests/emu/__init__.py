"""Test-only build of the planner with the CPU emulator backend.

``libgfech_emu.so`` = the product's planner and C ABI sources + a plain-loop
backend (``cpu_backend.cpp``).  Only CPU tests load it, to check the Chief's
bookkeeping without a GPU; the product binding never loads it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1806_04211_amd", "csrc")
SRCS = [os.path.join(CSRC, "chief.cpp"), os.path.join(CSRC, "api.cpp"), os.path.join(HERE, "cpu_backend.cpp")]
DEPS = SRCS + [os.path.join(CSRC, "backend.h"), os.path.join(CSRC, "chief.h"),
               os.path.join(ROOT, "include", "gfech.h")]
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(BUILD, "libgfech_emu.so")


def build(force: bool = False, extra_flags=()) -> str:
    newest = max(os.path.getmtime(p) for p in DEPS)
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < newest:
        os.makedirs(BUILD, exist_ok=True)
        tmp = LIB + f".tmp{os.getpid()}"
        cmd = ["g++", "-O1", "-g", "-std=c++17", "-shared", "-fPIC", "-pthread", "-Wall", "-Wno-unused-function",
               *extra_flags, "-o", tmp, *SRCS]
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    return LIB


_lib = None


def library():
    """The emulator build wrapped in the package's Python binding."""
    global _lib
    if _lib is None:
        from paper_1806_04211_amd.api import Library
        _lib = Library(ctypes.CDLL(build()))
    return _lib
