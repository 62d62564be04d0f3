"""Test infrastructure: the plain CPU oracle for Gaussian elimination over GF(p).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library (``paper_1806_04211_amd``)
never imports it and shares no code with it.

The whole-matrix result is the plain definition of Section 2.2 (Remark 2.3,
Eq. (1)) applied to the full matrix (Section 3.1, Eq. (2)): computed by a
plain Gauss-Jordan elimination in C (``gf_oracle.c``) with the paper's pivot
rule (the first non-zero entry of each row, rows in their original order,
Section 1).  ``jobs.py`` holds the plain definitions of the paper's jobs
(Section 4.1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gf_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc into oracle/_build/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        os.makedirs(_BUILD, exist_ok=True)
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def load_library(path: str):
    """Load and type a compiled oracle library (the default one, or a test variant)."""
    lib = ctypes.CDLL(path)
    i64p = ctypes.POINTER(ctypes.c_int64)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    lib.oracle_echelon.argtypes = [u8p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint32,
                                   i64p, i64p, i64p, u8p, u8p]
    lib.oracle_echelon.restype = ctypes.c_int
    lib.oracle_mad.argtypes = [u8p, u8p, u8p, u8p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                               ctypes.c_uint32]
    lib.oracle_mad.restype = ctypes.c_int
    lib.oracle_check_field.argtypes = [ctypes.c_uint32]
    lib.oracle_check_field.restype = ctypes.c_int
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.oracle_echelon_gf2.argtypes = [u64p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, i64p, i64p, i64p,
                                       u64p, u64p]
    lib.oracle_echelon_gf2.restype = ctypes.c_int
    lib.oracle_mad_gf2.argtypes = [u64p, u64p, u64p, u64p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                   ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
    lib.oracle_mad_gf2.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        _lib = load_library(build())
    return _lib


class OracleError(ValueError):
    pass


_ERRS = {1: "field: p must be a prime <= 251", 2: "range: entry >= p", 3: "out of memory", 4: "bad argument"}


def _u8(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _i64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


@dataclass
class Echelon:
    """Result of the whole-matrix echelonisation (Eq. (2)).

    Standard form: ``E`` (r x n RREF, pivots +1), ``T`` (m x m) with
    ``T @ A = [E; 0]`` mod p; rows of T are the pivot rows by increasing pivot
    column, then the non-selected rows ascending.

    Paper (negative) form, Remark 2.3: ``M`` (r x r), ``K`` ((m-r) x r),
    ``R`` (r x (n-r)) with
    ``[[M,0],[K,1]] [rho; rho_bar] A [gamma^tr gamma_bar^tr] = [[-1, R],[0,0]]``.
    """
    p: int
    m: int
    n: int
    rank: int
    gamma: np.ndarray      # pivot columns, ascending (int64, 0-based)
    rho: np.ndarray        # selected rows, ascending
    E: np.ndarray          # r x n
    T: np.ndarray          # m x m

    @property
    def gamma_bar(self):
        mask = np.ones(self.n, bool)
        mask[self.gamma] = False
        return np.nonzero(mask)[0].astype(np.int64)

    @property
    def rho_bar(self):
        mask = np.ones(self.m, bool)
        mask[self.rho] = False
        return np.nonzero(mask)[0].astype(np.int64)

    @property
    def M(self):
        # -T_top restricted to the selected-row columns (Remark 2.3: M = -(A[rho,gamma])^-1)
        return ((self.p - self.T[: self.rank][:, self.rho].astype(np.int64)) % self.p).astype(np.uint8)

    @property
    def K(self):
        return self.T[self.rank:][:, self.rho].copy()

    @property
    def R(self):
        # negative remnant: E = [1 | -R] after the column permutation
        return ((self.p - self.E[:, self.gamma_bar].astype(np.int64)) % self.p).astype(np.uint8)


def echelonize(A, p: int, lib=None) -> Echelon:
    """Whole-matrix echelonisation with transformation (the oracle proper).
    ``lib`` selects another compiled copy of the oracle (used by the tests
    that plant mistakes in a copy); by default the built oracle is used."""
    A = np.ascontiguousarray(np.asarray(A, dtype=np.uint8))
    if A.ndim != 2:
        raise OracleError("A must be 2-D")
    m, n = A.shape
    lib = lib or _load()
    k = max(1, min(m, n))
    piv = np.zeros(k, np.int64)
    sel = np.zeros(k, np.int64)
    E = np.zeros((max(m, 1), max(n, 1)), np.uint8)
    T = np.zeros((max(m, 1), max(m, 1)), np.uint8)
    r = np.zeros(1, np.int64)
    Ap = A if A.size else np.zeros((1, 1), np.uint8)
    rc = lib.oracle_echelon(_u8(Ap), m, n, max(n, 1), p, _i64(r), _i64(piv), _i64(sel), _u8(E), _u8(T))
    if rc:
        raise OracleError(_ERRS.get(rc, f"error {rc}"))
    r = int(r[0])
    return Echelon(p=p, m=m, n=n, rank=r, gamma=piv[:r].copy(), rho=sel[:r].copy(),
                   E=E[:r, :n].copy(), T=T[:m, :m].copy())


def mad_c(A, B, C, p: int):
    """(A + B @ C) mod p by the C triple loop (a second, independent MAD)."""
    B = np.ascontiguousarray(B, np.uint8)
    C = np.ascontiguousarray(C, np.uint8)
    a, b = B.shape
    b2, d = C.shape
    assert b == b2
    out = np.zeros((a, d), np.uint8)
    lib = _load()
    Ap = None if A is None else np.ascontiguousarray(A, np.uint8)
    rc = lib.oracle_mad(_u8(Ap) if Ap is not None else None, _u8(B), _u8(C), _u8(out), a, b, d, p)
    if rc:
        raise OracleError(_ERRS.get(rc, f"error {rc}"))
    return out


def is_field(p: int) -> bool:
    return _load().oracle_check_field(p) == 0


def _u64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


@dataclass
class EchelonGF2:
    """Result of the packed GF(2) oracle: E (r rows of ceil(n/64) words) and T
    (m rows of ceil(m/64) words), packed least significant bit first; rows as
    Echelon's."""
    m: int
    n: int
    rank: int
    gamma: np.ndarray
    rho: np.ndarray
    E: np.ndarray
    T: np.ndarray


def echelonize_gf2(W, n: int, lib=None) -> EchelonGF2:
    """Whole-matrix echelonisation over GF(2) of packed rows (Section 2.2 with
    p = 2: the same plain Gauss-Jordan, row operations as word XORs)."""
    W = np.ascontiguousarray(np.asarray(W, dtype=np.uint64))
    m = W.shape[0]
    wn, wm = (n + 63) // 64, (m + 63) // 64
    lib = lib or _load()
    k = max(1, min(m, n))
    piv = np.zeros(k, np.int64)
    sel = np.zeros(k, np.int64)
    E = np.zeros((max(m, 1), max(wn, 1)), np.uint64)
    T = np.zeros((max(m, 1), max(wm, 1)), np.uint64)
    r = np.zeros(1, np.int64)
    Wp = W if W.size else np.zeros((1, 1), np.uint64)
    rc = lib.oracle_echelon_gf2(_u64(Wp), m, n, max(W.shape[1] if W.ndim == 2 else 0, wn, 1), _i64(r), _i64(piv),
                                _i64(sel), _u64(E), _u64(T))
    if rc:
        raise OracleError(_ERRS.get(rc, f"error {rc}"))
    r = int(r[0])
    return EchelonGF2(m=m, n=n, rank=r, gamma=piv[:r].copy(), rho=sel[:r].copy(), E=E[:r, :wn].copy(),
                      T=T[:m, :wm].copy())


def mad_gf2(C, A, B, k: int, n: int):
    """(C + A B) over GF(2) on packed rows (C may be None): A has k columns, B and
    C n columns."""
    A = np.ascontiguousarray(A, np.uint64)
    B = np.ascontiguousarray(B, np.uint64)
    m = A.shape[0]
    wn = (n + 63) // 64
    out = np.zeros((m, wn), np.uint64)
    Cp = None if C is None else np.ascontiguousarray(C, np.uint64)
    lib = _load()
    rc = lib.oracle_mad_gf2(_u64(Cp) if Cp is not None else None, _u64(A), _u64(B), _u64(out), m, k, n,
                            A.shape[1], B.shape[1], wn)
    if rc:
        raise OracleError(_ERRS.get(rc, f"error {rc}"))
    return out
