"""Thin Python binding over the C ABI (argument marshalling only).

Every call goes straight to the same-named ``gfech_*`` entry point of a
loaded library; numpy arrays are host buffers, torch tensors on the GPU are
device buffers (their data pointers are passed through).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import _abi


class GfechError(RuntimeError):
    def __init__(self, status: int, detail: str = ""):
        self.status = status
        super().__init__(f"{_abi.STATUS_NAMES.get(status, status)}: {detail}")


@dataclass
class Outputs:
    """Everything a result holds, copied to host numpy arrays."""
    p: int
    m: int
    n: int
    rank: int
    gamma: np.ndarray
    rho: np.ndarray
    gamma_bar: np.ndarray
    rho_bar: np.ndarray
    R: np.ndarray | None
    M: np.ndarray | None
    K: np.ndarray | None
    E: np.ndarray | None = None
    T: np.ndarray | None = None
    variant: int = 0


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


class Result:
    """Owns one gfech_result*."""

    def __init__(self, lib, handle: int):
        self._lib = lib
        self._h = ctypes.c_void_p(handle)

    def __del__(self):
        self.free()

    def free(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.gfech_result_free(self._h)
            self._h = ctypes.c_void_p(0)

    def _check(self, st):
        if st != _abi.GFECH_OK:
            raise GfechError(st, self._lib.gfech_last_error().decode())

    @property
    def rank(self) -> int:
        return int(self._lib.gfech_rank(self._h))

    def shape(self):
        m, n, p = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_uint32()
        self._check(self._lib.gfech_shape(self._h, ctypes.byref(m), ctypes.byref(n), ctypes.byref(p)))
        return m.value, n.value, p.value

    def stats(self) -> dict:
        s = _abi.Stats()
        self._check(self._lib.gfech_get_stats(self._h, ctypes.byref(s)))
        return {name: getattr(s, name) for name, _ in _abi.Stats._fields_}

    def view(self) -> _abi.View:
        v = _abi.View()
        self._check(self._lib.gfech_device_view(self._h, ctypes.byref(v)))
        return v

    def pivots(self):
        r = self.rank
        g = np.zeros(r, np.int64)
        rho = np.zeros(r, np.int64)
        self._check(self._lib.gfech_pivots(self._h, _ptr(g), _ptr(rho)))
        return g, rho

    def nonpivots(self):
        m, n, _ = self.shape()
        r = self.rank
        gb = np.zeros(n - r, np.int64)
        rb = np.zeros(m - r, np.int64)
        self._check(self._lib.gfech_nonpivots(self._h, _ptr(gb), _ptr(rb)))
        return gb, rb

    def get_R(self):
        m, n, _ = self.shape()
        r = self.rank
        out = np.zeros((r, n - r), np.uint8)
        self._check(self._lib.gfech_get_R(self._h, _ptr(out), max(n - r, 1)))
        return out

    def get_M(self):
        r = self.rank
        out = np.zeros((r, r), np.uint8)
        self._check(self._lib.gfech_get_M(self._h, _ptr(out), max(r, 1)))
        return out

    def get_K(self):
        m, n, _ = self.shape()
        r = self.rank
        out = np.zeros((m - r, r), np.uint8)
        self._check(self._lib.gfech_get_K(self._h, _ptr(out), max(r, 1)))
        return out

    def expand_rref(self):
        m, n, _ = self.shape()
        out = np.zeros((self.rank, n), np.uint8)
        self._check(self._lib.gfech_expand_rref(self._h, _ptr(out), max(n, 1)))
        return out

    def expand_transform(self):
        m, n, _ = self.shape()
        out = np.zeros((m, m), np.uint8)
        self._check(self._lib.gfech_expand_transform(self._h, _ptr(out), max(m, 1)))
        return out

    def expand_rref_dev(self, out_ptr: int, lde: int, stream: int = 0):
        self._check(self._lib.gfech_expand_rref_dev(self._h, ctypes.c_void_p(out_ptr), lde, ctypes.c_void_p(stream)))

    def expand_transform_dev(self, out_ptr: int, ldt: int, stream: int = 0):
        self._check(self._lib.gfech_expand_transform_dev(self._h, ctypes.c_void_p(out_ptr), ldt,
                                                         ctypes.c_void_p(stream)))

    def outputs(self, expand: bool = True) -> Outputs:
        """Every output the result's variant includes (the others are None)."""
        m, n, p = self.shape()
        g, rho = self.pivots()
        gb, rb = self.nonpivots()
        v = int(self.stats()["variant"])
        has_r, has_t = v != _abi.WANT_RANK, v == _abi.WANT_RREF_T
        o = Outputs(p=p, m=m, n=n, rank=self.rank, gamma=g, rho=rho, gamma_bar=gb, rho_bar=rb,
                    R=self.get_R() if has_r else None, M=self.get_M() if has_t else None,
                    K=self.get_K() if has_t else None, variant=v)
        if expand:
            o.E = self.expand_rref() if has_r else None
            o.T = self.expand_transform() if has_t else None
        return o


def _opts(block_rows=0, block_cols=0, skip_range_check=False, profile=False, variant=0, timeout_ms=0):
    o = _abi.Opts()
    o.timeout_ms = int(timeout_ms)
    o.block_rows = int(block_rows)
    o.block_cols = int(block_cols)
    o.skip_range_check = 1 if skip_range_check else 0
    o.profile = int(profile)
    o.variant = int(variant)
    return o


class Library:
    """Calls into one loaded gfech library."""

    def __init__(self, lib):
        self.lib = _abi.declare(lib)

    def backend_name(self) -> str:
        return self.lib.gfech_backend_name().decode()

    def _check(self, st):
        if st != _abi.GFECH_OK:
            raise GfechError(st, self.lib.gfech_last_error().decode())

    def echelonise(self, A, p: int, block_rows=0, block_cols=0, variant=0, timeout_ms=0) -> Result:
        """A: host numpy (m x n, uint8).  variant: _abi.WANT_* (what is computed);
        timeout_ms > 0: the watchdog (GFECH_E_CANCELLED when it fires)."""
        A = np.ascontiguousarray(np.asarray(A, dtype=np.uint8))
        m, n = A.shape
        out = ctypes.c_void_p()
        o = _opts(block_rows, block_cols, variant=variant, timeout_ms=timeout_ms)
        self._check(self.lib.gfech_echelonise_u8(_ptr(A), m, n, max(n, 1), p, ctypes.byref(o), ctypes.byref(out)))
        return Result(self.lib, out.value)

    def echelonise_dev(self, ptr: int, m: int, n: int, lda: int, p: int, stream: int = 0, block_rows=0,
                       block_cols=0, skip_range_check=False, profile=False, variant=0, timeout_ms=0) -> Result:
        """ptr: device address of an m x n uint8 matrix with leading dimension lda."""
        out = ctypes.c_void_p()
        o = _opts(block_rows, block_cols, skip_range_check, profile, variant, timeout_ms)
        self._check(self.lib.gfech_echelonise_u8_dev(ctypes.c_void_p(ptr), m, n, lda, p, ctypes.byref(o),
                                                     ctypes.c_void_p(stream), ctypes.byref(out)))
        return Result(self.lib, out.value)

    def echelonise_gf2(self, W, n: int, block_rows=0, block_cols=0, variant=0, skip_range_check=False) -> Result:
        """W: host numpy uint64 (m x words), GF(2) rows packed least significant bit first."""
        W = np.ascontiguousarray(np.asarray(W, dtype=np.uint64))
        m = W.shape[0]
        ldw = W.shape[1] if W.ndim == 2 else 0
        out = ctypes.c_void_p()
        o = _opts(block_rows, block_cols, skip_range_check, variant=variant)
        self._check(self.lib.gfech_echelonise_gf2(_ptr(W), m, n, max(ldw, (n + 63) // 64, 1), ctypes.byref(o),
                                                  ctypes.byref(out)))
        return Result(self.lib, out.value)

    def echelonise_gf2_dev(self, ptr: int, m: int, n: int, ldw: int, stream: int = 0, block_rows=0, block_cols=0,
                           variant=0, skip_range_check=False) -> Result:
        """ptr: device address of m rows of ldw uint64 words (GF(2), packed)."""
        out = ctypes.c_void_p()
        o = _opts(block_rows, block_cols, skip_range_check, variant=variant)
        self._check(self.lib.gfech_echelonise_gf2_dev(ctypes.c_void_p(ptr), m, n, ldw, ctypes.byref(o),
                                                      ctypes.c_void_p(stream), ctypes.byref(out)))
        return Result(self.lib, out.value)

    def mad_dev(self, M, N, K, p, A, lda, B, ldb, D, ldd, C=0, ldc=0, brow=0, crow=0, stream=0):
        """MAD job on device addresses: D = (C + A B) mod p (C = 0 means none)."""
        self._check(self.lib.gfech_mad_dev(M, N, K, p, ctypes.c_void_p(A), lda, ctypes.c_void_p(B), ldb,
                                           ctypes.c_void_p(brow), ctypes.c_void_p(C), ldc, ctypes.c_void_p(crow),
                                           ctypes.c_void_p(D), ldd, ctypes.c_void_p(stream)))

    @staticmethod
    def mad_descs(descs):
        """A gfech_mad_desc array from dicts with its fields (device addresses)."""
        arr = (_abi.MadDesc * max(len(descs), 1))()
        for t, d in enumerate(descs):
            for k, v in d.items():
                setattr(arr[t], k, v)
        return arr

    def mad_batch_dev(self, descs, stream=0):
        """descs: list of dicts with the gfech_mad_desc fields, or an array from mad_descs."""
        arr = descs if isinstance(descs, ctypes.Array) else self.mad_descs(descs)
        self._check(self.lib.gfech_mad_batch_dev(len(descs), arr, ctypes.c_void_p(stream)))

    def mad_batch_dev_timed(self, descs, stream=0) -> float:
        """mad_batch_dev, returning the summed execution time (ms) of its MAD kernel launches."""
        arr = descs if isinstance(descs, ctypes.Array) else self.mad_descs(descs)
        ms = ctypes.c_double()
        self._check(self.lib.gfech_mad_batch_dev_timed(len(descs), arr, ctypes.c_void_p(stream), ctypes.byref(ms)))
        return ms.value

    def mad_gf2_dev(self, M, N, K, A, lda, B, ldb, D, ldd, C=0, ldc=0, stream=0):
        """MAD over GF(2) on packed rows (device addresses, leading dimensions in 64-bit words)."""
        vp = ctypes.c_void_p
        self._check(self.lib.gfech_mad_gf2_dev(M, N, K, vp(A), lda, vp(B), ldb, vp(C), ldc, vp(D), ldd, vp(stream)))

    def ech_dev(self, H, rows, cols, ldh, p, prow, qrow, pcol, qcol, M, ldm, K, ldk, R, ldr, stream=0) -> int:
        """ECH job on device addresses; returns the rank."""
        r = ctypes.c_int64()
        vp = ctypes.c_void_p
        self._check(self.lib.gfech_ech_dev(vp(H), rows, cols, ldh, p, vp(prow), vp(qrow), vp(pcol), vp(qcol),
                                           vp(M), ldm, vp(K), ldk, vp(R), ldr, ctypes.byref(r), vp(stream)))
        return r.value

    def ech_dev_noalloc(self, H, rows, cols, ldh, p, prow, qrow, pcol, qcol, M, ldm, K, ldk, R, ldr, rank_dev,
                        stream=0):
        """ECH job on device addresses with the library's fixed workspace; the rank
        goes to the device int32 at rank_dev; the work is queued on `stream`."""
        vp = ctypes.c_void_p
        self._check(self.lib.gfech_ech_dev_noalloc(vp(H), rows, cols, ldh, p, vp(prow), vp(qrow), vp(pcol),
                                                   vp(qcol), vp(M), ldm, vp(K), ldk, vp(R), ldr, vp(rank_dev),
                                                   vp(stream)))

    def server(self, hbm_budget_bytes: int = 0, max_active: int = 0, size_classes: int = 0) -> "Server":
        return Server(self, hbm_budget_bytes, max_active, size_classes)

    def echelonise_batch(self, problems, on_device: bool = False, stream: int = 0, block_rows=0, block_cols=0,
                         profile=False, variant=0):
        """problems: list of (A, p) with A a host numpy array (on_device=False) or
        (ptr, m, n, lda, p) tuples (on_device=True).  Returns (results, statuses)."""
        cnt = len(problems)
        arr = (_abi.Problem * max(cnt, 1))()
        keep = []
        for t, pr in enumerate(problems):
            if on_device:
                ptr, m, n, lda, p = pr
                arr[t].A = ptr
            else:
                A, p = pr
                A = np.ascontiguousarray(np.asarray(A, np.uint8))
                keep.append(A)
                m, n = A.shape
                lda = max(n, 1)
                arr[t].A = A.ctypes.data if A.size else 0
            arr[t].m, arr[t].n, arr[t].lda, arr[t].p = m, n, lda, p
        outs = (ctypes.c_void_p * max(cnt, 1))()
        sts = (ctypes.c_int * max(cnt, 1))()
        o = _opts(block_rows, block_cols, profile=profile, variant=variant)
        self.lib.gfech_echelonise_batch(cnt, arr, 1 if on_device else 0, ctypes.byref(o), ctypes.c_void_p(stream),
                                        outs, sts)
        res = [Result(self.lib, outs[t]) if outs[t] else None for t in range(cnt)]
        return res, [int(sts[t]) for t in range(cnt)]


class Server:
    """Owns one gfech_server* (continuous batching of elimination requests)."""

    def __init__(self, lib: "Library", hbm_budget_bytes: int = 0, max_active: int = 0, size_classes: int = 0):
        self._lib = lib.lib
        cfg = _abi.ServerCfg()
        cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        cfg.max_active = int(max_active)
        cfg.size_classes = int(size_classes)
        out = ctypes.c_void_p()
        st = self._lib.gfech_server_create(ctypes.byref(cfg), ctypes.byref(out))
        if st != _abi.GFECH_OK:
            raise GfechError(st, self._lib.gfech_last_error().decode())
        self._h = out

    def _check(self, st):
        if st != _abi.GFECH_OK:
            raise GfechError(st, self._lib.gfech_last_error().decode())

    def submit(self, A, p: int) -> int:
        """A: host numpy array (m x n uint8).  Returns the ticket."""
        A = np.ascontiguousarray(np.asarray(A, np.uint8))
        m, n = A.shape
        pr = _abi.Problem()
        pr.A = A.ctypes.data if A.size else 0
        pr.m, pr.n, pr.lda, pr.p = m, n, max(n, 1), p
        t = ctypes.c_uint64()
        self._check(self._lib.gfech_server_submit(self._h, ctypes.byref(pr), 0, ctypes.byref(t)))
        return t.value

    def submit_dev(self, ptr: int, m: int, n: int, lda: int, p: int) -> int:
        """ptr: device address of an m x n uint8 matrix.  Returns the ticket."""
        pr = _abi.Problem()
        pr.A = ptr
        pr.m, pr.n, pr.lda, pr.p = m, n, lda, p
        t = ctypes.c_uint64()
        self._check(self._lib.gfech_server_submit(self._h, ctypes.byref(pr), 1, ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int):
        """The Result when finished, else None."""
        out = ctypes.c_void_p()
        self._check(self._lib.gfech_server_poll(self._h, ticket, ctypes.byref(out)))
        return Result(self._lib, out.value) if out.value else None

    def stats(self) -> dict:
        s = _abi.ServerStats()
        self._check(self._lib.gfech_server_get_stats(self._h, ctypes.byref(s)))
        return {name: getattr(s, name) for name, _ in _abi.ServerStats._fields_}

    def cancel(self, ticket: int):
        self._check(self._lib.gfech_server_cancel(self._h, ticket))

    def wait(self, ticket: int) -> Result:
        out = ctypes.c_void_p()
        self._check(self._lib.gfech_server_wait(self._h, ticket, ctypes.byref(out)))
        return Result(self._lib, out.value)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.gfech_server_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        self.close()
