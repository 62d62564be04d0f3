"""Test infrastructure: plain definitions of the paper's jobs (Section 4.1).

Each function is the job's definition written out with numpy, 0-based, for
checking single GPU kernels and for tracing the worked example of
Section 2.2.  Index sets are ascending int arrays (Definition 2.1); bit
strings are uint8 arrays.

Readings of the paper used here (the text is inconsistent about bit
polarity): every bit string marks *new* elements with 1 and old ones with 0,
as UNH defines it.  RRF places its first matrix at the 0s, CRZ places the
existing columns at the 0s and zero columns at the 1s, ADI writes the
identity at the 1s, and MKR returns 0 for the elements of the smaller set.
"""
from __future__ import annotations

import numpy as np

from . import echelonize


def _u8(x):
    return np.asarray(x, dtype=np.int64)


def mul(A, B, p):
    """MUL: A x B mod p."""
    return ((_u8(A) @ _u8(B)) % p).astype(np.uint8)


def mad(A, B, C, p):
    """MAD: A + B x C mod p."""
    return ((_u8(A) + _u8(B) @ _u8(C)) % p).astype(np.uint8)


def ech(H, p):
    """ECH of Remark 2.3: returns (M, K, R, rho, gamma) with
    [[M,0],[K,1]] [rho; rho_bar] H [gamma^tr gamma_bar^tr] = [[-1, R],[0,0]]."""
    e = echelonize(H, p)
    return e.M, e.K, e.R, e.rho, e.gamma


def complement(S, size):
    mask = np.ones(size, bool)
    mask[np.asarray(S, np.int64)] = False
    return np.nonzero(mask)[0].astype(np.int64)


def cex(H, gamma):
    """CEX: (H x gamma^tr, H x gamma_bar^tr)."""
    H = np.asarray(H)
    g = np.asarray(gamma, np.int64)
    return H[:, g].copy(), H[:, complement(g, H.shape[1])].copy()


def rex(H, rho):
    """REX: (rho x H, rho_bar x H)."""
    H = np.asarray(H)
    r = np.asarray(rho, np.int64)
    return H[r].copy(), H[complement(r, H.shape[0])].copy()


def unh(rho1, rho2, alpha):
    """UNH: rho = rho1 united with the rho2-th elements of the complement of rho1;
    u marks the elements not in rho1 with 1."""
    rho1 = np.asarray(rho1, np.int64)
    x = complement(rho1, alpha)
    new = x[np.asarray(rho2, np.int64)]
    rho = np.sort(np.concatenate([rho1, new]))
    u = (~np.isin(rho, rho1)).astype(np.uint8)
    return rho, u


def un0(rho2, alpha):
    """UN0: UNH with an empty first set."""
    return unh(np.zeros(0, np.int64), rho2, alpha)


def mkr(rho1, rho2):
    """MKR for rho1 a subset of rho2: 0 at the elements of rho1, 1 at the new ones."""
    rho2 = np.asarray(rho2, np.int64)
    return (~np.isin(rho2, np.asarray(rho1, np.int64))).astype(np.uint8)


def rrf(u, B, C):
    """RRF: rows of B at the 0s of u, rows of C at the 1s, in order."""
    u = np.asarray(u, np.uint8)
    B = np.asarray(B)
    C = np.asarray(C)
    cols = B.shape[1] if B.ndim == 2 and B.shape[0] else C.shape[1]
    out = np.zeros((len(u), cols), np.uint8)
    out[u == 0] = B.reshape(-1, cols)
    out[u == 1] = C.reshape(-1, cols)
    return out


def crz(K, delta):
    """CRZ: existing columns of K at the 0s of delta, zero columns at the 1s."""
    delta = np.asarray(delta, np.uint8)
    K = np.asarray(K)
    out = np.zeros((K.shape[0], len(delta)), np.uint8)
    out[:, delta == 0] = K
    return out


def adi(V, delta):
    """ADI: V[t, position of the t-th 1 of delta] := 1."""
    V = np.array(V, dtype=np.uint8, copy=True)
    pos = np.nonzero(np.asarray(delta, np.uint8) == 1)[0]
    for t, c in enumerate(pos):
        V[t, c] = 1
    return V
