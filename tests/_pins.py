"""Independent checks that pin the oracle (and, reused, any echelon result).

Everything here avoids the oracle's own arithmetic: row spaces are
enumerated by brute force, rank counts come from the closed form for the
number of m x n matrices of rank r over F_q, and products use numpy int64.
"""
from __future__ import annotations

import itertools
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def matmul_mod(A, B, p):
    return (np.asarray(A, np.int64) @ np.asarray(B, np.int64)) % p


def rowspace(A, p):
    """Set of all F_p-linear combinations of the rows of A (brute force)."""
    A = np.asarray(A, np.int64)
    m, n = A.shape
    out = set()
    for coeffs in itertools.product(range(p), repeat=m):
        v = (np.asarray(coeffs, np.int64) @ A) % p if m else np.zeros(n, np.int64)
        out.add(tuple(int(x) for x in v))
    return out


def brute_rank(A, p):
    size = len(rowspace(A, p))
    r = 0
    while p ** r < size:
        r += 1
    assert p ** r == size
    return r


def count_rank(q, m, n, r):
    """Number of m x n matrices of rank r over F_q (standard closed form)."""
    num = 1
    den = 1
    for i in range(r):
        num *= (q ** m - q ** i) * (q ** n - q ** i)
        den *= (q ** r - q ** i)
    return num // den


def all_matrices(p, m, n):
    for entries in itertools.product(range(p), repeat=m * n):
        yield np.asarray(entries, np.uint8).reshape(m, n)


def is_rref(E, gamma, p):
    """E (r x n) is in reduced row echelon form with pivots +1 at gamma."""
    E = np.asarray(E, np.int64)
    r = E.shape[0]
    if len(gamma) != r:
        return False
    if r and np.any(np.diff(gamma) <= 0):
        return False
    for t in range(r):
        c = int(gamma[t])
        if np.any(E[t, :c] != 0) or E[t, c] != 1:
            return False
        col = E[:, c].copy()
        col[t] = 0
        if np.any(col != 0):
            return False
    return True


def check_result(A, p, rank, gamma, rho, E, T, *, who="result"):
    """Structural identities every correct result satisfies (Eq. (2) and the
    standard-form relations).  Raises AssertionError naming the first failure."""
    A = np.asarray(A, np.int64)
    m, n = A.shape
    r = int(rank)
    gamma = np.asarray(gamma, np.int64)
    rho = np.asarray(rho, np.int64)
    E = np.asarray(E, np.int64).reshape(r, n)
    T = np.asarray(T, np.int64).reshape(m, m)
    assert len(gamma) == r and len(rho) == r, f"{who}: pivot counts"
    assert is_rref(E, gamma, p), f"{who}: E not in RREF"
    TA = matmul_mod(T, A, p)
    assert np.array_equal(TA[:r], E % p), f"{who}: T*A top != E"
    assert not np.any(TA[r:]), f"{who}: T*A bottom != 0"
    rho_bar = np.setdiff1d(np.arange(m), rho)
    assert not np.any(T[:r][:, rho_bar]), f"{who}: T_top on non-selected columns != 0"
    assert np.array_equal(T[r:][:, rho_bar], np.eye(m - r, dtype=np.int64)), f"{who}: T_bot identity part"
    # Eq. (2) with explicit permutation matrices
    gamma_bar = np.setdiff1d(np.arange(n), gamma)
    M = (-T[:r][:, rho]) % p
    K = T[r:][:, rho]
    R = (-E[:, gamma_bar]) % p
    Prho = np.zeros((m, m), np.int64)
    Prho[np.arange(m), np.concatenate([rho, rho_bar])] = 1
    Pgam = np.zeros((n, n), np.int64)
    Pgam[np.concatenate([gamma, gamma_bar]), np.arange(n)] = 1
    L = np.zeros((m, m), np.int64)
    L[:r, :r] = M
    L[r:, :r] = K
    L[r:, r:] = np.eye(m - r, dtype=np.int64)
    lhs = matmul_mod(matmul_mod(matmul_mod(L, Prho, p), A, p), Pgam, p)
    rhs = np.zeros((m, n), np.int64)
    rhs[:r, :r] = (-np.eye(r, dtype=np.int64)) % p
    rhs[:r, r:] = R
    assert np.array_equal(lhs, rhs), f"{who}: Eq. (2) identity"


def lex_first_basis(A, p):
    """Rows i with A_i outside span(A_0..A_{i-1}), by brute-force row spaces."""
    A = np.asarray(A, np.int64)
    sel = []
    prev = {tuple([0] * A.shape[1])}
    for i in range(A.shape[0]):
        cur = rowspace(A[: i + 1], p)
        if len(cur) > len(prev):
            sel.append(i)
        prev = cur
    return np.asarray(sel, np.int64)
