"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds none of the elimination method's arithmetic: it only turns
(seed, stream, index) into field elements and builds the matrix families
the workloads need.  The paper uses uniformly random dense matrices and
states no distribution or seed; these generators fix one.

Generator: SplitMix64 (Steele, Lea and Flood, 2014).  The stream key is
``key = mix64(seed * 2**32 + stream)``; entry ``t`` (row-major index) takes
the SplitMix64 output ``mix64(key + (t + 1) * GAMMA)`` and maps its top 32
bits to [0, p) by the multiply-shift method (Lemire 2019) without the
rejection step, a bias below p / 2**32.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)
_PRIMES_251 = [q for q in range(2, 252) if all(q % d for d in range(2, int(q ** 0.5) + 1))]


def mix64(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, stream: int) -> np.uint64:
    return mix64(np.uint64((int(seed) << 32) + int(stream)) & np.uint64(0xFFFFFFFFFFFFFFFF))


def words(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    """SplitMix64 outputs for counters start..start+count-1."""
    key = stream_key(seed, stream)
    t = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(key + t * GAMMA)


def bounded(w: np.ndarray, p: int) -> np.ndarray:
    """Map 64-bit words to [0, p): (top32(w) * p) >> 32."""
    return (((w >> np.uint64(32)) * np.uint64(p)) >> np.uint64(32)).astype(np.uint8)


def uniform(seed: int, stream: int, m: int, n: int, p: int) -> np.ndarray:
    """m x n matrix with i.i.d. entries uniform in [0, p) (row-major counters)."""
    if m * n == 0:
        return np.zeros((m, n), np.uint8)
    return bounded(words(seed, stream, 0, m * n), p).reshape(m, n)


def uniform_rows(seed: int, stream: int, row0: int, rows: int, n: int, p: int) -> np.ndarray:
    """Rows row0..row0+rows-1 of ``uniform(seed, stream, *, n, p)`` (same counters)."""
    if rows * n == 0:
        return np.zeros((rows, n), np.uint8)
    return bounded(words(seed, stream, row0 * n, rows * n), p).reshape(rows, n)


def low_rank_product(seed: int, m: int, n: int, k: int, p: int) -> np.ndarray:
    """B @ C mod p with B (m x k) from stream 1 and C (k x n) from stream 2 (rank <= k).
    The product is formed in float64, exact while k (p - 1)^2 < 2^53 (every
    partial sum is then an integer below 2^53), else in int64."""
    if k * (p - 1) ** 2 < 2 ** 53:
        B = uniform(seed, 1, m, k, p).astype(np.float64)
        C = uniform(seed, 2, k, n, p).astype(np.float64)
        return np.remainder(B @ C, p).astype(np.uint8)
    B = uniform(seed, 1, m, k, p).astype(np.int64)
    C = uniform(seed, 2, k, n, p).astype(np.int64)
    return ((B @ C) % p).astype(np.uint8)


def deficient(seed: int, stream: int, m: int, n: int, p: int, frac_rows: float = 0.125) -> np.ndarray:
    """Uniform matrix in which a seeded subset S of rows (|S| ~ U[1, ceil(frac*m)]) is
    replaced by random combinations of the rows outside S."""
    A = uniform(seed, stream, m, n, p).astype(np.int64)
    if m < 2:
        return A.astype(np.uint8)
    rng = np.random.default_rng([seed, stream, 0xDEF])
    kmax = max(1, int(np.ceil(frac_rows * m)))
    k = int(rng.integers(1, min(kmax, m - 1) + 1))
    S = np.sort(rng.choice(m, size=k, replace=False))
    rest = np.setdiff1d(np.arange(m), S)
    coef = uniform(seed, stream + 0x10000, k, len(rest), p).astype(np.int64)
    A[S] = (coef @ A[rest]) % p
    return A.astype(np.uint8)


def batch_mix(seed: int, count: int, nmin: int = 32, nmax: int = 512,
              primes=(2, 3, 5, 7, 251), deficient_frac: float = 0.10):
    """The batched workload: ``count`` square matrices, n log-uniform in [nmin, nmax],
    p uniform from ``primes``, and a seeded 10 % made rank-deficient."""
    rng = np.random.default_rng([seed, 0xBA7C])
    ns = np.rint(np.exp(rng.uniform(np.log(nmin), np.log(nmax), count))).astype(int)
    ps = rng.choice(np.asarray(primes), size=count)
    defi = rng.random(count) < deficient_frac
    out = []
    for t in range(count):
        n, p = int(ns[t]), int(ps[t])
        if defi[t]:
            A = deficient(seed, 1000 + t, n, n, p)
        else:
            A = uniform(seed, 1000 + t, n, n, p)
        out.append((A, p))
    return out


def gf2_uniform_packed(seed: int, stream: int, m: int, n: int) -> np.ndarray:
    """m x n GF(2) matrix with i.i.d. Bernoulli(0.5) entries, packed in 64-bit
    words (bit b of word w = column 64 w + b): word w of row i is the
    SplitMix64 output of counter i * ceil(n / 64) + w, its bits past column
    n - 1 cleared."""
    nw = (n + 63) // 64
    if m * nw == 0:
        return np.zeros((m, nw), np.uint64)
    W = words(seed, stream, 0, m * nw).reshape(m, nw)
    if n % 64:
        W[:, -1] &= np.uint64((1 << (n % 64)) - 1)
    return W


def gf2_deficient_packed(seed: int, m: int, n: int, deficiency: int, terms: int = 64) -> np.ndarray:
    """The large GF(2) workload's construction, packed: rows 0 .. m - deficiency - 1
    i.i.d. Bernoulli(0.5) (stream 0), and each of the last `deficiency` rows the
    sum (XOR) of `terms` distinct earlier rows among the first m - deficiency,
    chosen by a seeded draw.  With probability about 1 - 2^-(n - m + deficiency)
    the rank is m - deficiency and the selected rows are exactly the first
    m - deficiency."""
    top = m - deficiency
    W = np.zeros((m, (n + 63) // 64), np.uint64)
    W[:top] = gf2_uniform_packed(seed, 0, top, n)
    idx = gf2_combination_rows(seed, top, deficiency, terms)
    for t in range(deficiency):
        W[top + t] = np.bitwise_xor.reduce(W[idx[t]], axis=0)
    return W


def gf2_combination_rows(seed: int, top: int, deficiency: int, terms: int) -> np.ndarray:
    """The earlier rows (deficiency x terms, distinct per row) whose sums form
    the appended rows of gf2_deficient_packed."""
    rng = np.random.default_rng([seed, 0x6F2])
    k = min(terms, top)
    return np.stack([rng.choice(top, size=k, replace=False) for _ in range(deficiency)]) if deficiency else \
        np.zeros((0, k), np.int64)


def gf2_pack(A: np.ndarray) -> np.ndarray:
    """Pack a 0/1 matrix row-wise into uint64 words, bit b of word w = column 64w+b."""
    A = np.asarray(A, np.uint8)
    m, n = A.shape
    nw = (n + 63) // 64
    pad = np.zeros((m, nw * 64), np.uint8)
    pad[:, :n] = A
    bits = pad.reshape(m, nw, 64).astype(np.uint64)
    return np.sum(bits << np.arange(64, dtype=np.uint64), axis=2, dtype=np.uint64)


def gf2_unpack(W: np.ndarray, n: int) -> np.ndarray:
    W = np.asarray(W, np.uint64)
    m, nw = W.shape
    bits = (W[:, :, None] >> np.arange(64, dtype=np.uint64)) & np.uint64(1)
    return bits.reshape(m, nw * 64)[:, :n].astype(np.uint8)


def primes_upto_251():
    return list(_PRIMES_251)
