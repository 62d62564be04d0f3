"""The same SplitMix64 streams as ``synth`` computed with torch int64 tensors
(on the GPU for the large workloads).  int64 products wrap modulo 2**64 like
the uint64 ones; logical right shifts are arithmetic shifts plus a mask."""
from __future__ import annotations

import torch


def _s64(x: int) -> int:
    x &= (1 << 64) - 1
    return x - (1 << 64) if x >= (1 << 63) else x


GAMMA = _s64(0x9E3779B97F4A7C15)
M1 = _s64(0xBF58476D1CE4E5B9)
M2 = _s64(0x94D049BB133111EB)


def _shr(z, s: int):
    return (z >> s) & ((1 << (64 - s)) - 1)


def mix64(z):
    z = (z ^ _shr(z, 30)) * M1
    z = (z ^ _shr(z, 27)) * M2
    return z ^ _shr(z, 31)


def stream_key(seed: int, stream: int) -> int:
    z = torch.tensor([_s64((int(seed) << 32) + int(stream))], dtype=torch.int64)
    return int(mix64(z)[0])


def uniform_rows(seed: int, stream: int, row0: int, rows: int, n: int, p: int, device="cuda") -> torch.Tensor:
    """Rows row0..row0+rows-1 of synth.uniform(seed, stream, *, n, p) as a uint8 tensor."""
    key = stream_key(seed, stream)
    t = torch.arange(row0 * n + 1, (row0 + rows) * n + 1, dtype=torch.int64, device=device)
    w = mix64(t * GAMMA + key)
    v = (_shr(w, 32) * p) >> 32
    return v.to(torch.uint8).reshape(rows, n)


def uniform(seed: int, stream: int, m: int, n: int, p: int, device="cuda", chunk_rows: int = 2048) -> torch.Tensor:
    out = torch.empty((m, n), dtype=torch.uint8, device=device)
    for r0 in range(0, m, chunk_rows):
        r = min(chunk_rows, m - r0)
        out[r0:r0 + r] = uniform_rows(seed, stream, r0, r, n, p, device)
    return out


def low_rank_product(seed: int, m: int, n: int, k: int, p: int, device="cuda", chunk_rows: int = 4096) -> torch.Tensor:
    """B @ C mod p with B (m x k) from stream 1 and C (k x n) from stream 2, as
    synth.low_rank_product; the product is exact in float64 (sums < 2**53)."""
    assert k * (p - 1) ** 2 < 2 ** 53
    C = uniform(seed, 2, k, n, p, device).to(torch.float64)
    out = torch.empty((m, n), dtype=torch.uint8, device=device)
    for r0 in range(0, m, chunk_rows):
        r = min(chunk_rows, m - r0)
        B = uniform_rows(seed, 1, r0, r, k, p, device).to(torch.float64)
        out[r0:r0 + r] = torch.remainder(B @ C, p).to(torch.uint8)
        del B
    del C
    return out


def gf2_uniform_packed(seed: int, stream: int, m: int, n: int, device="cuda", chunk_rows: int = 4096) -> torch.Tensor:
    """synth.gf2_uniform_packed as an int64 tensor (the same 64 bits per word)."""
    nw = (n + 63) // 64
    key = stream_key(seed, stream)
    out = torch.empty((m, nw), dtype=torch.int64, device=device)
    for r0 in range(0, m, chunk_rows):
        r = min(chunk_rows, m - r0)
        t = torch.arange(r0 * nw + 1, (r0 + r) * nw + 1, dtype=torch.int64, device=device)
        out[r0:r0 + r] = mix64(t * GAMMA + key).reshape(r, nw)
    if n % 64:
        out[:, -1] &= (1 << (n % 64)) - 1
    return out


def gf2_deficient_packed(seed: int, m: int, n: int, deficiency: int, terms: int = 64, device="cuda") -> torch.Tensor:
    """synth.gf2_deficient_packed as an int64 tensor on `device`."""
    import synth
    top = m - deficiency
    out = torch.empty((m, (n + 63) // 64), dtype=torch.int64, device=device)
    out[:top] = gf2_uniform_packed(seed, 0, top, n, device)
    if deficiency:
        idx = torch.from_numpy(synth.gf2_combination_rows(seed, top, deficiency, terms)).to(device)
        acc = torch.zeros((deficiency, out.shape[1]), dtype=torch.int64, device=device)
        for c in range(idx.shape[1]):
            acc ^= out[idx[:, c]]
        out[top:] = acc
    return out
