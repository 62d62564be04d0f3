"""Block-size tuner.

Section 3.1 leaves the block sizes open: larger blocks give fewer, larger
products (the MFMA kernel runs faster on them) but a longer chain of
ClearDown echelonisations on the critical path, and the paper reports a
too-large block costing about half again the run time (Section 6).  This
module picks them by measurement: for each size of a list it times
candidate (block rows, block columns) pairs on seeded synthetic matrices of
the benchmark's construction (B C mod p with inner dimension 0.975 n, so
rank-deficient like the 40000 x 40000 workload) through the C ABI, and
writes the fastest per size as a table; ``install`` hands a table to the
library (``gfech_set_blocking``), which then uses it whenever a call leaves
the block sizes to the library.  Block sizes never change results.
"""
from __future__ import annotations

import ctypes
import json
import math
import os
import time

from . import _abi

DEFAULT_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "blocking.json")
ROWS = (128, 256, 512)
COLS = (512, 1024, 1536, 2048, 3072, 4096)


def candidates(n: int):
    """(block rows, block columns) pairs worth timing for an n x n matrix."""
    out = [(r, c) for r in ROWS for c in COLS if r < n and c < n and r <= c]
    return out or [(n, n)]


def measure(lib, torch, n: int, p: int = 7, reps: int = 3, pairs=None, log=print):
    """Mean solve time (ms) of each candidate blocking on one n x n input."""
    from synth import torch_gen
    A = torch_gen.low_rank_product(0, n, n, max(1, int(round(0.975 * n))), p)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    rows = []
    for br, bc in pairs or candidates(n):
        lib.echelonise_dev(A.data_ptr(), n, n, n, p, stream=stream.cuda_stream, block_rows=br,
                           block_cols=bc).free()                        # warm-up
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lib.echelonise_dev(A.data_ptr(), n, n, n, p, stream=stream.cuda_stream, block_rows=br,
                               block_cols=bc).free()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        rows.append({"block_rows": br, "block_cols": bc, "ms": 1e3 * sum(ts) / len(ts)})
        log(f"tune n={n}: {br} x {bc}: {rows[-1]['ms']:.2f} ms")
    del A
    return rows


def tune(lib, torch, sizes=(1024, 2048, 4096, 8192, 16384, 40000), p: int = 7, reps: int = 3, log=print):
    """The table: one entry per size, covering max(m, n) up to the geometric
    mean of that size and the next (the last: every larger size)."""
    sizes = sorted(sizes)
    entries = []
    for k, n in enumerate(sizes):
        rows = measure(lib, torch, n, p, reps, log=log)
        best = min(rows, key=lambda r: r["ms"])
        hi = int(math.sqrt(n * sizes[k + 1])) if k + 1 < len(sizes) else 2 ** 31 - 1
        entries.append({"max_dim": hi, "block_rows": best["block_rows"], "block_cols": best["block_cols"],
                        "tuned_on": n, "ms": best["ms"], "candidates": rows})
    return {"p": p, "input": "B C mod p, inner dimension 0.975 n, seed 0", "entries": entries}


def save(table, path: str = DEFAULT_PATH):
    with open(path, "w") as f:
        json.dump(table, f, indent=1)


def install(lib, table) -> None:
    """Hand a table (a dict as written by tune, or a path to one) to the library."""
    if isinstance(table, str):
        with open(table) as f:
            table = json.load(f)
    ents = table["entries"]
    arr = (_abi.Blocking * max(len(ents), 1))()
    for t, e in enumerate(ents):
        arr[t].max_dim, arr[t].block_rows, arr[t].block_cols = e["max_dim"], e["block_rows"], e["block_cols"]
    lib._check(lib.lib.gfech_set_blocking(arr, len(ents)))


def install_default(lib) -> bool:
    """Install the package's tuned table when it exists; returns whether it did."""
    if not os.path.exists(DEFAULT_PATH):
        return False
    install(lib, DEFAULT_PATH)
    return True
