#!/usr/bin/env python3
"""Benchmark of the blocked Gaussian elimination over GF(p) on one MI355X.

Workload: a 40000 x 40000 matrix over GF(7) built as B * C mod 7 with B
(40000 x 39000) and C (39000 x 40000) i.i.d. uniform (seed 0; rank <= 39000),
stored one byte per entry and resident in HBM before timing starts.  One step
is one whole solve: Step 1 (ClearDown / Extend / UpdateRow /
UpdateRowTrafo), Step 2, Step 3 (PreClearUp / Copy / ClearUp) and the output
assembly (RREF remnant, rank, pivots, selected rows, M and K).

Prints one JSON line.  ``value`` is n^3/3 field multiply-adds per second of
the whole solve.  ``roofline`` describes the MAD kernel (int8 MFMA), timed
with device events on the stream it runs on.  ``cpu_baseline`` times the plain
CPU oracle on a smaller matrix of the same construction.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

INT8_PEAK_TOPS = 5000.0      # MI355X dense int8 MFMA, tera-ops per second (2 ops per multiply-add)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(n: int, k: int, p: int):
    """The oracle (single thread) on an n x n matrix of the same B*C construction."""
    import numpy as np

    import oracle
    import synth
    A = synth.low_rank_product(0, n, n, k, p)
    oracle.build()
    t0 = time.perf_counter()
    e = oracle.echelonize(A, p)
    dt = time.perf_counter() - t0
    return {"value": (n ** 3 / 3) / dt, "unit": "field mul-adds/s", "cores": 1, "kind": "oracle",
            "sample": f"{n}x{n} GF({p}) B*C with inner dimension {k} (rank {e.rank}), one solve, {dt:.2f} s",
            "seconds": dt}


def copy_calibration(torch, mib: int):
    """A streaming kernel of known traffic, three times: an elementwise negation
    that reads ``mib`` MiB and writes ``mib`` MiB (torch's elementwise kernel,
    not a DMA copy, so that per-dispatch counters see it).  The reading of an
    HBM byte counter for one dispatch, divided by the bytes it moved, is that
    counter's scale factor."""
    nbytes = mib << 20
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "launches": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=40000)
    ap.add_argument("--inner", type=int, default=39000)
    ap.add_argument("--p", type=int, default=7)
    ap.add_argument("--block", type=int, default=0, help="block size (0 = the library's choice)")
    ap.add_argument("--block-rows", type=int, default=0, help="block rows a_i (overrides --block)")
    ap.add_argument("--block-cols", type=int, default=0, help="block columns b_j (overrides --block)")
    ap.add_argument("--cpu-sample", type=int, default=2000, help="oracle sample size (0 = skip)")
    ap.add_argument("--no-kernel-events", action="store_true",
                    help="time the steps without per-launch device events (no roofline / kernel_ms)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the method here runs on a "
              "single MI355X and has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_mib > 0:
        copy_calibration(torch, args.copy_mib)
        return

    import paper_1806_04211_amd as gf
    from synth import torch_gen

    n, k, p = args.n, args.inner, args.p
    dev = torch.device("cuda:0")
    log(f"generating {n}x{n} GF({p}) = B*C (inner {k}) on the GPU")
    t0 = time.perf_counter()
    A = torch_gen.low_rank_product(0, n, n, k, p, device=dev)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log(f"input ready in {time.perf_counter() - t0:.1f} s")

    lib = gf.library()
    stream = torch.cuda.current_stream(dev)
    kw = dict(block_rows=args.block_rows or args.block, block_cols=args.block_cols or args.block)

    def solve(profile: int):
        """profile: 0 no device events, 1 every launch, 2 the MAD launches only"""
        return lib.echelonise_dev(A.data_ptr(), n, n, n, p, stream=stream.cuda_stream, profile=profile, **kw)

    rank = None
    for w in range(args.warmup):
        t1 = time.perf_counter()
        r = solve(0)
        rank = r.rank
        r.free()
        log(f"warmup {w}: {time.perf_counter() - t1:.3f} s, rank {rank}")

    # timed steps: device events around the MAD launches only (the roofline
    # kernel); every other launch runs without events
    times, stats = [], []
    torch.cuda.synchronize()
    for s in range(args.steps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = solve(0 if args.no_kernel_events else 2)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        times.append(dt)
        rank = r.rank
        stats.append(r.stats())
        r.free()
        log(f"step {s}: {dt:.3f} s, rank {rank}")
    # one more (untimed) solve with every launch timed, for the per-kind breakdown
    breakdown = None
    if not args.no_kernel_events:
        r = solve(1)
        breakdown = r.stats()
        r.free()

    mean = sum(times) / len(times)
    st = stats[-1]
    mac_mad = st["mac_cleardown"] + st["mac_updaterow"] + st["mac_trafo"] + st["mac_clearup"]
    mad_ms = sum(x["ms_mad"] for x in stats) / len(stats)
    mad_launches = st["launches_mad"]
    achieved = (2.0 * mac_mad) / (mad_ms * 1e-3) / 1e12 if mad_ms > 0 else 0.0
    lat = sorted(times)

    def pct(q):
        return lat[min(len(lat) - 1, int(round(q * (len(lat) - 1))))]

    out = {
        "metric": "GF(p) n^3/3 field mul-adds/s vs int8 MFMA peak; solves/s + p50/p99 latency",
        "value": (n ** 3 / 3) / mean,
        "unit": "field mul-adds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mean * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"{n}x{n} over GF({p}), B*C mod {p} with inner dimension {k}, seed 0",
                   "m": n, "n": n, "p": p, "rank": rank, "block_rows": st["block_rows"],
                   "block_cols": st["block_cols"], "parallelism": "single GPU"},
        "solves_per_s": 1.0 / mean,
        "latency_ms": {"p50": pct(0.5) * 1e3, "p99": pct(0.99) * 1e3},
        "work": {"mac_total": mac_mad + st["mac_ech"], "mac_mad": mac_mad, "mac_ech": st["mac_ech"],
                 "mac_alg_per_s": (mac_mad + st["mac_ech"]) / mean},
        "kernel_ms": None if breakdown is None else {
            "note": "one extra untimed solve with every launch timed",
            "mad": breakdown["ms_mad"], "ech": breakdown["ms_ech"], "small": breakdown["ms_small"],
            "launches_mad": breakdown["launches_mad"], "launches_ech": breakdown["launches_ech"],
            "launches_small": breakdown["launches_small"]},
        "roofline": {"bound": "mfma", "kernel": "k_gemm_modp (MAD mod p, int8 MFMA)",
                     "achieved": achieved, "peak": INT8_PEAK_TOPS, "unit": "TFLOP/s",
                     "frac": achieved / INT8_PEAK_TOPS, "traffic": None,
                     "per_launch": {"mac": mac_mad / max(mad_launches, 1),
                                    "avg_ms": mad_ms / max(mad_launches, 1)}},
        "check": {"rank": rank, "rank_expected": min(n, k)},
    }
    del A
    torch.cuda.empty_cache()
    if args.cpu_sample > 0:
        ns = args.cpu_sample
        log(f"oracle baseline on {ns}x{ns}")
        out["cpu_baseline"] = cpu_baseline(ns, int(round(ns * k / n)), p)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
