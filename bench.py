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


PROFILE = os.path.join(ROOT, "profiles", "k_gemm_modp_replay_40000_gf7.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1806_04211_amd", "csrc", "hip_backend.hip")
BLOCKING_TABLE = os.path.join(ROOT, "paper_1806_04211_amd", "blocking.json")


def block_size(n, tuned, rows=0, cols=0):
    """[block rows, block columns] a square n x n solve runs with: explicit
    sizes, else the tuned table's entry (when installed), else the library's
    built-in choice (256 x 2048 above 512 x 512, one block below)."""
    if rows or cols:
        return [rows or cols, cols or rows]
    if tuned:
        with open(BLOCKING_TABLE) as f:
            for e in json.load(f)["entries"]:
                if n <= e["max_dim"]:
                    return [e["block_rows"], e["block_cols"]]
    return [256, 2048] if n > 512 else [n, n]


def profiled_traffic():
    """HBM bytes per MAD launch from the committed counter summary, when it was
    taken on the current kernel source and, if it names one, the current
    blocking table (which decides the replayed launch); otherwise None."""
    import hashlib
    keys = ("source_sha256", "blocking_sha256", "traffic_bytes_per_launch")
    try:
        fields = {}
        for line in open(PROFILE):
            if ":" in line and line.split(":", 1)[0].strip() in keys:
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
        sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
        if "blocking_sha256" in fields:
            if fields["blocking_sha256"] != hashlib.sha256(open(BLOCKING_TABLE, "rb").read()).hexdigest():
                return None
        if fields.get("source_sha256") == sha and "traffic_bytes_per_launch" in fields:
            return float(fields["traffic_bytes_per_launch"])
    except OSError:
        pass
    return None


def exact_matmul_mod(X, Y, p, chunk_rows=4096):
    """(X @ Y) mod p for residue matrices on the host, exact: products in float32
    while every sum stays below 2^24 (then every partial sum is an exact
    integer), else in float64 (below 2^53); row chunks bound the memory."""
    import numpy as np
    k = X.shape[1]
    dt = np.float32 if k * (p - 1) ** 2 < 2 ** 24 else np.float64
    assert k * (p - 1) ** 2 < 2 ** 53
    Yf = Y.astype(dt)
    out = np.empty((X.shape[0], Y.shape[1]), np.int64)
    t0 = time.perf_counter()
    for r0 in range(0, X.shape[0], chunk_rows):
        out[r0:r0 + chunk_rows] = np.remainder(X[r0:r0 + chunk_rows].astype(dt) @ Yf, p).astype(np.int64)
        if time.perf_counter() - t0 > 20:         # progress of long host products
            log(f"  host product: {min(r0 + chunk_rows, X.shape[0])} of {X.shape[0]} rows")
            t0 = time.perf_counter()
    return out


def check_result(A_host, res, p, rank_expected, vectors=64, seed=0):
    """Checks of one timed solve's outputs, on the host and outside the library:
    the pinned rank; gamma and rho strictly increasing; R in reduced echelon
    shape (row t is zero in the non-pivot columns before its pivot column);
    and Eq. (2) by Freivalds' method with `vectors` random vectors X:
        -M (A X)[rho] = X[gamma] - R X[gamma_bar]     (T A X = E X, top rows)
        K (A X)[rho] + (A X)[rho_bar] = 0            (bottom rows)
    all mod p.  A wrong M, K, R, gamma or rho passes one vector with
    probability at most 1/p."""
    import numpy as np
    t0 = time.perf_counter()
    m, n = A_host.shape
    r = res.rank
    gamma, rho = res.pivots()
    gbar, rbar = res.nonpivots()
    log("  check: fetching R, M and K")
    R, M, K = res.get_R(), res.get_M(), res.get_K()
    out = {"rank": r, "rank_expected": rank_expected, "rank_ok": r == rank_expected}
    out["orders_ok"] = bool(np.all(np.diff(gamma) > 0) and np.all(np.diff(rho) > 0)
                            and len(np.intersect1d(gamma, gbar)) == 0 and len(np.intersect1d(rho, rbar)) == 0)
    # non-pivot columns before pivot column gamma[t]: gamma[t] - t of them
    lead = (gamma - np.arange(r))[:, None]
    out["rref_ok"] = bool(not np.any(R[np.arange(n - r)[None, :] < lead]))
    X = np.random.default_rng([seed, 0xF2E1]).integers(0, p, (n, vectors)).astype(np.uint8)
    log("  check: A X")
    Y = exact_matmul_mod(A_host, X, p)                      # A X, m x vectors
    log("  check: M (A X)[rho], R X[gamma_bar], K (A X)[rho]")
    Yr = Y[rho].astype(np.uint8)
    top_l = (-exact_matmul_mod(M, Yr, p)) % p
    top_r = (X[gamma].astype(np.int64) - exact_matmul_mod(R, X[gbar], p)) % p if n > r else X[gamma] % p
    bot = (exact_matmul_mod(K, Yr, p) + Y[rbar]) % p if m > r else np.zeros((0, vectors), np.int64)
    out["freivalds_vectors"] = vectors
    out["freivalds_ok"] = bool(np.array_equal(top_l, top_r) and not np.any(bot))
    out["ok"] = bool(out["rank_ok"] and out["orders_ok"] and out["rref_ok"] and out["freivalds_ok"])
    out["seconds"] = time.perf_counter() - t0
    return out


def read_mad_trace(path):
    """The descriptors of a GFECH_TRACE_MAD file: dicts with the engine
    iteration, launch number, kind (1 ClearDown, 2 UpdateRow, 3 UpdateRowTrafo,
    4 ClearUp), shapes, leading dimensions, flags and operand addresses."""
    keys = ("it", "launch", "kind", "M", "N", "K", "p", "lda", "ldb", "ldc", "ldd", "flags",
            "A", "B", "C", "D", "brow", "crow")
    out = []
    for line in open(path):
        f = line.split()
        if len(f) != len(keys):
            continue
        d = {}
        for k, v in zip(keys, f):
            d[k] = (0 if v == "(nil)" else int(v, 16)) if k in ("A", "B", "C", "D", "brow", "crow") else int(v)
        out.append(d)
    return out


def replay(torch, lib, descs, reps=10):
    """The traced descriptors as ONE grouped MAD launch, alone on the stream:
    operands rebased into one buffer of random residues that keeps their
    relative addresses (so sharing and alignment are those of the solve),
    gathered rows replaced by the identity.  Each launch is timed by the
    dispatch's own begin and end timestamps (the library's timed batch call),
    so the upload of the descriptor array is not counted.  Returns
    (multiply-adds, mean ms, operand bytes) of one launch."""
    p = descs[0]["p"]
    spans = []
    for d in descs:
        M, N, K = d["M"], d["N"], d["K"]
        spans += [(d["A"], (M - 1) * d["lda"] + K), (d["B"], (K - 1) * d["ldb"] + N + 16),
                  (d["D"], (M - 1) * d["ldd"] + N)]
        if d["C"]:
            spans.append((d["C"], (M - 1) * d["ldc"] + N + 16))
    lo = min(a for a, _ in spans)
    hi = max(a + n for a, n in spans)
    buf = torch.randint(0, p, (hi - lo + 256,), dtype=torch.uint8, device="cuda:0")
    base = buf.data_ptr()
    ident = torch.arange(max(max(d["K"], d["M"]) for d in descs), dtype=torch.int32, device="cuda:0")
    mad = [dict(M=d["M"], N=d["N"], K=d["K"], p=d["p"], A=base + d["A"] - lo, lda=d["lda"],
                B=base + d["B"] - lo, ldb=d["ldb"], brow=ident.data_ptr() if d["brow"] else 0,
                C=base + d["C"] - lo if d["C"] else 0, ldc=d["ldc"], crow=ident.data_ptr() if d["crow"] else 0,
                D=base + d["D"] - lo, ldd=d["ldd"]) for d in descs]
    stream = torch.cuda.current_stream()
    mad = lib.mad_descs(mad)                                  # marshalled once, outside the timed launches
    lib.mad_batch_dev(mad, stream=stream.cuda_stream)          # warm-up
    ms = [lib.mad_batch_dev_timed(mad, stream=stream.cuda_stream) for _ in range(reps)]
    del buf
    mac = sum(float(d["M"]) * d["N"] * d["K"] for d in descs)
    nbytes = sum(float(d["M"]) * d["K"] + float(d["K"]) * d["N"] + (2.0 if d["C"] else 1.0) * d["M"] * d["N"]
                 for d in descs)
    return mac, sum(ms) / len(ms), nbytes


def isolated_mad(torch, lib, trace_path):
    """Section 8(d)(i): the UpdateRow and UpdateRowTrafo products of the
    middle Step-1 iteration of the traced solve (one layer's worth: the
    priority products of layer L and the bulk sets of layer L - 1) as one
    grouped launch, and the largest ClearUp launch, each alone."""
    tr = read_mad_trace(trace_path)
    step1 = sorted({d["it"] for d in tr if d["kind"] == 1})
    mid = step1[len(step1) // 2]
    ur = [d for d in tr if d["it"] == mid and d["kind"] in (2, 3)]
    out = {}
    mac, ms, nb = replay(torch, lib, ur)
    out["updaterow_layer"] = {"iteration": mid, "descriptors": len(ur), "mac": mac, "ms": ms,
                              "int8_tops": 2 * mac / (ms * 1e-3) / 1e12, "operand_bytes": nb,
                              "shapes": sorted({(d["M"], d["N"], d["K"]) for d in ur},
                                               key=lambda x: -x[0] * x[1] * x[2])[:4]}
    cu = [d for d in tr if d["kind"] == 4]
    if cu:
        launches = {}
        for d in cu:
            launches.setdefault(d["launch"], []).append(d)
        big = max(launches.values(), key=lambda ds: sum(float(d["M"]) * d["N"] * d["K"] for d in ds))
        mac, ms, nb = replay(torch, lib, big)
        out["clearup_largest"] = {"descriptors": len(big), "mac": mac, "ms": ms,
                                  "int8_tops": 2 * mac / (ms * 1e-3) / 1e12, "operand_bytes": nb,
                                  "shapes": [(d["M"], d["N"], d["K"]) for d in big]}
    return out


def traced_isolated(torch, lib, solve):
    """One untimed solve with the MAD launch trace on, then isolated_mad."""
    import tempfile
    fd, path = tempfile.mkstemp(prefix="gfech_mad_trace_", suffix=".txt")
    os.close(fd)
    os.environ["GFECH_TRACE_MAD"] = path
    try:
        solve(0).free()
    finally:
        del os.environ["GFECH_TRACE_MAD"]
    try:
        iso = isolated_mad(torch, lib, path)
    finally:
        os.unlink(path)
    log(f"isolated: {json.dumps(iso)}")
    return iso


def summarize_replay_profile(prof_dir, pmc_dir, copy_dir, reps=10):
    """Figures of a `rocprofv3` run of `bench.py --replay-only` (kernel trace in
    prof_dir, FETCH_SIZE / WRITE_SIZE in pmc_dir, the copy calibration in
    copy_dir, CSV output).  The replays are the last 2 (reps + 1) MAD
    dispatches: the UpdateRow layer launch (one warm-up, `reps` timed), then
    the largest ClearUp launch the same way; the warm-ups are dropped."""
    import csv
    import glob

    def rows(d, suffix):
        path = glob.glob(os.path.join(d, "*" + suffix))[0]
        return list(csv.DictReader(open(path)))

    def mad(rs):
        return [r for r in rs if "k_gemm_modp" in r["Kernel_Name"]]

    trace = mad(rows(prof_dir, "kernel_trace.csv"))[-2 * (reps + 1):]
    fetch = mad(rows(pmc_dir, "fetch_counter_collection.csv") if glob.glob(os.path.join(pmc_dir, "fetch*")) else [])
    write = mad(rows(pmc_dir, "write_counter_collection.csv") if glob.glob(os.path.join(pmc_dir, "write*")) else [])
    cf = [float(r["Counter_Value"]) for r in rows(copy_dir, "fetch_counter_collection.csv") if "neg" in r["Kernel_Name"]]
    cw = [float(r["Counter_Value"]) for r in rows(copy_dir, "write_counter_collection.csv") if "neg" in r["Kernel_Name"]]
    copy_kib = 1024 * 1024        # bench.py --copy-mib 1024: reads and writes 1 GiB per dispatch
    f_scale = copy_kib / (sum(cf) / len(cf))
    w_scale = copy_kib / (sum(cw) / len(cw))
    out = {"fetch_scale": f_scale, "write_scale": w_scale}
    for name, lo in (("updaterow_layer", 0), ("clearup_largest", reps + 1)):
        sel = slice(lo + 1, lo + reps + 1)
        us = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in trace[sel]]
        ent = {"dispatches": len(us), "grid": int(trace[lo].get("Grid_Size_X") or trace[lo].get("Grid_Size") or 0),
               "mean_us": sum(us) / len(us)}
        if fetch and write:
            fk = [float(r["Counter_Value"]) for r in fetch[-2 * (reps + 1):][sel]]
            wk = [float(r["Counter_Value"]) for r in write[-2 * (reps + 1):][sel]]
            ent["fetch_kib"] = sum(fk) / len(fk)
            ent["write_kib"] = sum(wk) / len(wk)
            ent["traffic_bytes"] = 1024 * (ent["fetch_kib"] * f_scale + ent["write_kib"] * w_scale)
        out[name] = ent
    return out


def percentile(xs, q):
    xs = sorted(xs)
    return xs[min(len(xs) - 1, int(round(q * (len(xs) - 1))))] if xs else 0.0


def batch_inputs(torch, count, seed=0):
    """The batched workload of synth.batch_mix (n log-uniform in [32, 512],
    p from {2, 3, 5, 7, 251}, 10 % rank-deficient), in one device buffer:
    uniform matrices generated on the device, deficient ones on the host."""
    import numpy as np

    import synth
    from synth import torch_gen
    rng = np.random.default_rng([seed, 0xBA7C])
    ns = np.rint(np.exp(rng.uniform(np.log(32), np.log(512), count))).astype(int)
    ps = rng.choice(np.asarray([2, 3, 5, 7, 251]), size=count)
    defi = rng.random(count) < 0.10
    offs = np.concatenate([[0], np.cumsum(ns.astype(np.int64) ** 2)])
    buf = torch.empty(int(offs[-1]), dtype=torch.uint8, device="cuda:0")
    for t in range(count):
        n, p = int(ns[t]), int(ps[t])
        if defi[t]:
            A = torch.from_numpy(synth.deficient(seed, 1000 + t, n, n, p).ravel()).to("cuda:0")
        else:
            A = torch_gen.uniform(seed, 1000 + t, n, n, p).reshape(-1)
        buf[int(offs[t]):int(offs[t + 1])] = A
    torch.cuda.synchronize()
    return buf, [(int(buf.data_ptr() + offs[t]), int(ns[t]), int(ns[t]), int(ns[t]), int(ps[t])) for t in range(count)]


def run_batch(torch, args):
    """Many small matrices: one batched call against one call per matrix."""
    import paper_1806_04211_amd as gf
    lib = gf.library()
    t0 = time.perf_counter()
    buf, probs = batch_inputs(torch, args.count)
    log(f"{len(probs)} matrices ready in {time.perf_counter() - t0:.1f} s")
    stream = torch.cuda.current_stream().cuda_stream

    def batched():
        res, sts = lib.echelonise_batch(probs, on_device=True, stream=stream)
        assert all(st == 0 for st in sts)
        return res

    for _ in range(args.warmup):
        [r.free() for r in batched()]
    times = []
    for s in range(args.steps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res = batched()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
        ranks = [r.rank for r in res]
        bst = res[0].stats()                    # launch counts of the whole engine run
        [r.free() for r in res]
        log(f"batched step {s}: {times[-1]:.3f} s")
    # the plain path: one call (one launch sequence) per matrix
    lat = []
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for (ptr, m, n, lda, p) in probs:
        t2 = time.perf_counter()
        r = lib.echelonise_dev(ptr, m, n, lda, p, stream=stream)
        lat.append(time.perf_counter() - t2)
        r.free()
    per_call = time.perf_counter() - t1
    mean = sum(times) / len(times)
    print(json.dumps({
        "metric": "batched solves/s (4096 matrices n in [32, 512], one call) vs one call per matrix",
        "value": len(probs) / mean, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": mean * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"{len(probs)} square matrices, n log-uniform in [32, 512], p from {{2, 3, 5, 7, 251}}, "
                               "10 % rank-deficient, seed 0", "count": len(probs)},
        "per_call": {"solves_per_s": len(probs) / per_call, "latency_ms": {"p50": percentile(lat, 0.5) * 1e3,
                                                                           "p99": percentile(lat, 0.99) * 1e3}},
        "speedup_vs_per_call": per_call / mean,
        "rank_sum": int(sum(ranks)),
        "launches_per_batch": bst["launches"], "host_syncs_per_batch": bst["syncs"],
    }), flush=True)


def serve_request(rng_seed, t):
    """Request t of the serving workload: n log-uniform in [64, 8192],
    m = n U[0.75, 1.25], p from {2, 3, 5, 251}, uniform entries of stream t."""
    import numpy as np
    rng = np.random.default_rng([rng_seed, 0x5E7E, t])
    n = int(np.rint(np.exp(rng.uniform(np.log(64), np.log(8192)))))
    m = max(1, int(round(n * rng.uniform(0.75, 1.25))))
    p = int(rng.choice([2, 3, 5, 251]))
    return m, n, p


def run_serve(torch, args):
    """The serving workload: `requests` requests (n log-uniform in [64, 8192],
    m = n U[0.75, 1.25], p from {2, 3, 5, 251}, uniform entries from a
    per-request seed), Poisson arrivals at `load` x the server's capacity,
    through the server (continuous batching, size classes) and, on the same
    arrivals, through one plain call at a time (first come, first served).

    Inputs are generated on the device when a request arrives (a few tens of
    microseconds; all 20000 would take about 140 GB at once).  Three phases:
    (1) every request alone through one plain call: its service time;
    (2) the server's capacity mu: all requests through the server with the
        submitted-but-unfinished inputs kept under `window_gb` (a saturated
        queue that does not hold every input at once);
    (3) Poisson arrivals at lambda = load x mu through the server: latency =
        completion - arrival.  The plain path's latencies on the same arrivals
        follow from (1): each request starts when it has arrived and the
        previous one has finished."""
    import numpy as np

    import paper_1806_04211_amd as gf
    from synth import torch_gen
    lib = gf.library()
    nreq = args.requests
    shapes = [serve_request(0, t) for t in range(nreq)]

    def make(t):
        m, n, p = shapes[t]
        return torch_gen.uniform(0, 2000 + t, m, n, p)

    # (1) the plain path: one call per request, its service time alone
    service = []
    t0 = time.perf_counter()
    for t in range(nreq):
        m, n, p = shapes[t]
        A = make(t)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = lib.echelonise_dev(A.data_ptr(), m, n, n, p)
        service.append(time.perf_counter() - t1)
        r.free()
        del A
        if t % 2000 == 1999:
            log(f"plain path: {t + 1} requests, {sum(service):.1f} s of service")
    log(f"plain path: {sum(service):.2f} s of service for {nreq} requests ({time.perf_counter() - t0:.1f} s)")

    srv = lib.server(hbm_budget_bytes=args.budget_gb << 30, size_classes=args.size_classes)
    cur = torch.cuda.current_stream()

    def collect(pending, done_at, t0):
        for tk in list(pending):
            r = srv.poll(tk)
            if r is not None:
                done_at[pending.pop(tk)[0]] = time.perf_counter() - t0
                r.free()

    # (2) capacity: a saturated queue, bounded by the bytes of waiting inputs
    window = args.window_gb << 30
    pending, done_at = {}, {}
    t0 = time.perf_counter()
    for t in range(nreq):
        m, n, p = shapes[t]
        while sum(v[1] for v in pending.values()) + m * n > window and pending:
            collect(pending, done_at, t0)
        A = make(t)
        cur.synchronize()                  # the generation only, not the server's streams
        pending[srv.submit_dev(A.data_ptr(), m, n, n, p)] = (t, m * n)
        del A
        collect(pending, done_at, t0)
    while pending:
        collect(pending, done_at, t0)
    burst = time.perf_counter() - t0
    mu = nreq / burst
    lam = args.load * mu
    log(f"server capacity {mu:.1f} solves/s ({burst:.1f} s); plain path {nreq / sum(service):.1f} solves/s; "
        f"arrival rate {lam:.1f}/s")

    # (3) Poisson arrivals through the server
    arrivals = np.cumsum(np.random.default_rng(0).exponential(1.0 / lam, nreq))
    pending, done_at = {}, {}
    t0 = time.perf_counter()
    for t in range(nreq):
        while time.perf_counter() - t0 < arrivals[t]:
            collect(pending, done_at, t0)
        m, n, p = shapes[t]
        A = make(t)
        cur.synchronize()                  # the generation only, not the server's streams
        pending[srv.submit_dev(A.data_ptr(), m, n, n, p)] = (t, m * n)
        del A
        if t % 2000 == 1999:
            log(f"served: {t + 1} requests submitted, {len(done_at)} finished")
    while pending:
        collect(pending, done_at, t0)
    span = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    lat = [done_at[t] - arrivals[t] for t in range(nreq)]
    # the plain path on the same arrivals: one request at a time, first come first served
    fin, plain_lat = 0.0, []
    for t in range(nreq):
        fin = max(fin, arrivals[t]) + service[t]
        plain_lat.append(fin - arrivals[t])
    small = [t for t in range(nreq) if max(shapes[t][:2]) <= 512]
    if args.dump_latencies:
        with open(args.dump_latencies, "w") as f:
            f.write("t m n p arrival_s served_ms plain_ms service_ms\n")
            for t in range(nreq):
                m, n, p = shapes[t]
                f.write(f"{t} {m} {n} {p} {arrivals[t]:.6f} {lat[t] * 1e3:.3f} {plain_lat[t] * 1e3:.3f} "
                        f"{service[t] * 1e3:.3f}\n")
    print(json.dumps({
        "metric": "served solves/s and p50/p99 latency (Poisson arrivals, continuous batching) vs one call at a time",
        "value": nreq / span, "unit": "solves/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": span * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"{nreq} requests, n log-uniform in [64, 8192], m = n U[0.75, 1.25], p from "
                               f"{{2, 3, 5, 251}}, Poisson arrivals at {args.load} x the server's capacity "
                               f"({lam:.1f}/s), budget {args.budget_gb} GB, {args.size_classes or 3} size classes",
                   "requests": nreq, "arrival_rate": lam, "capacity": mu, "budget_gb": args.budget_gb},
        "latency_ms": {"p50": percentile(lat, 0.5) * 1e3, "p99": percentile(lat, 0.99) * 1e3,
                       "p99_small": percentile([lat[t] for t in small], 0.99) * 1e3},
        "server": {"peak_gb_in_flight": st["peak_bytes_in_flight"] / 2 ** 30, "peak_active": st["peak_active"]},
        "plain": {"solves_per_s": nreq / fin, "service_s": sum(service),
                  "latency_ms": {"p50": percentile(plain_lat, 0.5) * 1e3, "p99": percentile(plain_lat, 0.99) * 1e3,
                                 "p99_small": percentile([plain_lat[t] for t in small], 0.99) * 1e3}},
    }), flush=True)


def run_gf2(torch, args):
    """The largest single instance: n x n over GF(2), packed in 64-bit words on
    the device (rows 0 .. n - 1001 i.i.d. Bernoulli(0.5) from seed 4, the last
    1000 rows sums of 64 distinct earlier rows), through gfech_echelonise_gf2_dev.
    The solve's result is checked on the host: rank n - 1000 and the first
    n - 1000 rows selected (pinned by the construction), and Freivalds on Eq. (2)."""
    import numpy as np

    import paper_1806_04211_amd as gf
    from paper_1806_04211_amd import tune
    from synth import torch_gen
    lib = gf.library()
    tuned = tune.install_default(lib)
    n, d = args.gf2_n, 1000
    words = (n + 63) // 64
    t0 = time.perf_counter()
    W = torch_gen.gf2_deficient_packed(4, n, n, d)
    torch.cuda.synchronize()
    log(f"{n}x{n} GF(2) packed input ({W.numel() * 8 / 2**30:.1f} GiB) ready in {time.perf_counter() - t0:.1f} s")
    stream = torch.cuda.current_stream()

    def solve(variant=0):
        return lib.echelonise_gf2_dev(W.data_ptr(), n, n, words, stream=stream.cuda_stream, variant=variant)

    for w in range(args.warmup):
        t1 = time.perf_counter()
        r = solve()
        log(f"warmup {w}: {time.perf_counter() - t1:.2f} s, rank {r.rank}")
        r.free()
    times, last, st = [], None, None
    for s in range(args.steps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = solve()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
        st = r.stats()
        if last is not None:
            last.free()
        last = r
        log(f"step {s}: {times[-1]:.2f} s, rank {r.rank}")
    mean = sum(times) / len(times)
    mac = st["mac_cleardown"] + st["mac_updaterow"] + st["mac_trafo"] + st["mac_clearup"] + st["mac_ech"]
    out = {
        "metric": "GF(p) n^3/3 field mul-adds/s vs int8 MFMA peak; solves/s + p50/p99 latency",
        "value": (n ** 3 / 3) / mean, "unit": "field mul-adds/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": mean * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"{n}x{n} over GF(2), bit-packed in 64-bit words, rank deficiency {d} (rows "
                               f"{n - d}.. are sums of 64 earlier rows), seed 4", "m": n, "n": n, "p": 2,
                   "rank": last.rank, "block_grid": [st["block_rows"], st["block_cols"]],
                   "block_size": block_size(n, tuned),
                   "blocking": "tuned table" if tuned else "built-in", "parallelism": "single GPU"},
        "work": {"mac_total": mac, "mac_alg_per_s": mac / mean},
        "roofline": {"bound": "mfma", "kernel": "k_gemm_modp (MAD mod p, int8 MFMA, unpacked GF(2))",
                     "solve_wide": {"achieved": 2 * (mac - st["mac_ech"]) / mean / 1e12,
                                    "frac": 2 * (mac - st["mac_ech"]) / mean / 1e12 / INT8_PEAK_TOPS}},
    }
    if not args.no_check:
        log("checking the last timed solve on the host (pins and Freivalds, 64 vectors)")
        t1 = time.perf_counter()
        A_host = np.unpackbits(W.cpu().numpy().view(np.uint8), axis=1, bitorder="little")[:, :n]
        del W
        torch.cuda.empty_cache()
        chk = check_result(A_host, last, 2, n - d)
        gamma, rho = last.pivots()
        chk["rho_first_rows_ok"] = bool(np.array_equal(rho, np.arange(n - d)))
        chk["ok"] = chk["ok"] and chk["rho_first_rows_ok"]
        chk["seconds"] = time.perf_counter() - t1
        out["check"] = chk
        log(f"check: {chk}")
    last.free()
    print(json.dumps(out), flush=True)


def run_gf2_mad(torch, args):
    """GF(2) products two ways on the same logical shapes: the byte path's MAD
    (int8 MFMA on one byte per entry, p = 2) against the four-Russians MAD on
    packed rows; device events around 5 launches each after one untimed."""
    import paper_1806_04211_amd as gf
    lib = gf.library()
    stream = torch.cuda.current_stream()
    rows = []
    for (M, N, K) in ((256, 32768, 2048), (4096, 20480, 2048), (8192, 8192, 8192), (32768, 40000, 4096)):
        res = {"shape": [M, N, K]}
        # bytes: operands of 0/1 entries
        A8 = torch.randint(0, 2, (M, K), dtype=torch.uint8, device="cuda:0")
        B8 = torch.randint(0, 2, (K, N), dtype=torch.uint8, device="cuda:0")
        C8 = torch.randint(0, 2, (M, N), dtype=torch.uint8, device="cuda:0")
        # packed: random words with the pad bits cleared
        wk, wn = (K + 63) // 64, (N + 63) // 64
        Ap = torch.randint(-2 ** 62, 2 ** 62, (M, wk), dtype=torch.int64, device="cuda:0")
        Bp = torch.randint(-2 ** 62, 2 ** 62, (K, wn), dtype=torch.int64, device="cuda:0")
        Cp = torch.randint(-2 ** 62, 2 ** 62, (M, wn), dtype=torch.int64, device="cuda:0")
        if N % 64:
            Bp[:, -1] &= (1 << (N % 64)) - 1
            Cp[:, -1] &= (1 << (N % 64)) - 1
        runs = {
            "int8_mfma_bytes": lambda: lib.mad_dev(M, N, K, 2, A8.data_ptr(), K, B8.data_ptr(), N, C8.data_ptr(), N,
                                                    C=C8.data_ptr(), ldc=N, stream=stream.cuda_stream),
            "four_russians_packed": lambda: lib.mad_gf2_dev(M, N, K, Ap.data_ptr(), wk, Bp.data_ptr(), wn,
                                                            Cp.data_ptr(), wn, C=Cp.data_ptr(), ldc=wn,
                                                            stream=stream.cuda_stream)}
        for name, fn in runs.items():
            fn()
            ms = []
            for _ in range(5):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                fn()
                e1.record(stream)
                e1.synchronize()
                ms.append(e0.elapsed_time(e1))
            t = sum(ms) / len(ms)
            res[name] = {"ms": t, "gf2_mac_per_s": M * N * K / (t * 1e-3)}
        res["packed_speedup"] = res["int8_mfma_bytes"]["ms"] / res["four_russians_packed"]["ms"]
        log(f"gf2 mad {M}x{N}x{K}: bytes {res['int8_mfma_bytes']['ms']:.3f} ms, packed "
            f"{res['four_russians_packed']['ms']:.3f} ms")
        rows.append(res)
        del A8, B8, C8, Ap, Bp, Cp
        torch.cuda.empty_cache()
    print(json.dumps({"gf2_mad": rows}), flush=True)


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
    ap.add_argument("--summarize-profile", nargs=3, metavar=("TRACE_DIR", "PMC_DIR", "COPY_DIR"),
                    help="print the figures of a rocprofv3 run of --replay-only (no GPU needed)")
    ap.add_argument("--tune", action="store_true",
                    help="run the block-size tuner and write its table to gpurun_out/blocking.json")
    ap.add_argument("--replay-only", action="store_true",
                    help="only a traced solve and the isolated replays of its launches (for kernel profiles)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the timing of the variants without the transformation")
    ap.add_argument("--no-check", action="store_true",
                    help="skip the host-side check (Freivalds) of the last timed solve; only its rank is reported")
    ap.add_argument("--no-kernel-events", action="store_true",
                    help="time the steps without per-launch device events (no roofline / kernel_ms)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (calibrates HBM byte counters)")
    ap.add_argument("--gf2-n", type=int, default=200000, help="gf2: the matrix size")
    ap.add_argument("--workload", choices=["single", "batch", "serve", "gf2", "gf2mad"], default="single",
                    help="single: the one large matrix (default); batch: many small matrices in one call; "
                         "serve: a Poisson stream of requests through the server")
    ap.add_argument("--count", type=int, default=4096, help="batch: number of matrices")
    ap.add_argument("--requests", type=int, default=20000, help="serve: number of requests")
    ap.add_argument("--load", type=float, default=0.8,
                    help="serve: arrival rate as a fraction of the server's capacity")
    ap.add_argument("--budget-gb", type=int, default=200, help="serve: device-memory admission budget")
    ap.add_argument("--window-gb", type=int, default=32,
                    help="serve: inputs waiting in the server at most while its capacity is measured")
    ap.add_argument("--size-classes", type=int, default=0, help="serve: size classes of the server (0 = 3)")
    ap.add_argument("--dump-latencies", default="", help="serve: write every request's latencies to this file")
    ap.add_argument("--hw-queues", type=int, default=-1,
                    help="hardware queues of the process (GPU_MAX_HW_QUEUES, at most 32; 0 = the environment's; "
                         "default: 16 for the serving workload, whose size classes each run their own streams, "
                         "else the environment's)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the method here runs on a "
              "single MI355X and has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    if args.summarize_profile:
        print(json.dumps(summarize_replay_profile(*args.summarize_profile), indent=1))
        return
    if args.hw_queues < 0:
        args.hw_queues = 16 if args.workload == "serve" else 0
    if args.hw_queues > 0:
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(args.hw_queues, 32))     # before the runtime starts
    import torch

    if args.copy_mib > 0:
        copy_calibration(torch, args.copy_mib)
        return
    if args.workload == "batch":
        run_batch(torch, args)
        return
    if args.workload == "serve":
        run_serve(torch, args)
        return
    if args.workload == "gf2":
        run_gf2(torch, args)
        return
    if args.workload == "gf2mad":
        run_gf2_mad(torch, args)
        return

    import paper_1806_04211_amd as gf
    from paper_1806_04211_amd import tune
    from synth import torch_gen

    if args.tune:
        # the block-size tuner; the table goes to gpurun_out/ (copied into the package by hand)
        table = tune.tune(gf.library(), torch, log=log)
        os.makedirs(os.path.join(ROOT, "gpurun_out"), exist_ok=True)
        tune.save(table, os.path.join(ROOT, "gpurun_out", "blocking.json"))
        print(json.dumps(table), flush=True)
        return
    tuned = tune.install_default(gf.library())

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
        """profile: 0 no device events, 1 every launch, 2 the MAD launches only,
        3 every fourth MAD launch"""
        return lib.echelonise_dev(A.data_ptr(), n, n, n, p, stream=stream.cuda_stream, profile=profile, **kw)

    if args.replay_only:
        # for profiling: one traced solve, then the isolated launches alone
        iso = traced_isolated(torch, lib, solve)
        print(json.dumps({"isolated": iso}), flush=True)
        return

    rank = None
    for w in range(args.warmup):
        t1 = time.perf_counter()
        r = solve(0)
        rank = r.rank
        r.free()
        log(f"warmup {w}: {time.perf_counter() - t1:.3f} s, rank {rank}")

    # timed steps: no device events at all
    times, stats = [], []
    last = None
    torch.cuda.synchronize()
    for s in range(args.steps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = solve(0)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        times.append(dt)
        rank = r.rank
        stats.append(r.stats())
        if last is not None:
            last.free()
        last = r                      # the last timed solve's result is checked below
        log(f"step {s}: {dt:.3f} s, rank {rank}")
    # two more (untimed) solves: one with device events around a pseudo-random
    # quarter of the MAD launches (the in-situ figure: an event pair costs host
    # time on the issuing thread, so the timed steps carry none), one with
    # every launch timed, for the per-kind breakdown
    breakdown, sampled = None, None
    if not args.no_kernel_events:
        r = solve(3)
        sampled = r.stats()
        r.free()
        r = solve(1)
        breakdown = r.stats()
        r.free()

    mean = sum(times) / len(times)
    st = stats[-1]
    mac_mad = st["mac_cleardown"] + st["mac_updaterow"] + st["mac_trafo"] + st["mac_clearup"]
    # the timed (sampled) MAD launches of the sampled solve
    mad_ms = sampled["ms_mad"] if sampled else 0.0
    mad_launches = sampled["launches_mad"] if sampled else 0
    mac_timed = sampled["mac_mad_timed"] if sampled else 0.0
    achieved = (2.0 * mac_timed) / (mad_ms * 1e-3) / 1e12 if mad_ms > 0 else 0.0
    # MAD launches of one solve (the solve with every launch timed counts them)
    all_mad_launches = breakdown["launches_mad"] if breakdown else 0
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
                   "m": n, "n": n, "p": p, "rank": rank, "block_grid": [st["block_rows"], st["block_cols"]],
                   "block_size": block_size(n, tuned, kw["block_rows"], kw["block_cols"]),
                   "blocking": "tuned table" if tuned and not (kw["block_rows"] or kw["block_cols"]) else
                               "explicit" if (kw["block_rows"] or kw["block_cols"]) else "built-in",
                   "parallelism": "single GPU"},
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
                     "frac": achieved / INT8_PEAK_TOPS, "traffic": profiled_traffic(),
                     "per_launch": {"mac": mac_timed / max(mad_launches, 1),
                                    "bytes": st["mad_bytes"] / all_mad_launches if all_mad_launches else None,
                                    "avg_ms": mad_ms / max(mad_launches, 1),
                                    "timed_launches": mad_launches, "launches_per_solve": all_mad_launches}},
    }
    # Section 8(d)(i): one layer's UpdateRow launch and the largest ClearUp
    # launch replayed alone at their traced shapes.  The isolated layer launch
    # is the roofline figure; the in-situ one (sampled launches of an untimed
    # solve, which overlap on four streams) and the solve-wide MAD rate stand
    # beside it.
    if not args.no_kernel_events:
        roof = out["roofline"]
        roof["in_situ"] = {"achieved": roof["achieved"], "frac": roof["frac"], "per_launch": roof.pop("per_launch"),
                           "note": "sampled MAD launches of one untimed solve (contended: four streams overlap)"}
        roof["solve_wide"] = {"achieved": 2 * mac_mad / mean / 1e12, "frac": 2 * mac_mad / mean / 1e12 / INT8_PEAK_TOPS,
                              "note": "all MAD multiply-adds of a solve over its wall time"}
        iso = traced_isolated(torch, lib, solve)
        u = iso["updaterow_layer"]
        roof["achieved"] = u["int8_tops"]
        roof["frac"] = u["int8_tops"] / INT8_PEAK_TOPS
        roof["measured"] = ("isolated: the UpdateRow / UpdateRowTrafo products of one mid-solve Step-1 iteration "
                            "as one grouped launch, alone, each of 10 launches timed by its dispatch timestamps")
        roof["isolated"] = iso
        roof["traffic"] = profiled_traffic()
    # the variants without the transformation (Section 1), one solve each after
    # a warm-up, beside the full solve's mean
    if not args.no_variants:
        out["variants_ms"] = {"rref_and_transform": mean * 1e3}
        for name, v in (("rref_only", 1), ("rank_only", 2)):
            lib.echelonise_dev(A.data_ptr(), n, n, n, p, stream=stream.cuda_stream, variant=v, **kw).free()
            vt = []
            for _ in range(2):
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                r = lib.echelonise_dev(A.data_ptr(), n, n, n, p, stream=stream.cuda_stream, variant=v, **kw)
                torch.cuda.synchronize()
                vt.append(time.perf_counter() - t1)
                assert r.rank == rank
                r.free()
            out["variants_ms"][name] = min(vt) * 1e3
            log(f"variant {name}: {min(vt) * 1e3:.1f} ms")
    # the last timed solve's outputs, checked on the host (outside the library)
    if args.no_check:
        out["check"] = {"rank": rank, "rank_expected": min(n, k)}
        last.free()
    else:
        log("checking the last timed solve on the host (Freivalds, 64 vectors)")
        A_host = A.cpu().numpy()
        out["check"] = check_result(A_host, last, p, min(n, k))
        last.free()
        del A_host
        log(f"check: {out['check']}")
    del A
    torch.cuda.empty_cache()
    if args.cpu_sample > 0:
        ns = args.cpu_sample
        log(f"oracle baseline on {ns}x{ns}")
        out["cpu_baseline"] = cpu_baseline(ns, int(round(ns * k / n)), p)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
