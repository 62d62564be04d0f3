"""The serving API (continuous batching) through the C ABI on the test-only
CPU emulator backend: every result equals the oracle's and the result of the
same problem solved alone, whatever else is in flight."""
import numpy as np
import pytest

import oracle
import synth
from paper_1806_04211_amd.api import GfechError
from tests import emu
from tests.test_chief_emu import compare


@pytest.fixture(scope="module")
def lib():
    return emu.library()


def mixed_requests(seed, count):
    rng = np.random.default_rng([seed, 77])
    out = []
    for t in range(count):
        p = int(rng.choice([2, 3, 5, 251]))
        n = int(rng.integers(1, 90)) if t % 4 else int(rng.integers(513, 640))   # some need several blocks
        m = max(1, int(round(n * rng.uniform(0.75, 1.25))))
        A = synth.deficient(seed, t, m, n, p) if t % 5 == 0 and m > 2 else synth.uniform(seed, t, m, n, p)
        out.append((A, p))
    return out


def test_results_same_alone_and_in_the_mix(lib):
    reqs = mixed_requests(1, 14)
    srv = lib.server()
    tickets = [srv.submit(A, p) for A, p in reqs]
    got = {t: srv.wait(t) for t in reversed(tickets)}
    for (A, p), t in zip(reqs, tickets):
        o = got[t].outputs()
        compare(o, oracle.echelonize(A, p), f"{A.shape} p={p}")
        compare(o, lib.echelonise(A, p).outputs(), f"alone {A.shape} p={p}")
    srv.close()


def test_requests_join_while_others_run(lib):
    """Submissions interleaved with polls: later requests join an engine that
    is already working on earlier ones."""
    reqs = mixed_requests(2, 10)
    srv = lib.server()
    tickets, results = [], {}
    for A, p in reqs:
        tickets.append(srv.submit(A, p))
        for t in tickets:
            if t not in results:
                r = srv.poll(t)
                if r is not None:
                    results[t] = r
    for t in tickets:
        if t not in results:
            results[t] = srv.wait(t)
    for (A, p), t in zip(reqs, tickets):
        compare(results[t].outputs(), oracle.echelonize(A, p), f"{A.shape} p={p}")
    srv.close()


def test_memory_budget_admission(lib):
    """A budget that holds only one or two requests at a time still finishes
    all of them; a request larger than the budget alone is refused."""
    reqs = mixed_requests(3, 6)
    srv = lib.server(hbm_budget_bytes=16 << 20)
    big = np.zeros((3000, 3000), np.uint8)
    with pytest.raises(GfechError) as ex:
        srv.submit(big, 3)
    assert ex.value.status == 5
    tickets = [srv.submit(A, p) for A, p in reqs]
    for (A, p), t in zip(reqs, tickets):
        compare(srv.wait(t).outputs(), oracle.echelonize(A, p))
    st = srv.stats()
    assert st["admitted"] == st["finished"] == len(reqs)
    assert 0 < st["peak_bytes_in_flight"] <= 16 << 20
    srv.close()


def test_errors_and_tickets(lib):
    srv = lib.server(max_active=2)
    with pytest.raises(GfechError) as ex:
        srv.submit(np.full((3, 3), 7, np.uint8), 7)
    assert ex.value.status == 3
    with pytest.raises(GfechError) as ex:
        srv.submit(np.zeros((3, 3), np.uint8), 4)
    assert ex.value.status == 2
    t = srv.submit(np.eye(4, dtype=np.uint8), 5)
    r = srv.wait(t)
    assert r.rank == 4
    with pytest.raises(GfechError) as ex:
        srv.poll(t)                      # answered once
    assert ex.value.status == 1
    e = srv.submit(np.zeros((0, 5), np.uint8), 5)
    assert srv.wait(e).rank == 0
    srv.close()


def test_cancel_queued_and_running(lib):
    """A cancelled request answers GFECH_E_CANCELLED unless it had already
    finished (then its result is right); when it was dropped or stopped, the
    others are unaffected and the server keeps working afterwards."""
    srv = lib.server(max_active=1)
    big = synth.uniform(3, 1, 1500, 300, 7)        # 6 block rows: several iterations
    small = [(synth.uniform(3, 2 + t, 40, 50, 5), 5) for t in range(3)]
    tb = srv.submit(big, 7)
    ts = [srv.submit(A, p) for A, p in small]
    srv.cancel(ts[1])
    srv.cancel(tb)
    for tk, (A, p) in ((tb, (big, 7)), (ts[1], small[1])):
        try:
            compare(srv.wait(tk).outputs(), oracle.echelonize(A, p))
        except GfechError as e:
            assert e.status == 7
    for t in (0, 2):
        compare(srv.wait(ts[t]).outputs(), oracle.echelonize(*small[t]))
    with pytest.raises(GfechError) as ex:
        srv.cancel(12345)
    assert ex.value.status == 1
    srv.close()


def test_watchdog_cancels_and_library_recovers(lib):
    A = synth.uniform(4, 1, 400, 400, 7)
    with pytest.raises(GfechError) as ex:
        lib.echelonise(A, 7, block_rows=8, block_cols=8, timeout_ms=1)
    assert ex.value.status == 7
    B = synth.deficient(4, 2, 60, 70, 7)
    compare(lib.echelonise(B, 7, block_rows=8, block_cols=8, timeout_ms=60000).outputs(), oracle.echelonize(B, 7))


@pytest.mark.parametrize("classes", [1, 2, 3])
def test_size_classes_give_the_same_results(lib, classes):
    """One engine for every size, or one per size class (each with its own
    backend instance and worker thread): the same results, equal to the
    oracle's."""
    rng = np.random.default_rng(classes)
    reqs = []
    for t in range(12):
        n = int(rng.choice([20, 300, 700, 2100]))
        m = max(1, int(round(n * rng.uniform(0.75, 1.25))))
        p = int(rng.choice([2, 3, 251]))
        reqs.append((synth.uniform(classes, t, m, n if n < 2000 else 120, p), p))
    srv = lib.server(size_classes=classes)
    tickets = [srv.submit(A, p) for A, p in reqs]
    for (A, p), t in zip(reqs, tickets):
        compare(srv.wait(t).outputs(), oracle.echelonize(A, p), f"{A.shape} p={p}")
    st = srv.stats()
    assert st["admitted"] == st["finished"] == len(reqs)
    srv.close()
