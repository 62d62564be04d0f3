"""Serving on the GPU (continuous batching) through the C ABI: requests of
varying size and field submitted while others run; every result equals the
oracle's and the same problem solved alone, bit for bit."""
import numpy as np
import pytest

import oracle
import synth
from paper_1806_04211_amd.api import GfechError
from tests.gpu_util import dev, gpu_library, say, torch_cuda
from tests.test_gpu_parity import compare

pytestmark = pytest.mark.gpu


def mixed(seed, count):
    rng = np.random.default_rng([seed, 55])
    out = []
    for t in range(count):
        p = int(rng.choice([2, 3, 5, 251]))
        n = int(np.rint(np.exp(rng.uniform(np.log(8), np.log(1100)))))     # some span several blocks
        m = max(1, int(round(n * rng.uniform(0.75, 1.25))))
        A = synth.deficient(seed, t, m, n, p) if t % 4 == 0 and m > 2 else synth.uniform(seed, t, m, n, p)
        out.append((A, p))
    return out


def test_server_mix_matches_oracle_and_solo():
    lib = gpu_library()
    reqs = mixed(7, 24)
    say(f"server mix of {len(reqs)}: largest {max(A.shape for A, _ in reqs)}")
    srv = lib.server()
    tickets = [srv.submit(A, p) for A, p in reqs]
    results = {t: srv.wait(t) for t in tickets}
    for (A, p), t in zip(reqs, tickets):
        o = results[t].outputs()
        compare(o, oracle.echelonize(A, p), f"{A.shape} p={p}")
        compare(o, lib.echelonise(A, p).outputs(), f"solo {A.shape} p={p}")
    srv.close()


def test_server_device_inputs_and_budget():
    torch = torch_cuda()
    lib = gpu_library()
    reqs = mixed(8, 10)
    bufs = [dev(torch, A) for A, _ in reqs]
    srv = lib.server(hbm_budget_bytes=64 << 20, max_active=3)
    tickets = [srv.submit_dev(b.data_ptr(), A.shape[0], A.shape[1], A.shape[1], p) for b, (A, p) in zip(bufs, reqs)]
    for (A, p), t in zip(reqs, tickets):
        compare(srv.wait(t).outputs(), oracle.echelonize(A, p), f"{A.shape} p={p}")
    with pytest.raises(GfechError) as ex:
        srv.submit(np.zeros((8000, 8000), np.uint8), 3)
    assert ex.value.status == 5
    st = srv.stats()
    assert st["admitted"] == st["finished"] == len(reqs)
    assert 0 < st["peak_bytes_in_flight"] <= 64 << 20 and 1 <= st["peak_active"] <= 3
    srv.close()


def test_server_cancel_and_device_inputs_reused_at_once():
    """Device inputs are copied before submit returns (the caller overwrites
    its buffer right away); a cancelled request answers GFECH_E_CANCELLED or,
    if it had already finished, the right result; the rest are unaffected."""
    torch = torch_cuda()
    lib = gpu_library()
    reqs = mixed(9, 8)
    srv = lib.server()
    tickets = []
    buf = torch.empty(max(A.size for A, _ in reqs), dtype=torch.uint8, device="cuda:0")
    for A, p in reqs:
        buf[: A.size] = torch.from_numpy(A.ravel().copy()).to("cuda:0")
        torch.cuda.synchronize()             # the server's streams do not wait for torch's
        tickets.append(srv.submit_dev(buf.data_ptr(), A.shape[0], A.shape[1], A.shape[1], p))
        buf.fill_(255)                       # not a residue: a late copy would be refused or wrong
    torch.cuda.synchronize()
    srv.cancel(tickets[3])
    for t, ((A, p), tk) in enumerate(zip(reqs, tickets)):
        try:
            compare(srv.wait(tk).outputs(), oracle.echelonize(A, p), f"request {t}")
        except GfechError as e:
            assert t == 3 and e.status == 7
    srv.close()


def test_watchdog_cancels_a_long_solve():
    torch = torch_cuda()
    lib = gpu_library()
    from synth import torch_gen
    say("watchdog: 6000 x 6000 GF(7) with a 1 ms limit")
    A = torch_gen.uniform(0, 3, 6000, 6000, 7)
    with pytest.raises(GfechError) as ex:
        lib.echelonise_dev(A.data_ptr(), 6000, 6000, 6000, 7, timeout_ms=1)
    assert ex.value.status == 7
    B = synth.deficient(1, 5, 700, 600, 7)
    compare(lib.echelonise(B, 7, timeout_ms=60000).outputs(), oracle.echelonize(B, 7), "after the watchdog")
