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
    srv.close()
