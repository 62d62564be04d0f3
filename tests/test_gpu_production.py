"""End-to-end parity at the library's default blocking (256-row by 2048-column
blocks above 512 x 512): several block rows and several 2048-wide block
columns, so the schedule that produces the large benchmark runs (the four
lanes with their near / mid / far sets, the three copies of the job scratch,
products with an inner dimension near 2048, the leading-columns ECH and its
rerun) is compared with the oracle bit for bit on every output."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import gpu_library, say, torch_cuda
from tests.test_gpu_parity import compare

pytestmark = pytest.mark.gpu


def _zero_band(seed, m, n, p):
    """Uniform rows with a band of zero columns across a block-column boundary
    and duplicated rows: whole block columns hold few or no pivots, so later
    block columns take rows that earlier ones left unselected."""
    A = synth.uniform(seed, 0, m, n, p)
    A[:300, :2500] = 0
    A[:, 4000:4300] = 0
    A[5::7] = A[3::7][: len(A[5::7])]
    return A


CASES = [
    # (name, m, n, p, input)
    ("lowrank-gf7", 1024, 10752, 7, lambda: synth.low_rank_product(3, 1024, 10752, 1000, 7)),
    ("uniform-gf251", 1024, 10752, 251, lambda: synth.uniform(4, 0, 1024, 10752, 251)),
    ("deficient-gf2", 1100, 10000, 2, lambda: synth.deficient(5, 0, 1100, 10000, 2)),
    ("zeroband-gf3", 600, 6200, 3, lambda: _zero_band(6, 600, 6200, 3)),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_default_blocking_matches_oracle(case):
    lib = gpu_library()
    name, m, n, p, make = case
    A = make()
    assert A.shape == (m, n)
    say(f"echelonise {name} {m}x{n} GF({p}) at the default blocking")
    res = lib.echelonise(A, p)
    st = res.stats()
    # the default blocking: 256-row blocks and 2048-wide block columns
    assert st["block_rows"] == -(-m // 256) and st["block_cols"] == -(-n // 2048)
    assert st["block_rows"] >= 3 and st["block_cols"] >= 4
    out = res.outputs()
    res.free()
    say(f"oracle {name}")
    compare(out, oracle.echelonize(A, p), name)


def test_batch_sample_of_the_batched_workload():
    """A sample of the batched workload (n log-uniform in [32, 512], p from
    {2, 3, 5, 7, 251}, 10 % rank-deficient) in one call, each member against
    the oracle."""
    lib = gpu_library()
    mix = synth.batch_mix(11, 64)
    ps = [p for _, p in mix]
    ns = [A.shape[0] for A, _ in mix]
    assert 251 in ps and max(ns) > 400
    say("batch sample of 64, n up to 512")
    res, sts = lib.echelonise_batch(mix)
    assert all(s == 0 for s in sts)
    deficient = 0
    for t, ((A, p), r) in enumerate(zip(mix, res)):
        e = oracle.echelonize(A, p)
        deficient += e.rank < A.shape[0]
        compare(r.outputs(), e, f"problem {t} n={A.shape[0]} p={p}")
        r.free()
    assert deficient >= 3


def test_gf2_packed_default_blocking_matches_oracle():
    """Bit-packed GF(2) rows unpacked straight into the block-row panels, at
    the default blocking (several 2048-wide block columns)."""
    lib = gpu_library()
    m, n = 1000, 6500
    A = synth.uniform(12, 0, m, n, 2)
    A[:, 300:2500] = 0
    A[7::9] = A[2::9][: len(A[7::9])]
    say(f"echelonise gf2 packed {m}x{n} at the default blocking")
    out = lib.echelonise_gf2(synth.gf2_pack(A), n).outputs()
    compare(out, oracle.echelonize(A, 2), "gf2 packed")


def test_gf2_large_construction_pins_and_freivalds():
    """The large GF(2) workload's construction at 12000 x 12000 (deficiency
    100): its pinned rank and selected rows, and Freivalds on Eq. (2) with 64
    vectors, computed on the host outside the library."""
    torch = torch_cuda()
    lib = gpu_library()
    import bench
    from synth import torch_gen
    n, d = 12000, 100
    W = torch_gen.gf2_deficient_packed(4, n, n, d)
    say(f"echelonise gf2 packed {n}x{n}, deficiency {d}")
    res = lib.echelonise_gf2_dev(W.data_ptr(), n, n, W.shape[1])
    A = np.unpackbits(W.cpu().numpy().view(np.uint8), axis=1, bitorder="little")[:, :n]
    chk = bench.check_result(A, res, 2, n - d)
    gamma, rho = res.pivots()
    res.free()
    assert chk["ok"], chk
    assert np.array_equal(rho, np.arange(n - d))


def test_gf2_8192_matches_packed_oracle():
    """8192 x 8192 over GF(2) (the large construction, deficiency 50) against
    the packed oracle, element by element: rank, pivots, selected rows, E and
    T (unpacked from the oracle's words)."""
    torch = torch_cuda()
    lib = gpu_library()
    from synth import torch_gen
    n, d = 8192, 50
    W = torch_gen.gf2_deficient_packed(7, n, n, d, terms=9)
    say(f"echelonise gf2 packed {n}x{n}")
    res = lib.echelonise_gf2_dev(W.data_ptr(), n, n, W.shape[1])
    st = res.stats()
    assert st["block_cols"] >= 2 and st["block_rows"] >= 16
    out = res.outputs()
    res.free()
    say("packed oracle")
    e = oracle.echelonize_gf2(W.cpu().numpy().view(np.uint64), n)
    assert out.rank == e.rank == n - d
    assert np.array_equal(out.gamma, e.gamma) and np.array_equal(out.rho, e.rho)
    assert np.array_equal(out.E, synth.gf2_unpack(e.E, n))
    assert np.array_equal(out.T, synth.gf2_unpack(e.T, n))


def test_grouped_clearup_matches_oracle(monkeypatch):
    """ClearUp groups of about 300 pivots (GFECH_CLEARUP_GROUP) at the default
    blocking: several groups, each cleared inside and then applied to every
    row above it in one product, compared with the oracle."""
    monkeypatch.setenv("GFECH_CLEARUP_GROUP", "300")
    lib = gpu_library()
    A = synth.low_rank_product(7, 1024, 6200, 1000, 7)
    say("echelonise 1024x6200 GF(7), ClearUp groups of 300 pivots")
    out = lib.echelonise(A, 7).outputs()
    compare(out, oracle.echelonize(A, 7), "grouped ClearUp")
