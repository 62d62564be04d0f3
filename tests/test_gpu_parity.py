"""End-to-end parity on the GPU through the C ABI: every output of the
blocked method (rank, pivots, selected rows, R, M, K, the RREF E and T)
against the oracle, bit for bit."""
import numpy as np
import pytest

import oracle
import synth
from tests import _pins as P
from tests.gpu_util import dev, gpu_library, say, torch_cuda

pytestmark = pytest.mark.gpu


def compare(o, e, where=""):
    assert o.rank == e.rank, where
    for name in ("gamma", "rho", "gamma_bar", "rho_bar", "R", "M", "K", "E", "T"):
        assert np.array_equal(getattr(o, name), getattr(e, name)), f"{where}: {name}"


CASES = [
    # (m, n, p, block_rows, block_cols, kind)
    (40, 40, 3, 8, 8, "uniform"),
    (96, 64, 2, 32, 16, "deficient"),
    (64, 96, 251, 16, 32, "uniform"),
    (130, 130, 7, 64, 64, "lowrank"),
    (200, 150, 5, 48, 37, "deficient"),
    (257, 257, 251, 128, 128, "uniform"),
    (300, 300, 3, 300, 300, "deficient"),
    (512, 512, 7, 128, 128, "lowrank"),
    (333, 500, 2, 100, 125, "uniform"),
]


def make(kind, m, n, p, seed):
    if kind == "uniform":
        return synth.uniform(seed, 0, m, n, p)
    if kind == "deficient":
        return synth.deficient(seed, 0, m, n, p)
    return synth.low_rank_product(seed, m, n, min(m, n) * 3 // 4, p)


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}-p{c[2]}-b{c[3]}x{c[4]}-{c[5]}" for c in CASES])
def test_blocked_method_matches_oracle(case):
    lib = gpu_library()
    m, n, p, br, bc, kind = case
    say(f"echelonise {case}")
    A = make(kind, m, n, p, seed=m + n)
    o = lib.echelonise(A, p, block_rows=br, block_cols=bc).outputs()
    compare(o, oracle.echelonize(A, p), str(case))


def test_device_input_and_default_blocking():
    torch = torch_cuda()
    import paper_1806_04211_amd as gf
    A = synth.uniform(0, 0, 1000, 1000, 3)          # the 1000 x 1000 GF(3) workload, seed 0
    say("echelonise 1000x1000 GF(3) seed 0 (device input)")
    t = torch.from_numpy(A).to("cuda:0")
    o = gf.echelonise_tensor(t, 3).outputs()
    compare(o, oracle.echelonize(A, 3), "1000x1000")


def test_device_range_check():
    torch = torch_cuda()
    import paper_1806_04211_amd as gf
    A = np.zeros((20, 20), np.uint8)
    A[3, 4] = 7
    with pytest.raises(gf.GfechError) as ex:
        gf.echelonise_tensor(torch.from_numpy(A).to("cuda:0"), 7)
    assert ex.value.status == 3


def test_batch_mixed_sizes_and_fields():
    lib = gpu_library()
    mix = synth.batch_mix(5, 48, nmin=8, nmax=160)
    say("batch of 48")
    res, sts = lib.echelonise_batch(mix)
    assert all(s == 0 for s in sts)
    for t, ((A, p), r) in enumerate(zip(mix, res)):
        compare(r.outputs(), oracle.echelonize(A, p), f"problem {t}")


def test_full_rank_inverse():
    lib = gpu_library()
    p = 251
    A = synth.uniform(8, 0, 192, 192, p)
    say("inverse 192")
    o = lib.echelonise(A, p, block_rows=64, block_cols=64).outputs()
    assert o.rank == 192
    assert np.array_equal(P.matmul_mod(o.T, A, p), np.eye(192))
    assert np.array_equal(P.matmul_mod(A, o.T, p), np.eye(192))


def test_profile_levels_time_the_mad_launches():
    """Device-event timing leaves the results alone; level 2 times every MAD
    launch (their multiply-adds are the method's MAD work), level 3 about a
    quarter of them."""
    torch = torch_cuda()
    lib = gpu_library()
    m = n = 768
    p = 7
    A = synth.uniform(5, 0, m, n, p)
    say("echelonise 768x768 GF(7) blocks 128x128, profile levels 0 2 3")
    t = torch.from_numpy(A).to("cuda:0")
    e = oracle.echelonize(A, p)
    runs = {}
    for level in (0, 2, 3):
        r = lib.echelonise_dev(t.data_ptr(), m, n, n, p, block_rows=128, block_cols=128, profile=level)
        torch.cuda.synchronize()
        compare(r.outputs(), e, f"profile {level}")
        runs[level] = r.stats()
        r.free()
    s0, s2, s3 = runs[0], runs[2], runs[3]
    mad_total = s0["mac_cleardown"] + s0["mac_updaterow"] + s0["mac_trafo"] + s0["mac_clearup"]
    assert s0["launches_mad"] == 0 and s0["mac_mad_timed"] == 0
    assert s2["launches_mad"] > 8 and s2["ms_mad"] > 0
    assert s2["mac_mad_timed"] == mad_total
    assert 0 < s3["launches_mad"] < s2["launches_mad"]
    assert 0 < s3["mac_mad_timed"] < mad_total


@pytest.mark.parametrize("variant", [1, 2])
def test_variants_at_default_blocking(variant):
    """The reduced echelon form alone and the rank alone (several block rows
    and 2048-wide block columns) equal the oracle's outputs."""
    lib = gpu_library()
    m, n, p = 768, 5000, 5
    A = synth.deficient(9, 1, m, n, p)
    A[:, 100:2300] = 0
    say(f"echelonise {m}x{n} GF({p}) variant {variant}")
    o = lib.echelonise(A, p, variant=variant).outputs()
    e = oracle.echelonize(A, p)
    assert o.variant == variant and o.rank == e.rank
    for name in ("gamma", "rho", "gamma_bar", "rho_bar"):
        assert np.array_equal(getattr(o, name), getattr(e, name)), name
    assert o.M is None and o.K is None and o.T is None
    if variant == 1:
        assert np.array_equal(o.R, e.R) and np.array_equal(o.E, e.E)
    else:
        assert o.R is None and o.E is None


@pytest.mark.parametrize("shape", [(300, 200, 96, 80), (700, 1100, 0, 0), (64, 65, 0, 0)])
def test_gf2_packed_input(shape):
    """Bit-packed GF(2) input (host and device), unpacked on the device, equals
    the oracle over p = 2."""
    torch = torch_cuda()
    lib = gpu_library()
    m, n, br, bc = shape
    A = synth.deficient(2, 77, m, n, 2)
    W = synth.gf2_pack(A)
    e = oracle.echelonize(A, 2)
    say(f"echelonise gf2 packed {m}x{n} (host input)")
    compare(lib.echelonise_gf2(W, n, block_rows=br, block_cols=bc).outputs(), e, "host")
    say(f"echelonise gf2 packed {m}x{n} (device input, ldw {W.shape[1] + 1})")
    Wd = np.concatenate([W, np.zeros((m, 1), np.uint64)], axis=1)
    t = torch.from_numpy(Wd.view(np.int64).copy()).to("cuda:0")
    r = lib.echelonise_gf2_dev(t.data_ptr(), m, n, Wd.shape[1], block_rows=br, block_cols=bc)
    compare(r.outputs(), e, "device")
    if n % 64:
        Wd[5, n // 64] |= np.uint64(1) << np.uint64(63)
        t = torch.from_numpy(Wd.view(np.int64).copy()).to("cuda:0")
        import paper_1806_04211_amd as gf
        with pytest.raises(gf.GfechError) as ex:
            lib.echelonise_gf2_dev(t.data_ptr(), m, n, Wd.shape[1])
        assert ex.value.status == 3


def test_batch_device_inputs_range_checked_together():
    """Device inputs of a batch are range-checked in one pass: the problem with
    an entry >= p is refused, the others are solved."""
    torch = torch_cuda()
    lib = gpu_library()
    mix = synth.batch_mix(21, 12, nmin=8, nmax=120)
    bufs = [dev(torch, A) for A, _ in mix]
    bad_t = 5
    A5, p5 = mix[bad_t]
    A5 = A5.copy()
    A5[A5.shape[0] // 2, 1] = p5          # not a residue
    bufs[bad_t] = dev(torch, A5)
    probs = [(b.data_ptr(), A.shape[0], A.shape[1], A.shape[1], p) for b, (A, p) in zip(bufs, mix)]
    say("batch of 12 device inputs, one out of range")
    res, sts = lib.echelonise_batch(probs, on_device=True)
    for t, ((A, p), r, s) in enumerate(zip(mix, res, sts)):
        if t == bad_t:
            assert s == 3 and r is None
        else:
            assert s == 0
            compare(r.outputs(), oracle.echelonize(A, p), f"problem {t}")
