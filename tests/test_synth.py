"""The seeded input generators: published SplitMix64 outputs, ranges, and
the rank structure the workloads promise."""
import numpy as np

import oracle
import synth


def test_splitmix64_published_sequence():
    # SplitMix64 started from state 0 (Steele, Lea and Flood 2014; Vigna's reference code)
    got = synth.mix64(np.arange(1, 5, dtype=np.uint64) * synth.GAMMA)
    assert [int(x) for x in got] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                    0x06C45D188009454F, 0xF88BB8A8724C81EC]


def test_uniform_range_and_determinism():
    for p in (2, 3, 7, 251):
        A = synth.uniform(0, 0, 64, 80, p)
        assert A.dtype == np.uint8 and A.max() < p
        assert np.array_equal(A, synth.uniform(0, 0, 64, 80, p))
        assert not np.array_equal(A, synth.uniform(1, 0, 64, 80, p))
    A = synth.uniform(3, 5, 40, 33, 7)
    assert np.array_equal(A[10:17], synth.uniform_rows(3, 5, 10, 7, 33, 7))


def test_low_rank_product_rank():
    A = synth.low_rank_product(0, 60, 70, 50, 7)
    assert oracle.echelonize(A, 7).rank <= 50


def test_deficient_is_deficient():
    for t in range(5):
        A = synth.deficient(0, t, 40, 40, 5)
        assert oracle.echelonize(A, 5).rank < 40


def test_gf2_pack_roundtrip():
    A = synth.uniform(4, 0, 7, 130, 2)
    W = synth.gf2_pack(A)
    assert W.shape == (7, 3)
    assert np.array_equal(synth.gf2_unpack(W, 130), A)
    assert int(W[0, 0]) & 1 == int(A[0, 0])


def test_low_rank_product_float_path_is_exact():
    # the float64 product equals the plain int64 one (sums below 2^53)
    for (m, n, k, p) in ((30, 40, 20, 7), (64, 50, 33, 251), (17, 9, 5, 2)):
        B = synth.uniform(1, 1, m, k, p).astype(np.int64)
        C = synth.uniform(1, 2, k, n, p).astype(np.int64)
        assert np.array_equal(synth.low_rank_product(1, m, n, k, p), ((B @ C) % p).astype(np.uint8))


def test_gf2_deficient_packed_pins():
    """The large GF(2) construction at a small size: pad bits clear, rank
    m - deficiency, selected rows the first m - deficiency (the pins its full
    size is checked by), through the oracle."""
    m, n, d = 150, 200, 12
    W = synth.gf2_deficient_packed(4, m, n, d, terms=9)
    assert not np.any(W[:, -1] >> np.uint64(n % 64))
    e = oracle.echelonize(synth.gf2_unpack(W, n), 2)
    assert e.rank == m - d
    assert np.array_equal(e.rho, np.arange(m - d))
