"""Pins of the packed GF(2) oracle (oracle_echelon_gf2, oracle_mad_gf2): it
must satisfy the structural identities of Eq. (2) on its own (checked after
unpacking by tests/_pins.check_result), match brute-force row spaces on every
tiny matrix, agree with the byte oracle over p = 2 (itself pinned to the
paper's worked example), and fail a pin for each planted mistake."""
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from tests import _pins as P


def unpacked(e, n):
    E = synth.gf2_unpack(e.E, n) if e.rank else np.zeros((0, n), np.uint8)
    T = synth.gf2_unpack(e.T, e.m) if e.m else np.zeros((0, 0), np.uint8)
    return E, T


@pytest.mark.parametrize("shape", [(2, 3), (3, 3), (3, 2), (4, 2)])
def test_exhaustive_tiny(shape):
    m, n = shape
    for A in P.all_matrices(2, m, n):
        e = oracle.echelonize_gf2(synth.gf2_pack(A), n)
        assert len(P.rowspace(A, 2)) == 2 ** e.rank
        assert np.array_equal(e.rho, P.lex_first_basis(A, 2))
        E, T = unpacked(e, n)
        P.check_result(A, 2, e.rank, e.gamma, e.rho, E, T)


@pytest.mark.parametrize("shape", [(1, 1), (5, 70), (70, 5), (64, 64), (65, 129), (130, 100), (200, 200)])
def test_matches_byte_oracle_and_identities(shape):
    m, n = shape
    for seed in range(3):
        A = synth.deficient(seed, m + n, m, n, 2) if m > 2 else synth.uniform(seed, 1, m, n, 2)
        if n > 3:
            A[:, n // 3] = 0
        e = oracle.echelonize_gf2(synth.gf2_pack(A), n)
        b = oracle.echelonize(A, 2)
        assert e.rank == b.rank
        assert np.array_equal(e.gamma, b.gamma) and np.array_equal(e.rho, b.rho)
        E, T = unpacked(e, n)
        assert np.array_equal(E, b.E) and np.array_equal(T, b.T)
        if m * n <= 130 * 100:
            P.check_result(A, 2, e.rank, e.gamma, e.rho, E, T)


def test_large_construction_pins():
    """The large GF(2) workload's construction at 600 x 700: rank and selected
    rows as pinned, T A = [E; 0] by packed parity."""
    m, n, d = 600, 700, 40
    W = synth.gf2_deficient_packed(4, m, n, d, terms=11)
    e = oracle.echelonize_gf2(W, n)
    assert e.rank == m - d and np.array_equal(e.rho, np.arange(m - d))
    A = synth.gf2_unpack(W, n)
    E, T = unpacked(e, n)
    TA = P.matmul_mod(T, A, 2)
    assert np.array_equal(TA[: e.rank], E) and not np.any(TA[e.rank:])


def test_mad_gf2_against_byte_products():
    rng = np.random.default_rng(0)
    for (m, k, n) in ((1, 1, 1), (7, 65, 130), (33, 200, 64), (64, 64, 200)):
        A = rng.integers(0, 2, (m, k)).astype(np.uint8)
        B = rng.integers(0, 2, (k, n)).astype(np.uint8)
        C = rng.integers(0, 2, (m, n)).astype(np.uint8)
        got = oracle.mad_gf2(synth.gf2_pack(C), synth.gf2_pack(A), synth.gf2_pack(B), k, n)
        assert np.array_equal(synth.gf2_unpack(got, n), (C.astype(np.int64) + A.astype(np.int64) @ B) % 2)
        # closed form: all-ones operands give the parity of k in every entry
        ones = oracle.mad_gf2(None, synth.gf2_pack(np.ones((m, k), np.uint8)),
                              synth.gf2_pack(np.ones((k, n), np.uint8)), k, n)
        assert np.all(synth.gf2_unpack(ones, n) == k % 2)


def test_pad_bits_rejected():
    W = synth.gf2_pack(np.eye(3, dtype=np.uint8))
    W[1, 0] |= np.uint64(1) << np.uint64(5)
    with pytest.raises(oracle.OracleError):
        oracle.echelonize_gf2(W, 4)


MUTANTS = {
    "no_back_reduction": ("for (int64_t k = 0; k < w; ++k) s[k] ^= row[k];", ";"),
    "last_nonzero_pivot": ("if ((row[j / 64] >> (j % 64)) & 1u) { c = j; break; }",
                           "if ((row[j / 64] >> (j % 64)) & 1u) { c = j; }"),
    "identity_not_augmented": ("W[i * w + wn + i / 64] |= 1ull << (i % 64);", ";"),
    "unsorted_pivots": ("b > 0 && piv_col[b - 1] > piv_col[b]", "0"),
    "identity_bit_off_by_one": ("W[i * w + wn + i / 64] |= 1ull << (i % 64);",
                                "W[i * w + wn + (i + 1) / 64] |= 1ull << ((i + 1) % 64);"),
}


def _pins_fail(lib):
    try:
        for (m, n) in ((2, 3), (3, 3)):
            for A in P.all_matrices(2, m, n):
                e = oracle.echelonize_gf2(synth.gf2_pack(A), n, lib=lib)
                if len(P.rowspace(A, 2)) != 2 ** e.rank:
                    return True
                E, T = unpacked(e, n)
                P.check_result(A, 2, e.rank, e.gamma, e.rho, E, T)
        A = synth.deficient(3, 3, 70, 90, 2)
        e = oracle.echelonize_gf2(synth.gf2_pack(A), 90, lib=lib)
        E, T = unpacked(e, 90)
        P.check_result(A, 2, e.rank, e.gamma, e.rho, E, T)
    except (AssertionError, oracle.OracleError):
        return True
    return False


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "gf_oracle.c")).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, name
    path = tmp_path / "mut.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-shared", "-fPIC", "-o", str(so), str(path)])
    assert _pins_fail(oracle.load_library(str(so))), f"mutant {name} passed every pin"


def test_unmutated_oracle_passes_quick_pins():
    assert not _pins_fail(oracle._load())
