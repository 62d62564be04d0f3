"""Pins for the CPU oracle: the paper's worked example, brute force on tiny
inputs, the closed-form rank counts, known inverses, special cases, and
copies of the oracle with planted mistakes that these pins must catch."""
import os
import re
import shutil
import subprocess
import tempfile
from collections import Counter

import numpy as np
import pytest

import oracle
from oracle import jobs
from tests import _pins as P

PRIMES = [2, 3, 5, 7, 11, 13, 127, 251]


# ---------------------------------------------------------------- worked example (Section 2.2)

def test_example_block_ech_matches_paper():
    g = P.load_golden("paper_example_gf3.json")
    C = np.array(g["C"], np.uint8)
    M, K, R, rho, gamma = jobs.ech(C[:3, :3], 3)
    exp = g["ech_top_left"]
    assert M.tolist() == exp["M"]
    assert K.tolist() == exp["K"]
    assert R.tolist() == exp["R"]
    assert rho.tolist() == exp["rho"]
    assert gamma.tolist() == exp["gamma"]


def test_example_block_ech_identity_matches_printed_rhs():
    g = P.load_golden("paper_example_gf3.json")
    C = np.array(g["C"], np.int64)[:3, :3]
    M, K, R, rho, gamma = jobs.ech(C, 3)
    L = np.zeros((3, 3), np.int64)
    L[:2, :2] = M
    L[2:, :2] = K
    L[2, 2] = 1
    PH = C[np.concatenate([rho, jobs.complement(rho, 3)])][:, np.concatenate([gamma, jobs.complement(gamma, 3)])]
    assert P.matmul_mod(L, PH, 3).tolist() == g["ech_top_left_rhs"]


def test_example_top_right_update():
    """UpdateRow with i = 1 on the top-right block (Section 2.2)."""
    g = P.load_golden("paper_example_gf3.json")
    C = np.array(g["C"], np.uint8)
    M, K, R, rho, gamma = jobs.ech(C[:3, :3], 3)
    V, W = jobs.rex(C[:3, 3:], rho)
    assert V.tolist() == g["top_right_selected_rows"]
    assert W.tolist() == g["top_right_nonselected_rows"]
    assert jobs.mad(W, K, V, 3).tolist() == g["top_right_nonselected_after"]
    assert jobs.mul(M, V, 3).tolist() == g["top_right_selected_after"]


def test_example_bottom_left_clear_and_bottom_right_mad():
    """ClearDown's CEX+MAD and UpdateRow's MAD (1) on the bottom blocks (Section 2.2)."""
    g = P.load_golden("paper_example_gf3.json")
    C = np.array(g["C"], np.uint8)
    M, K, R, rho, gamma = jobs.ech(C[:3, :3], 3)
    A, Ap = jobs.cex(C[3:, :3], gamma)
    assert A.tolist() == g["bottom_left_pivot_cols"]
    assert Ap.tolist() == g["bottom_left_nonpivot_cols"]
    assert jobs.mad(Ap, A, R, 3).tolist() == g["bottom_left_nonpivot_after"]
    V, _ = jobs.rex(C[:3, 3:], rho)
    X = jobs.mul(M, V, 3)
    assert jobs.mad(C[3:, 3:], A, X, 3).tolist() == g["bottom_right_after"]


def test_example_intermediate_matrix():
    g = P.load_golden("paper_example_gf3.json")
    C = np.array(g["C"], np.uint8)
    M, K, R, rho, gamma = jobs.ech(C[:3, :3], 3)
    V, W = jobs.rex(C[:3, 3:], rho)
    A, Ap = jobs.cex(C[3:, :3], gamma)
    X = jobs.mul(M, V, 3)
    top = np.zeros((3, 6), np.uint8)
    top[:2, :3] = [[2, 0, 0], [0, 2, 0]]   # -1 on the pivots
    top[:2, 2:3] = R
    top[2, :3] = 0
    top[:2, 3:] = X
    top[2:, 3:] = jobs.mad(W, K, V, 3)
    bot = np.zeros((3, 6), np.uint8)
    bot[:, 2:3] = jobs.mad(Ap, A, R, 3)
    bot[:, 3:] = jobs.mad(C[3:, 3:], A, X, 3)
    assert np.vstack([top, bot]).tolist() == g["intermediate"]


def test_example_whole_matrix_identities():
    g = P.load_golden("paper_example_gf3.json")
    C = np.array(g["C"], np.uint8)
    e = oracle.echelonize(C, 3)
    P.check_result(C, 3, e.rank, e.gamma, e.rho, e.E, e.T, who="oracle")
    assert e.rank == P.brute_rank(C, 3)


# ---------------------------------------------------------------- brute force on all tiny inputs

@pytest.mark.parametrize("p,m,n", [(2, 3, 3), (3, 2, 3), (2, 2, 4), (5, 2, 2), (2, 4, 2)])
def test_exhaustive_rank_rowspace_and_rref(p, m, n):
    hist = Counter()
    for A in P.all_matrices(p, m, n):
        e = oracle.echelonize(A, p)
        rs = P.rowspace(A, p)
        assert len(rs) == p ** e.rank
        assert P.rowspace(e.E, p) == rs          # same row space, and E is RREF: E is the RREF
        assert P.is_rref(e.E, e.gamma, p)
        P.check_result(A, p, e.rank, e.gamma, e.rho, e.E, e.T)
        hist[e.rank] += 1
    for r in range(min(m, n) + 1):
        assert hist[r] == P.count_rank(p, m, n, r), (r, hist)


@pytest.mark.parametrize("p,m,n", [(2, 4, 3), (3, 3, 2), (2, 3, 4)])
def test_exhaustive_selected_rows_are_lex_first_basis(p, m, n):
    for A in P.all_matrices(p, m, n):
        e = oracle.echelonize(A, p)
        assert e.rho.tolist() == P.lex_first_basis(A, p).tolist()


# ---------------------------------------------------------------- closed forms and identities

@pytest.mark.parametrize("p", PRIMES)
def test_unitriangular_inverse_closed_form(p):
    """U = 1 + N, N strictly upper triangular: U^-1 = sum_k (-N)^k (finite, N nilpotent)."""
    rng = np.random.default_rng(p)
    n = 9
    N = np.triu(rng.integers(0, p, (n, n)), 1)
    U = (np.eye(n, dtype=np.int64) + N) % p
    inv = np.eye(n, dtype=np.int64)
    term = np.eye(n, dtype=np.int64)
    for _ in range(n):
        term = P.matmul_mod(term, (-N) % p, p)
        inv = (inv + term) % p
    e = oracle.echelonize(U.astype(np.uint8), p)
    assert e.rank == n
    assert np.array_equal(e.T.astype(np.int64), inv)
    assert np.array_equal(e.M.astype(np.int64), (-inv) % p)


@pytest.mark.parametrize("p", PRIMES)
def test_full_rank_transform_is_inverse(p):
    rng = np.random.default_rng(100 + p)
    for n in (1, 2, 5, 17):
        for _ in range(20):
            A = rng.integers(0, p, (n, n)).astype(np.uint8)
            e = oracle.echelonize(A, p)
            if e.rank < n:
                continue
            assert e.gamma.tolist() == list(range(n)) and e.rho.tolist() == list(range(n))
            assert np.array_equal(P.matmul_mod(e.T, A, p), np.eye(n))
            assert np.array_equal(P.matmul_mod(A, e.T, p), np.eye(n))


@pytest.mark.parametrize("p", PRIMES)
@pytest.mark.parametrize("shape", [(7, 7), (12, 5), (5, 12), (1, 9), (9, 1), (16, 16)])
def test_random_identities(p, shape):
    rng = np.random.default_rng(hash((p,) + shape) % 2 ** 32)
    m, n = shape
    for trial in range(6):
        A = rng.integers(0, p, (m, n)).astype(np.uint8)
        if trial % 2 and m > 2:
            # rank deficiency: some rows become combinations of others
            k = rng.integers(1, m)
            idx = rng.choice(m, size=k, replace=False)
            rest = np.setdiff1d(np.arange(m), idx)
            coef = rng.integers(0, p, (k, len(rest)))
            A[idx] = P.matmul_mod(coef, A[rest], p)
        e = oracle.echelonize(A, p)
        P.check_result(A, p, e.rank, e.gamma, e.rho, e.E, e.T)


def test_prefix_rank_property():
    """Pivots among the first k columns = rank of those columns (Section 3.1, after Eq. (3))."""
    rng = np.random.default_rng(7)
    p = 3
    A = rng.integers(0, p, (10, 12)).astype(np.uint8)
    A[3] = (A[0] + 2 * A[1]) % p
    e = oracle.echelonize(A, p)
    for k in range(0, 13):
        sub = oracle.echelonize(A[:, :k], p)
        assert int(np.sum(e.gamma < k)) == sub.rank


# ---------------------------------------------------------------- special and degenerate cases

@pytest.mark.parametrize("p", [2, 3, 251])
def test_zero_matrix(p):
    e = oracle.echelonize(np.zeros((4, 6), np.uint8), p)
    assert e.rank == 0 and np.array_equal(e.T, np.eye(4))


@pytest.mark.parametrize("p", [2, 3, 251])
def test_identity(p):
    e = oracle.echelonize(np.eye(5, dtype=np.uint8), p)
    assert e.rank == 5
    assert np.array_equal(e.M.astype(np.int64), (-np.eye(5, dtype=np.int64)) % p)
    assert e.K.shape == (0, 5) and e.R.shape == (5, 0)


@pytest.mark.parametrize("p", [2, 5, 251])
def test_duplicate_row_gives_minus_unit_K(p):
    rng = np.random.default_rng(p)
    A = rng.integers(0, p, (4, 6)).astype(np.uint8)
    A = np.vstack([A, A[1:2]])
    e = oracle.echelonize(A, p)
    if 1 in e.rho.tolist() and 4 not in e.rho.tolist():
        s = e.rho.tolist().index(1)
        krow = e.K[list(e.rho_bar).index(4)].astype(np.int64)
        exp = np.zeros(e.rank, np.int64)
        exp[s] = p - 1
        assert np.array_equal(krow, exp)


def test_empty_shapes():
    e = oracle.echelonize(np.zeros((0, 5), np.uint8), 3)
    assert e.rank == 0 and e.T.shape == (0, 0)
    e = oracle.echelonize(np.zeros((3, 0), np.uint8), 3)
    assert e.rank == 0 and np.array_equal(e.T, np.eye(3))


def test_errors():
    with pytest.raises(oracle.OracleError):
        oracle.echelonize(np.zeros((2, 2), np.uint8), 4)
    with pytest.raises(oracle.OracleError):
        oracle.echelonize(np.zeros((2, 2), np.uint8), 257)
    with pytest.raises(oracle.OracleError):
        oracle.echelonize(np.full((2, 2), 3, np.uint8), 3)


def test_mad_two_ways():
    rng = np.random.default_rng(0)
    for p in (2, 7, 251):
        A = rng.integers(0, p, (5, 7)).astype(np.uint8)
        B = rng.integers(0, p, (5, 9)).astype(np.uint8)
        C = rng.integers(0, p, (9, 7)).astype(np.uint8)
        assert np.array_equal(oracle.mad_c(A, B, C, p), jobs.mad(A, B, C, p))
    # closed form: ones x ones = k
    assert np.all(oracle.mad_c(None, np.ones((3, 10), np.uint8), np.ones((10, 4), np.uint8), 7) == 3)


def test_bitset_jobs_definitions():
    rho, u = jobs.unh([1, 4], [0, 2], 6)       # complement of {1,4} = {0,2,3,5}; picks 0 and 3
    assert rho.tolist() == [0, 1, 3, 4] and u.tolist() == [1, 0, 1, 0]
    rho, u = jobs.un0([1, 2], 4)
    assert rho.tolist() == [1, 2] and u.tolist() == [1, 1]
    assert jobs.mkr([2, 7], [1, 2, 5, 7]).tolist() == [1, 0, 1, 0]
    out = jobs.rrf([1, 0, 0, 1], np.array([[1, 1], [2, 2]]), np.array([[5, 5], [6, 6]]))
    assert out.tolist() == [[5, 5], [1, 1], [2, 2], [6, 6]]
    assert jobs.crz(np.array([[1, 2]]), [0, 1, 0]).tolist() == [[1, 0, 2]]
    assert jobs.adi(np.zeros((2, 3)), [1, 0, 1]).tolist() == [[1, 0, 0], [0, 0, 1]]


# ---------------------------------------------------------------- planted mistakes must be caught

MUTANTS = {
    "no_back_reduction": ("if (g) row_axpy(s, row, p - g, p, w);", ";"),
    "wrong_sign_reduce": ("if (f) row_axpy(row, W + piv_row[t] * w, p - f, p, w);",
                          "if (f) row_axpy(row, W + piv_row[t] * w, f, p, w);"),
    "last_nonzero_pivot": ("if (row[j]) { c = j; break; }", "if (row[j]) { c = j; }"),
    "no_scale": ("row_scale(row, inv_mod(row[c], p), p, w);", ";"),
    "bad_inverse": ("return pow_mod(a, p - 2, p);", "return pow_mod(a, p - 1, p);"),
    "identity_not_augmented": ("W[i * w + n + i] = 1;", ";"),
    "unsorted_pivots": ("while (b >= 0 && piv_col[b] > c)", "while (0)"),
}


def _pins_fail(lib):
    """Run a quick set of pins against an oracle library; True if any pin fails."""
    g = P.load_golden("paper_example_gf3.json")
    C = np.array(g["C"], np.uint8)
    try:
        b = oracle.echelonize(C[:3, :3], 3, lib=lib)
        if b.M.tolist() != g["ech_top_left"]["M"] or b.K.tolist() != g["ech_top_left"]["K"] \
                or b.R.tolist() != g["ech_top_left"]["R"]:
            return True
        for p, m, n in [(2, 3, 3), (3, 2, 3)]:
            for A in P.all_matrices(p, m, n):
                e = oracle.echelonize(A, p, lib=lib)
                if len(P.rowspace(A, p)) != p ** e.rank:
                    return True
                P.check_result(A, p, e.rank, e.gamma, e.rho, e.E, e.T)
        rng = np.random.default_rng(5)
        for p in (5, 251):
            A = rng.integers(0, p, (6, 8)).astype(np.uint8)
            A[4] = A[0]
            e = oracle.echelonize(A, p, lib=lib)
            P.check_result(A, p, e.rank, e.gamma, e.rho, e.E, e.T)
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
    lib = oracle.load_library(str(so))
    assert _pins_fail(lib), f"mutant {name} passed every pin"


def test_unmutated_oracle_passes_quick_pins():
    assert not _pins_fail(oracle._load())
