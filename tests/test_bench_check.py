"""The benchmark's host-side check of a solve (rank, orders, reduced echelon
shape, Freivalds on Eq. (2)) accepts the oracle's outputs and rejects each
planted mistake.  CPU only: the outputs come from the oracle."""
import numpy as np
import pytest

import bench
import oracle
import synth


class _Fake:
    """The getters of a library result, answered from oracle outputs."""

    def __init__(self, e, **override):
        self.e = e
        self.o = override

    @property
    def rank(self):
        return self.o.get("rank", self.e.rank)

    def pivots(self):
        return self.o.get("gamma", self.e.gamma), self.e.rho

    def nonpivots(self):
        return self.e.gamma_bar, self.e.rho_bar

    def get_R(self):
        return self.o.get("R", self.e.R)

    def get_M(self):
        return self.o.get("M", self.e.M)

    def get_K(self):
        return self.o.get("K", self.e.K)


@pytest.mark.parametrize("p", [2, 7, 251])
def test_check_accepts_oracle_and_rejects_mistakes(p):
    A = synth.deficient(3, p, 90, 120, p)
    A[:, 2] = 0                       # a non-pivot column before most pivots
    e = oracle.echelonize(A, p)
    assert 0 < e.rank < 90
    assert bench.check_result(A, _Fake(e), p, e.rank)["ok"]
    # a wrong rank expectation
    assert not bench.check_result(A, _Fake(e), p, e.rank + 1)["rank_ok"]
    # one entry of M, K or R changed
    for name in ("M", "K", "R"):
        X = getattr(e, name).copy()
        X[len(X) // 2, X.shape[1] // 3] = (int(X[len(X) // 2, X.shape[1] // 3]) + 1) % p
        got = bench.check_result(A, _Fake(e, **{name: X}), p, e.rank)
        assert not got["freivalds_ok"] and not got["ok"], name
    # a non-zero entry left of a pivot: the reduced echelon shape check
    R = e.R.copy()
    t = int(np.argmax(e.gamma - np.arange(e.rank) > 0))
    assert e.gamma[t] - t > 0
    R[t, 0] = 1
    assert not bench.check_result(A, _Fake(e, R=R), p, e.rank)["rref_ok"]
    # pivot columns out of order
    g = e.gamma.copy()
    g[[0, 1]] = g[[1, 0]]
    assert not bench.check_result(A, _Fake(e, gamma=g), p, e.rank)["ok"]


def test_exact_matmul_mod_matches_int64():
    rng = np.random.default_rng(0)
    for p, k in ((7, 5000), (251, 300), (251, 3000)):
        X = rng.integers(0, p, (50, k)).astype(np.uint8)
        Y = rng.integers(0, p, (k, 9)).astype(np.uint8)
        exp = (X.astype(np.int64) @ Y.astype(np.int64)) % p
        assert np.array_equal(bench.exact_matmul_mod(X, Y, p, chunk_rows=16), exp)


def test_mad_trace_matches_the_work_counters(tmp_path, monkeypatch):
    """The opt-in launch trace (read by the benchmark's isolated replay) lists
    every MAD descriptor once, with its kind: per kind, the traced
    multiply-adds equal the result's work counters (emulator build)."""
    from tests import emu
    lib = emu.library()
    path = tmp_path / "trace.txt"
    monkeypatch.setenv("GFECH_TRACE_MAD", str(path))
    A = synth.deficient(4, 4, 60, 50, 7)
    res = lib.echelonise(A, 7, block_rows=8, block_cols=12)
    st = res.stats()
    tr = bench.read_mad_trace(str(path))
    assert tr and all(d["A"] and d["D"] and d["p"] == 7 for d in tr)
    mac = {k: sum(float(d["M"]) * d["N"] * d["K"] for d in tr if d["kind"] == k) for k in (1, 2, 3, 4)}
    assert mac[1] == st["mac_cleardown"] and mac[2] == st["mac_updaterow"]
    assert mac[3] == st["mac_trafo"] and mac[4] == st["mac_clearup"]
    assert len({d["it"] for d in tr if d["kind"] == 1}) > 3


def test_committed_profile_matches_the_sources():
    """The committed rocprofv3 summary of the isolated MAD launches was taken on
    the current kernel source and blocking table, so the benchmark reports its
    traffic figure (a kernel or table change needs a new profile)."""
    import bench
    assert bench.profiled_traffic() is not None
