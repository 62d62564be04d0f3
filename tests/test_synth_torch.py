"""The torch generator reproduces the numpy one bit for bit (CPU torch here)."""
import numpy as np
import torch

import synth
from synth import torch_gen


def test_uniform_matches_numpy():
    for p in (2, 7, 251):
        a = synth.uniform(3, 4, 37, 53, p)
        b = torch_gen.uniform(3, 4, 37, 53, p, device="cpu", chunk_rows=10).numpy()
        assert np.array_equal(a, b)


def test_low_rank_product_matches_numpy():
    a = synth.low_rank_product(0, 30, 40, 20, 7)
    b = torch_gen.low_rank_product(0, 30, 40, 20, 7, device="cpu", chunk_rows=7).numpy()
    assert np.array_equal(a, b)


def test_gf2_packed_generators_match_numpy():
    for (m, n, d) in ((40, 130, 5), (9, 64, 0), (70, 200, 20)):
        a = synth.gf2_deficient_packed(3, m, n, d, terms=7)
        b = torch_gen.gf2_deficient_packed(3, m, n, d, terms=7, device="cpu").numpy().view(np.uint64)
        assert np.array_equal(a, b)
