"""Host checks of the float-quotient reductions the HIP kernels use, in the
same float32 arithmetic (round to nearest even, as the GPU's v_mul_f32):

* v mod p for v < 2^22 with inv = fl(1/p): q = trunc(fl(v inv)) is floor(v / p)
  or one less, so r = v - q p lies in [0, 2p) and one conditional subtraction
  finishes;
* v mod p for v < 2^17 with inv17 = fl(fl(1/p) (1 + 2^-18)): q is floor(v / p)
  exactly, so r = v - q p needs no correction (also with fl(1/p) one ulp off).

Exhaustive over every p <= 251 for the 2^17 form; for the 2^22 form over all
v below 2^22 for a spread of primes and the largest."""
import numpy as np
import pytest

PRIMES = [p for p in range(2, 252) if all(p % d for d in range(2, int(p ** 0.5) + 1))]


def _inv17(p, ulp=0):
    inv = np.float32(1.0) / np.float32(p)
    if ulp:
        inv = np.nextafter(inv, np.float32(np.inf) if ulp > 0 else np.float32(0))
    return np.float32(inv * np.float32(1.0 + 2.0 ** -18))


@pytest.mark.parametrize("ulp", [0, -1, 1])
def test_mod17_quotient_exact(ulp):
    v = np.arange(0, 1 << 17, dtype=np.int64)
    vf = v.astype(np.float32)
    for p in range(2, 252):
        q = np.trunc(vf * _inv17(p, ulp)).astype(np.int64)
        assert np.array_equal(q, v // p), p


def test_mod17_fails_beyond_its_range():
    # the bound is not idle: 2^22 inputs do produce an off-by-one quotient
    v = np.arange(1 << 17, 1 << 22, dtype=np.int64)
    vf = v.astype(np.float32)
    assert any(not np.array_equal(np.trunc(vf * _inv17(p)).astype(np.int64), v // p) for p in PRIMES)


@pytest.mark.parametrize("p", [2, 3, 7, 43, 127, 251])
def test_mod22_one_correction(p):
    v = np.arange(0, 1 << 22, dtype=np.int64)
    inv = np.float32(1.0) / np.float32(p)
    q = np.trunc(v.astype(np.float32) * inv).astype(np.int64)
    r = v - q * p
    assert r.min() >= 0 and r.max() < 2 * p
    assert np.array_equal(np.where(r >= p, r - p, r), v % p)
