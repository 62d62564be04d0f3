"""Per-kernel parity on the GPU through the C ABI: the MAD job (int8 MFMA,
mod p) and the ECH job, against the oracle's plain definitions."""
import numpy as np
import pytest

import oracle
from oracle import jobs
import synth
from tests.gpu_util import dev, gpu_library, say, torch_cuda

pytestmark = pytest.mark.gpu

MAD_SHAPES = [(1, 1, 1), (17, 33, 5), (128, 128, 64), (130, 257, 65), (300, 129, 200), (64, 1000, 3),
              (513, 70, 130), (7, 9, 300), (256, 384, 1024),
              # 16-byte aligned rows: interior tiles stream through LDS (p <= 127), with a K
              # tail, a single K step, and edge tiles in the same launch
              (512, 256, 208), (256, 256, 96), (600, 400, 320), (256, 128, 64)]
PRIMES = [2, 3, 7, 127, 131, 251]


@pytest.mark.parametrize("p", PRIMES)
@pytest.mark.parametrize("shape", MAD_SHAPES)
def test_mad_plain(shape, p):
    torch = torch_cuda()
    lib = gpu_library()
    M, N, K = shape
    say(f"mad {shape} p={p}")
    rng = np.random.default_rng(M * 7 + N * 13 + K + p)
    A = rng.integers(0, p, (M, K)).astype(np.uint8)
    B = rng.integers(0, p, (K, N)).astype(np.uint8)
    C = rng.integers(0, p, (M, N)).astype(np.uint8)
    dA, dB, dC = dev(torch, A), dev(torch, B), dev(torch, C)
    dD = torch.zeros(M * N, dtype=torch.uint8, device="cuda:0")
    lib.mad_dev(M, N, K, p, dA.data_ptr(), K, dB.data_ptr(), N, dD.data_ptr(), N, C=dC.data_ptr(), ldc=N)
    torch.cuda.synchronize()
    assert np.array_equal(dD.cpu().numpy().reshape(M, N), jobs.mad(C, A, B, p))
    # without C, in place and adversarial all-(p-1) operands
    A[:] = p - 1
    B[:] = p - 1
    dA, dB = dev(torch, A), dev(torch, B)
    lib.mad_dev(M, N, K, p, dA.data_ptr(), K, dB.data_ptr(), N, dC.data_ptr(), N, C=dC.data_ptr(), ldc=N)
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy().reshape(M, N), jobs.mad(C, A, B, p))


@pytest.mark.parametrize("p", [3, 251])
def test_mad_unaligned_strided_and_gathered(p):
    """Operands at odd byte offsets with odd leading dimensions, B and C rows gathered."""
    torch = torch_cuda()
    lib = gpu_library()
    rng = np.random.default_rng(p)
    M, N, K = 203, 157, 91
    lda, ldb, ldc, ldd = K + 5, N + 3, N + 7, N + 1
    say(f"mad unaligned p={p}")
    Abuf = rng.integers(0, p, (M, lda)).astype(np.uint8)
    Bbuf = rng.integers(0, p, (2 * K, ldb)).astype(np.uint8)
    Cbuf = rng.integers(0, p, (2 * M, ldc)).astype(np.uint8)
    brow = rng.choice(2 * K, size=K, replace=False).astype(np.int32)
    crow = rng.choice(2 * M, size=M, replace=False).astype(np.int32)
    offA, offB, offC, offD = 3, 1, 2, 5
    dA = dev(torch, np.concatenate([np.zeros(offA, np.uint8), Abuf.ravel()]))
    dB = dev(torch, np.concatenate([np.zeros(offB, np.uint8), Bbuf.ravel()]))
    dC = dev(torch, np.concatenate([np.zeros(offC, np.uint8), Cbuf.ravel()]))
    dD = torch.zeros(offD + M * ldd, dtype=torch.uint8, device="cuda:0")
    db, dc = dev(torch, brow), dev(torch, crow)
    lib.mad_dev(M, N, K, p, dA.data_ptr() + offA, lda, dB.data_ptr() + offB, ldb, dD.data_ptr() + offD, ldd,
                C=dC.data_ptr() + offC, ldc=ldc, brow=db.data_ptr(), crow=dc.data_ptr())
    torch.cuda.synchronize()
    got = dD.cpu().numpy()[offD:].reshape(M, ldd)[:, :N]
    exp = jobs.mad(Cbuf[crow, :N], Abuf[:, :K], Bbuf[brow, :N], p)
    assert np.array_equal(got, exp)


def test_mad_batch_grouped():
    torch = torch_cuda()
    lib = gpu_library()
    rng = np.random.default_rng(1)
    descs, keep, exps = [], [], []
    for t in range(40):
        M, N, K = (int(x) for x in rng.integers(1, 260, 3))
        p = int(rng.choice(PRIMES))
        A = rng.integers(0, p, (M, K)).astype(np.uint8)
        B = rng.integers(0, p, (K, N)).astype(np.uint8)
        dA, dB = dev(torch, A), dev(torch, B)
        dD = torch.zeros(M * N, dtype=torch.uint8, device="cuda:0")
        keep += [dA, dB, dD]
        descs.append(dict(M=M, N=N, K=K, p=p, A=dA.data_ptr(), lda=K, B=dB.data_ptr(), ldb=N, D=dD.data_ptr(),
                          ldd=N))
        exps.append((dD, jobs.mul(A, B, p), M, N))
    say("mad batch of 40")
    lib.mad_batch_dev(descs)
    torch.cuda.synchronize()
    for dD, exp, M, N in exps:
        assert np.array_equal(dD.cpu().numpy().reshape(M, N), exp)
    say("mad batch of 40, timed")
    for dD, _, _, _ in exps:
        dD.zero_()
    torch.cuda.synchronize()
    ms = lib.mad_batch_dev_timed(descs)
    assert 0 < ms < 1000
    for dD, exp, M, N in exps:
        assert np.array_equal(dD.cpu().numpy().reshape(M, N), exp)


ECH_SHAPES = [(1, 1), (5, 9), (9, 5), (64, 64), (100, 37), (37, 100), (300, 300), (513, 200), (200, 700),
              # blocks of at most 256 rows (working matrix in LDS when p <= 46): full panels, ragged
              # last panels, more columns than fit, one column
              (256, 288), (256, 256), (250, 301), (256, 33), (129, 400), (64, 1500), (256, 1)]


@pytest.mark.parametrize("p", [2, 3, 5, 7, 43, 47, 251])
@pytest.mark.parametrize("shape", ECH_SHAPES)
def test_ech_block(shape, p):
    rows, cols = shape
    say(f"ech {shape} p={p}")
    H = synth.deficient(p, rows * 1000 + cols, rows, cols, p) if rows > 3 else synth.uniform(p, 9, rows, cols, p)
    check_ech(H, p)


def _structured(kind, rows, cols, p):
    H = synth.uniform(p, rows * 7 + cols, rows, cols, p)
    if kind == "zero_lead":        # the first 70 rows zero: the first 64 unselected rows are no candidates
        H[:70] = 0
    elif kind == "zero_stripes":   # every 3rd row zero and a zero column band
        H[::3] = 0
        H[:, 40:90] = 0
    elif kind == "late_rank":      # only the last 30 rows independent of the rest
        H[: rows - 30] = np.outer(np.arange(rows - 30) % p, H[rows - 30]) % p
    return H


# blocks whose pivot search by one wave finds every pivot (uniform) or misses a
# column while later rows could hold its pivot (the others)
@pytest.mark.parametrize("p", [2, 7, 43])
@pytest.mark.parametrize("kind", ["uniform", "zero_lead", "zero_stripes", "late_rank"])
@pytest.mark.parametrize("shape", [(256, 288), (200, 150), (100, 300)])
def test_ech_block_structured(shape, kind, p):
    rows, cols = shape
    say(f"ech structured {kind} {shape} p={p}")
    check_ech(_structured(kind, rows, cols, p), p)


def check_ech(H, p):
    torch = torch_cuda()
    lib = gpu_library()
    rows, cols = H.shape
    mr = min(rows, cols)
    dH = dev(torch, H)
    i32 = lambda k: torch.zeros(max(k, 1), dtype=torch.int32, device="cuda:0")
    u8 = lambda k: torch.zeros(max(k, 1), dtype=torch.uint8, device="cuda:0")
    prow, qrow, pcol, qcol = i32(mr), i32(rows), i32(mr), i32(cols)
    dM, dK, dR = u8(mr * mr), u8(rows * mr), u8(mr * cols)
    r = lib.ech_dev(dH.data_ptr(), rows, cols, cols, p, prow.data_ptr(), qrow.data_ptr(), pcol.data_ptr(),
                    qcol.data_ptr(), dM.data_ptr(), mr, dK.data_ptr(), mr, dR.data_ptr(), cols)
    torch.cuda.synchronize()
    M, K, R, rho, gamma = jobs.ech(H, p)
    assert r == len(rho)
    P = prow.cpu().numpy()[:r]
    # pivot rows in pivot (column) order; the oracle lists them ascending
    assert sorted(P.tolist()) == rho.tolist()
    assert pcol.cpu().numpy()[:r].tolist() == gamma.tolist()
    assert qrow.cpu().numpy()[: rows - r].tolist() == jobs.complement(rho, rows).tolist()
    assert qcol.cpu().numpy()[: cols - r].tolist() == jobs.complement(gamma, cols).tolist()
    perm = np.searchsorted(rho, P)            # our column u is the oracle's column perm[u]
    gM = dM.cpu().numpy()[: mr * mr].reshape(mr, mr)[:r, :r]
    gK = dK.cpu().numpy()[: rows * mr].reshape(rows, mr)[: rows - r, :r]
    gR = dR.cpu().numpy()[: mr * cols].reshape(mr, cols)[:r, : cols - r]
    assert np.array_equal(gM, M[:, perm])
    assert np.array_equal(gK, K[:, perm])
    assert np.array_equal(gR, R)


@pytest.mark.parametrize("K", [64, 130, 200, 256, 300])
@pytest.mark.parametrize("with_crow", [False, True])
def test_mad_gathered_aligned(K, with_crow):
    """Gathered B rows on 16-byte aligned operands: K up to 4 steps streams
    through LDS with the row numbers loaded first (K = 130 and 200 end in a
    tail step, K = 300 takes the register path); edge tiles in M and N."""
    torch = torch_cuda()
    lib = gpu_library()
    p = 43
    rng = np.random.default_rng(K + 7 * with_crow)
    M, N = 300, 400
    Abuf = rng.integers(0, p, (M, K)).astype(np.uint8)
    Bbuf = rng.integers(0, p, (K + 37, N)).astype(np.uint8)
    Cbuf = rng.integers(0, p, (M + 11, N)).astype(np.uint8)
    brow = rng.integers(0, K + 37, size=K).astype(np.int32)          # repeats allowed
    crow = rng.choice(M + 11, size=M, replace=False).astype(np.int32)
    dA, dB, dC = dev(torch, Abuf), dev(torch, Bbuf), dev(torch, Cbuf)
    dD = torch.zeros(M * N, dtype=torch.uint8, device="cuda:0")
    db, dc = dev(torch, brow), dev(torch, crow)
    say(f"mad gathered aligned K={K} crow={with_crow}")
    lib.mad_dev(M, N, K, p, dA.data_ptr(), K, dB.data_ptr(), N, dD.data_ptr(), N,
                C=dC.data_ptr(), ldc=N, brow=db.data_ptr(), crow=dc.data_ptr() if with_crow else 0)
    torch.cuda.synchronize()
    cin = Cbuf[crow] if with_crow else Cbuf[:M]
    assert np.array_equal(dD.cpu().numpy().reshape(M, N), jobs.mad(cin, Abuf, Bbuf[brow], p))


def test_mad_batch_streamed():
    """More descriptors than travel as kernel arguments, 16-byte aligned rows
    (interior tiles stream through LDS), with C, over p <= 127."""
    torch = torch_cuda()
    lib = gpu_library()
    rng = np.random.default_rng(2)
    descs, keep, exps = [], [], []
    for t in range(40):
        M = int(rng.choice([256, 300, 512]))
        N = int(rng.choice([128, 144, 256, 400]))
        K = int(rng.choice([64, 80, 192, 256]))
        p = int(rng.choice([2, 7, 43, 127]))
        A = rng.integers(0, p, (M, K)).astype(np.uint8)
        B = rng.integers(0, p, (K, N)).astype(np.uint8)
        C = rng.integers(0, p, (M, N)).astype(np.uint8)
        dA, dB, dC = dev(torch, A), dev(torch, B), dev(torch, C)
        dD = torch.zeros(M * N, dtype=torch.uint8, device="cuda:0")
        keep += [dA, dB, dC, dD]
        descs.append(dict(M=M, N=N, K=K, p=p, A=dA.data_ptr(), lda=K, B=dB.data_ptr(), ldb=N, C=dC.data_ptr(),
                          ldc=N, D=dD.data_ptr(), ldd=N))
        exps.append((dD, jobs.mad(C, A, B, p), M, N))
    say("mad batch of 40, streamed")
    lib.mad_batch_dev(descs)
    torch.cuda.synchronize()
    for dD, exp, M, N in exps:
        assert np.array_equal(dD.cpu().numpy().reshape(M, N), exp)


# inner dimensions of the large solves' products (2048-wide block columns) and beyond,
# on 16-byte aligned rows so interior tiles take the streamed path; even step
# counts from 4 up move A two steps at a time (6 and 10 steps: the transfer
# schedule's first and last steps overlap), an odd count (5) one step at a time
LONG_K_SHAPES = [(256, 512, 2048), (512, 384, 4096), (300, 272, 2048), (512, 256, 384), (256, 512, 640),
                 (512, 512, 320)]


@pytest.mark.parametrize("p", [2, 7, 127, 131, 251])
@pytest.mark.parametrize("shape", LONG_K_SHAPES)
def test_mad_long_k(shape, p):
    torch = torch_cuda()
    lib = gpu_library()
    M, N, K = shape
    say(f"mad long K {shape} p={p}")
    rng = np.random.default_rng(M + N + K + p)
    A = rng.integers(0, p, (M, K)).astype(np.uint8)
    B = rng.integers(0, p, (K, N)).astype(np.uint8)
    C = rng.integers(0, p, (M, N)).astype(np.uint8)
    dA, dB, dC = dev(torch, A), dev(torch, B), dev(torch, C)
    dD = torch.zeros(M * N, dtype=torch.uint8, device="cuda:0")
    lib.mad_dev(M, N, K, p, dA.data_ptr(), K, dB.data_ptr(), N, dD.data_ptr(), N, C=dC.data_ptr(), ldc=N)
    torch.cuda.synchronize()
    assert np.array_equal(dD.cpu().numpy().reshape(M, N), oracle.mad_c(C, A, B, p))


def _extremes(p):
    """Residues whose centred int8 forms have the largest magnitudes: for
    p <= 127 every residue is its own form and p - 1 is the largest; for p > 127
    the residues 127 and 128 have the forms 127 and 128 - p (the most negative)."""
    return [p - 1, p - 2] if p <= 127 else [127, 128]


@pytest.mark.parametrize("p", [7, 127, 131, 251])
@pytest.mark.parametrize("K", [2048, 4096])
def test_mad_extreme_operands(K, p):
    """Every product at the largest magnitudes of either sign, summed over long
    inner dimensions: all-equal blocks (the largest sums of one sign) and
    seeded mixtures of the two extreme residues (sums of both signs)."""
    torch = torch_cuda()
    lib = gpu_library()
    M, N = 256, 256
    hi, lo = _extremes(p)
    rng = np.random.default_rng(K + p)
    cases = {
        "hi*hi": (np.full((M, K), hi, np.uint8), np.full((K, N), hi, np.uint8)),
        "hi*lo": (np.full((M, K), hi, np.uint8), np.full((K, N), lo, np.uint8)),
        "lo*lo": (np.full((M, K), lo, np.uint8), np.full((K, N), lo, np.uint8)),
        "mixed": (rng.choice([hi, lo], (M, K)).astype(np.uint8), rng.choice([hi, lo], (K, N)).astype(np.uint8)),
    }
    C = np.full((M, N), p - 1, np.uint8)
    dC = dev(torch, C)
    for name, (A, B) in cases.items():
        say(f"mad extreme {name} K={K} p={p}")
        dA, dB = dev(torch, A), dev(torch, B)
        dD = torch.zeros(M * N, dtype=torch.uint8, device="cuda:0")
        lib.mad_dev(M, N, K, p, dA.data_ptr(), K, dB.data_ptr(), N, dD.data_ptr(), N, C=dC.data_ptr(), ldc=N)
        torch.cuda.synchronize()
        assert np.array_equal(dD.cpu().numpy().reshape(M, N), jobs.mad(C, A, B, p)), name


GF2_MAD_SHAPES = [(1, 1, 1), (300, 1000, 77), (256, 1024, 64), (513, 2100, 1030), (1000, 65, 4100), (70, 3000, 9)]


@pytest.mark.parametrize("shape", GF2_MAD_SHAPES)
def test_mad_gf2_packed(shape):
    """The four-Russians MAD over GF(2) on packed rows against the packed
    oracle's MAD: with and without C, in place, and with row strides above
    the words a row needs."""
    torch = torch_cuda()
    lib = gpu_library()
    M, N, K = shape
    say(f"mad gf2 packed {shape}")
    rng = np.random.default_rng(M + N + K)
    A = synth.gf2_pack(rng.integers(0, 2, (M, K)).astype(np.uint8))
    B = synth.gf2_pack(rng.integers(0, 2, (K, N)).astype(np.uint8))
    C = synth.gf2_pack(rng.integers(0, 2, (M, N)).astype(np.uint8))
    exp = oracle.mad_gf2(C, A, B, K, N)
    # bits of A past K - 1 are ignored: set them
    Ax = A.copy()
    if K % 64:
        Ax[:, -1] |= ~((np.uint64(1) << np.uint64(K % 64)) - np.uint64(1))
    pad = lambda X, k: np.concatenate([X, np.zeros((X.shape[0], k), np.uint64)], axis=1)
    t = lambda X: torch.from_numpy(np.ascontiguousarray(X).view(np.int64)).to("cuda:0")
    dA, dB, dC = t(pad(Ax, 1)), t(pad(B, 2)), t(C)
    dD = torch.zeros_like(dC)
    wa, wb, wn = Ax.shape[1] + 1, B.shape[1] + 2, C.shape[1]
    lib.mad_gf2_dev(M, N, K, dA.data_ptr(), wa, dB.data_ptr(), wb, dD.data_ptr(), wn, C=dC.data_ptr(), ldc=wn)
    torch.cuda.synchronize()
    assert np.array_equal(dD.cpu().numpy().view(np.uint64), exp)
    lib.mad_gf2_dev(M, N, K, dA.data_ptr(), wa, dB.data_ptr(), wb, dD.data_ptr(), wn)
    torch.cuda.synchronize()
    assert np.array_equal(dD.cpu().numpy().view(np.uint64), oracle.mad_gf2(None, A, B, K, N))
    lib.mad_gf2_dev(M, N, K, dA.data_ptr(), wa, dB.data_ptr(), wb, dC.data_ptr(), wn, C=dC.data_ptr(), ldc=wn)
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy().view(np.uint64), exp)
