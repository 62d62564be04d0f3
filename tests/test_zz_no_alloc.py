"""The allocation-free ECH entry point (workspace in the library's fixed
device array, rank written to device memory) against gfech_ech_dev, bit for
bit, on two calls in a row (the second smaller), through the C ABI."""
import numpy as np
import pytest

import synth
from tests.gpu_util import gpu_library, say, torch_cuda

pytestmark = pytest.mark.gpu


def _buffers(torch, rows, cols):
    mr = min(rows, cols)
    i32 = lambda k: torch.full((max(k, 1),), -7, dtype=torch.int32, device="cuda:0")
    u8 = lambda k: torch.full((max(k, 1),), 0xEE, dtype=torch.uint8, device="cuda:0")
    return dict(prow=i32(mr), qrow=i32(rows), pcol=i32(mr), qcol=i32(cols), M=u8(mr * mr), K=u8(rows * mr),
                R=u8(mr * cols))


def _outputs(b, r, rows, cols):
    mr = min(rows, cols)
    return (b["prow"].cpu().numpy()[:r], b["qrow"].cpu().numpy()[: rows - r], b["pcol"].cpu().numpy()[:r],
            b["qcol"].cpu().numpy()[: cols - r], b["M"].cpu().numpy()[: mr * mr].reshape(mr, mr)[:r, :r],
            b["K"].cpu().numpy()[: rows * mr].reshape(rows, mr)[: rows - r, :r],
            b["R"].cpu().numpy()[: mr * cols].reshape(mr, cols)[:r, : cols - r])


def _run_both(torch, lib, H, p):
    rows, cols = H.shape
    mr = min(rows, cols)
    dH = torch.from_numpy(H.ravel().copy()).to("cuda:0")
    a, b = _buffers(torch, rows, cols), _buffers(torch, rows, cols)
    r_ref = lib.ech_dev(dH.data_ptr(), rows, cols, cols, p, a["prow"].data_ptr(), a["qrow"].data_ptr(),
                        a["pcol"].data_ptr(), a["qcol"].data_ptr(), a["M"].data_ptr(), mr, a["K"].data_ptr(), mr,
                        a["R"].data_ptr(), cols)
    rank_dev = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    lib.ech_dev_noalloc(dH.data_ptr(), rows, cols, cols, p, b["prow"].data_ptr(), b["qrow"].data_ptr(),
                        b["pcol"].data_ptr(), b["qcol"].data_ptr(), b["M"].data_ptr(), mr, b["K"].data_ptr(), mr,
                        b["R"].data_ptr(), cols, rank_dev.data_ptr(), stream=stream)
    torch.cuda.synchronize()
    r = int(rank_dev.cpu().numpy()[0])
    assert r == r_ref
    for x, y in zip(_outputs(a, r, rows, cols), _outputs(b, r, rows, cols)):
        assert np.array_equal(x, y)
    return r


def test_noalloc_ech_matches_ech_dev_twice():
    torch = torch_cuda()
    lib = gpu_library()
    # first call: more than 512 rows (the global-memory ECH, all of its
    # workspace in the fixed array); second, smaller: the panel ECH over a
    # field above 46 (workspace in the fixed array too), over the first's contents
    for (rows, cols, p) in ((600, 700, 251), (150, 200, 131)):
        say(f"ech noalloc {rows}x{cols} p={p}")
        H = synth.deficient(p, rows + cols, rows, cols, p)
        r = _run_both(torch, lib, H, p)
        assert 0 < r < rows


def test_noalloc_ech_limits():
    torch = torch_cuda()
    lib = gpu_library()
    import paper_1806_04211_amd as gf
    rank_dev = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")
    # a workspace above the fixed array is refused before anything is queued
    with pytest.raises(gf.GfechError) as ex:
        lib.ech_dev_noalloc(1, 3000, 5000, 5000, 7, 1, 1, 1, 1, 1, 3000, 1, 3000, 1, 5000, rank_dev.data_ptr())
    assert ex.value.status == 5
    # an empty block writes rank 0 on the device
    lib.ech_dev_noalloc(0, 0, 10, 10, 7, 0, 0, 0, 0, 0, 0, 0, 0, 0, 10, rank_dev.data_ptr(),
                        stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert int(rank_dev.cpu().numpy()[0]) == 0
