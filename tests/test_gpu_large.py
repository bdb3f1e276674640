"""Matrices of 1.48e9 entries (fp32, height 8) and 2.08e9 entries (fp64,
height 32; the library accepts up to 2^31 - 2^16): every index and byte
offset of the path runs in its upper range.  Built on the device (no host copy, no oracle at this size); checked by
properties that hold at any size, exactly:

* rows of 22 ones with distinct columns in ascending order, so y = A*1 is 22
  in every row (exact in fp32) for the strip-group, column-blocked and split
  products;
* CSR -> CMRS -> CSR reproduces row_ptr and col_ind exactly;
* StripPtr[s] = RowPtr[s*h], and inside every strip the packed words ascend
  (the reorder of Sec. 4), RowInStrip < h.
"""
import pytest
import torch

pytestmark = pytest.mark.gpu

ROWS = 1 << 26


@pytest.fixture(scope="module")
def C():
    from paper_1203_2946_amd import cmrs
    return cmrs


@pytest.mark.parametrize("PER_ROW,HEIGHT,dtype", [(22, 8, torch.float32), (31, 32, torch.float64)])
def test_large_index_range(C, PER_ROW, HEIGHT, dtype):
    dev = torch.device("cuda:0")
    cols = ROWS
    stride = cols // PER_ROW
    nnz = ROWS * PER_ROW
    assert 2 ** 30 < nnz <= 2 ** 31 - 2 ** 16
    row_ptr = torch.arange(0, nnz + 1, PER_ROW, dtype=torch.int32, device=dev)
    r = torch.arange(ROWS, dtype=torch.int32, device=dev).repeat_interleave(PER_ROW)
    j = torch.arange(PER_ROW, dtype=torch.int32, device=dev).repeat(ROWS)
    col_ind = j * stride + r % stride              # ascending inside each row, < cols
    del r, j
    val = torch.ones(nnz, dtype=dtype, device=dev)
    try:
        M = C.from_csr(row_ptr, col_ind, val, cols, HEIGHT, sort=True)
        torch.cuda.synchronize()
        strips = M.strips
        assert torch.equal(M.strip_ptr[:-1].to(torch.int64), row_ptr[::HEIGHT][:strips].to(torch.int64))
        assert int(M.strip_ptr[-1]) == nnz
        w = M.col_word.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        assert int((w & ((1 << M.bits) - 1)).max()) < HEIGHT
        starts = torch.zeros(nnz, dtype=torch.bool, device=dev)
        starts[M.strip_ptr[:-1].to(torch.int64)] = True
        asc = (w[1:] >= w[:-1]) | starts[1:]
        assert bool(asc.all()), "words descend inside a strip"
        del w, starts, asc

        x = torch.ones(cols, dtype=dtype, device=dev)
        y = C.spmv(M, x)
        torch.cuda.synchronize()
        assert bool((y == PER_ROW).all())
        plan = C.colblock_plan(M, 4)
        y.zero_()
        C.spmv_colblock(M, plan, x, out=y, schedule="concurrent")
        torch.cuda.synchronize()
        assert bool((y == PER_ROW).all())
        del plan
        sp = C.split_plan(M)
        y.zero_()
        C.spmv_split(M, sp, x, out=y)
        torch.cuda.synchronize()
        assert bool((y == PER_ROW).all())
        del sp, y, x

        rp2, ci2, v2 = C.to_csr(M)
        torch.cuda.synchronize()
        assert torch.equal(rp2, row_ptr)
        assert torch.equal(ci2, col_ind)
        assert bool((v2 == 1).all())
    finally:
        torch.cuda.empty_cache()
