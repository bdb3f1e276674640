"""cmrs_spmv_colblock_noalloc (partial sums in the library's static device
scratch) against cmrs_spmv_colblock with a caller workspace: the same
kernels, so the same bits.  Two calls in a row on one GPU, the second with a
smaller matrix (the scratch keeps the first call's contents), in every value
precision; each result also within the oracle's bound."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

U64, U32, U16 = 2.0 ** -53, 2.0 ** -24, 2.0 ** -8


@pytest.fixture(scope="module")
def C():
    from paper_1203_2946_amd import cmrs
    return cmrs


def _pair(C, A, x64, height, nb, dtype):
    rp, ci, v, hv = G.upload(A, dtype)
    M = C.from_csr(rp, ci, v, A.cols, height, sort=True)
    plan = C.colblock_plan(M, nb)
    xt, xs64 = G.xy_vector(x64, dtype)
    y_ref = C.spmv_colblock(M, plan, xt, schedule="concurrent")
    y = torch.full_like(y_ref, float("nan"))
    C.spmv_colblock_noalloc(M, plan, xt, out=y)
    torch.cuda.synchronize()
    assert torch.equal(y.view(torch.int32 if y.dtype == torch.float32 else torch.int64),
                       y_ref.view(torch.int32 if y.dtype == torch.float32 else torch.int64)), \
        f"noalloc differs from the workspace call (h={height} nb={nb} {dtype})"
    return y.cpu().numpy().astype(np.float64), hv, xs64


def _bound_ok(A, x64, y, dtype, hv, xs64):
    k = np.diff(A.row_ptr).astype(np.float64)
    if dtype == "f64":
        yref = oracle.csr_spmv(A.row_ptr, A.col_ind, A.val, x64)
        tol = 4.0 * k * U64 * oracle.csr_absmv(A.row_ptr, A.col_ind, A.val, x64)
    else:
        v64 = G.vals_as_f64(hv, dtype)
        yref = oracle.csr_spmv(A.row_ptr, A.col_ind, v64, xs64)
        tol = 4.0 * k * U32 * oracle.csr_absmv(A.row_ptr, A.col_ind, v64, xs64)
    assert np.all(np.abs(y - yref) <= tol)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_noalloc_two_calls_second_smaller(C, dtype):
    # First call: the largest fp64 case the 32 MiB scratch holds with 4 blocks (2^20 rows).
    big = synth.poisson_rows(1 << 20, 16.0, seed=0) if dtype == "f64" else synth.poisson_rows(1 << 19, 16.0, seed=2)
    xb = synth.normal_vector(big.cols, seed=1)
    print(f"noalloc {dtype}: first call rows={big.rows} h=32 nb=4", flush=True)
    y1, hv1, xs1 = _pair(C, big, xb, 32, 4, dtype)
    _bound_ok(big, xb, y1, dtype, hv1, xs1)
    # Second call: fewer rows, other height and block count, ragged last strip, long rows.
    small = synth.zipf_clustered(100_003, seed=5)
    xs = synth.uniform_vector(small.cols, seed=6)
    print(f"noalloc {dtype}: second call rows={small.rows} h=7 nb=8", flush=True)
    y2, hv2, xs2 = _pair(C, small, xs, 7, 8, dtype)
    _bound_ok(small, xs, y2, dtype, hv2, xs2)


def test_noalloc_one_block_and_limit(C):
    A = synth.random_csr(3000, 2000, max_row=40, seed=3, int_values=True)
    x = np.random.default_rng(3).integers(-7, 8, A.cols).astype(np.float64)
    rp, ci, v, _ = G.upload(A)
    M = C.from_csr(rp, ci, v, A.cols, 4, sort=True)
    plan = C.colblock_plan(M, 1)
    y = C.spmv_colblock_noalloc(M, plan, torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy(), oracle.csr_spmv(A.row_ptr, A.col_ind, A.val, x))
    # Beyond the scratch: refused before any launch, y untouched.
    B = synth.poisson_rows(1 << 21, 2.0, seed=4)
    rp, ci, v, _ = G.upload(B)
    MB = C.from_csr(rp, ci, v, B.cols, 4, sort=True)
    pb = C.colblock_plan(MB, 4)
    yb = torch.full((B.rows,), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(C.CmrsError):
        C.spmv_colblock_noalloc(MB, pb, torch.ones(B.cols, dtype=torch.float64, device="cuda"), out=yb)
    torch.cuda.synchronize()
    assert bool((yb == 7.0).all())
