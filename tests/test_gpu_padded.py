"""GPU parity of the padded CMRS of Sec. 6.7.

Conversion: bit-exact against the reference arrangement (oracle/padded.py)
on small matrices and on sampled strips of large ones, and the Sec. 6.7
constraints checked on the whole result.  SpMV: the fp64 bound
|y - y_ref|_i <= 4 k_i 2^-53 (|A||x|)_i against the CSR product (the
padding adds nothing, even where x holds inf), fp32/bf16 on rounded inputs.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import padded as P
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

U64, U32 = 2.0 ** -53, 2.0 ** -24


@pytest.fixture(scope="module")
def C():
    from paper_1203_2946_amd import cmrs
    return cmrs


def _convert(C, A, height, dtype="f64"):
    rp, ci, v, hv = G.upload(A, dtype)
    M = C.padded_from_csr(rp, ci, v, A.cols, height)
    torch.cuda.synchronize()
    return M, hv


CASES = {
    "random": lambda: synth.random_csr(700, 500, max_row=40, seed=1),
    "laplace": lambda: synth.laplace2d(40, 23),
    "zipf": lambda: synth.zipf_clustered(3000, kmax=400, seed=2),
    "empty_rows": lambda: synth.random_csr(900, 300, max_row=3, seed=3),
    "dense": lambda: synth.dense_as_sparse(70, seed=4),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("height", [1, 2, 5, 8, 16, 32])
def test_conversion_bit_exact(C, name, height):
    A = CASES[name]()
    M, hv = _convert(C, A, height)
    sp, w, v = P.arrange(A.row_ptr, A.col_ind, hv, height)
    assert np.array_equal(M.strip_ptr.cpu().numpy(), sp)
    assert np.array_equal(M.col_word.cpu().numpy().view(np.uint32), w)
    assert np.array_equal(G.val_bits(M.val), v.view(np.uint64))
    assert M.bits == P.padded_bits(height)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_conversion_moves_value_bits(C, dtype):
    A = synth.random_csr(500, 400, max_row=25, seed=5)
    M, hv = _convert(C, A, 16, dtype)
    sp, w, v = P.arrange(A.row_ptr, A.col_ind, hv, 16)
    assert np.array_equal(M.col_word.cpu().numpy().view(np.uint32), w)
    assert np.array_equal(G.val_bits(M.val), G.np_bits(v))


def test_constraints_and_sampled_strips_at_scale(C):
    """C2-shaped matrix (Poisson 16 per row, 2^18 rows) at height 16: the
    constraints on every strip, and 200 sampled strips equal the reference
    arrangement of their rows."""
    A = synth.poisson_rows(1 << 18, 16.0, seed=7)
    M, hv = _convert(C, A, 16)
    sp = M.strip_ptr.cpu().numpy().astype(np.int64)
    w = M.col_word.cpu().numpy().view(np.uint32)
    v = M.val.cpu().numpy()
    strips = sp.size - 1
    rng = np.random.default_rng(0)
    for s in np.unique(np.concatenate([[0, strips - 1], rng.integers(0, strips, 200)])):
        r0, r1 = 16 * s, min(A.rows, 16 * s + 16)
        a, b = A.row_ptr[r0], A.row_ptr[r1]
        sub_rp = A.row_ptr[r0:r1 + 1] - a
        ssp, sw, sv = P.arrange(sub_rp, A.col_ind[a:b], hv[a:b], 16)
        assert np.array_equal(w[sp[s]:sp[s + 1]], sw) and np.array_equal(v[sp[s]:sp[s + 1]], sv), s
    # Whole-matrix constraints through a vectorised check: strips hold whole
    # chunks; padding entries are exactly the words 16 with value 0.
    assert np.all(np.diff(sp) % 64 == 0)
    pad = (w & 31) == 16
    assert np.all(v[pad] == 0) and np.all(w[pad] == 16)
    assert int((~pad).sum()) == A.nnz


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("height", [1, 4, 16, 32])
def test_spmv_fp64(C, name, height):
    A = CASES[name]()
    M, hv = _convert(C, A, height)
    x = synth.normal_vector(A.cols, seed=height)
    y = C.padded_spmv(M, torch.from_numpy(x).cuda()).cpu().numpy()
    ref = oracle.csr_spmv(A.row_ptr, A.col_ind, A.val, x)
    tol = oracle.spmv_bound(A.row_ptr, A.col_ind, A.val, x, U64, factor=4.0)
    assert np.all(np.abs(y - ref) <= tol)
    empty = np.diff(A.row_ptr) == 0
    assert np.all(y[empty] == 0) and not np.signbit(y[empty]).any()


def test_padding_ignores_x(C):
    """Column 0 unused by the matrix and x[0] = inf: padding entries point at
    column 0 with value 0 but are skipped, so y stays finite and exact."""
    A = synth.random_csr(400, 300, max_row=20, seed=9, int_values=True)
    keep = A.col_ind != 0
    rp = np.concatenate([[0], np.cumsum([keep[A.row_ptr[i]:A.row_ptr[i + 1]].sum() for i in range(A.rows)])])
    B = synth.Csr(A.rows, A.cols, rp.astype(np.int32), A.col_ind[keep], A.val[keep], "no column 0")
    M, _ = _convert(C, B, 16)
    x = np.random.default_rng(1).integers(-4, 5, B.cols).astype(np.float64)
    x[0] = np.inf
    y = C.padded_spmv(M, torch.from_numpy(x).cuda()).cpu().numpy()
    assert np.all(np.isfinite(y))
    assert np.array_equal(y, oracle.csr_spmv(B.row_ptr, B.col_ind, B.val, x))


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_spmv_low_precision(C, dtype):
    A = synth.poisson_rows(30_000, 11.0, seed=3)
    M, hv = _convert(C, A, 16, dtype)
    x64 = synth.normal_vector(A.cols, seed=2)
    xt, xs = G.xy_vector(x64, dtype)
    y = C.padded_spmv(M, xt).cpu().numpy().astype(np.float64)
    v64 = G.vals_as_f64(hv, dtype)
    ref = oracle.csr_spmv(A.row_ptr, A.col_ind, v64, xs)
    tol = oracle.spmv_bound(A.row_ptr, A.col_ind, v64, xs, U32, factor=4.0)
    assert np.all(np.abs(y - ref) <= tol)


def test_no_entries(C):
    A = synth.random_csr(333, 50, max_row=0, seed=1)
    M, _ = _convert(C, A, 16)
    assert M.nnz == 0 and np.all(M.strip_ptr.cpu().numpy() == 0)
    y = C.padded_spmv(M, torch.ones(A.cols, dtype=torch.float64, device="cuda")).cpu().numpy()
    assert np.all(y == 0) and not np.signbit(y).any()
