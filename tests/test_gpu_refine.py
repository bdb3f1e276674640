"""fp64 where a solver's stability needs it: mixed-precision iterative
refinement through the library's SpMV (fp64 residual r = b - A x, inner
Jacobi sweeps with the fp32 or bf16-value product) reaches the fp64 level,
while the same iteration with a low-precision residual stalls at the low
precision.  Matrix: the skewed-row pattern plus a dominant diagonal, with a
known solution; b from the oracle."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def C():
    from paper_1203_2946_amd import cmrs
    return cmrs


def _system(n, seed):
    B = synth.zipf_clustered(n, seed=seed)
    N = sp.csr_matrix((B.val, B.col_ind, B.row_ptr), shape=(B.rows, B.cols))
    d = 2.0 * np.asarray(abs(N).sum(axis=1)).ravel() + 1.0
    A = (N + sp.diags(d)).tocsr()
    A.sort_indices()
    rp, ci, v = A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64)
    xs = synth.uniform_vector(n, seed=seed + 1)
    return rp, ci, v, d, xs, oracle.csr_spmv(rp, ci, v, xs)


def _refine(C, M64, ML, b, dinv, outer, resid64):
    x = torch.zeros_like(b)
    for _ in range(outer):
        r = b - C.spmv(M64, x) if resid64 else (b.float() - C.spmv(ML, x.float())).double()
        r32 = r.float()
        d = torch.zeros_like(r32)
        for _ in range(3):
            d = d + dinv.float() * (r32 - C.spmv(ML, d))
        x = x + d.double()
    return x


@pytest.mark.parametrize("low", ["f32", "bf16"])
def test_fp64_residual_reaches_fp64(C, low):
    rp_h, ci_h, v_h, d, xs, b = _system(150_000, 3)
    dev = torch.device("cuda:0")
    rp, ci = torch.from_numpy(rp_h).to(dev), torch.from_numpy(ci_h).to(dev)
    M64 = C.from_csr(rp, ci, torch.from_numpy(v_h).to(dev), len(xs), 8, sort=True)
    lv = (torch.from_numpy(synth.round_to_f32(v_h)) if low == "f32"
          else torch.from_numpy(synth.round_to_bf16_bits(v_h).view(np.int16).copy()).view(torch.bfloat16))
    ML = C.from_csr(rp, ci, lv.to(dev), len(xs), 8, sort=True)
    bt, dinv, xst = (torch.from_numpy(t).to(dev) for t in (b, 1.0 / d, xs))
    e64 = float((_refine(C, M64, ML, bt, dinv, 25, True) - xst).abs().max()) / float(np.abs(xs).max())
    elow = float((_refine(C, M64, ML, bt, dinv, 25, False) - xst).abs().max()) / float(np.abs(xs).max())
    # fp64 residual: within a few ulps of fp64 times the condition (about 3 here)
    assert e64 < 1e-14, e64
    # low-precision residual: stuck at the low precision's rounding level
    assert elow > 1e3 * e64 and elow > 1e-9, (elow, e64)
