"""GPU parity of the split schedule (heavy strips cut into chunks, chunk sums
added in chunk order) against the fp64 oracle.

Bars as in test_gpu_spmv.py: bit-exact on integer data (every summation
order is exact there); fp64 4 k_i 2^-53 (|A||x|)_i; fp32 / bf16 the
arithmetic bound on the rounded inputs and the total bound against the fp64
data.  Also: determinism across calls and plan rebuilds, calls in a row,
HIP graph replay."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests import gpu_util as G
from tests.test_gpu_spmv import Bounds, assert_fp64_bound, assert_low_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def C():
    from paper_1203_2946_amd import cmrs
    return cmrs


def long_row_matrix(seed, rows=5000, cols=30000, longs=((0, 12000), (1, 3000), (17, 20000), (2500, 5000),
                                                           (4999, 7000)), int_values=False):
    rng = np.random.default_rng(seed)
    k = rng.integers(0, 3, rows)
    for r, n in longs:
        k[r] = n
    cl = [np.sort(rng.choice(cols, size=int(kk), replace=False)) for kk in k]
    rp = np.zeros(rows + 1, np.int64)
    np.cumsum(k, out=rp[1:])
    nnz = int(k.sum())
    val = rng.integers(-8, 9, nnz).astype(np.float64) if int_values else rng.standard_normal(nnz)
    return synth.Csr(rows, cols, rp.astype(np.int32), np.concatenate(cl).astype(np.int32), val)


def run_split(C, A, x64, height, dtype="f64", sort=True, long_len=0, chunk_len=0):
    rp, ci, v, hv = G.upload(A, dtype)
    M = C.from_csr(rp, ci, v, A.cols, height, sort=sort)
    plan = C.split_plan(M, long_len, chunk_len)
    xt, xs64 = G.xy_vector(x64, dtype)
    y = C.spmv_split(M, plan, xt)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64), hv, xs64, M, plan, xt


@pytest.mark.parametrize("height", [1, 2, 3, 8, 16, 32])
@pytest.mark.parametrize("lens", [(0, 0), (1, 1), (1, 7), (40, 64), (100, 1000), (5000, 3000)])
def test_integer_exact(C, height, lens):
    A = long_row_matrix(height, int_values=True)
    x = np.random.default_rng(height).integers(-7, 8, A.cols).astype(np.float64)
    y, *_ = run_split(C, A, x, height, sort=height % 2 == 0, long_len=lens[0], chunk_len=lens[1])
    assert np.array_equal(y, oracle.csr_spmv(A.row_ptr, A.col_ind, A.val, x))


@pytest.mark.parametrize("height", [1, 4, 8, 32])
def test_fp64_bound_and_deterministic(C, height):
    A = long_row_matrix(10 + height)
    x = synth.normal_vector(A.cols, seed=1)
    y, _, _, M, plan, xt = run_split(C, A, x, height)
    assert_fp64_bound(A, x, y)
    ref = torch.from_numpy(y).cuda()
    for _ in range(10):
        assert torch.equal(C.spmv_split(M, plan, xt), ref)
    # a rebuilt plan gives the same bits
    plan2 = C.split_plan(M)
    for _ in range(3):
        assert torch.equal(C.spmv_split(M, plan2, xt), ref)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("height", [2, 8, 16])
def test_low_precision(C, dtype, height):
    A = long_row_matrix(20 + height)
    x = synth.normal_vector(A.cols, seed=2)
    y, hv, xs, *_ = run_split(C, A, x, height, dtype, long_len=64, chunk_len=512)
    assert_low_bound(A, hv, dtype, xs, x, y)


def test_random_and_edges(C):
    A = synth.random_csr(2000, 1500, max_row=60, seed=5, explicit_zeros=True, canonical=False, duplicates=True)
    x = synth.normal_vector(A.cols, seed=3)
    for h in (1, 5, 8, 32):
        for lens in ((0, 0), (10, 16)):
            y, *_ = run_split(C, A, x, h, sort=False, long_len=lens[0], chunk_len=lens[1])
            assert_fp64_bound(A, x, y)
    # no entries, ragged last strip, one-row matrix with a single long row
    E = synth.Csr(37, 11, np.zeros(38, np.int32), np.zeros(0, np.int32), np.zeros(0))
    y, *_ = run_split(C, E, np.ones(11), 4)
    assert np.all(y == 0) and not np.signbit(y).any()
    one = long_row_matrix(7, rows=1, cols=40000, longs=((0, 33333),))
    x = synth.normal_vector(one.cols, seed=4)
    for h in (1, 32):
        y, *_ = run_split(C, one, x, h, long_len=100, chunk_len=700)
        assert_fp64_bound(one, x, y)


@pytest.fixture(scope="module")
def c3():
    return synth.zipf_clustered(2_000_000, seed=0)


@pytest.fixture(scope="module")
def c3b(c3):
    return Bounds(c3, synth.uniform_vector(c3.cols, seed=1))


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_c3_full(C, c3, c3b, dtype):
    """The skewed-row workload at full size (rows of up to 10^4 entries)."""
    for h, lens in ((4, (0, 0)), (8, (0, 0)), (16, (0, 0)), (8, (256, 2048)), (32, (0, 512))):
        y, *_ = run_split(C, c3, c3b.x64, h, dtype, long_len=lens[0], chunk_len=lens[1])
        c3b.check(y, dtype, f"h={h} lens={lens}")


def test_c2_full_no_heavy(C):
    """Uniform rows: no strip is heavy, the product is the strip-group one."""
    A = synth.poisson_rows(1 << 20, 16.0, seed=0)
    x = synth.normal_vector(A.cols, seed=1)
    b = Bounds(A, x)
    for h in (2, 32):
        y, *_ = run_split(C, A, x, h)
        b.check(y, "f64", f"h={h}")


def test_graph_replay(C):
    """Plan and product captured in one HIP graph (no memset nodes), replayed
    with eager work in between: every replay equals the eager result."""
    A = long_row_matrix(3)
    x = synth.normal_vector(A.cols, seed=5)
    rp, ci, v, _ = G.upload(A)
    M = C.from_csr(rp, ci, v, A.cols, 8, sort=True)
    xt = torch.from_numpy(x).cuda()
    plan = C.split_plan(M, 64, 256)
    y_eager = C.spmv_split(M, plan, xt).clone()
    y = torch.empty_like(y_eager)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            C.split_plan(M, 64, 256, out=plan)
            C.spmv_split(M, plan, xt, out=y)
    torch.cuda.current_stream().wait_stream(s)
    for i in range(4):
        y.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, y_eager), f"replay {i}"
        assert torch.equal(C.spmv_split(M, plan, xt), y_eager)
    assert_fp64_bound(A, x, y_eager.cpu().numpy())
