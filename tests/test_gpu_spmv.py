"""GPU parity of the CMRS SpMV against the fp64 oracle (plain CSR product).

Bars (each written in the test that uses it):
  fp64:  |y - y_ref|_i <= 4 k_i 2^-53 (|A||x|)_i        (y_ref on the same inputs)
  fp32:  |y - y_ref~|_i <= 4 k_i 2^-24 (|A~||x~|)_i     (arithmetic, on the rounded inputs)
         |y - y_ref|_i  <= 2 (k_i + 2) 2^-24 (|A||x|)_i (total, against the fp64 data)
  bf16 values, fp32 x/y: |y - y_ref|_i <= 2 (2^-8 + (k_i + 2) 2^-24) (|A||x|)_i
  exact cases (integer data, permutation, identity, Laplacian times ones): bit-exact.
k_i = 0 rows must be exactly +0.0.
"""
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


def run(C, A, x64, height, dtype="f64", sort=False, variant="auto"):
    rp, ci, v, hv = G.upload(A, dtype)
    M = C.from_csr(rp, ci, v, A.cols, height, sort=sort)
    xt, xs64 = G.xy_vector(x64, dtype)
    y = C.spmv(M, xt, variant=variant)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64), hv, xs64


def assert_fp64_bound(A, x, y):
    yref = oracle.csr_spmv(A.row_ptr, A.col_ind, A.val, x)
    tol = oracle.spmv_bound(A.row_ptr, A.col_ind, A.val, x, U64, factor=4.0)
    err = np.abs(y - yref)
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, f"{bad.size} rows out of bound, first {bad[:5]}, err {err[bad[:5]]}, tol {tol[bad[:5]]}"
    empty = np.diff(A.row_ptr) == 0
    assert np.all(y[empty] == 0) and not np.signbit(y[empty]).any()


def assert_low_bound(A, hv, dtype, xs64, x64, y):
    """fp32 / bf16 paths: arithmetic bound on the rounded inputs and total
    bound against the original fp64 data."""
    v64 = G.vals_as_f64(hv, dtype)
    yref_r = oracle.csr_spmv(A.row_ptr, A.col_ind, v64, xs64)
    tol_r = oracle.spmv_bound(A.row_ptr, A.col_ind, v64, xs64, U32, factor=4.0)
    assert np.all(np.abs(y - yref_r) <= tol_r), "arithmetic bound on rounded inputs"
    yref = oracle.csr_spmv(A.row_ptr, A.col_ind, A.val, x64)
    k = np.diff(A.row_ptr).astype(np.float64)
    absmv = oracle.csr_absmv(A.row_ptr, A.col_ind, A.val, x64)
    rep = U16 if dtype == "bf16" else 0.0
    tol = 2.0 * (rep + (k + 2) * U32) * absmv
    assert np.all(np.abs(y - yref) <= tol), "total bound against fp64 data"
    empty = k == 0
    assert np.all(y[empty] == 0) and not np.signbit(y[empty]).any()


HEIGHTS = [1, 2, 3, 4, 5, 7, 8, 12, 16, 17, 31, 32]


VARIANTS = ["lds", "reg", "lds_nt", "reg_nt", "group", "group_nt"]


@pytest.mark.parametrize("height", HEIGHTS)
@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("sort", [False, True])
def test_integer_exact(C, height, variant, sort):
    A = synth.random_csr(1200, 700, max_row=40, seed=height, int_values=True, canonical=False, duplicates=not sort)
    x = np.random.default_rng(height).integers(-7, 8, A.cols).astype(np.float64)
    y, _, _ = run(C, A, x, height, sort=sort, variant=variant)
    assert np.array_equal(y, oracle.csr_spmv(A.row_ptr, A.col_ind, A.val, x))


@pytest.mark.parametrize("height", HEIGHTS)
@pytest.mark.parametrize("variant", VARIANTS)
def test_random_fp64_bound(C, height, variant):
    A = synth.random_csr(2000, 1500, max_row=60, seed=100 + height, explicit_zeros=True)
    x = synth.normal_vector(A.cols, seed=height)
    y, _, _ = run(C, A, x, height, sort=height % 2 == 0, variant=variant)
    assert_fp64_bound(A, x, y)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("height", [1, 2, 4, 8, 16, 32, 6])
@pytest.mark.parametrize("variant", ["lds", "reg", "group_nt"])
def test_random_low_precision(C, dtype, height, variant):
    A = synth.random_csr(1500, 1100, max_row=50, seed=200 + height)
    x = synth.normal_vector(A.cols, seed=3)
    y, hv, xs = run(C, A, x, height, dtype, sort=True, variant=variant)
    assert_low_bound(A, hv, dtype, xs, x, y)


@pytest.mark.parametrize("height", [2, 4, 8])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_laplacian_64(C, height, dtype):
    A = synth.laplace2d(64)
    x = synth.uniform_vector(A.cols, seed=0)
    for sort in (False, True):
        y, hv, xs = run(C, A, x, height, dtype, sort=sort)
        if dtype == "f64":
            assert_fp64_bound(A, x, y)
        else:
            assert_low_bound(A, hv, dtype, xs, x, y)
        ones, _, _ = run(C, A, np.ones(A.cols), height, dtype, sort=sort)
        assert np.array_equal(ones, oracle.csr_spmv(A.row_ptr, A.col_ind, A.val, np.ones(A.cols)))


@pytest.mark.parametrize("height", [1, 4, 32])
def test_permutation_identity_exact(C, height):
    P = synth.permutation(100000, seed=7)
    x = synth.normal_vector(P.cols, seed=8)
    for sort in (False, True):
        y, _, _ = run(C, P, x, height, sort=sort)
        assert np.array_equal(y, x[P.col_ind])
    E = synth.identity(4099)
    y, _, _ = run(C, E, x[:4099], height)
    assert np.array_equal(y, x[:4099])


def test_dense_as_sparse(C):
    A = synth.dense_as_sparse(1024, seed=1)
    x = synth.uniform_vector(1024, seed=2)
    for h in (1, 4, 16):
        y, _, _ = run(C, A, x, h, sort=True)
        assert_fp64_bound(A, x, y)
        d = oracle.csr_to_dense(A.row_ptr, A.col_ind, A.val, A.cols)
        yd = oracle.dense_matvec(d, x)
        tol = oracle.spmv_bound(A.row_ptr, A.col_ind, A.val, x, U64, factor=4.0)
        assert np.all(np.abs(y - yd) <= tol)


def test_edges(C):
    # no entries: every row +0.0
    A = synth.Csr(37, 11, np.zeros(38, np.int32), np.zeros(0, np.int32), np.zeros(0))
    for h in (1, 4, 32):
        y, _, _ = run(C, A, np.ones(11), h)
        assert np.all(y == 0) and not np.signbit(y).any()
    # products that are all -0.0 give +0.0
    A = synth.Csr(2, 2, np.array([0, 2, 3], np.int32), np.array([0, 1, 0], np.int32), np.array([-0.0, 0.0, -1.0]))
    y, _, _ = run(C, A, np.array([1.0, -1.0]), 2)
    assert y[0] == 0 and not np.signbit(y[0]) and y[1] == -1.0
    # rectangular, ragged last strip
    A = synth.random_csr(1001, 77, max_row=30, seed=9)
    x = synth.normal_vector(77, seed=1)
    for h in (3, 8, 32):
        y, _, _ = run(C, A, x, h)
        assert_fp64_bound(A, x, y)
    A = synth.random_csr(33, 9000, max_row=900, seed=10)
    x = synth.normal_vector(9000, seed=1)
    for h in (1, 16):
        y, _, _ = run(C, A, x, h, sort=True)
        assert_fp64_bound(A, x, y)


def test_rows_zero_noop(C):
    A = synth.Csr(0, 4, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    rp, ci, v, _ = G.upload(A)
    M = C.from_csr(rp, ci, v, 4, 2)
    y = torch.empty(0, dtype=torch.float64, device="cuda")
    C.spmv(M, torch.ones(4, dtype=torch.float64, device="cuda"), out=y)
    torch.cuda.synchronize()


def test_deterministic(C):
    A = synth.zipf_clustered(200000, seed=3)
    x = synth.uniform_vector(A.cols, seed=4)
    rp, ci, v, _ = G.upload(A)
    for h, variant in ((8, "lds"), (4, "reg"), (32, "lds"), (8, "group_nt"), (1, "group")):
        M = C.from_csr(rp, ci, v, A.cols, h, sort=True)
        xt = torch.from_numpy(x).cuda()
        ref = C.spmv(M, xt, variant=variant).clone()
        for _ in range(20):
            assert torch.equal(C.spmv(M, xt, variant=variant), ref)
        assert_fp64_bound(A, x, ref.cpu().numpy())


def test_long_rows(C):
    """Rows of thousands of entries next to empty and one-entry rows."""
    rng = np.random.default_rng(5)
    k = rng.integers(0, 3, 5000)
    k[[0, 1, 17, 2500, 4999]] = [12000, 3000, 20000, 5000, 7000]
    cols = 30000
    cl = [np.sort(rng.choice(cols, size=int(kk), replace=False)) for kk in k]
    rp = np.zeros(5001, np.int64)
    np.cumsum(k, out=rp[1:])
    A = synth.Csr(5000, cols, rp.astype(np.int32), np.concatenate(cl).astype(np.int32),
                  rng.standard_normal(int(k.sum())))
    x = synth.normal_vector(cols, seed=6)
    for h in (1, 2, 8, 32):
        for variant in ("lds", "reg", "group", "group_nt"):
            y, _, _ = run(C, A, x, h, sort=True, variant=variant)
            assert_fp64_bound(A, x, y)


@pytest.fixture(scope="module")
def c2():
    return synth.poisson_rows(1 << 20, 16.0, seed=0)


@pytest.fixture(scope="module")
def c2x(c2):
    return synth.normal_vector(c2.cols, seed=1)


class Bounds:
    """Oracle references and elementwise tolerances of one workload, computed
    once: fp64 4 k u |A||x|; fp32 / bf16 the arithmetic bound on the rounded
    inputs and the total bound against the fp64 data (as assert_low_bound)."""

    def __init__(self, A, x64):
        self.A, self.x64 = A, x64
        self.k = np.diff(A.row_ptr).astype(np.float64)
        self.absmv = oracle.csr_absmv(A.row_ptr, A.col_ind, A.val, x64)
        self.yref = oracle.csr_spmv(A.row_ptr, A.col_ind, A.val, x64)
        self._low = {}

    def check(self, y, dtype, what=""):
        A = self.A
        if dtype == "f64":
            tol = 4.0 * self.k * U64 * self.absmv
            bad = np.nonzero(np.abs(y - self.yref) > tol)[0]
            assert bad.size == 0, f"{what}: {bad.size} rows out of the fp64 bound, first {bad[:5]}"
        else:
            if dtype not in self._low:
                hv = G.host_vals(A.val, dtype)
                v64 = G.vals_as_f64(hv, dtype)
                xs = synth.round_to_f32(self.x64).astype(np.float64)
                self._low[dtype] = (oracle.csr_spmv(A.row_ptr, A.col_ind, v64, xs),
                                    4.0 * self.k * U32 * oracle.csr_absmv(A.row_ptr, A.col_ind, v64, xs))
            yr, tr = self._low[dtype]
            assert np.all(np.abs(y - yr) <= tr), f"{what}: arithmetic bound on rounded inputs"
            rep = U16 if dtype == "bf16" else 0.0
            tol = 2.0 * (rep + (self.k + 2) * U32) * self.absmv
            assert np.all(np.abs(y - self.yref) <= tol), f"{what}: total bound against fp64 data"
        empty = self.k == 0
        assert np.all(y[empty] == 0) and not np.signbit(y[empty]).any()


@pytest.fixture(scope="module")
def c2b(c2, c2x):
    return Bounds(c2, c2x)


@pytest.mark.parametrize("height", [1, 2, 4, 8, 16, 32])
def test_c2_full_fp64(C, c2, c2x, c2b, height):
    """Every one-wave and strip-group variant the benchmark sweeps, at full
    size (one wave per strip with non-temporal loads included)."""
    for variant in ("auto", "lds", "lds_nt", "reg", "group_nt"):
        y, _, _ = run(C, c2, c2x, height, sort=True, variant=variant)
        c2b.check(y, "f64", f"h={height} {variant}")


@pytest.mark.parametrize("height", [1, 2, 4, 8, 16, 32])
def test_c2_full_fp32(C, c2, c2x, c2b, height):
    for variant in ("auto", "lds", "lds_nt"):
        y, _, _ = run(C, c2, c2x, height, "f32", sort=True, variant=variant)
        c2b.check(y, "f32", f"h={height} {variant}")


@pytest.mark.parametrize("height", [1, 2, 4, 8, 16, 32])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_c2_full_colblock_concurrent(C, c2, c2x, c2b, height, dtype):
    """The concurrent (4 and 8 blocks) and phased (4, 8, 16 blocks)
    column-blocked schedules at every height (the benchmark's and the
    selector's colblock classes), full size:
    the launcher picks its group width from the run length, so every width
    these heights reach on this matrix is exercised."""
    rp, ci, v, _ = G.upload(c2, dtype)
    M = C.from_csr(rp, ci, v, c2.cols, height, sort=True)
    xt, _ = G.xy_vector(c2x, dtype)
    for nb in (4, 8, 16):
        plan = C.colblock_plan(M, nb)
        for schedule in ("concurrent", "phased"):
            if schedule == "concurrent" and nb == 16:
                continue
            y = C.spmv_colblock(M, plan, xt, schedule=schedule)
            torch.cuda.synchronize()
            c2b.check(y.cpu().numpy().astype(np.float64), dtype, f"h={height} nb={nb} {schedule}")


@pytest.fixture(scope="module")
def c3():
    return synth.zipf_clustered(2_000_000, seed=0)


@pytest.fixture(scope="module")
def c3b(c3):
    return Bounds(c3, synth.uniform_vector(c3.cols, seed=1))


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_c3_full(C, c3, c3b, dtype):
    x = c3b.x64
    for h, variant in ((4, "auto"), (8, "auto"), (16, "auto"), (8, "group_nt"), (8, "lds"), (16, "lds_nt")):
        y, hv, xs = run(C, c3, x, h, dtype, sort=True, variant=variant)
        c3b.check(y, dtype, f"h={h} {variant}")


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_c3_full_colblock_concurrent(C, c3, c3b, dtype):
    rp, ci, v, _ = G.upload(c3, dtype)
    xt, _ = G.xy_vector(c3b.x64, dtype)
    for h in (4, 16):
        M = C.from_csr(rp, ci, v, c3.cols, h, sort=True)
        for nb in (4, 8):
            plan = C.colblock_plan(M, nb)
            for schedule in ("concurrent", "phased"):
                y = C.spmv_colblock(M, plan, xt, schedule=schedule)
                torch.cuda.synchronize()
                c3b.check(y.cpu().numpy().astype(np.float64), dtype, f"h={h} nb={nb} {schedule}")


def run_colblock(C, A, x64, height, nb, dtype="f64", variant="auto", schedule="passes"):
    rp, ci, v, hv = G.upload(A, dtype)
    M = C.from_csr(rp, ci, v, A.cols, height, sort=True)
    plan = C.colblock_plan(M, nb)
    xt, xs64 = G.xy_vector(x64, dtype)
    y = C.spmv_colblock(M, plan, xt, variant=variant, schedule=schedule)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64), hv, xs64, M, plan


@pytest.mark.parametrize("nb", [1, 2, 3, 7, 16, 64])
@pytest.mark.parametrize("height", [1, 4, 8, 32])
def test_colblock(C, nb, height):
    A = synth.random_csr(3000, 2000, max_row=40, seed=nb + height, int_values=True)
    x = np.random.default_rng(nb).integers(-7, 8, A.cols).astype(np.float64)
    for variant, schedule in (("lds", "passes"), ("reg", "passes"), ("group_nt", "passes"), ("auto", "concurrent"),
                              ("auto", "phased")):
        y, _, _, M, plan = run_colblock(C, A, x, height, nb, variant=variant, schedule=schedule)
        assert np.array_equal(y, oracle.csr_spmv(A.row_ptr, A.col_ind, A.val, x))
    if nb > 1:
        # plan: first entry of each strip at or beyond each block boundary
        sp = M.strip_ptr.cpu().numpy()
        col = G.words(M.col_word) >> M.bits
        split = plan.split.cpu().numpy()[: M.strips * (nb - 1)].reshape(M.strips, nb - 1)
        bw = -(-A.cols // nb)
        for s in range(0, M.strips, max(1, M.strips // 50)):
            c = col[sp[s]:sp[s + 1]]
            for b in range(1, nb):
                assert split[s, b - 1] == sp[s] + int(np.sum(c < b * bw))


def test_colblock_bounds_fp64_fp32(C):
    A = synth.poisson_rows(300000, 16.0, seed=5)
    x = synth.normal_vector(A.cols, seed=6)
    for nb, schedule in ((2, "passes"), (4, "passes"), (8, "concurrent"), (3, "concurrent"), (8, "phased"),
                         (5, "phased")):
        y, _, _, _, _ = run_colblock(C, A, x, 8, nb, schedule=schedule)
        assert_fp64_bound(A, x, y)
        y, hv, xs, _, _ = run_colblock(C, A, x, 8, nb, "f32", schedule=schedule)
        assert_low_bound(A, hv, "f32", xs, x, y)
        y, hv, xs, _, _ = run_colblock(C, A, x, 8, nb, "bf16", schedule=schedule)
        assert_low_bound(A, hv, "bf16", xs, x, y)


@pytest.mark.parametrize("height", [1, 8, 32])
def test_colblock_concurrent_long_rows_and_c2(C, c2, c2x, height):
    """Concurrent schedule on the full n = 2^20 workload and on rows long
    enough to take the whole-wave path inside a column block."""
    y, _, _, _, _ = run_colblock(C, c2, c2x, height, 8, schedule="concurrent")
    assert_fp64_bound(c2, c2x, y)
    rng = np.random.default_rng(11)
    k = rng.integers(0, 3, 3000)
    k[[0, 5, 2999]] = [20000, 9000, 4000]
    cols = 40000
    cl = [np.sort(rng.choice(cols, size=int(kk), replace=False)) for kk in k]
    rp = np.zeros(3001, np.int64)
    np.cumsum(k, out=rp[1:])
    A = synth.Csr(3000, cols, rp.astype(np.int32), np.concatenate(cl).astype(np.int32), rng.standard_normal(int(k.sum())))
    x = synth.normal_vector(cols, seed=3)
    for nb in (2, 8):
        for schedule in ("concurrent", "phased"):
            y, _, _, _, _ = run_colblock(C, A, x, height, nb, schedule=schedule)
            assert_fp64_bound(A, x, y)


def test_colblock_needs_sorted(C):
    A = synth.random_csr(100, 100, seed=1)
    rp, ci, v, _ = G.upload(A)
    M = C.from_csr(rp, ci, v, A.cols, 4, sort=False)
    with pytest.raises(C.CmrsError):
        C.colblock_plan(M, 4)
