"""GPU parity of the multi-right-hand-side and batched CMRS products.

Every column y_k = A x_k is held to the bars of the single-vector product
(same per-row error bounds, see test_gpu_spmv.py):
  fp64: |y_k - y_ref,k|_i <= 4 k_i 2^-53 (|A||x_k|)_i
  fp32 / bf16 values with fp32 X: 4 k_i 2^-24 (|A~||x~_k|)_i on the rounded inputs.
Empty rows give +0.  A batch tile is computed exactly as cmrs_spmm computes
those strips with the same group width, so batched and single results are
compared bit for bit; a HIP-graph replay of a batch is compared bit for bit
with the eager launch.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

U64, U32 = 2.0 ** -53, 2.0 ** -24


@pytest.fixture(scope="module")
def C():
    from paper_1203_2946_amd import cmrs
    return cmrs


def _rhs(A, nrhs, dtype, seed, ld=None):
    """X (cols x nrhs, leading dimension ld) on the device and its fp64 values."""
    ld = nrhs if ld is None else ld
    g = np.random.default_rng(seed)
    X64 = g.normal(size=(A.cols, nrhs))
    Xs = X64 if dtype == "f64" else synth.round_to_f32(X64).astype(np.float64)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    full = torch.full((A.cols, ld), float("nan"), dtype=tdt, device="cuda")
    full[:, :nrhs] = torch.from_numpy(Xs).to(tdt).cuda()
    return full[:, :nrhs], Xs


def _slots(height, nrhs):
    return (1 << (height - 1).bit_length()) * (1 << (nrhs - 1).bit_length())


def _check_cols(A, hv, dtype, Xs, Y):
    v64 = G.vals_as_f64(hv, dtype)
    u = U64 if dtype == "f64" else U32
    empty = np.diff(A.row_ptr) == 0
    for k in range(Xs.shape[1]):
        x = np.ascontiguousarray(Xs[:, k])
        ref = oracle.csr_spmv(A.row_ptr, A.col_ind, v64, x)
        tol = oracle.spmv_bound(A.row_ptr, A.col_ind, v64, x, u, factor=4.0)
        err = np.abs(Y[:, k] - ref)
        bad = np.nonzero(err > tol)[0]
        assert bad.size == 0, f"rhs {k}: {bad.size} rows out of bound, first {bad[:5]}"
        assert np.all(Y[empty, k] == 0) and not np.signbit(Y[empty, k]).any()


MATS = {
    "laplace": lambda: synth.laplace2d(64, 37),
    "random": lambda: synth.random_csr(3000, 2500, max_row=30, seed=3),
    "zipf": lambda: synth.zipf_clustered(6000, seed=5),
    "stencil": lambda: synth.stencil27(14, 13, 12, seed=6),
    "banded": lambda: synth.banded(4000, 33, seed=7),
    "empty_rows": lambda: synth.random_csr(2000, 2000, max_row=2, seed=8),
}


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("height", [1, 3, 4, 8, 32])
@pytest.mark.parametrize("nrhs", [1, 2, 3, 5, 8])
def test_spmm_fp64(C, name, height, nrhs):
    A = MATS[name]()
    rp, ci, v, hv = G.upload(A, "f64")
    M = C.from_csr(rp, ci, v, A.cols, height, sort=(height % 2 == 0))
    X, Xs = _rhs(A, nrhs, "f64", seed=height * 10 + nrhs)
    if _slots(height, nrhs) * 64 * 8 > 65536:
        # The partial sums of one wave would exceed 64 KiB of LDS.
        with pytest.raises(C.CmrsError) as ei:
            C.spmm(M, X)
        assert ei.value.status == C.CMRS_ERR_NOT_SUPPORTED
        return
    Y = C.spmm(M, X)
    torch.cuda.synchronize()
    _check_cols(A, hv, "f64", Xs, Y.cpu().numpy())


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("height", [2, 8, 16])
@pytest.mark.parametrize("nrhs", [1, 4, 7])
def test_spmm_low_precision(C, dtype, height, nrhs):
    A = synth.poisson_rows(20_000, 9.0, seed=height + nrhs)
    rp, ci, v, hv = G.upload(A, dtype)
    M = C.from_csr(rp, ci, v, A.cols, height, sort=True)
    X, Xs = _rhs(A, nrhs, dtype, seed=nrhs)
    Y = C.spmm(M, X)
    torch.cuda.synchronize()
    _check_cols(A, hv, dtype, Xs, Y.cpu().numpy().astype(np.float64))


@pytest.mark.parametrize("group", [1, 2, 8, 16])
def test_spmm_groups_and_padded_blocks(C, group):
    """Explicit group widths, X and Y with leading dimensions above nrhs:
    padding columns of Y are left untouched."""
    A = synth.zipf_clustered(5000, seed=11)
    nrhs = 3
    rp, ci, v, hv = G.upload(A, "f64")
    M = C.from_csr(rp, ci, v, A.cols, 8, sort=True)
    X, Xs = _rhs(A, nrhs, "f64", seed=group, ld=5)
    Yfull = torch.full((A.rows, 7), -123.0, dtype=torch.float64, device="cuda")
    Y = Yfull[:, :nrhs]
    C.spmm(M, X, out=Y, group=group)
    torch.cuda.synchronize()
    full = Yfull.cpu().numpy()
    assert np.all(full[:, nrhs:] == -123.0)
    _check_cols(A, hv, "f64", Xs, full[:, :nrhs])
    # Deterministic: a second call gives the same bits.
    Y2 = C.spmm(M, X, group=group)
    torch.cuda.synchronize()
    assert np.array_equal(Y2.cpu().numpy().view(np.uint64), full[:, :nrhs].copy().view(np.uint64))


@pytest.mark.parametrize("dtype,group,nrhs,ld", [("f64", 64, 8, 8), ("f64", 16, 5, 6), ("f64", 16, 4, 4),
                                                  ("f64", 16, 7, 7), ("f32", 16, 7, 8), ("f32", 64, 3, 4),
                                                  ("f64", 4, 6, 6), ("f64", 2, 8, 9), ("f32", 2, 5, 5)])
def test_spmm_several_passes_per_wave(C, dtype, group, nrhs, ld):
    """A single launch large enough that each wave takes 2-8 consecutive
    passes (the pipelined loop: the next step's loads are issued before this
    step's additions, clamped at strip and tile ends).  X rows 16-byte
    aligned with nrhs below the bucket (vector loads for the lower half of the
    bucket, single loads above), and unaligned ones.  Chunk lanes (groups of 2
    or 4 lanes sharing entries, each gathering one 16-byte chunk): with the
    chunk moved back to end at nrhs (5-7 right-hand sides), with a group as
    narrow as the chunk count (one entry slot per strip: fp64 group 4 with 4
    chunks, fp32 group 2 with 2), and too narrow for them (fp64 group 2 with
    4 chunks: one lane per entry).  Columns within the bounds; the persistent
    batched launch of the same matrix and group gives the same bits."""
    A = synth.poisson_rows(400_000, 6.0, seed=nrhs + group)
    rp, ci, v, hv = G.upload(A, dtype)
    M = C.from_csr(rp, ci, v, A.cols, 2, sort=True)
    X, Xs = _rhs(A, nrhs, dtype, seed=nrhs, ld=ld)
    Y = C.spmm(M, X, group=group)
    torch.cuda.synchronize()
    y = Y.cpu().numpy().astype(np.float64)
    _check_cols(A, hv, dtype, Xs, y)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    Yb = torch.full((A.rows, nrhs), float("nan"), dtype=tdt, device="cuda")
    plan = C.spmm_plan([M], [X], [Yb], tile_nnz=200_000, group=group)
    C.spmm_batched(plan)
    torch.cuda.synchronize()
    ut = np.uint64 if dtype == "f64" else np.uint32
    assert np.array_equal(Yb.cpu().numpy().view(ut), Y.cpu().numpy().view(ut))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("rows,max_row", [(3, 2), (9, 1), (37, 3), (200, 6)])
def test_spmm_tiny_matrices_chunk_lanes(C, dtype, rows, max_row):
    """Matrices of a handful of entries (4 or more, so chunk lanes run): most
    of a group's vector stream loads are moved back from past the last entry
    or lie wholly past their strip, for 3-8 right-hand sides, groups of 4 and
    16 lanes, heights 1, 2 and 4; the batched launch gives the same bits."""
    A = synth.random_csr(rows, 50, max_row=max_row, seed=rows)
    if A.nnz < 4:
        A = synth.random_csr(rows, 50, max_row=max_row + 2, seed=rows + 1, empty_row_frac=0.0)
    assert A.nnz >= 4
    rp, ci, v, hv = G.upload(A, dtype)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    ut = np.uint64 if dtype == "f64" else np.uint32
    for h in (1, 2, 4):
        M = C.from_csr(rp, ci, v, A.cols, h, sort=True)
        for nrhs in (3, 5, 6, 8):
            for group in (4, 16):
                X, Xs = _rhs(A, nrhs, dtype, seed=nrhs * 7 + group)
                Y = C.spmm(M, X, group=group)
                torch.cuda.synchronize()
                _check_cols(A, hv, dtype, Xs, Y.cpu().numpy().astype(np.float64))
                Yb = torch.full((A.rows, nrhs), float("nan"), dtype=tdt, device="cuda")
                plan = C.spmm_plan([M], [X], [Yb], group=group)
                C.spmm_batched(plan)
                torch.cuda.synchronize()
                assert np.array_equal(Yb.cpu().numpy().view(ut), Y.cpu().numpy().view(ut)), (h, nrhs, group)


def test_spmm_no_entries(C):
    A = synth.random_csr(777, 300, max_row=0, seed=1)
    assert A.nnz == 0
    rp, ci, v, hv = G.upload(A, "f64")
    M = C.from_csr(rp, ci, v, A.cols, 4)
    X, _ = _rhs(A, 4, "f64", seed=0)
    Y = C.spmm(M, X)
    torch.cuda.synchronize()
    y = Y.cpu().numpy()
    assert np.all(y == 0) and not np.signbit(y).any()


def _batch(C, seed, count, dtype="f64", max_rows=30_000):
    """count mixed matrices (stencil, banded, Poisson, Zipf), heights 1..32,
    1..8 right-hand sides, some with padded leading dimensions."""
    g = np.random.default_rng(seed)
    mats, Xs, Ys, host = [], [], [], []
    tdt = torch.float64 if dtype == "f64" else torch.float32
    for i in range(count):
        n = int(g.integers(500, max_rows))
        kind = i % 4
        if kind == 0:
            nx = max(2, round(n ** (1 / 3)))
            A = synth.stencil27(nx, nx, max(2, n // (nx * nx)), seed=i)
        elif kind == 1:
            A = synth.banded(n, int(g.integers(8, 65)), seed=i)
        elif kind == 2:
            A = synth.poisson_rows(n, float(g.uniform(2, 30)), seed=i)
        else:
            A = synth.zipf_clustered(n, kmax=max(4, n // 16), seed=i)
        nrhs = int(g.integers(1, 9))
        h = int(g.choice([hh for hh in (1, 2, 3, 4, 8, 16, 32) if _slots(hh, nrhs) <= 128]))
        rp, ci, v, hv = G.upload(A, dtype)
        M = C.from_csr(rp, ci, v, A.cols, h, sort=bool(i % 3))
        ld = nrhs + int(g.integers(0, 2))
        X, Xh = _rhs(A, nrhs, dtype, seed=1000 + i, ld=ld)
        Y = torch.full((A.rows, nrhs), float("nan"), dtype=tdt, device="cuda")
        mats.append(M)
        Xs.append(X)
        Ys.append(Y)
        host.append((A, hv, Xh))
    return mats, Xs, Ys, host


@pytest.mark.parametrize("tile_nnz,group", [(0, 0), (2000, 0), (50_000, 4), (1, 1)])
def test_batched_matches_single_and_oracle(C, tile_nnz, group):
    mats, Xs, Ys, host = _batch(C, seed=tile_nnz + group, count=24)
    plan = C.spmm_plan(mats, Xs, Ys, tile_nnz=tile_nnz, group=group)
    assert plan.tiles >= len(mats)
    C.spmm_batched(plan)
    torch.cuda.synchronize()
    first = [Y.cpu().numpy().copy() for Y in Ys]
    for (A, hv, Xh), y in zip(host, first):
        _check_cols(A, hv, "f64", Xh, y)
    # The same plan again (the queue was reset by the last wave): same bits.
    for Y in Ys:
        Y.fill_(float("nan"))
    C.spmm_batched(plan)
    torch.cuda.synchronize()
    for Y, y in zip(Ys, first):
        assert np.array_equal(Y.cpu().numpy().view(np.uint64), y.view(np.uint64))
    # Each matrix alone through cmrs_spmm with the plan's group width.
    for M, X, y in zip(mats, Xs, first):
        ys = C.spmm(M, X, group=group)
        torch.cuda.synchronize()
        assert np.array_equal(ys.cpu().numpy().view(np.uint64), y.view(np.uint64))


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_batched_low_precision(C, dtype):
    mats, Xs, Ys, host = _batch(C, seed=77, count=12, dtype=dtype)
    plan = C.spmm_plan(mats, Xs, Ys)
    C.spmm_batched(plan)
    torch.cuda.synchronize()
    for (A, hv, Xh), Y in zip(host, Ys):
        _check_cols(A, hv, dtype, Xh, Y.cpu().numpy().astype(np.float64))


def test_batched_graph_replay(C):
    """Capture one batched launch in a HIP graph; every replay (with eager
    work and synchronisations between them) reproduces the eager bits."""
    mats, Xs, Ys, host = _batch(C, seed=5, count=16)
    plan = C.spmm_plan(mats, Xs, Ys, tile_nnz=4000)
    C.spmm_batched(plan)
    torch.cuda.synchronize()
    eager = [Y.cpu().numpy().copy() for Y in Ys]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            C.spmm_batched(plan)
    torch.cuda.synchronize()
    for rep in range(4):
        for Y in Ys:
            Y.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for Y, y in zip(Ys, eager):
            assert np.array_equal(Y.cpu().numpy().view(np.uint64), y.view(np.uint64)), f"replay {rep}"
        C.spmm(mats[0], Xs[0])  # eager work between replays
        torch.cuda.synchronize()


def test_batched_single_tile_per_matrix_and_empty(C):
    """Matrices without rows or entries inside a batch; more workgroups than
    tiles (late workgroups find the queue empty)."""
    A0 = synth.random_csr(0, 10, max_row=1, seed=1)
    A1 = synth.random_csr(100, 100, max_row=0, seed=2)
    A2 = synth.laplace2d(30)
    mats, Xs, Ys, host = [], [], [], []
    for i, A in enumerate([A0, A1, A2]):
        rp, ci, v, hv = G.upload(A, "f64")
        M = C.from_csr(rp, ci, v, A.cols, 4)
        X, Xh = _rhs(A, 2, "f64", seed=i)
        Y = torch.full((A.rows, 2), float("nan"), dtype=torch.float64, device="cuda")
        mats.append(M)
        Xs.append(X)
        Ys.append(Y)
        host.append((A, hv, Xh))
    plan = C.spmm_plan(mats, Xs, Ys, blocks_per_cu=8)
    for _ in range(3):
        C.spmm_batched(plan)
    torch.cuda.synchronize()
    for (A, hv, Xh), Y in zip(host, Ys):
        if A.rows:
            _check_cols(A, hv, "f64", Xh, Y.cpu().numpy())


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batched_full_workload_sampled_rows(C, dtype):
    """The full uneven batch (256 matrices, 10k-500k rows, 1.1e9 entries) in
    fp64 and fp32 with the default plan, one persistent launch: 16 sampled
    rows of every matrix and every right-hand side against the oracle's row
    sums (fp32: on the fp32 values and x, with the fp32 bound)."""
    from synth import gpu_families as F
    tdt = torch.float64 if dtype == "f64" else torch.float32
    u = U64 if dtype == "f64" else U32
    W = F.batched_workload(seed=0)
    mats, Xs, Ys, keep = [], [], [], []
    for i, (fam, rp, ci, val, cols, r) in enumerate(W):
        val = val.to(tdt)
        mats.append(C.from_csr(rp, ci, val, cols, 4, sort=True))
        X = torch.randn(cols, r, dtype=torch.float64, device="cuda").to(tdt)
        Xs.append(X)
        Ys.append(torch.full((rp.numel() - 1, r), float("nan"), dtype=tdt, device="cuda"))
        keep.append((rp, ci, val))
    plan = C.spmm_plan(mats, Xs, Ys)
    C.spmm_batched(plan)
    torch.cuda.synchronize()
    g = np.random.default_rng(0)
    for (rp, ci, val), X, Y in zip(keep, Xs, Ys):
        rows = rp.numel() - 1
        sample = np.unique(np.concatenate([[0, rows - 1], g.integers(0, rows, 14)]))
        hrp = rp.cpu().numpy()
        Xh = X.cpu().numpy().astype(np.float64)
        Yh = Y.cpu().numpy().astype(np.float64)
        for i in sample:
            a, b = int(hrp[i]), int(hrp[i + 1])
            sub_rp = np.array([0, b - a], dtype=np.int32)
            cols_i = ci[a:b].cpu().numpy()
            vals_i = val[a:b].cpu().numpy().astype(np.float64)
            for k in range(X.shape[1]):
                xk = np.ascontiguousarray(Xh[:, k])
                ref = oracle.csr_spmv(sub_rp, cols_i, vals_i, xk)[0]
                tol = oracle.spmv_bound(sub_rp, cols_i, vals_i, xk, u, factor=4.0)[0]
                assert abs(Yh[i, k] - ref) <= tol, (i, k)


def test_autotuner_and_graph_runner(C):
    """batched.tune picks one of its candidate plans, whose results match the
    oracle; a Graph of it replays the same bits."""
    from paper_1203_2946_amd import batched as B
    mats, Xs, Ys, host = _batch(C, seed=31, count=10)
    plan, tun, table = B.tune(mats, Xs, Ys, candidates={"tile_nnz": (2000, 20000), "group": (0, 4),
                                                        "blocks_per_cu": (1, 4)}, reps=2)
    assert len(table) == 8 and tun in [t for t, _ in table]
    assert min(ms for _, ms in table) == [ms for t, ms in table if t == tun][0]
    g = B.Graph(plan)
    for Y in Ys:
        Y.fill_(float("nan"))
    g.replay()
    torch.cuda.synchronize()
    first = [Y.cpu().numpy().copy() for Y in Ys]
    for (A, hv, Xh), y in zip(host, first):
        _check_cols(A, hv, "f64", Xh, y)
    g.replay()
    torch.cuda.synchronize()
    for Y, y in zip(Ys, first):
        assert np.array_equal(Y.cpu().numpy().view(np.uint64), y.view(np.uint64))
    assert B.batch_bytes(mats, [X.shape[1] for X in Xs]) > 0
