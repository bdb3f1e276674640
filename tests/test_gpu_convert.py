"""GPU parity of the conversions (CSR -> CMRS, CMRS -> CSR) against the oracle.

Bar: bit-exact on every array (strip pointers, packed words, value bits),
through the C ABI, for every height 1..32, sorted and unsorted, on seeded
inputs that span many strips and a ragged last strip, at full workload sizes,
and on the edge cases (no rows, no entries, empty rows and strips, strips
longer than a wave's and a workgroup's sort capacity, rectangular shapes).
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import synth
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_example.json")


@pytest.fixture(scope="module")
def C():
    from paper_1203_2946_amd import cmrs
    return cmrs


def check_from_csr(C, A, height, sort, dtype="f64", in_place=False):
    rp, ci, v, hv = G.upload(A, dtype)
    M = C.from_csr(rp, ci, v, A.cols, height, sort=sort, in_place=in_place)
    torch.cuda.synchronize()
    esp, ew, ev = oracle.csr_to_cmrs(A.row_ptr, A.col_ind, hv, A.cols, height, sorted_=sort)
    assert np.array_equal(M.strip_ptr.cpu().numpy(), esp), "strip_ptr"
    assert np.array_equal(G.words(M.col_word), ew), "col_word"
    assert np.array_equal(G.val_bits(M.val), G.np_bits(ev)), "val"
    return M, hv


def check_round_trip(C, A, M, hv):
    rp2, ci2, v2 = C.to_csr(M)
    torch.cuda.synchronize()
    erp, eci, ev = oracle.cmrs_to_csr(M.strip_ptr.cpu().numpy(), G.words(M.col_word), G.val_bits(M.val).view(hv.dtype),
                                      A.rows, M.height)
    assert np.array_equal(rp2.cpu().numpy(), erp), "row_ptr vs oracle"
    assert np.array_equal(ci2.cpu().numpy(), eci), "col_ind vs oracle"
    assert np.array_equal(G.val_bits(v2), G.np_bits(ev)), "val vs oracle"
    return rp2, ci2, v2


def test_paper_example(C):
    P = json.load(open(GOLDEN))
    c = P["crs"]
    A = synth.Csr(5, 5, np.array(c["RowPtr"], np.int32), np.array(c["ColInd"], np.int32),
                  np.array(c["Val"], np.float64))
    for key, sort in (("cmrs_h2", False), ("cmrs_h2_sorted", True)):
        M, _ = check_from_csr(C, A, 2, sort)
        exp = P[key]
        w = G.words(M.col_word)
        assert M.strip_ptr.cpu().tolist() == exp["StripPtr"]
        assert (w >> 4).tolist() == exp["ColInd"]
        assert (w & 15).tolist() == exp["RowInStrip"]
        assert M.val.cpu().tolist() == [float(a) for a in exp["Val"]]


@pytest.mark.parametrize("height", list(range(1, 33)))
@pytest.mark.parametrize("sort", [False, True])
def test_random_all_heights(C, height, sort):
    A = synth.random_csr(517, 300, max_row=20, seed=height, canonical=sort or height % 2 == 0,
                         duplicates=(not sort) and height % 3 == 0, explicit_zeros=True)
    M, hv = check_from_csr(C, A, height, sort)
    rp2, ci2, v2 = check_round_trip(C, A, M, hv)
    # round trip returns the input itself (sorted: the input is canonical)
    assert np.array_equal(rp2.cpu().numpy(), A.row_ptr) and np.array_equal(ci2.cpu().numpy(), A.col_ind)
    assert np.array_equal(G.val_bits(v2), A.val.view(np.uint64))


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("sort", [False, True])
@pytest.mark.parametrize("height", [2, 4, 8])
def test_laplacian_64(C, dtype, sort, height):
    A = synth.laplace2d(64)
    M, hv = check_from_csr(C, A, height, sort, dtype)
    rp2, ci2, v2 = check_round_trip(C, A, M, hv)
    assert np.array_equal(rp2.cpu().numpy(), A.row_ptr) and np.array_equal(ci2.cpu().numpy(), A.col_ind)
    assert np.array_equal(G.val_bits(v2), G.np_bits(hv))


@pytest.mark.parametrize("height", [3, 8, 32])
def test_in_place_unsorted(C, height):
    A = synth.random_csr(300, 200, max_row=12, seed=11, canonical=False)
    rp, ci, v, hv = G.upload(A)
    ci_ptr, v_ptr = ci.data_ptr(), v.data_ptr()
    M = C.from_csr(rp, ci, v, A.cols, height, in_place=True)
    assert M.col_word.data_ptr() == ci_ptr and M.val.data_ptr() == v_ptr
    torch.cuda.synchronize()
    esp, ew, ev = oracle.csr_to_cmrs(A.row_ptr, A.col_ind, hv, A.cols, height)
    assert np.array_equal(M.strip_ptr.cpu().numpy(), esp)
    assert np.array_equal(G.words(M.col_word), ew)
    assert np.array_equal(G.val_bits(M.val), G.np_bits(ev))


def test_edge_empty(C):
    # no rows
    A0 = synth.Csr(0, 5, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    for sort in (False, True):
        M = C.from_csr(*G.upload(A0)[:3], A0.cols, 4, sort=sort)
        rp2, ci2, v2 = C.to_csr(M)
        torch.cuda.synchronize()
        assert M.strip_ptr.cpu().tolist() == [0]
        assert rp2.cpu().tolist() == [0] and ci2.numel() == 0
    # rows but no entries
    A1 = synth.Csr(10, 3, np.zeros(11, np.int32), np.zeros(0, np.int32), np.zeros(0))
    for sort in (False, True):
        M, hv = check_from_csr(C, A1, 4, sort)
        check_round_trip(C, A1, M, hv)
    # single row, single column
    A2 = synth.Csr(1, 1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([2.5]))
    for h in (1, 2, 32):
        M, hv = check_from_csr(C, A2, h, True)
        check_round_trip(C, A2, M, hv)


@pytest.mark.parametrize("shape", [(1000, 37), (37, 5000)])
def test_rectangular(C, shape):
    A = synth.random_csr(shape[0], shape[1], max_row=30, seed=4)
    for h in (1, 5, 16):
        for sort in (False, True):
            M, hv = check_from_csr(C, A, h, sort)
            check_round_trip(C, A, M, hv)


def _long_strip_matrix(rows, cols, long_rows, long_len, seed):
    """Mostly short rows plus a few rows of long_len entries (long strips)."""
    rng = np.random.default_rng(seed)
    k = rng.integers(0, 4, rows)
    k[long_rows] = long_len
    cl = [np.sort(rng.choice(cols, size=int(kk), replace=False)) for kk in k]
    col = np.concatenate(cl)
    rp = np.zeros(rows + 1, np.int64)
    np.cumsum(k, out=rp[1:])
    return synth.Csr(rows, cols, rp.astype(np.int32), col.astype(np.int32), rng.standard_normal(col.size))


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_long_strips_sorted(C, dtype):
    """Strips beyond the per-wave (1024) and per-workgroup (16384) LDS sort
    capacities take the workgroup and the global-workspace sort paths."""
    A = _long_strip_matrix(4000, 60000, [5, 6, 1000, 1001, 1002, 3999], 9000, seed=1)
    for h in (2, 4, 8):
        M, hv = check_from_csr(C, A, h, True, dtype)
        rp2, ci2, v2 = check_round_trip(C, A, M, hv)
        assert np.array_equal(ci2.cpu().numpy(), A.col_ind)


def test_long_strips_unsorted_noncanonical(C):
    A = _long_strip_matrix(3000, 40000, [7, 8, 9], 20000, seed=2)
    rng = np.random.default_rng(3)
    for i in range(A.rows):
        a, b = A.row_ptr[i], A.row_ptr[i + 1]
        A.col_ind[a:b] = rng.permutation(A.col_ind[a:b])
    for h in (4, 16, 32):
        M, hv = check_from_csr(C, A, h, False)
        rp2, ci2, v2 = check_round_trip(C, A, M, hv)
        assert np.array_equal(ci2.cpu().numpy(), A.col_ind)
        M2, hv2 = check_from_csr(C, A, h, True)   # sorted from non-canonical input: oracle decides
        check_round_trip(C, A, M2, hv2)


@pytest.fixture(scope="module")
def c2():
    return synth.poisson_rows(1 << 20, 16.0, seed=0)


@pytest.fixture(scope="module")
def c3():
    return synth.zipf_clustered(2_000_000, seed=0)


@pytest.mark.parametrize("height", [1, 2, 4, 8, 16, 32])
def test_c2_full_size(C, c2, height):
    """n = 2^20, Poisson(16) rows: bit-exact conversion both ways, sorted."""
    M, hv = check_from_csr(C, c2, height, True)
    rp2, ci2, v2 = C.to_csr(M)
    torch.cuda.synchronize()
    assert np.array_equal(rp2.cpu().numpy(), c2.row_ptr) and np.array_equal(ci2.cpu().numpy(), c2.col_ind)
    assert np.array_equal(G.val_bits(v2), c2.val.view(np.uint64))


@pytest.mark.parametrize("height,sort", [(2, True), (8, True), (8, False), (16, False), (32, True)])
def test_c3_full_size(C, c3, height, sort):
    """n = 2e6, Zipf(2) rows up to 10000 entries: long strips in sorted mode."""
    M, hv = check_from_csr(C, c3, height, sort)
    rp2, ci2, v2 = C.to_csr(M)
    torch.cuda.synchronize()
    assert np.array_equal(rp2.cpu().numpy(), c3.row_ptr) and np.array_equal(ci2.cpu().numpy(), c3.col_ind)
    assert np.array_equal(G.val_bits(v2), c3.val.view(np.uint64))


def test_validate_csr(C):
    A = synth.random_csr(100, 50, seed=1)
    rp, ci, _, _ = G.upload(A)
    assert C.validate_csr(rp, ci, A.cols) == 0
    bad = ci.clone()
    bad[3] = 50
    assert C.validate_csr(rp, bad, A.cols) & 4
    rpb = rp.clone()
    rpb[10] = rpb[11] + 1
    assert C.validate_csr(rpb, ci, A.cols) & 2
    rpc = rp.clone()
    rpc[-1] += 1
    assert C.validate_csr(rpc, ci, A.cols) & 1


def _run_totals_matrix(totals, run_rows, cols, spread, seed):
    """Rows grouped in runs of run_rows rows; run i holds totals[i] entries,
    all in its first row (spread=False) or dealt round-robin over its rows."""
    rng = np.random.default_rng(seed)
    k = np.zeros(len(totals) * run_rows, np.int64)
    for i, t in enumerate(totals):
        if spread:
            k[i * run_rows:(i + 1) * run_rows] = t // run_rows
            k[i * run_rows:i * run_rows + t % run_rows] += 1
        else:
            k[i * run_rows] = t
    cl = [np.sort(rng.choice(cols, size=int(kk), replace=False)) for kk in k]
    col = np.concatenate(cl) if cl else np.zeros(0)
    rp = np.zeros(k.size + 1, np.int64)
    np.cumsum(k, out=rp[1:])
    return synth.Csr(k.size, cols, rp.astype(np.int32), col.astype(np.int32), rng.standard_normal(col.size))


@pytest.mark.parametrize("spread", [False, True])
@pytest.mark.parametrize("height", [2, 3, 16, 32])
def test_run_boundaries(C, height, spread):
    """Runs of whole strips of up to 32 rows with 0, 1, 63, 64, 767, 768, 769
    and 1500 entries: the conversions' register and streaming paths and their
    cut-over, empty runs between full ones, and a ragged last run."""
    run_rows = (32 // height) * height
    A = _run_totals_matrix([0, 767, 768, 769, 0, 0, 1, 63, 64, 1500, 768, 5], run_rows, 4000, spread, seed=height)
    A = synth.Csr(A.rows - 3, A.cols, A.row_ptr[:-3].copy(), A.col_ind[:A.row_ptr[-4]].copy(),
                  A.val[:A.row_ptr[-4]].copy())
    for sort in (False, True):
        M, hv = check_from_csr(C, A, height, sort)
        rp2, ci2, v2 = check_round_trip(C, A, M, hv)
        assert np.array_equal(rp2.cpu().numpy(), A.row_ptr) and np.array_equal(ci2.cpu().numpy(), A.col_ind)
        assert np.array_equal(G.val_bits(v2), A.val.view(np.uint64))


@pytest.mark.parametrize("spread", [False, True])
@pytest.mark.parametrize("height", [2, 5, 32])
def test_shared_long_runs(C, height, spread):
    """CMRS -> CSR runs of more than 2048 entries are shared by the waves of a
    workgroup: runs just below and above that length, several long runs in one
    workgroup (runs 4..7), a long run between short ones and a long ragged last
    run, sorted and unsorted."""
    run_rows = (32 // height) * height
    totals = [2047, 2048, 2049, 10, 5000, 9001, 3000, 2100, 0, 64, 4097, 1, 6000]
    A = _run_totals_matrix(totals, run_rows, 20000, spread, seed=40 + height)
    A = synth.Csr(A.rows - 2, A.cols, A.row_ptr[:-2].copy(), A.col_ind[:A.row_ptr[-3]].copy(),
                  A.val[:A.row_ptr[-3]].copy())
    for sort in (False, True):
        M, hv = check_from_csr(C, A, height, sort)
        rp2, ci2, v2 = check_round_trip(C, A, M, hv)
        assert np.array_equal(rp2.cpu().numpy(), A.row_ptr) and np.array_equal(ci2.cpu().numpy(), A.col_ind)
        assert np.array_equal(G.val_bits(v2), A.val.view(np.uint64))


def _rows_matrix(rng, rows, cols, lengths, col_fn, canonical=True):
    cl = []
    for i, k in enumerate(lengths):
        c = col_fn(i, int(k)) if k else np.zeros(0, np.int64)
        c = np.sort(c) if canonical else c
        cl.append(c)
    rp = np.zeros(rows + 1, np.int64)
    np.cumsum([c.size for c in cl], out=rp[1:])
    col = np.concatenate(cl).astype(np.int32) if cl else np.zeros(0, np.int32)
    return synth.Csr(rows, cols, rp.astype(np.int32), col, rng.standard_normal(col.size))


@pytest.mark.parametrize("height", [4, 8])
def test_both_lists_many_mid_strips(C, height):
    """One launch sorts both lists of strips the group kernel leaves: more
    mid-size strips (257..1024 entries, one wave each) than the launch has
    waves (256 workgroups x 16), so waves take several in turn, together with
    long strips (one workgroup each) that hold a few workgroups back while
    the others start on the mid-size ones."""
    rng = np.random.default_rng(77 + height)
    strips = 5000
    rows, cols = strips * height, 1 << 20
    k = rng.integers(300 // height, 1000 // height, rows)
    k[[3, 4000, rows - 1]] = 3000                                         # three long strips
    A = _rows_matrix(rng, rows, cols, k, lambda i, n: rng.choice(cols, n, replace=False))
    per_strip = np.add.reduceat(np.diff(A.row_ptr), np.arange(0, rows, height))
    assert int(np.sum((per_strip > 256) & (per_strip <= 1024))) > 256 * 16
    assert int(np.sum(per_strip > 1024)) == 3
    M, hv = check_from_csr(C, A, height, True)
    check_round_trip(C, A, M, hv)


@pytest.mark.parametrize("height", [16, 32])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_tall_strips_bucket_sort(C, height, dtype):
    """Strips of 320..1100 entries on average (the one-wave bucket sort of
    tall strips): uniform columns, unsorted rows with duplicate columns,
    columns bunched in two clusters far apart (more than 64 keys in one
    bucket: the bitonic fallback), a few strips beyond 1024 entries (the
    workgroup list), empty strips and a ragged last strip."""
    rng = np.random.default_rng(height)
    rows, cols = 40 * height + 5, 1 << 22
    mean = 1100 // height + 1
    k = rng.poisson(mean, rows)
    k[rng.random(rows) < 0.05] = 0
    k[: height] = 0                      # an empty first strip
    k[3 * height + 1] = 3000             # strips past 1024 entries
    A = _rows_matrix(rng, rows, cols, k, lambda i, n: rng.choice(cols, size=n, replace=False))
    check_from_csr(C, A, height, True, dtype)
    # unsorted rows with duplicates inside a row
    B = _rows_matrix(rng, rows, cols, k, lambda i, n: rng.integers(0, cols, n), canonical=False)
    check_from_csr(C, B, height, True, dtype)
    # two tight clusters at both ends of the column range
    Cl = _rows_matrix(rng, rows, cols, k, lambda i, n: np.where(
        rng.random(n) < 0.5, rng.integers(0, 40, n), cols - 1 - rng.integers(0, 40, n)), canonical=False)
    check_from_csr(C, Cl, height, True, dtype)
    # band around the diagonal plus scattered columns (the skewed workload's shape)
    D = _rows_matrix(rng, rows, cols, k, lambda i, n: np.unique(np.concatenate(
        [np.clip(i + rng.integers(-512, 513, max(1, 7 * n // 10)), 0, cols - 1), rng.integers(0, cols, n // 3)])))
    check_from_csr(C, D, height, True, dtype)


@pytest.mark.parametrize("height", [2, 3, 7, 12, 24, 32])
@pytest.mark.parametrize("dtype", ["f64", "bf16"])
def test_workgroup_merge_strips(C, height, dtype):
    """Listed strips of 1025..16384 entries with rows sorted by column (the
    workgroup's merge of the row runs): one dominant row among short ones,
    rows of equal length, repeated columns inside a row (ties keep CSR
    order), empty rows inside a strip, a strip of exactly 16384 entries and
    one of 16385 (the workspace path), columns in a band around the diagonal
    plus scattered ones (the skewed workload's shape)."""
    rng = np.random.default_rng(100 + height)
    strips = 24
    rows, cols = strips * height - 1, 1 << 21
    k = rng.poisson(6, rows)
    k[rng.random(rows) < 0.2] = 0
    for s in range(strips):
        r0 = s * height
        if s % 4 == 0:
            k[r0 + (s // 4) % height] = int(rng.integers(1100, 12000))       # one dominant row
        elif s % 4 == 1:
            k[r0: r0 + height] = 16384 // height + 40                    # rows of equal length
    k = k[:rows]
    # strip 2: exactly 16384 entries, strip 3: 16385
    for s, want in ((2, 16384), (3, 16385)):
        seg = k[s * height:(s + 1) * height]
        seg[:] = want // height
        seg[0] += want - int(seg.sum())
    assert int(k[2 * height:3 * height].sum()) == 16384 and int(k[3 * height:4 * height].sum()) == 16385

    def cols_of(i, n):
        near = np.clip(i * (cols // rows) + rng.integers(-512, 513, n), 0, cols - 1)
        far = rng.integers(0, cols, n)
        c = np.where(rng.random(n) < 0.7, near, far)
        if i % 3 == 0:
            c[: n // 4] = c[0]                                           # repeated columns
        return c
    A = _rows_matrix(rng, rows, cols, k, cols_of)
    M, hv = check_from_csr(C, A, height, True, dtype)
    check_round_trip(C, A, M, hv)


@pytest.mark.parametrize("height", [1, 2, 32])
def test_long_strip_single_descent(C, height):
    """Listed strips whose rows are sorted but for one descending pair, placed
    where the workgroup sort's check pairs entries across waves (entry 63|64,
    1023|1024, 1087|1088 of the strip) or inside a wave (500|501): each strip
    must still come out in (column, row, CSR order)."""
    rng = np.random.default_rng(7 + height)
    cuts = [63, 1023, 1087, 500]
    rows, cols = len(cuts) * height, 1 << 20
    k = np.zeros(rows, np.int64)
    k[::height] = 3000                       # one long first row per strip
    if height > 1:
        k[1::height] = 5
    A = _rows_matrix(rng, rows, cols, k, lambda i, n: rng.choice(cols, size=n, replace=False))
    for s, c in enumerate(cuts):
        a = A.row_ptr[s * height] + c        # a pair inside the long row
        A.col_ind[a], A.col_ind[a + 1] = A.col_ind[a + 1], A.col_ind[a]
    M, hv = check_from_csr(C, A, height, True)
    check_round_trip(C, A, M, hv)


@pytest.mark.parametrize("seed", range(6))
def test_long_strips_random_mixes(C, seed):
    """Listed strips (past 1024 entries) from random mixes of row lengths: empty
    rows, short rows (the gathered short-row list, up to and past its 512-entry
    capacity), rows just over the 64-entry short-row limit, and long rows (one
    or several per strip); repeated columns inside rows; heights 2..32 with
    ragged last strips; every value type."""
    rng = np.random.default_rng(1000 + seed)
    height = int(rng.choice([2, 3, 8, 16, 24, 32]))
    dtype = ["f64", "f32", "bf16"][seed % 3]
    strips = 20
    rows, cols = strips * height - int(rng.integers(0, height)), 1 << 21
    kinds = rng.choice(5, size=rows, p=[0.15, 0.45, 0.15, 0.1, 0.15])
    lo_hi = [(0, 1), (1, 11), (20, 65), (65, 200), (1000, 6000)]
    k = np.array([rng.integers(*lo_hi[t]) for t in kinds], dtype=np.int64)
    if height >= 16:                      # strip 0: short rows past the 512-entry list
        k[:height] = 40
        k[0] = 2000

    def cols_of(i, n):
        c = rng.integers(0, cols, n)
        if rng.random() < 0.3 and n > 2:
            c[: n // 3] = c[0]                                           # repeated columns
        return c
    A = _rows_matrix(rng, rows, cols, k, cols_of)
    M, hv = check_from_csr(C, A, height, True, dtype)
    check_round_trip(C, A, M, hv)


@pytest.mark.parametrize("height", [8, 16, 32])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_to_csr_staged_runs(C, height, dtype):
    """CMRS -> CSR where runs of rows are long enough on average for the output
    to be staged in LDS: runs below and above the stage's 640 entries and past
    the shared-run length (2048), empty rows, an empty run of rows, a ragged
    last strip; sorted and unsorted strips."""
    rng = np.random.default_rng(300 + height)
    rows, cols = 32 * 40 + 7, 1 << 20
    k = rng.poisson(16, rows)
    k[rng.random(rows) < 0.1] = 0
    k[32:64] = 0                                  # an empty run of 32 rows
    k[96:128] = 25                                # a run of 800 entries
    k[160] = 2500                                 # a run past 2048 entries
    A = _rows_matrix(rng, rows, cols, k, lambda i, n: rng.choice(cols, size=n, replace=False))
    for sort in (True, False):
        M, hv = check_from_csr(C, A, height, sort, dtype)
        rp2, ci2, v2 = check_round_trip(C, A, M, hv)
        assert np.array_equal(rp2.cpu().numpy(), A.row_ptr)


def test_graph_replay_sorted_conversion(C):
    """CSR -> CMRS sorted (short strips in groups, strips listed for one wave,
    long strips for a workgroup with its shared counter, a strip past the
    workgroup's LDS) and CMRS -> CSR captured in one HIP graph: its counters
    are cleared by a kernel, not a memset node.  Every replay, with eager
    work and the outputs scrambled in between, equals the eager result."""
    A = _long_strip_matrix(4000, 60000, [5, 6, 1000, 1001, 1002, 3999], 9000, seed=4)
    h = 8
    rp, ci, v, hv = G.upload(A)
    ws = torch.empty(max(1, C.from_csr_workspace_bytes(A.rows, A.nnz, h, True)), dtype=torch.uint8, device="cuda")
    M = C.from_csr(rp, ci, v, A.cols, h, sort=True, workspace=ws)
    torch.cuda.synchronize()
    ref_w, ref_v, ref_sp = M.col_word.clone(), M.val.clone(), M.strip_ptr.clone()
    back = (torch.empty_like(rp), torch.empty_like(ci), torch.empty_like(v))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            C.from_csr(rp, ci, v, A.cols, h, sort=True, workspace=ws, out=M)
            C.to_csr(M, out=back)
    torch.cuda.current_stream().wait_stream(s)
    for i in range(4):
        M.col_word.fill_(-1)
        M.strip_ptr.fill_(-1)
        M.val.fill_(float("nan"))
        for t in back:
            t.fill_(-7)
        C.from_csr(rp, ci, v, A.cols, 2, sort=True)       # eager work in between
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(M.col_word, ref_w) and torch.equal(M.strip_ptr, ref_sp), f"replay {i}: CMRS"
        assert np.array_equal(G.val_bits(M.val), G.val_bits(ref_v)), f"replay {i}: values"
        assert torch.equal(back[0], rp) and torch.equal(back[1], ci), f"replay {i}: CSR"
        assert np.array_equal(G.val_bits(back[2]), G.val_bits(v)), f"replay {i}: CSR values"
    check_from_csr(C, A, h, True)
