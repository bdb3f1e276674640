"""Pins of the padded-CMRS reference (Sec. 6.7) on the CPU."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import brute
from oracle import padded as P

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_example.json")


def test_paper_example_height2_by_hand():
    """The 5x5 matrix of Sec. 2.3 at height 2, arranged by hand from the
    rule: strip 0 = rows 0 and 1 (2 entries each, row 0 first), strip 1 =
    row 3 (3 entries, more left, so first) then row 2, strip 2 = row 4; each
    strip one chunk of 64 with padding words (RowInStrip 2, column 0)."""
    crs = json.load(open(GOLDEN))["crs"]
    sp, w, v = P.arrange(crs["RowPtr"], crs["ColInd"], np.asarray(crs["Val"], float), 2)
    assert list(sp) == [0, 64, 128, 192]
    assert list(w[:4]) == [0 << 4 | 0, 3 << 4 | 0, 1 << 4 | 1, 4 << 4 | 1] and list(v[:4]) == [1, 2, 3, 4]
    assert all(w[4:64] == 2) and all(v[4:64] == 0)
    assert list(w[64:69]) == [2 << 4 | 1, 3 << 4 | 1, 4 << 4 | 1, 2 << 4 | 0, 4 << 4 | 0]
    assert list(v[64:69]) == [7, 8, 9, 5, 6]
    assert all(w[69:128] == 2)
    assert w[128] == 4 << 4 and v[128] == 10 and all(w[129:] == 2)


def test_padded_bits():
    assert [P.padded_bits(h) for h in (1, 2, 3, 4, 7, 8, 15, 16, 17, 31, 32)] == [4, 4, 4, 4, 4, 4, 4, 5, 5, 5, 6]


@pytest.mark.parametrize("height", [1, 2, 3, 8, 16, 32])
@pytest.mark.parametrize("seed", [0, 1])
def test_arrangement_meets_the_constraints(height, seed):
    A = synth.random_csr(300, 200, max_row=40, seed=seed)
    sp, w, v = P.arrange(A.row_ptr, A.col_ind, A.val, height)
    P.check_constraints(A.row_ptr, A.col_ind, A.val, height, sp, w, v)


def test_long_rows_need_one_chunk_per_eight_entries():
    # One row of 100 entries in a strip of 16: at least ceil(100/8) = 13 chunks,
    # and the greedy rule reaches that bound.
    A = synth.random_csr(16, 500, max_row=0, seed=0)
    row_ptr = np.zeros(17, np.int64)
    row_ptr[4:] = 100
    col = np.arange(100, dtype=np.int32) * 3
    sp, w, v = P.arrange(row_ptr, col, np.ones(100), 16)
    assert sp[-1] == 13 * 64
    P.check_constraints(row_ptr, col, np.ones(100), 16, sp, w, v)
    assert A.nnz == 0


def test_full_chunks_without_padding():
    # height 8, every row 8 entries: 64 entries, exactly one full chunk per strip.
    n = 64
    row_ptr = np.arange(n + 1) * 8
    col = np.tile(np.arange(8), n).astype(np.int32)
    sp, w, v = P.arrange(row_ptr, col, np.arange(8.0 * n), 8)
    assert list(sp) == [64 * s for s in range(n // 8 + 1)]
    assert not np.any((w & 15) == 8)


def test_checker_rejects_broken_arrangements():
    A = synth.random_csr(64, 64, max_row=20, seed=3)
    sp, w, v = P.arrange(A.row_ptr, A.col_ind, A.val, 4)
    P.check_constraints(A.row_ptr, A.col_ind, A.val, 4, sp, w, v)
    # A padding value that is not zero.
    pad = np.nonzero((w & 15) == 4)[0][0]
    v2 = v.copy()
    v2[pad] = 1.0
    with pytest.raises(AssertionError):
        P.check_constraints(A.row_ptr, A.col_ind, A.val, 4, sp, w, v2)
    # Two entries of one chunk swapped across rows: the run structure breaks
    # or the per-row entry lists differ.
    real = np.nonzero((w & 15) != 4)[0]
    i, j = real[0], real[-1]
    w3 = w.copy()
    w3[i], w3[j] = w3[j], w3[i]
    with pytest.raises(AssertionError):
        P.check_constraints(A.row_ptr, A.col_ind, A.val, 4, sp, w3, v)


@pytest.mark.parametrize("height", [1, 4, 16])
def test_product_of_padded_arrays_is_the_matrix_product(height):
    A = synth.random_csr(120, 90, max_row=30, seed=height, int_values=True)
    x = np.random.default_rng(height).integers(-5, 6, A.cols).astype(float)
    sp, w, v = P.arrange(A.row_ptr, A.col_ind, A.val, height)
    y = P.spmv_by_definition(sp, w, v, A.rows, height, x)
    dense = brute.dense_from_coo(A.rows, A.cols, brute.coo_from_csr(A.row_ptr, A.col_ind, A.val))
    assert np.array_equal(y, np.asarray(brute.dense_matvec(dense, list(x))))
