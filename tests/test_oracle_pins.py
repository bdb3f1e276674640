"""Pins of the CPU oracle against what the paper and plain mathematics fix.

None of these compares the oracle with itself: the expected values are the
arrays printed in the paper (tests/golden/paper_example.json), brute force in
pure Python (oracle/brute.py), exact rational arithmetic, closed forms, and
special matrices whose product is known exactly.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_example.json")


@pytest.fixture(scope="module")
def paper():
    with open(GOLDEN) as f:
        return json.load(f)


def _crs_M(paper):
    c = paper["crs"]
    return (np.array(c["RowPtr"], np.int32), np.array(c["ColInd"], np.int32), np.array(c["Val"], np.float64))


def _unpack(word, bits):
    word = np.asarray(word, dtype=np.uint32)
    return (word >> bits).astype(np.int64), (word & ((1 << bits) - 1)).astype(np.int64)


# ------------------------------------------------------------ printed example
def test_crs_of_M_matches_dense_and_coo(paper):
    """The printed CRS/COO arrays describe the printed dense M (Sec. 2.3)."""
    rp, ci, v = _crs_M(paper)
    dense = oracle.csr_to_dense(rp, ci, v, 5)
    assert dense.tolist() == [[float(a) for a in r] for r in paper["dense_M"]]
    coo = paper["coo"]
    rows = np.repeat(np.arange(5), np.diff(rp))
    assert rows.tolist() == coo["RowInd"]


def test_cmrs_h2_unsorted_printed(paper):
    rp, ci, v = _crs_M(paper)
    sp, w, vo = oracle.csr_to_cmrs(rp, ci, v, 5, height=2, sorted_=False)
    exp = paper["cmrs_h2"]
    col, ris = _unpack(w, oracle.bits_for_height(2))
    assert sp.tolist() == exp["StripPtr"]
    assert col.tolist() == exp["ColInd"]
    assert ris.tolist() == exp["RowInStrip"]
    assert vo.tolist() == [float(a) for a in exp["Val"]]


def test_cmrs_h2_sorted_printed(paper):
    rp, ci, v = _crs_M(paper)
    sp, w, vo = oracle.csr_to_cmrs(rp, ci, v, 5, height=2, sorted_=True)
    exp = paper["cmrs_h2_sorted"]
    col, ris = _unpack(w, oracle.bits_for_height(2))
    assert sp.tolist() == exp["StripPtr"]
    assert col.tolist() == exp["ColInd"]
    assert ris.tolist() == exp["RowInStrip"]
    assert vo.tolist() == [float(a) for a in exp["Val"]]


def test_packed_word_layout_B4(paper):
    """Sec. 4: RowInStrip in the low 4 bits, the column above them."""
    rp, ci, v = _crs_M(paper)
    _, w, _ = oracle.csr_to_cmrs(rp, ci, v, 5, height=2)
    exp = paper["cmrs_h2"]
    assert w.tolist() == [(c << 4) | r for c, r in zip(exp["ColInd"], exp["RowInStrip"])]


def test_spmv_of_M_by_brute_force(paper):
    """y = M x with the dense M printed in Sec. 2.3; integers, so exact."""
    rp, ci, v = _crs_M(paper)
    dense = [[float(a) for a in r] for r in paper["dense_M"]]
    for x in ([1.0] * 5, [1.0, 2.0, 3.0, 4.0, 5.0], [-3.0, 0.5, 7.0, -1.0, 2.0]):
        y = oracle.csr_spmv(rp, ci, v, np.array(x))
        assert y.tolist() == brute.dense_matvec(dense, x)


def test_transposed_product_is_rejected(paper):
    """M is not symmetric: M^T x differs from M x, so an operand swap cannot pass."""
    rp, ci, v = _crs_M(paper)
    dense = np.array(paper["dense_M"], dtype=np.float64)
    x = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    y = oracle.csr_spmv(rp, ci, v, x)
    assert not np.array_equal(y, dense.T @ x)
    assert y.tolist() == [9.0, 26.0, 45.0, 98.0, 50.0]


# ------------------------------------------------------------ definitions
@pytest.mark.parametrize("height", [1, 2, 3, 4, 5, 7, 8, 16, 32])
def test_other_heights_on_M(paper, height):
    """StripPtr[j] = RowPtr[j*height], StripPtr[strips] = nnz, RowInStrip = row mod height (Sec. 3)."""
    rp, ci, v = _crs_M(paper)
    sp, w, _ = oracle.csr_to_cmrs(rp, ci, v, 5, height=height)
    strips = -(-5 // height)
    assert sp.tolist() == [int(rp[j * height]) for j in range(strips)] + [10]
    _, ris = _unpack(w, oracle.bits_for_height(height))
    rows = np.repeat(np.arange(5), np.diff(rp))
    assert ris.tolist() == (rows % height).tolist()


def test_height1_equals_crs():
    """Sec. 3: with height 1 CMRS and CRS coincide."""
    A = synth.random_csr(40, 30, seed=3)
    sp, w, vo = oracle.csr_to_cmrs(A.row_ptr, A.col_ind, A.val, A.cols, height=1)
    assert np.array_equal(sp, A.row_ptr)
    col, ris = _unpack(w, oracle.bits_for_height(1))
    assert np.array_equal(col, A.col_ind) and not ris.any()
    assert np.array_equal(vo.view(np.uint64), A.val.view(np.uint64))


def test_bits_for_height():
    assert [oracle.bits_for_height(h) for h in (1, 2, 4, 8, 9, 16, 17, 32)] == [4, 4, 4, 4, 4, 4, 5, 5]
    assert oracle.num_strips(5, 2) == 3 and oracle.num_strips(0, 4) == 0 and oracle.num_strips(8, 4) == 2


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("height", [1, 2, 3, 4, 8])
@pytest.mark.parametrize("sorted_", [False, True])
def test_cmrs_matches_definition_brute(seed, height, sorted_):
    """C oracle vs the literal entry-by-entry construction in pure Python."""
    A = synth.random_csr(23, 17, max_row=6, seed=seed, canonical=bool(seed % 2), duplicates=seed >= 4)
    sp, w, vo = oracle.csr_to_cmrs(A.row_ptr, A.col_ind, A.val, A.cols, height=height, sorted_=sorted_)
    coo = brute.coo_from_csr(A.row_ptr, A.col_ind, A.val)
    esp, ecol, eris, evals = brute.cmrs_by_definition(A.rows, height, coo, sorted_=sorted_)
    col, ris = _unpack(w, oracle.bits_for_height(height))
    assert sp.tolist() == esp
    assert col.tolist() == ecol
    assert ris.tolist() == eris
    assert vo.tolist() == [float(a) for a in evals]


# ------------------------------------------------------------ round trips
@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("height", [1, 2, 3, 5, 8, 16, 32])
def test_round_trip_unsorted_any_csr(seed, height):
    """to_csr(from_csr(A)) == A bit for bit for any valid CRS in unsorted mode
    (shuffled columns, duplicates, explicit zeros included)."""
    A = synth.random_csr(37, 29, max_row=9, seed=seed, canonical=seed % 2 == 0, duplicates=seed % 3 == 0,
                         explicit_zeros=True)
    sp, w, vo = oracle.csr_to_cmrs(A.row_ptr, A.col_ind, A.val, A.cols, height=height)
    rp, ci, v = oracle.cmrs_to_csr(sp, w, vo, A.rows, height)
    assert np.array_equal(rp, A.row_ptr) and np.array_equal(ci, A.col_ind)
    assert np.array_equal(v.view(np.uint64), A.val.view(np.uint64))


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("height", [1, 2, 4, 7, 8, 32])
def test_round_trip_sorted_canonical(seed, height):
    A = synth.random_csr(41, 33, max_row=10, seed=seed, explicit_zeros=True)
    sp, w, vo = oracle.csr_to_cmrs(A.row_ptr, A.col_ind, A.val, A.cols, height=height, sorted_=True)
    rp, ci, v = oracle.cmrs_to_csr(sp, w, vo, A.rows, height)
    assert np.array_equal(rp, A.row_ptr) and np.array_equal(ci, A.col_ind)
    assert np.array_equal(v.view(np.uint64), A.val.view(np.uint64))


def test_sorted_strip_invariants():
    A = synth.poisson_rows(4096, mean=6, seed=1)
    h = 8
    sp, w, vo = oracle.csr_to_cmrs(A.row_ptr, A.col_ind, A.val, A.cols, height=h, sorted_=True)
    col, ris = _unpack(w, oracle.bits_for_height(h))
    key = col * 64 + ris
    for s in range(len(sp) - 1):
        seg = key[sp[s]:sp[s + 1]]
        assert np.all(np.diff(seg) >= 0)
    # the multiset of (row, col, val) is unchanged
    strip_of = np.repeat(np.arange(len(sp) - 1), np.diff(sp))
    rows = strip_of * h + ris
    a = sorted(zip(rows.tolist(), col.tolist(), vo.tolist()))
    crow = np.repeat(np.arange(A.rows), np.diff(A.row_ptr))
    b = sorted(zip(crow.tolist(), A.col_ind.tolist(), A.val.tolist()))
    assert a == b


def test_cmrs_to_csr_rejects_bad_row():
    # strip 0 of a 3-row matrix with height 4 cannot hold row 3
    sp = np.array([0, 1], np.int32)
    w = np.array([(0 << 4) | 3], np.uint32)
    with pytest.raises(ValueError):
        oracle.cmrs_to_csr(sp, w, np.ones(1), 3, 4)


def test_csr_to_cmrs_rejects_bad_column():
    with pytest.raises(ValueError):
        oracle.csr_to_cmrs(np.array([0, 1], np.int32), np.array([5], np.int32), np.ones(1), 3, height=2)


# ------------------------------------------------------------ SpMV pins
@pytest.mark.parametrize("seed", range(10))
def test_spmv_integer_values_exact(seed):
    """Small integers: every partial sum is exact, so any correct summation
    order gives the same bits as the dense brute force."""
    A = synth.random_csr(30, 25, max_row=12, seed=seed, int_values=True, duplicates=seed % 2 == 1)
    x = np.random.default_rng(seed).integers(-5, 6, A.cols).astype(np.float64)
    y = oracle.csr_spmv(A.row_ptr, A.col_ind, A.val, x)
    dense = brute.dense_from_coo(A.rows, A.cols, brute.coo_from_csr(A.row_ptr, A.col_ind, A.val))
    assert y.tolist() == brute.dense_matvec(dense, x.tolist())


@pytest.mark.parametrize("seed", range(10))
def test_spmv_within_gamma_k_of_exact(seed):
    """|y - y_exact|_i <= gamma_{k_i} (|A||x|)_i (Higham, recursive summation),
    with y_exact in rational arithmetic.  A dropped term, a wrong sign or a
    wrong index would break this by O(1), not by rounding."""
    A = synth.random_csr(25, 40, max_row=15, seed=100 + seed)
    x = np.random.default_rng(seed).standard_normal(A.cols)
    y = oracle.csr_spmv(A.row_ptr, A.col_ind, A.val, x)
    ex = brute.exact_matvec(A.rows, brute.coo_from_csr(A.row_ptr, A.col_ind, A.val), x.tolist())
    absmv = oracle.csr_absmv(A.row_ptr, A.col_ind, A.val, x)
    k = np.diff(A.row_ptr)
    u = Fraction(1, 2**53)
    for i in range(A.rows):
        ki = int(k[i])
        gamma = ki * u / (1 - ki * u) if ki else Fraction(0)
        err = abs(Fraction(float(y[i])) - ex[i])
        assert err <= gamma * Fraction(float(absmv[i])) * (1 + Fraction(1, 2**40))
        if ki == 0:
            assert y[i] == 0.0 and not np.signbit(y[i])


def test_dense_as_sparse_matches_dense():
    A = synth.dense_as_sparse(64, seed=2, m=48)
    x = synth.uniform_vector(48, seed=5)
    y = oracle.csr_spmv(A.row_ptr, A.col_ind, A.val, x)
    d = oracle.csr_to_dense(A.row_ptr, A.col_ind, A.val, A.cols)
    # same entries in the same order: identical bits
    assert np.array_equal(y, oracle.dense_matvec(d, x))
    ex = brute.exact_matvec(A.rows, brute.coo_from_csr(A.row_ptr, A.col_ind, A.val), x.tolist())
    bound = oracle.spmv_bound(A.row_ptr, A.col_ind, A.val, x, 2.0**-53, factor=1.0)
    assert all(abs(float(Fraction(float(y[i])) - ex[i])) <= bound[i] for i in range(A.rows))


def test_permutation_and_identity_exact():
    P = synth.permutation(1000, seed=7)
    x = synth.normal_vector(1000, seed=8)
    y = oracle.csr_spmv(P.row_ptr, P.col_ind, P.val, x)
    assert np.array_equal(y, x[P.col_ind])
    E = synth.identity(500)
    assert np.array_equal(oracle.csr_spmv(E.row_ptr, E.col_ind, E.val, x[:500]), x[:500])


def test_laplacian_ones_closed_form():
    """5-point Laplacian times ones: 4 - (number of neighbours) = 0 inside,
    1 on edges, 2 at the four corners; 64x64 grid has 5*64^2 - 4*64 entries."""
    A = synth.laplace2d(64)
    assert A.nnz == 5 * 64 * 64 - 4 * 64 == 20224
    y = oracle.csr_spmv(A.row_ptr, A.col_ind, A.val, np.ones(A.cols))
    g = y.reshape(64, 64)
    assert g[1:-1, 1:-1].max() == 0 and g[1:-1, 1:-1].min() == 0
    assert (g[0, 1:-1] == 1).all() and (g[-1, 1:-1] == 1).all() and (g[1:-1, 0] == 1).all() and (g[1:-1, -1] == 1).all()
    assert g[0, 0] == g[0, -1] == g[-1, 0] == g[-1, -1] == 2


def test_negative_zero_products_give_positive_zero():
    """The sum starts from +0.0 (Algorithm 1 zero-fills its buffer): a row whose
    products are all -0.0 yields +0.0."""
    rp = np.array([0, 2], np.int32)
    ci = np.array([0, 1], np.int32)
    v = np.array([-0.0, 0.0])
    y = oracle.csr_spmv(rp, ci, v, np.array([1.0, -1.0]))
    assert y[0] == 0.0 and not np.signbit(y[0])


# ------------------------------------------------------------ |A||x| pins
def test_absmv_of_M_with_signed_x(paper):
    """|M||x| for the printed M and a signed x equals M|x| (all entries of M are
    positive), here [9, 26, 45, 98, 50]; the plain product with the same signed
    x differs, so an absolute value dropped on either factor fails."""
    rp, ci, v = _crs_M(paper)
    xs = np.array([1.0, -2.0, 3.0, -4.0, 5.0])
    a = oracle.csr_absmv(rp, ci, v, xs)
    assert a.tolist() == [9.0, 26.0, 45.0, 98.0, 50.0]
    assert oracle.csr_absmv(rp, ci, -v, xs).tolist() == a.tolist()
    assert not np.array_equal(oracle.csr_spmv(rp, ci, v, xs), a)


@pytest.mark.parametrize("seed", range(8))
def test_absmv_integer_exact(seed):
    """Small signed integers: every partial sum of |a||x| is exact, so the
    oracle must equal the rational definition bit for bit (duplicates, empty
    rows and explicit zeros included)."""
    A = synth.random_csr(40, 30, max_row=14, seed=300 + seed, int_values=True, duplicates=True,
                         explicit_zeros=seed % 2 == 0)
    x = np.random.default_rng(seed).integers(-6, 7, A.cols).astype(np.float64)
    a = oracle.csr_absmv(A.row_ptr, A.col_ind, A.val, x)
    ex = brute.exact_absmv(A.rows, brute.coo_from_csr(A.row_ptr, A.col_ind, A.val), x.tolist())
    assert [Fraction(float(t)) for t in a] == ex
    k = np.diff(A.row_ptr)
    assert np.all(a[k == 0] == 0.0)


@pytest.mark.parametrize("seed", range(8))
def test_absmv_within_gamma_k_of_exact(seed):
    """Random real data: all terms are non-negative, so recursive summation of
    k_i rounded products is within gamma_{k_i} of the exact sum, relatively.
    A row counted twice, a wrong range end or a missing term is off by O(1)."""
    A = synth.random_csr(30, 50, max_row=20, seed=400 + seed, duplicates=seed % 2 == 1, explicit_zeros=True)
    x = np.random.default_rng(seed).standard_normal(A.cols)
    a = oracle.csr_absmv(A.row_ptr, A.col_ind, A.val, x)
    ex = brute.exact_absmv(A.rows, brute.coo_from_csr(A.row_ptr, A.col_ind, A.val), x.tolist())
    k = np.diff(A.row_ptr)
    u = Fraction(1, 2**53)
    for i in range(A.rows):
        ki = int(k[i])
        gamma = ki * u / (1 - ki * u) if ki else Fraction(0)
        assert abs(Fraction(float(a[i])) - ex[i]) <= gamma * ex[i]
        assert a[i] >= 0.0


def test_absmv_dominates_product():
    """|y_i| <= (|A||x|)_i for the exact product, with equality for rows whose
    products share one sign (here: non-negative data)."""
    A = synth.random_csr(50, 40, max_row=12, seed=9)
    x = synth.normal_vector(A.cols, seed=10)
    coo = brute.coo_from_csr(A.row_ptr, A.col_ind, A.val)
    ex_y = brute.exact_matvec(A.rows, coo, x.tolist())
    ex_a = brute.exact_absmv(A.rows, coo, x.tolist())
    assert all(abs(yi) <= ai for yi, ai in zip(ex_y, ex_a))
    pos = np.abs(A.val)
    xp = np.abs(x)
    assert np.array_equal(oracle.csr_absmv(A.row_ptr, A.col_ind, A.val, x),
                          oracle.csr_spmv(A.row_ptr, A.col_ind, pos, xp))


# ------------------------------------------------------------ precision helpers
def test_bf16_rounding_rne():
    # 1 + 2^-8 is halfway between bf16 neighbours 1 and 1 + 2^-7: ties to even -> 1
    vals = np.array([1.0, 1.0 + 2**-8, 1.0 + 3 * 2**-8, -2.5, 1.0 + 2**-8 + 2**-30, 3.0e-39, 0.0])
    b = synth.round_to_bf16_bits(vals)
    back = synth.bf16_bits_to_f64(b)
    assert back[0] == 1.0
    assert back[1] == 1.0
    assert back[2] == 1.0 + 4 * 2**-8
    assert back[3] == -2.5
    assert back[4] == 1.0 + 2**-7
    assert back[6] == 0.0
    # subnormal range: quantum 2^-133
    assert back[5] == np.rint(3.0e-39 / 2.0**-133) * 2.0**-133
    rng = np.random.default_rng(0)
    x = rng.standard_normal(10000)
    r = synth.bf16_bits_to_f64(synth.round_to_bf16_bits(x))
    assert np.all(np.abs(r - x) <= 2.0**-8 * np.abs(x))  # unit roundoff of 8 significant bits
