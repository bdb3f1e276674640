"""Pins of the selector reference (features, MLP, Adam) on the CPU.

The selector learns the outcome of the paper's brute-force search over strip
heights and kernel options (Sec. 6.3, 6.8).  Its reference in
oracle/selector_ref.py is pinned here against hand-counted features, central
finite differences of the loss and Adam's closed-form first step.
"""
import math
import os

import numpy as np
import pytest

from oracle import selector_ref as R


def test_row_len_bins_by_hand():
    # Half octaves: [2^p, 1.5*2^p) -> 1 + 2p, [1.5*2^p, 2^(p+1)) -> 2 + 2p.
    expect = {0: 0, 1: 1, 2: 3, 3: 4, 4: 5, 5: 5, 6: 6, 7: 6, 8: 7, 11: 7, 12: 8, 15: 8, 16: 9,
              256: 17, 383: 17, 384: 18, 511: 18, 512: 19, 10 ** 6: 19}
    for ln, b in expect.items():
        assert R.row_len_bin(ln) == b, ln


def test_row_len_bins_against_real_log():
    for ln in range(1, 600):
        p = math.floor(math.log2(ln))
        half = 1 if ln / 2 ** p >= 1.5 else 0
        assert R.row_len_bin(ln) == min(19, 1 + 2 * p + half)


def test_dist_bins_by_hand():
    expect = {0: 0, 1: 1, 2: 2, 3: 2, 4: 3, 7: 3, 8: 4, 2 ** 13: 14, 2 ** 14 - 1: 14, 2 ** 14: 15, 10 ** 9: 15}
    for d, b in expect.items():
        assert R.dist_bin(d) == b, d


def test_features_hand_counted():
    # 4 x 8 (column scale 2): row 0 {0, 3}, row 1 empty, row 2 {4, 5, 6, 7},
    # row 3 {0}.  Centres 0, 2, 4, 6; distances 0,3 | - | 0,1,2,3 | 6.
    row_ptr = [0, 2, 2, 6, 7]
    col_ind = [0, 3, 4, 5, 6, 7, 0]
    f = R.features(row_ptr, col_ind, 8)
    rh = np.zeros(20)
    rh[[3, 0, 5, 1]] = 1  # lengths 2, 0, 4, 1
    dh = np.zeros(16)
    dh[0], dh[1], dh[2], dh[3] = 2, 1, 3, 1
    np.testing.assert_array_equal(f[:20], (rh / 4).astype(np.float32))
    np.testing.assert_array_equal(f[20:36], (dh / 7).astype(np.float32))
    np.testing.assert_allclose(f[36:], [2 / 22, 3 / 26, math.log2(2.75) / 14, math.log2(5) / 14], rtol=1e-6)


def test_features_identity_and_empty():
    n = 100
    f = R.features(np.arange(n + 1), np.arange(n), n)
    assert f[1] == 1.0 and f[:20].sum() == 1.0
    assert f[20] == 1.0 and f[20:36].sum() == 1.0
    np.testing.assert_allclose(f[36:], [math.log2(100) / 22, math.log2(101) / 26, 1 / 14, 1 / 14], rtol=1e-6)
    g = R.features(np.zeros(11, np.int64), np.zeros(0, np.int64), 10)
    assert g[0] == 1.0 and g[20:36].sum() == 0.0 and g[37] == 0.0 and g[39] == 0.0


def test_feature_fractions_sum_to_one():
    import synth
    for A in (synth.poisson_rows(3000, 9.0, 5), synth.random_csr(500, 700, 40, seed=2)):
        f = R.features(A.row_ptr, A.col_ind, A.cols)
        assert abs(float(f[:20].sum()) - 1.0) < 1e-5
        assert abs(float(f[20:36].sum()) - 1.0) < 1e-5


def _params(seed, scale=0.3):
    g = np.random.default_rng(seed)
    n = sum(a * b + b for a, b in R.SHAPES)
    assert n == 8344
    return g.normal(0, scale, n)


def test_forward_layer_order_and_layout():
    # W1 = [I | 0], W2 = I, W3 = first 24 columns of I, zero biases: Y equals
    # relu(X)[:, :24]; a transposed or misplaced block breaks it.
    W1 = np.zeros((40, 64))
    W1[np.arange(40), np.arange(40)] = 1
    W3 = np.zeros((64, 24))
    W3[np.arange(24), np.arange(24)] = 1
    p = np.concatenate([W1.ravel(), np.zeros(64), np.eye(64).ravel(), np.zeros(64), W3.ravel(), np.zeros(24)])
    X = np.random.default_rng(0).normal(size=(7, 40))
    Y = R.mlp_forward(X, p)[2]
    np.testing.assert_array_equal(Y, np.maximum(X, 0)[:, :24])
    # A bias on the last layer shifts every row.
    p[-24:] = np.arange(24)
    np.testing.assert_array_equal(R.mlp_forward(X, p)[2], np.maximum(X, 0)[:, :24] + np.arange(24))


def test_gradient_finite_differences():
    g = np.random.default_rng(1)
    X = g.normal(size=(6, 40))
    T = g.normal(size=(6, 24))
    p = _params(2)
    grad = R.mlp_backward(X, T, p)[0]
    idx = np.concatenate([g.choice(8344, 150, replace=False), np.arange(2560, 2624), np.arange(8320, 8344)])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (R.mse(X, T, p + e) - R.mse(X, T, p - e)) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * (1 + abs(grad[i])), i


def test_adam_first_step_closed_form():
    g = np.random.default_rng(3)
    p = g.normal(size=50)
    gr = g.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    lr, eps = 1e-2, 1e-8
    p1, m1, v1 = R.adam(p, gr, m, v, lr, 0.9, 0.999, eps, 1)
    # After one step the bias-corrected moments are g and g^2 exactly.
    np.testing.assert_allclose(p1, p - lr * gr / (np.abs(gr) + eps), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m1, 0.1 * gr, rtol=1e-15)
    np.testing.assert_allclose(v1, 0.001 * gr * gr, rtol=1e-12)
    # A zero gradient from zero moments leaves the parameters alone.
    p2, _, _ = R.adam(p, np.zeros(50), m, v, lr, 0.9, 0.999, eps, 1)
    np.testing.assert_array_equal(p2, p)


DATA = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1203_2946_amd", "data")


@pytest.mark.skipif(not os.path.exists(os.path.join(DATA, "selector_weights.npz")), reason="no trained weights")
def test_committed_weights_regret_fp64():
    """The committed weights, run by the fp64 reference on the held-out part
    of the committed timing set, pick classes within 5 % (geometric mean) of
    the measured best, and beat the best single fixed class."""
    d = np.load(os.path.join(DATA, "selector_timings.npz"), allow_pickle=False)
    w = np.load(os.path.join(DATA, "selector_weights.npz"), allow_pickle=False)
    X, t = d["features"], d["times_ms"]
    te = np.arange(int(w["n_train"]), X.shape[0])
    Y = R.mlp_forward(X[te].astype(np.float64), w["params"].astype(np.float64))[2]
    choice = Y.argmin(axis=1)
    best = t[te].min(axis=1)

    def gm(c):
        return float(np.exp(np.mean(np.log(t[te][np.arange(te.size), c] / best)))) - 1

    r = gm(choice)
    fixed = min(gm(np.full(te.size, c)) for c in range(24))
    assert r <= 0.05, r
    assert r < fixed, (r, fixed)
