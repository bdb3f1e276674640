"""Reference of the learned configuration selector (TEST INFRASTRUCTURE ONLY).

Only ``tests/`` and ``bench.py``'s CPU leg may use it.  The selector turns the
paper's brute-force tuning of the strip height and kernel options over
measured times (Sec. 6.3, with the tuning headroom of Sec. 6.8) into a
prediction; this module holds, written independently of the HIP kernels:

  * ``features``: the 40 structure features, by their definitions, with
    Python integers for every bin decision;
  * ``mlp_forward`` / ``mlp_backward``: the 40 -> 64 -> 64 -> 24 ReLU network
    and its gradient of the mean squared error, in fp64 numpy;
  * ``adam``: one Adam step (Kingma and Ba, Algorithm 1), fp64.

Pins (CPU tests): feature bins of hand-checked matrices, gradients against
central finite differences, Adam's first step against its closed form.
"""
from __future__ import annotations

import numpy as np

N_FEATURES, HIDDEN, N_CLASSES = 40, 64, 24
ROW_BINS, DIST_BINS = 20, 16
SHAPES = ((N_FEATURES, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, N_CLASSES))


def row_len_bin(length: int) -> int:
    """Half-octave bin of a row length: 0 for an empty row; with
    p = floor(log2 len), 1 + 2p for len < 1.5 * 2^p, else 2 + 2p; capped at 19."""
    if length <= 0:
        return 0
    p = int(length).bit_length() - 1
    b = 1 + 2 * p + (1 if 2 * length >= 3 * (1 << p) else 0)
    return min(b, ROW_BINS - 1)


def dist_bin(d: int) -> int:
    """0 for distance 0, b for a distance in [2^(b-1), 2^b), capped at 15."""
    if d <= 0:
        return 0
    return min(int(d).bit_length(), DIST_BINS - 1)


def feature_counts(row_ptr, col_ind, cols):
    """Integer histograms (row-length bins, distance bins) and the maximum
    row length.  An entry (r, c) has distance |c - floor(r * cols / rows)|, the
    product taken in binary64 as the features define it."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_ind = np.asarray(col_ind, dtype=np.int64)
    rows = row_ptr.size - 1
    lens = np.diff(row_ptr)
    rh = np.zeros(ROW_BINS, np.int64)
    for ln, cnt in zip(*np.unique(lens, return_counts=True)):
        rh[row_len_bin(int(ln))] += int(cnt)
    dh = np.zeros(DIST_BINS, np.int64)
    if col_ind.size:
        scale = float(cols) / rows
        r = np.repeat(np.arange(rows, dtype=np.int64), lens)
        center = np.floor(r.astype(np.float64) * scale).astype(np.int64)
        d = np.abs(col_ind - center)
        for dv, cnt in zip(*np.unique(d, return_counts=True)):
            dh[dist_bin(int(dv))] += int(cnt)
    return rh, dh, int(lens.max()) if rows else 0


def features(row_ptr, col_ind, cols) -> np.ndarray:
    """The 40 features in float32: row-length fractions, distance fractions,
    log2(rows)/22, log2(nnz+1)/26, log2(nnz/rows+1)/14, log2(max len+1)/14."""
    rows = len(row_ptr) - 1
    nnz = len(col_ind)
    rh, dh, mx = feature_counts(row_ptr, col_ind, cols)
    f = np.zeros(N_FEATURES, np.float32)
    f32 = np.float32
    if rows:
        f[:ROW_BINS] = rh.astype(f32) / f32(rows)
    if nnz:
        f[ROW_BINS:ROW_BINS + DIST_BINS] = dh.astype(f32) / f32(nnz)
    mean = f32(nnz) / f32(rows) if rows else f32(0)
    f[36] = np.log2(f32(max(rows, 1))) / f32(22)
    f[37] = np.log2(f32(nnz) + f32(1)) / f32(26)
    f[38] = np.log2(mean + f32(1)) / f32(14)
    f[39] = np.log2(f32(mx) + f32(1)) / f32(14)
    return f


def unpack(params):
    """Split the packed vector into [(W, b)] with W of shape (nin, nout)."""
    params = np.asarray(params, dtype=np.float64)
    out, o = [], 0
    for nin, nout in SHAPES:
        W = params[o:o + nin * nout].reshape(nin, nout)
        o += nin * nout
        b = params[o:o + nout]
        o += nout
        out.append((W, b))
    assert o == params.size
    return out


def mlp_forward(X, params):
    """Activations (H1, H2, Y): H1 = relu(X W1 + b1), H2 = relu(H1 W2 + b2),
    Y = H2 W3 + b3."""
    (W1, b1), (W2, b2), (W3, b3) = unpack(params)
    X = np.asarray(X, dtype=np.float64)
    H1 = np.maximum(X @ W1 + b1, 0.0)
    H2 = np.maximum(H1 @ W2 + b2, 0.0)
    Y = H2 @ W3 + b3
    return H1, H2, Y


def mse(X, T, params) -> float:
    Y = mlp_forward(X, params)[2]
    return float(np.mean((Y - np.asarray(T, np.float64)) ** 2))


def mlp_backward(X, T, params):
    """Gradient of mse() with respect to the packed parameters (chain rule
    through the three layers, ReLU derivative taken as 0 at 0)."""
    (W1, b1), (W2, b2), (W3, b3) = unpack(params)
    X = np.asarray(X, dtype=np.float64)
    H1, H2, Y = mlp_forward(X, params)
    dY = 2.0 * (Y - np.asarray(T, np.float64)) / Y.size
    gW3, gb3 = H2.T @ dY, dY.sum(0)
    dH2 = (dY @ W3.T) * (H2 > 0)
    gW2, gb2 = H1.T @ dH2, dH2.sum(0)
    dH1 = (dH2 @ W2.T) * (H1 > 0)
    gW1, gb1 = X.T @ dH1, dH1.sum(0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3]), dY, dH2, dH1


def adam(p, g, m, v, lr, b1, b2, eps, step):
    """One bias-corrected Adam step; returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
