"""Seeded synthetic sparse matrices in canonical CSR form (int32 indices).

Every generator is deterministic in its arguments (numpy ``default_rng``, PCG64)
and returns a :class:`Csr`.  "Canonical" means: ``row_ptr[0] == 0``, columns
strictly increasing inside each row, no duplicate entries.  ``random_csr`` can
also produce non-canonical input (unsorted columns, duplicates, explicit zeros)
for the conversion tests.

Workload families (the paper's test set, UF SMC, is not available, so these
stand in for it):
  * ``laplace2d``      2-D 5-point Laplacian (values 4 / -1), natural order
  * ``poisson_rows``   row lengths max(1, Poisson(mean)), distinct uniform
                       columns, N(0,1) values
  * ``zipf_clustered`` row lengths min(Zipf(a), kmax); round(0.7 k) distinct
                       columns drawn from the +-half_window band around the
                       diagonal, the rest distinct and uniform; U[-1,1] values
  * ``permutation``, ``identity``, ``dense_as_sparse`` (the paper's p7 and
    dense4 kinds of special matrices, at any size)
  * ``stencil27``, ``banded``, ``dense_blocks`` (batched / selector families)
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Csr:
    rows: int
    cols: int
    row_ptr: np.ndarray   # int32 [rows+1]
    col_ind: np.ndarray   # int32 [nnz]
    val: np.ndarray       # float64 [nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.col_ind.size)

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))


def _rng(seed):
    return np.random.default_rng(seed)


def _finish(rows, cols, lengths, col_ind, val, name):
    row_ptr = np.zeros(rows + 1, dtype=np.int64)
    np.cumsum(lengths, out=row_ptr[1:])
    assert row_ptr[-1] < 2**31
    return Csr(rows, cols, row_ptr.astype(np.int32), np.ascontiguousarray(col_ind, dtype=np.int32),
               np.ascontiguousarray(val, dtype=np.float64), name)


# ---------------------------------------------------------------- vectors
def uniform_vector(n: int, seed: int = 0, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return _rng(seed).uniform(lo, hi, n)


def normal_vector(n: int, seed: int = 0) -> np.ndarray:
    return _rng(seed).standard_normal(n)


# ---------------------------------------------------------------- precision
def round_to_f32(a: np.ndarray) -> np.ndarray:
    """fp64 -> fp32, round to nearest even (numpy cast)."""
    return np.asarray(a, dtype=np.float64).astype(np.float32)


def round_to_bf16_bits(a: np.ndarray) -> np.ndarray:
    """fp64 -> bfloat16 bit patterns (uint16), round to nearest even directly
    from fp64 (no intermediate fp32 rounding).  bfloat16 keeps 8 significant
    bits and the fp32 exponent range; below 2^-126 its quantum is 2^-133."""
    a = np.asarray(a, dtype=np.float64)
    m, e = np.frexp(a)                      # a = m * 2^e, 0.5 <= |m| < 1
    e = np.maximum(e, -125)
    ulp = np.ldexp(1.0, e - 8)
    r = np.rint(a / ulp) * ulp              # exact: power-of-two scaling, rint is RNE
    f = r.astype(np.float32)                # exact: r is representable in bf16 (subset of fp32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


def bf16_bits_to_f64(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------- families
def laplace2d(nx: int, ny: int | None = None) -> Csr:
    """5-point Laplacian on an nx*ny grid, row i = y*nx + x, diagonal 4,
    neighbours -1, columns ascending."""
    ny = nx if ny is None else ny
    n = nx * ny
    idx = np.arange(n, dtype=np.int64)
    gx, gy = idx % nx, idx // nx
    offs = [(-nx, gy > 0), (-1, gx > 0), (0, np.ones(n, bool)), (1, gx < nx - 1), (nx, gy < ny - 1)]
    cols = np.stack([idx + o for o, _ in offs], axis=1)
    mask = np.stack([m for _, m in offs], axis=1)
    vals = np.where(np.arange(5)[None, :] == 2, 4.0, -1.0) * np.ones((n, 5))
    lengths = mask.sum(axis=1)
    return _finish(n, n, lengths, cols[mask], vals[mask], f"laplace2d_{nx}x{ny}")


def _dedupe_rows(rows_of, cols, n, rng, redraw):
    """Make columns distinct inside each row.  ``rows_of`` is the row id of each
    entry (grouped by row).  Rows that contain a repeated column are redrawn by
    ``redraw(row) -> sorted distinct columns`` in increasing row order."""
    key = rows_of.astype(np.int64) * n + cols
    order = np.argsort(key, kind="stable")
    key = key[order]
    cols = cols[order]
    dup = np.nonzero(key[1:] == key[:-1])[0]
    if dup.size:
        bad_rows = np.unique(rows_of[order][dup + 1])
        starts = np.searchsorted(rows_of, bad_rows, side="left")
        ends = np.searchsorted(rows_of, bad_rows, side="right")
        for r, a, b in zip(bad_rows, starts, ends):
            cols[a:b] = redraw(int(r), b - a)
    return cols


def poisson_rows(n: int = 1 << 20, mean: float = 16.0, seed: int = 0) -> Csr:
    """Square n*n matrix; k_i = max(1, Poisson(mean)); k_i distinct columns
    uniform in [0, n), ascending; values N(0,1)."""
    rng = _rng(seed)
    k = np.maximum(1, rng.poisson(mean, n)).astype(np.int64)
    nnz = int(k.sum())
    rows_of = np.repeat(np.arange(n, dtype=np.int64), k)
    cols = rng.integers(0, n, nnz, dtype=np.int64)

    def redraw(r, m):
        return np.sort(rng.choice(n, size=m, replace=False))

    cols = _dedupe_rows(rows_of, cols, n, rng, redraw)
    val = rng.standard_normal(nnz)
    return _finish(n, n, k, cols, val, f"poisson{mean:g}_n{n}_s{seed}")


def zipf_clustered(n: int = 2_000_000, a: float = 2.0, kmax: int = 10_000, near_frac: float = 0.7,
                   half_window: int = 512, seed: int = 0) -> Csr:
    """Square n*n matrix with skewed rows.
    k_i = min(Zipf(a), kmax) (numpy's zipf, >= 1);
    k_near = round-half-up(near_frac * k_i), capped at the band size, columns
    drawn distinct from [i-half_window, i+half_window] intersected with [0, n);
    the other k_i - k_near columns distinct and uniform over [0, n) among the
    columns not yet taken; columns ascending; values U[-1,1]."""
    rng = _rng(seed)
    k = np.minimum(rng.zipf(a, n), kmax).astype(np.int64)
    i = np.arange(n, dtype=np.int64)
    lo = np.maximum(0, i - half_window)
    hi = np.minimum(n - 1, i + half_window)
    wsize = hi - lo + 1
    tenths = int(round(near_frac * 10))
    k_near = np.minimum((tenths * k + 5) // 10, wsize)
    k_far = k - k_near
    nnz = int(k.sum())
    rows_of = np.repeat(i, k)
    # entry t of row i is "near" for t < k_near[i]
    starts = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(k, out=starts[1:])
    t = np.arange(nnz, dtype=np.int64) - starts[rows_of]
    is_near = t < k_near[rows_of]
    cols = np.empty(nnz, dtype=np.int64)
    nn = int(is_near.sum())
    r_near = rows_of[is_near]
    cols[is_near] = lo[r_near] + rng.integers(0, wsize[r_near], nn, dtype=np.int64)
    cols[~is_near] = rng.integers(0, n, nnz - nn, dtype=np.int64)

    def redraw(r, m):
        kn = int(k_near[r])
        near = lo[r] + rng.choice(int(wsize[r]), size=kn, replace=False)
        taken = set(near.tolist())
        far = []
        while len(far) < m - kn:
            need = m - kn - len(far)
            for c in rng.integers(0, n, need).tolist():
                if c not in taken:
                    taken.add(c)
                    far.append(c)
        return np.sort(np.concatenate([near, np.asarray(far, dtype=np.int64)]))

    cols = _dedupe_rows(rows_of, cols, n, rng, redraw)
    val = rng.uniform(-1.0, 1.0, nnz)
    return _finish(n, n, k, cols, val, f"zipf{a:g}_n{n}_s{seed}")


def permutation(n: int, seed: int = 0) -> Csr:
    """Random n*n permutation matrix: row i has a single 1 in column p(i)."""
    p = _rng(seed).permutation(n)
    return _finish(n, n, np.ones(n, np.int64), p, np.ones(n), f"perm_n{n}_s{seed}")


def identity(n: int) -> Csr:
    return _finish(n, n, np.ones(n, np.int64), np.arange(n), np.ones(n), f"eye_n{n}")


def dense_as_sparse(n: int, seed: int = 0, m: int | None = None) -> Csr:
    """Dense n*m matrix (all entries stored), values U[-1,1]."""
    m = n if m is None else m
    rng = _rng(seed)
    cols = np.tile(np.arange(m, dtype=np.int64), n)
    return _finish(n, m, np.full(n, m, np.int64), cols, rng.uniform(-1, 1, n * m), f"dense_{n}x{m}_s{seed}")


def random_csr(rows: int, cols: int, max_row: int = 8, seed: int = 0, *, canonical: bool = True,
               duplicates: bool = False, explicit_zeros: bool = False, int_values: bool = False,
               empty_row_frac: float = 0.2) -> Csr:
    """Small random CSR for conversion / brute-force tests.
    Row lengths uniform in [0, max_row] with a fraction of rows forced empty.
    canonical=False shuffles columns inside rows; duplicates=True repeats some
    (row, col) pairs; explicit_zeros=True stores some 0.0 values;
    int_values=True draws small integers (exact in any summation order)."""
    rng = _rng(seed)
    k = rng.integers(0, max_row + 1, rows)
    k[rng.random(rows) < empty_row_frac] = 0
    k = np.minimum(k, cols if not duplicates else 4 * cols)
    col_list = []
    for i in range(rows):
        if duplicates and k[i] > 1:
            c = rng.integers(0, cols, k[i])
        else:
            c = rng.choice(cols, size=min(int(k[i]), cols), replace=False)
            k[i] = c.size
        c = np.sort(c)
        if not canonical:
            rng.shuffle(c)
        col_list.append(c)
    col = np.concatenate(col_list) if col_list else np.zeros(0, np.int64)
    nnz = col.size
    if int_values:
        val = rng.integers(-8, 9, nnz).astype(np.float64)
    else:
        val = rng.standard_normal(nnz)
    if explicit_zeros and nnz:
        val[rng.random(nnz) < 0.2] = 0.0
    return _finish(rows, cols, k, col, val, f"rand_{rows}x{cols}_s{seed}")


def stencil27(nx: int, ny: int, nz: int, seed: int = 0) -> Csr:
    """3-D 27-point stencil on nx*ny*nz, natural order, values N(0,1)."""
    n = nx * ny * nz
    idx = np.arange(n, dtype=np.int64)
    gx, gy, gz = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    cols, masks = [], []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                ok = (gx + dx >= 0) & (gx + dx < nx) & (gy + dy >= 0) & (gy + dy < ny) & (gz + dz >= 0) & (gz + dz < nz)
                cols.append(idx + dx + dy * nx + dz * nx * ny)
                masks.append(ok)
    cols = np.stack(cols, axis=1)
    mask = np.stack(masks, axis=1)
    lengths = mask.sum(axis=1)
    val = _rng(seed).standard_normal(int(lengths.sum()))
    return _finish(n, n, lengths, cols[mask], val, f"stencil27_{nx}x{ny}x{nz}_s{seed}")


def banded(n: int, bandwidth: int, fill: float = 0.6, seed: int = 0) -> Csr:
    """n*n band matrix: each entry with |i-j| <= bandwidth is stored with
    probability ``fill`` (the diagonal always), values N(0,1)."""
    rng = _rng(seed)
    offs = np.arange(-bandwidth, bandwidth + 1, dtype=np.int64)
    i = np.arange(n, dtype=np.int64)[:, None]
    cols = i + offs[None, :]
    mask = (cols >= 0) & (cols < n) & ((rng.random(cols.shape) < fill) | (offs[None, :] == 0))
    lengths = mask.sum(axis=1)
    val = rng.standard_normal(int(lengths.sum()))
    return _finish(n, n, lengths, cols[mask], val, f"banded{bandwidth}_n{n}_s{seed}")


def dense_blocks(n: int, block: int = 32, blocks_per_row: int = 2, seed: int = 0) -> Csr:
    """Block-sparse n*n matrix made of dense block*block tiles: each block row
    holds the diagonal tile plus ``blocks_per_row - 1`` distinct random tiles."""
    rng = _rng(seed)
    nb = -(-n // block)
    col_blocks = []
    for b in range(nb):
        others = rng.choice(nb, size=min(nb, blocks_per_row), replace=False).tolist()
        cb = sorted(set([b] + others))[:max(1, blocks_per_row)]
        if b not in cb:
            cb = sorted(set(cb[:-1] + [b]))
        col_blocks.append(cb)
    lengths = np.zeros(n, np.int64)
    cols = []
    for i in range(n):
        cb = col_blocks[i // block]
        c = np.concatenate([np.arange(b * block, min(n, (b + 1) * block)) for b in cb])
        lengths[i] = c.size
        cols.append(c)
    col = np.concatenate(cols)
    return _finish(n, n, lengths, col, rng.standard_normal(col.size), f"dblock{block}_n{n}_s{seed}")
