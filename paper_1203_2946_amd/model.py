"""Byte, flop and coalescing models used to report CMRS measurements.

Pure arithmetic on sizes; no device code.  Paper: Koza et al., arXiv:1203.2946.

* ``beta_plus`` / ``beta_minus``: bytes an SpMV must move when the input
  vector is fully cached (+) or read once per nonzero (-), Eq. (6.1),
  generalised to rows != cols and to separate x / y element sizes:
      beta+ = (s_v + s_i) nnz + s_i (strips + 1) + s_x cols + s_y rows
      beta- = beta+ + s_x (nnz - cols)
  (the paper counts s_i * strips for the strip pointers and 2 s_v rows for x
  and y of a square matrix).
* ``flops``: 2 nnz - rows, Sec. 6.4.
* ``f_model`` / ``a_model``: Eq. (5.1) and Eq. (5.2), the ratio of bytes
  transferred to bytes requested when a wave reads h*mu contiguous b-byte
  items in lambda-byte segments, and the predicted CMRS / vector-kernel
  speedup.
* ``expected_segments``: Appendix A, S = 1 + (n - b) / lambda.
"""
from __future__ import annotations

S_I = 4  # bytes of one packed column word / strip pointer


def dtype_size(name: str) -> int:
    return {"f64": 8, "f32": 4, "bf16": 2}[name]


def beta_plus(nnz: int, rows: int, cols: int, strips: int, s_v: int, s_x: int, s_y: int) -> int:
    return (s_v + S_I) * nnz + S_I * (strips + 1) + s_x * cols + s_y * rows


def beta_minus(nnz: int, rows: int, cols: int, strips: int, s_v: int, s_x: int, s_y: int) -> int:
    return beta_plus(nnz, rows, cols, strips, s_v, s_x, s_y) + s_x * (nnz - cols)


def paper_beta(nnz: int, rows: int, strips: int, s_v: int):
    """Eq. (6.1) exactly as printed (square matrix, x and y of size s_v)."""
    bm = (2 * s_v + S_I) * nnz + S_I * strips + s_v * rows
    bp = (s_v + S_I) * nnz + S_I * strips + 2 * s_v * rows
    return bm, bp


def flops(nnz: int, rows: int) -> int:
    return 2 * nnz - rows


def from_csr_bytes(nnz: int, rows: int, strips: int, s_v: int, moves_val: bool = True) -> int:
    """Reads RowPtr, ColInd (and Val), writes StripPtr, words (and Val)."""
    return S_I * (rows + 1) + S_I * nnz * 2 + S_I * (strips + 1) + (2 * s_v * nnz if moves_val else 0)


def to_csr_bytes(nnz: int, rows: int, strips: int, s_v: int) -> int:
    """Reads StripPtr, words, Val; writes RowPtr, ColInd, Val."""
    return S_I * (strips + 1) + S_I * nnz * 2 + 2 * s_v * nnz + S_I * (rows + 1)


def f_model(h: float, mu: float, lam: float = 128.0, b: float = 4.0) -> float:
    """Eq. (5.1): f(h, mu) = 1 + (lambda - b) / (h mu b)."""
    return 1.0 + (lam - b) / (h * mu * b)


def a_model(h: float, mu: float, lam: float = 128.0, b: float = 4.0) -> float:
    """Eq. (5.2), exact ratio f(1, mu) / f(h, mu)."""
    return f_model(1, mu, lam, b) / f_model(h, mu, lam, b)


def a_model_approx(h: float, mu: float, lam: float = 128.0, b: float = 4.0) -> float:
    """Eq. (5.2), the approximation 1 + (h - 1) / (1 + h mu b / lambda)."""
    return 1.0 + (h - 1.0) / (1.0 + h * mu * b / lam)


def expected_segments(n: int, lam: int, b: int) -> float:
    """Appendix A: mean number of lambda-byte segments touched by an n-byte,
    b-aligned chunk placed uniformly at random: 1 + (n - b) / lambda."""
    return 1.0 + (n - b) / lam
