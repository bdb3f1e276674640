"""CMRS oracle: a plain CPU reference of what the CMRS hot path computes.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU library never
calls it and shares no code with it.

The arithmetic lives in ``cmrs_oracle.c`` (plain C, fp64, built with
``-ffp-contract=off``); this module only marshals numpy arrays through ctypes.
``brute.py`` holds independent pure-Python definitions for tiny cases that pin
the C code.  Paper: Koza et al., arXiv:1203.2946.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cmrs_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE binary64, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def build_baseline(out_dir: str) -> str:
    """Compile the same C source for the CPU-baseline timing: -O3
    -march=native (for the host it runs on, so call it there) and -fopenmp
    for ora_csr_spmv_par; still -ffp-contract=off, so results are unchanged.
    Returns the path of the shared library."""
    os.makedirs(out_dir, exist_ok=True)
    path = os.path.join(out_dir, "liboracle_baseline%d.so" % os.getpid())
    subprocess.check_call(["gcc", "-O3", "-march=native", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                           "-fopenmp", "-fPIC", "-shared", "-o", path, _SRC, "-lm"])
    return path


def _bind(lib):
    i32, u32p, i32p, vp = ctypes.c_int32, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    lib.ora_num_strips.argtypes = [i32, i32]
    lib.ora_num_strips.restype = i32
    lib.ora_bits_for_height.argtypes = [i32]
    lib.ora_bits_for_height.restype = i32
    lib.ora_csr_spmv.argtypes = [i32, i32p, i32p, dp, dp, dp]
    lib.ora_csr_spmv.restype = None
    lib.ora_csr_spmv_par.argtypes = [i32, i32p, i32p, dp, dp, dp, i32]
    lib.ora_csr_spmv_par.restype = i32
    lib.ora_csr_absmv.argtypes = [i32, i32p, i32p, dp, dp, dp]
    lib.ora_csr_absmv.restype = None
    lib.ora_csr_to_dense.argtypes = [i32, i32, i32p, i32p, dp, dp]
    lib.ora_csr_to_dense.restype = None
    lib.ora_dense_matvec.argtypes = [i32, i32, dp, dp, dp]
    lib.ora_dense_matvec.restype = None
    lib.ora_csr_to_cmrs.argtypes = [i32, i32, i32, i32p, i32p, vp, i32, i32, i32, i32, i32p, u32p, vp]
    lib.ora_csr_to_cmrs.restype = i32
    lib.ora_cmrs_to_csr.argtypes = [i32, i32, i32, i32, i32p, u32p, vp, i32, i32p, i32p, vp]
    lib.ora_cmrs_to_csr.restype = i32
    return lib


def _load(path: str | None = None):
    """The oracle library (the test build), or the library at ``path``."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build(force=True)
    _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_strips(rows: int, height: int) -> int:
    return int(_load().ora_num_strips(rows, height))


def bits_for_height(height: int) -> int:
    return int(_load().ora_bits_for_height(height))


def csr_spmv(row_ptr, col_ind, val, x, lib=None) -> np.ndarray:
    """y = A x in fp64, serial CRS order, sum from +0.0."""
    lib = lib or _load()
    row_ptr, col_ind, val, x = _i32(row_ptr), _i32(col_ind), _f64(val), _f64(x)
    rows = row_ptr.size - 1
    y = np.empty(rows, dtype=np.float64)
    lib.ora_csr_spmv(rows, _p(row_ptr, ctypes.c_int32), _p(col_ind, ctypes.c_int32),
                     _p(val, ctypes.c_double), _p(x, ctypes.c_double), _p(y, ctypes.c_double))
    return y


def csr_spmv_par(row_ptr, col_ind, val, x, threads: int, lib=None):
    """ora_csr_spmv_par: the same y over nnz-balanced row ranges on
    ``threads`` OpenMP threads (lib: a handle from _load(build_baseline(..)));
    returns (y, threads used)."""
    lib = lib or _load()
    row_ptr, col_ind, val, x = _i32(row_ptr), _i32(col_ind), _f64(val), _f64(x)
    rows = row_ptr.size - 1
    y = np.empty(rows, dtype=np.float64)
    used = lib.ora_csr_spmv_par(rows, _p(row_ptr, ctypes.c_int32), _p(col_ind, ctypes.c_int32),
                                _p(val, ctypes.c_double), _p(x, ctypes.c_double), _p(y, ctypes.c_double), threads)
    return y, int(used)


def csr_absmv(row_ptr, col_ind, val, x) -> np.ndarray:
    """(|A||x|)_i in fp64."""
    lib = _load()
    row_ptr, col_ind, val, x = _i32(row_ptr), _i32(col_ind), _f64(val), _f64(x)
    rows = row_ptr.size - 1
    out = np.empty(rows, dtype=np.float64)
    lib.ora_csr_absmv(rows, _p(row_ptr, ctypes.c_int32), _p(col_ind, ctypes.c_int32),
                      _p(val, ctypes.c_double), _p(x, ctypes.c_double), _p(out, ctypes.c_double))
    return out


def csr_to_dense(row_ptr, col_ind, val, cols: int) -> np.ndarray:
    lib = _load()
    row_ptr, col_ind, val = _i32(row_ptr), _i32(col_ind), _f64(val)
    rows = row_ptr.size - 1
    dense = np.empty((rows, cols), dtype=np.float64)
    lib.ora_csr_to_dense(rows, cols, _p(row_ptr, ctypes.c_int32), _p(col_ind, ctypes.c_int32),
                         _p(val, ctypes.c_double), _p(dense, ctypes.c_double))
    return dense


def dense_matvec(dense, x) -> np.ndarray:
    lib = _load()
    dense, x = _f64(dense), _f64(x)
    rows, cols = dense.shape
    y = np.empty(rows, dtype=np.float64)
    lib.ora_dense_matvec(rows, cols, _p(dense, ctypes.c_double), _p(x, ctypes.c_double), _p(y, ctypes.c_double))
    return y


def csr_to_cmrs(row_ptr, col_ind, val, cols: int, height: int, sorted_: bool = False, bits: int | None = None):
    """CRS -> CMRS.  Returns (strip_ptr int32, word uint32, val) with val of the
    input's dtype, moved bit for bit."""
    lib = _load()
    row_ptr, col_ind = _i32(row_ptr), _i32(col_ind)
    val = np.ascontiguousarray(val)
    rows = row_ptr.size - 1
    nnz = col_ind.size
    if bits is None:
        bits = bits_for_height(height)
    strips = num_strips(rows, height)
    strip_ptr = np.empty(strips + 1, dtype=np.int32)
    word = np.empty(nnz, dtype=np.uint32)
    val_out = np.empty_like(val)
    rc = lib.ora_csr_to_cmrs(rows, cols, nnz, _p(row_ptr, ctypes.c_int32), _p(col_ind, ctypes.c_int32),
                             val.ctypes.data_as(ctypes.c_void_p), val.itemsize, height, bits, int(bool(sorted_)),
                             _p(strip_ptr, ctypes.c_int32), _p(word, ctypes.c_uint32),
                             val_out.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise ValueError("oracle csr_to_cmrs rejected the input")
    return strip_ptr, word, val_out


def cmrs_to_csr(strip_ptr, word, val, rows: int, height: int, bits: int | None = None):
    """CMRS -> CRS.  Returns (row_ptr int32, col_ind int32, val)."""
    lib = _load()
    strip_ptr = _i32(strip_ptr)
    word = np.ascontiguousarray(word, dtype=np.uint32)
    val = np.ascontiguousarray(val)
    nnz = word.size
    if bits is None:
        bits = bits_for_height(height)
    row_ptr = np.empty(rows + 1, dtype=np.int32)
    col_ind = np.empty(nnz, dtype=np.int32)
    val_out = np.empty_like(val)
    rc = lib.ora_cmrs_to_csr(rows, nnz, height, bits, _p(strip_ptr, ctypes.c_int32), _p(word, ctypes.c_uint32),
                             val.ctypes.data_as(ctypes.c_void_p), val.itemsize,
                             _p(row_ptr, ctypes.c_int32), _p(col_ind, ctypes.c_int32),
                             val_out.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise ValueError("oracle cmrs_to_csr rejected the input")
    return row_ptr, col_ind, val_out


def spmv_bound(row_ptr, col_ind, val, x, unit_roundoff: float, factor: float = 4.0, extra: float = 0.0):
    """Componentwise tolerance  factor * (k_i + extra) * u * (|A||x|)_i  used by
    the parity tests (fp64: factor 4, extra 0, u = 2^-53)."""
    k = np.diff(_i32(row_ptr)).astype(np.float64)
    return factor * (k + extra) * unit_roundoff * csr_absmv(row_ptr, col_ind, val, x)
