"""CPU checks of the C ABI: the library loads, exports every function that
include/cmrs.h declares, and its host-side logic (sizes, argument validation)
behaves as documented.  No call here reaches a kernel launch."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cmrs.h")


@pytest.fixture(scope="module")
def C():
    from paper_1203_2946_amd import cmrs
    return cmrs


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cmrs_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("cmrs_from_csr", "cmrs_to_csr", "cmrs_spmv", "cmrs_num_strips", "cmrs_bits_for_height",
              "cmrs_status_string", "cmrs_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(C):
    lib = ctypes.CDLL(C.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert sorted(C.EXPORTED) == sorted(declared_functions())


def test_abi_version(C):
    assert C.abi_version() == 2


def test_host_helpers(C):
    assert C.num_strips(5, 2) == 3 and C.num_strips(0, 7) == 0 and C.num_strips(2**31 - 1, 32) == 2**26
    assert C.num_strips(-1, 2) == -1 and C.num_strips(4, 0) == -1
    assert [C.bits_for_height(h) for h in (1, 2, 3, 16, 17, 32)] == [4, 4, 4, 4, 5, 5]
    assert C.bits_for_height(0) == -1 and C.bits_for_height(33) == -1
    assert C.lib.cmrs_status_string(3).decode() == "CMRS_ERR_NOT_SUPPORTED"
    assert C.lib.cmrs_status_string(99).decode() == "CMRS_UNKNOWN_STATUS"


def test_workspace_sizes(C):
    assert C.from_csr_workspace_bytes(100, 1000, 8, sort=False) == 0
    ws = C.from_csr_workspace_bytes(100, 1000, 8, sort=True)
    assert ws >= 16 * 1000
    assert C.from_csr_workspace_bytes(100, 0, 8, sort=True) == 0


FAKE = 0x1000  # never dereferenced: every call below fails its host checks first


def _from_csr(C, **kw):
    a = dict(rows=4, cols=4, nnz=4, row_ptr=FAKE, col_ind=FAKE, val=FAKE, dtype=0, height=2, flags=0,
             sp=FAKE, cw=FAKE + 64, vo=FAKE + 128, ws=None, wsb=0)
    a.update(kw)
    return C.lib.cmrs_from_csr(a["rows"], a["cols"], a["nnz"], a["row_ptr"], a["col_ind"], a["val"], a["dtype"],
                               a["height"], a["flags"], a["sp"], a["cw"], a["vo"], a["ws"], a["wsb"], None)


@pytest.mark.parametrize("kw,status", [
    (dict(rows=-1), 1), (dict(nnz=-3), 1), (dict(height=0), 1), (dict(height=33), 1), (dict(flags=2), 1),
    (dict(dtype=7), 1), (dict(row_ptr=None), 1), (dict(col_ind=None), 1), (dict(sp=None), 1),
    (dict(cols=2**28 + 1), 2), (dict(cols=2**27 + 1, height=17), 2),
    (dict(flags=1, ws=None, wsb=0), 5),
    (dict(flags=1, cw=FAKE + 8, col_ind=FAKE + 8, ws=FAKE, wsb=1 << 20), 1),
    (dict(cw=FAKE + 4, col_ind=FAKE), 1),
])
def test_from_csr_rejects(C, kw, status):
    assert _from_csr(C, **kw) == status
    assert C.lib.cmrs_last_error().decode() != ""


def _mat(C, **kw):
    d = dict(rows=4, cols=4, nnz=4, height=2, bits=4, sorted=0, val_dtype=0, strip_ptr=FAKE, col_word=FAKE,
             val=FAKE)
    d.update(kw)
    return C.CmrsMatDesc(**d)


@pytest.mark.parametrize("kw,xy,variant,status", [
    (dict(height=0), 0, 0, 1), (dict(bits=5), 0, 0, 1), (dict(val_dtype=9), 0, 0, 1),
    (dict(strip_ptr=None), 0, 0, 1), (dict(cols=2**28 + 1), 0, 0, 2),
    (dict(), 1, 0, 3), (dict(val_dtype=1), 0, 0, 3), (dict(val_dtype=2), 2, 0, 3),
    (dict(), 0, 9, 1),
])
def test_spmv_rejects(C, kw, xy, variant, status):
    d = _mat(C, **kw)
    assert C.lib.cmrs_spmv(ctypes.byref(d), FAKE, FAKE + 4096, xy, variant, None) == status


def test_spmv_rejects_overlap_and_null(C):
    d = _mat(C)
    assert C.lib.cmrs_spmv(ctypes.byref(d), FAKE, FAKE + 8, 0, 0, None) == 1      # x and y overlap
    assert C.lib.cmrs_spmv(ctypes.byref(d), FAKE, None, 0, 0, None) == 1
    assert C.lib.cmrs_spmv(None, FAKE, FAKE + 4096, 0, 0, None) == 1


def test_spmv_empty_matrix_is_noop(C):
    d = _mat(C, rows=0, nnz=0, strip_ptr=None, col_word=None, val=None)
    assert C.lib.cmrs_spmv(ctypes.byref(d), None, None, 0, 0, None) == 0


def test_to_csr_rejects(C):
    d = _mat(C)
    assert C.lib.cmrs_to_csr(ctypes.byref(d), None, FAKE, FAKE, None, 0, None) == 1
    assert C.lib.cmrs_to_csr(ctypes.byref(d), FAKE + 4096, FAKE, FAKE + 8192, None, 0, None) == 1  # col_ind_out overlaps col_word
    d2 = _mat(C, nnz=-1)
    assert C.lib.cmrs_to_csr(ctypes.byref(d2), FAKE, FAKE, FAKE, None, 0, None) == 1


def test_validate_rejects(C):
    assert C.lib.cmrs_validate_csr(-1, 4, 4, FAKE, FAKE, FAKE, None) == 1
    assert C.lib.cmrs_validate_csr(4, 4, 4, None, FAKE, FAKE, None) == 1


# ----------------------------------------------------------------- multi-RHS and batches
@pytest.mark.parametrize("nrhs,ldx,ldy,xy,group,status", [
    (0, 4, 4, 0, 0, 1), (9, 9, 9, 0, 0, 1), (2, 1, 2, 0, 0, 1), (2, 2, 1, 0, 0, 1),
    (2, 2, 2, 1, 0, 3),                       # fp64 values with fp32 X/Y
    (2, 2, 2, 0, 3, 1), (2, 2, 2, 0, 128, 1), # group not a power of two / above 64
])
def test_spmm_rejects(C, nrhs, ldx, ldy, xy, group, status):
    d = _mat(C)
    assert C.lib.cmrs_spmm(ctypes.byref(d), nrhs, FAKE, ldx, FAKE + 1 << 20, ldy, xy, group, None) == status


def test_spmm_lds_limit(C):
    # 32 rows x 8 right-hand sides x 64 lanes of fp64 partials = 128 KiB per wave.
    big = _mat(C, rows=64, cols=64, height=32, bits=5)
    assert C.lib.cmrs_spmm(ctypes.byref(big), 8, FAKE, 8, FAKE + (1 << 20), 8, 0, 0, None) == 3
    m, r = _batch(C, [big], [8])
    assert C.lib.cmrs_spmm_plan_bytes(1, m, r, None) == 0


def test_spmm_rejects_overlap_and_accepts_empty(C):
    d = _mat(C)
    # X spans 4 rows x ld 8 doubles; Y starts inside it.
    assert C.lib.cmrs_spmm(ctypes.byref(d), 2, FAKE, 8, FAKE + 100, 2, 0, 0, None) == 1
    e = _mat(C, rows=0, nnz=0, strip_ptr=None, col_word=None, val=None)
    assert C.lib.cmrs_spmm(ctypes.byref(e), 3, None, 3, None, 3, 0, 0, None) == 0


def _batch(C, mats, nrhs):
    n = len(mats)
    return (C.CmrsMatDesc * n)(*mats), (ctypes.c_int32 * n)(*nrhs)


def test_spmm_plan_bytes_counts_tiles(C):
    # 1000 rows, height 4: 250 strips of 108 entries; one right-hand side
    # unrolls 8 entries per slot: 108 / 8 -> 16 slots, 4 strips per pass;
    # 32768 / 108 -> 300 strips per tile: one tile.  Header 1024 B, one 96 B
    # descriptor, one 16 B tile.
    m, r = _batch(C, [_mat(C, rows=1000, cols=1000, nnz=27000, height=4)], [1])
    assert C.lib.cmrs_spmm_plan_bytes(1, m, r, None) == 1024 + 96 + 16
    tun = C.SpmmTuning(1000, 0, 0, 0)       # 1000 / 108 -> 9 -> 8 strips per tile: 32 tiles
    assert C.lib.cmrs_spmm_plan_bytes(1, m, r, ctypes.byref(tun)) == 1024 + 96 + 16 * 32
    m2, r2 = _batch(C, [_mat(C, rows=1000, cols=1000, nnz=27000, height=4), _mat(C, rows=0, nnz=0)], [1, 8])
    assert C.lib.cmrs_spmm_plan_bytes(2, m2, r2, None) == 1024 + 2 * 96 + 16
    bad = C.SpmmTuning(0, 0, 0, 1)           # reserved field set
    assert C.lib.cmrs_spmm_plan_bytes(1, m, r, ctypes.byref(bad)) == 0
    m3, r3 = _batch(C, [_mat(C)], [9])
    assert C.lib.cmrs_spmm_plan_bytes(1, m3, r3, None) == 0


def test_spmm_plan_rejects(C):
    mats, nrhs = _batch(C, [_mat(C), _mat(C)], [1, 1])
    ld = (ctypes.c_int32 * 2)(1, 1)
    plan = C.SpmmPlanStruct()
    X = (ctypes.c_void_p * 2)(FAKE, FAKE)               # shared X is fine
    Y_ok = (ctypes.c_void_p * 2)(FAKE + 4096, FAKE + 8192)
    Y_clash = (ctypes.c_void_p * 2)(FAKE + 4096, FAKE + 4096 + 16)
    Y_on_x = (ctypes.c_void_p * 2)(FAKE + 4096, FAKE + 8)
    def call(Y, desc=FAKE + 1 << 20, nbytes=1 << 16, tun=None):
        return C.lib.cmrs_spmm_plan(2, mats, nrhs, X, ld, Y, ld, 0, tun, desc, nbytes, ctypes.byref(plan), None)
    assert call(Y_clash) == 1
    assert call(Y_on_x) == 1
    assert call(Y_ok, nbytes=16) == 5                   # plan buffer too small
    assert call(Y_ok, desc=FAKE + 3) == 5 or call(Y_ok, desc=FAKE + 3) == 1
    assert call(Y_ok, tun=ctypes.byref(C.SpmmTuning(0, 3, 0, 0))) == 1
    mixed, nr = _batch(C, [_mat(C), _mat(C, val_dtype=1)], [1, 1])
    assert C.lib.cmrs_spmm_plan(2, mixed, nr, X, ld, Y_ok, ld, 0, None, FAKE, 1 << 16, ctypes.byref(plan),
                                None) == 3


def test_spmm_batched_rejects_corrupt_plan(C):
    p = C.SpmmPlanStruct()
    assert C.lib.cmrs_spmm_batched(ctypes.byref(p), None) == 0          # zero tiles: nothing to do
    p.tiles, p.count, p.grid, p.waves, p.max_slots, p.lds_bytes, p.desc = 3, 1, 2, 7, 4, 4 * 64 * 8 * 4, FAKE
    assert C.lib.cmrs_spmm_batched(ctypes.byref(p), None) == 1          # waves not a multiple of grid
    p.waves, p.max_slots = 8, 3
    assert C.lib.cmrs_spmm_batched(ctypes.byref(p), None) == 1          # slot count not a power of two
    p.max_slots, p.lds_bytes = 4, 1024
    assert C.lib.cmrs_spmm_batched(ctypes.byref(p), None) == 1          # LDS below 4 waves x 4 slots x 64 x 8 B
    assert C.lib.cmrs_spmm_batched(None, None) == 1


def test_sizes_above_max_index_rejected(C):
    """rows or nnz above CMRS_MAX_INDEX (2^31 - 2^16) return INDEX_OVERFLOW (2)
    from the host checks, before anything is enqueued."""
    big = 2**31 - 2**16 + 1
    assert _from_csr(C, nnz=big) == 2
    assert _from_csr(C, rows=big) == 2
    d = _mat(C, nnz=big)
    assert C.lib.cmrs_to_csr(ctypes.byref(d), FAKE + 4096, FAKE + 8192, FAKE + 16384, None, 0, None) == 2
    assert C.lib.cmrs_spmv(ctypes.byref(d), FAKE + 4096, FAKE + 8192, 0, 0, None) == 2
    d = _mat(C, rows=big)
    assert C.lib.cmrs_spmv(ctypes.byref(d), FAKE + 4096, FAKE + 8192, 0, 0, None) == 2
    assert C.lib.cmrs_validate_csr(big, 4, 4, FAKE, FAKE, FAKE, None) == 2


def test_colblock_noalloc_host_checks(C):
    """The allocation-free column-blocked product refuses, before any device
    call, partial sums beyond its static scratch and the same bad arguments
    as cmrs_spmv_colblock."""
    big = 1 << 21                                  # fp64, 4 blocks: 4 * 2^21 * 8 B = 64 MiB > 32 MiB
    d = _mat(C, rows=big, cols=big, nnz=4, height=4, sorted=1)
    assert C.lib.cmrs_spmv_colblock_noalloc(ctypes.byref(d), FAKE, FAKE + (1 << 30), 0, 0, 4, FAKE,
                                            1 << 30, None) == 5
    assert "scratch" in C.lib.cmrs_last_error().decode()
    assert C.lib.cmrs_spmv_colblock_workspace(ctypes.byref(d), 4, 1) == 4 * big * 8 > C.NOALLOC_SCRATCH_BYTES
    ok = _mat(C, rows=1 << 20, cols=1 << 20, nnz=4, height=4, sorted=1)
    assert C.lib.cmrs_spmv_colblock_workspace(ctypes.byref(ok), 4, 1) == C.NOALLOC_SCRATCH_BYTES
    unsorted = _mat(C, sorted=0)
    assert C.lib.cmrs_spmv_colblock_noalloc(ctypes.byref(unsorted), FAKE, FAKE + 4096, 0, 0, 4, FAKE, 64, None) == 1
    small = _mat(C, sorted=1)
    assert C.lib.cmrs_spmv_colblock_noalloc(ctypes.byref(small), FAKE, FAKE + 4096, 0, 0, 4, None, 0, None) == 5
    assert C.lib.cmrs_spmv_colblock_noalloc(ctypes.byref(small), FAKE, FAKE + 4096, 0, 0, 65, FAKE, 64, None) == 1
    assert C.lib.cmrs_spmv_colblock_noalloc(ctypes.byref(small), FAKE, FAKE + 8, 0, 0, 4, FAKE, 64, None) == 1


def test_split_plan_host_checks(C):
    d = _mat(C, rows=1000, cols=1000, nnz=5000, height=8, sorted=0)
    n0 = C.lib.cmrs_spmv_split_plan_bytes(ctypes.byref(d), 0, 0)
    assert n0 > 0 and n0 % 256 == 0
    assert C.lib.cmrs_spmv_split_plan_bytes(ctypes.byref(d), -1, 0) == 0
    assert C.lib.cmrs_spmv_split_plan_bytes(ctypes.byref(_mat(C, height=0)), 0, 0) == 0
    p = C.SplitPlanStruct()
    assert C.lib.cmrs_spmv_split_plan(ctypes.byref(d), 0, 0, None, 0, ctypes.byref(p), None) == 5
    assert C.lib.cmrs_spmv_split_plan(ctypes.byref(d), 0, 0, FAKE + 4, n0, ctypes.byref(p), None) == 5  # misaligned
    assert C.lib.cmrs_spmv_split_plan(ctypes.byref(d), 0, 0, FAKE, n0 - 1, ctypes.byref(p), None) == 5
    assert C.lib.cmrs_spmv_split_plan(ctypes.byref(d), -2, 0, FAKE, n0, ctypes.byref(p), None) == 1
    assert C.lib.cmrs_spmv_split_plan(ctypes.byref(d), 0, 0, FAKE, n0, None, None) == 1
    # a plan for another shape, or with fields that do not match the matrix, is refused before any launch
    bad = C.SplitPlanStruct(999, 5000, 8, 8, 128, 1024, 1, 1, FAKE, n0)
    assert C.lib.cmrs_spmv_split(ctypes.byref(d), ctypes.byref(bad), FAKE + (1 << 20), FAKE + (1 << 21), 0, None) == 1
    bad = C.SplitPlanStruct(1000, 5000, 8, 8, 0, 1024, 1, 1, FAKE, n0)
    assert C.lib.cmrs_spmv_split(ctypes.byref(d), ctypes.byref(bad), FAKE + (1 << 20), FAKE + (1 << 21), 0, None) == 1
    assert C.lib.cmrs_spmv_split(ctypes.byref(d), None, FAKE + (1 << 20), FAKE + (1 << 21), 0, None) == 1
    assert C.lib.cmrs_spmv_split(ctypes.byref(d), None, FAKE + (1 << 20), FAKE + (1 << 21), 1, None) == 3
