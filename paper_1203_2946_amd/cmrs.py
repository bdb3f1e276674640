"""Python binding of libcmrs.so (argument marshalling only).

Every computation runs in the library's HIP kernels; this module checks
tensor devices, dtypes and contiguity, allocates outputs and workspaces with
torch, and passes raw device pointers plus torch's current HIP stream through
the C ABI declared in include/cmrs.h.  Importing it fails loudly when the
library is not built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcmrs.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_1203_2946_amd.build` "
                      "(or __graft_entry__.build()) first")
lib = ctypes.CDLL(LIB_PATH)

# ----------------------------------------------------------------- C ABI
CMRS_OK = 0
CMRS_ERR_INVALID_VALUE = 1
CMRS_ERR_INDEX_OVERFLOW = 2
CMRS_ERR_NOT_SUPPORTED = 3
CMRS_ERR_DEVICE = 4
CMRS_ERR_WORKSPACE = 5

CMRS_R64F, CMRS_R32F, CMRS_R16BF = 0, 1, 2
CMRS_SORT = 1
CMRS_MAX_HEIGHT = 32
SPMV_AUTO, SPMV_LDS, SPMV_REG, SPMV_LDS_NT, SPMV_REG_NT, SPMV_GROUP, SPMV_GROUP_NT = 0, 1, 2, 3, 4, 5, 6
VARIANTS = {"auto": SPMV_AUTO, "lds": SPMV_LDS, "reg": SPMV_REG, "lds_nt": SPMV_LDS_NT, "reg_nt": SPMV_REG_NT,
            "group": SPMV_GROUP, "group_nt": SPMV_GROUP_NT}

_DT = {torch.float64: CMRS_R64F, torch.float32: CMRS_R32F, torch.bfloat16: CMRS_R16BF}


class CmrsMatDesc(ctypes.Structure):
    _fields_ = [
        ("rows", ctypes.c_int32), ("cols", ctypes.c_int32), ("nnz", ctypes.c_int32),
        ("height", ctypes.c_int32), ("bits", ctypes.c_int32), ("sorted", ctypes.c_int32),
        ("val_dtype", ctypes.c_int), ("strip_ptr", ctypes.c_void_p), ("col_word", ctypes.c_void_p),
        ("val", ctypes.c_void_p),
    ]


_i32, _u32, _sz, _vp = ctypes.c_int32, ctypes.c_uint32, ctypes.c_size_t, ctypes.c_void_p
_DP = ctypes.POINTER(CmrsMatDesc)
lib.cmrs_abi_version.argtypes, lib.cmrs_abi_version.restype = [], _i32
lib.cmrs_num_strips.argtypes, lib.cmrs_num_strips.restype = [_i32, _i32], _i32
lib.cmrs_bits_for_height.argtypes, lib.cmrs_bits_for_height.restype = [_i32], _i32
lib.cmrs_from_csr_workspace.argtypes, lib.cmrs_from_csr_workspace.restype = [_i32, _i32, _i32, _u32], _sz
lib.cmrs_from_csr.argtypes = [_i32, _i32, _i32, _vp, _vp, _vp, ctypes.c_int, _i32, _u32, _vp, _vp, _vp, _vp, _sz, _vp]
lib.cmrs_from_csr.restype = ctypes.c_int
lib.cmrs_to_csr_workspace.argtypes, lib.cmrs_to_csr_workspace.restype = [_DP], _sz
lib.cmrs_to_csr.argtypes = [_DP, _vp, _vp, _vp, _vp, _sz, _vp]
lib.cmrs_to_csr.restype = ctypes.c_int
lib.cmrs_spmv.argtypes = [_DP, _vp, _vp, ctypes.c_int, _i32, _vp]
lib.cmrs_spmv.restype = ctypes.c_int
lib.cmrs_colblock_plan_bytes.argtypes, lib.cmrs_colblock_plan_bytes.restype = [_DP, _i32], _sz
lib.cmrs_colblock_plan.argtypes = [_DP, _i32, _vp, _sz, _vp]
lib.cmrs_colblock_plan.restype = ctypes.c_int
lib.cmrs_spmv_colblock_workspace.argtypes, lib.cmrs_spmv_colblock_workspace.restype = [_DP, _i32, _i32], _sz
lib.cmrs_spmv_colblock.argtypes = [_DP, _vp, _vp, ctypes.c_int, _i32, _i32, _vp, _sz, _i32, _vp, _sz, _vp]
lib.cmrs_spmv_colblock.restype = ctypes.c_int
lib.cmrs_spmv_colblock_noalloc.argtypes = [_DP, _vp, _vp, ctypes.c_int, _i32, _i32, _vp, _sz, _vp]
lib.cmrs_spmv_colblock_noalloc.restype = ctypes.c_int
NOALLOC_SCRATCH_BYTES = 32 << 20  # CMRS_NOALLOC_SCRATCH_BYTES


class SplitPlanStruct(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32), ("nnz", ctypes.c_int32), ("height", ctypes.c_int32),
                ("group", ctypes.c_int32), ("long_len", ctypes.c_int32), ("chunk_len", ctypes.c_int32),
                ("max_heavy", ctypes.c_int32), ("max_chunks", ctypes.c_int32), ("buf", ctypes.c_void_p),
                ("bytes", ctypes.c_size_t)]


lib.cmrs_spmv_split_plan_bytes.argtypes = [_DP, _i32, _i32]
lib.cmrs_spmv_split_plan_bytes.restype = _sz
lib.cmrs_spmv_split_plan.argtypes = [_DP, _i32, _i32, _vp, _sz, ctypes.POINTER(SplitPlanStruct), _vp]
lib.cmrs_spmv_split_plan.restype = ctypes.c_int
lib.cmrs_spmv_split.argtypes = [_DP, ctypes.POINTER(SplitPlanStruct), _vp, _vp, ctypes.c_int, _vp]
lib.cmrs_spmv_split.restype = ctypes.c_int
lib.cmrs_calib_stream_read.argtypes = [_vp, _vp, _i32, ctypes.c_int, _i32, _vp, _vp]
lib.cmrs_calib_stream_read.restype = ctypes.c_int
lib.cmrs_calib_gather.argtypes = [_vp, ctypes.c_int64, _vp, ctypes.c_int, _vp, _vp]
lib.cmrs_calib_gather.restype = ctypes.c_int
class SpmmTuning(ctypes.Structure):
    _fields_ = [("tile_nnz", ctypes.c_int32), ("group", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class SpmmPlanStruct(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("tiles", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int32), ("val_dtype", ctypes.c_int32), ("xy_dtype", ctypes.c_int32),
                ("max_slots", ctypes.c_int32), ("waves", ctypes.c_int32), ("desc", ctypes.c_void_p),
                ("desc_bytes", ctypes.c_size_t)]


_PI32 = ctypes.POINTER(ctypes.c_int32)
_PVP = ctypes.POINTER(ctypes.c_void_p)
lib.cmrs_spmm.argtypes = [_DP, _i32, _vp, _i32, _vp, _i32, ctypes.c_int, _i32, _vp]
lib.cmrs_spmm.restype = ctypes.c_int
lib.cmrs_spmm_plan_bytes.argtypes = [_i32, _DP, _PI32, ctypes.POINTER(SpmmTuning)]
lib.cmrs_spmm_plan_bytes.restype = _sz
lib.cmrs_spmm_plan.argtypes = [_i32, _DP, _PI32, _PVP, _PI32, _PVP, _PI32, ctypes.c_int,
                               ctypes.POINTER(SpmmTuning), _vp, _sz, ctypes.POINTER(SpmmPlanStruct), _vp]
lib.cmrs_spmm_plan.restype = ctypes.c_int
lib.cmrs_spmm_batched.argtypes = [ctypes.POINTER(SpmmPlanStruct), _vp]
lib.cmrs_spmm_batched.restype = ctypes.c_int
lib.cmrs_padded_bits.argtypes, lib.cmrs_padded_bits.restype = [_i32], _i32
lib.cmrs_padded_plan_workspace.argtypes, lib.cmrs_padded_plan_workspace.restype = [_i32, _i32], _sz
lib.cmrs_padded_plan.argtypes = [_i32, _i32, _vp, _i32, _vp, ctypes.POINTER(ctypes.c_int64), _vp, _sz, _vp]
lib.cmrs_padded_plan.restype = ctypes.c_int
lib.cmrs_padded_from_csr.argtypes = [_i32, _i32, _i32, _vp, _vp, _vp, ctypes.c_int, _i32, _vp, _i32, _vp, _vp, _vp]
lib.cmrs_padded_from_csr.restype = ctypes.c_int
lib.cmrs_padded_spmv.argtypes = [_DP, _vp, _vp, ctypes.c_int, _vp]
lib.cmrs_padded_spmv.restype = ctypes.c_int
lib.cmrs_features.argtypes = [_i32, _i32, _i32, _vp, _vp, _vp, _vp, _sz, _vp]
lib.cmrs_features.restype = ctypes.c_int
lib.cmrs_mlp_forward.argtypes = [_i32, _vp, _vp, _vp, _vp, _vp, _vp]
lib.cmrs_mlp_forward.restype = ctypes.c_int
lib.cmrs_mlp_backward.argtypes = [_i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
lib.cmrs_mlp_backward.restype = ctypes.c_int
lib.cmrs_mse_grad.argtypes = [_i32, _vp, _vp, _vp, ctypes.c_float, _vp]
lib.cmrs_mse_grad.restype = ctypes.c_int
lib.cmrs_adam_step.argtypes = [_i32, _vp, _vp, _vp, _vp] + [ctypes.c_float] * 4 + [_i32, _vp]
lib.cmrs_adam_step.restype = ctypes.c_int
lib.cmrs_validate_csr.argtypes = [_i32, _i32, _i32, _vp, _vp, _vp, _vp]
lib.cmrs_validate_csr.restype = ctypes.c_int
lib.cmrs_status_string.argtypes, lib.cmrs_status_string.restype = [ctypes.c_int], ctypes.c_char_p
lib.cmrs_last_error.argtypes, lib.cmrs_last_error.restype = [], ctypes.c_char_p

EXPORTED = ["cmrs_abi_version", "cmrs_num_strips", "cmrs_bits_for_height", "cmrs_from_csr_workspace",
            "cmrs_from_csr", "cmrs_to_csr_workspace", "cmrs_to_csr", "cmrs_spmv", "cmrs_validate_csr",
            "cmrs_colblock_plan_bytes", "cmrs_colblock_plan", "cmrs_spmv_colblock_workspace", "cmrs_spmv_colblock",
            "cmrs_spmv_colblock_noalloc", "cmrs_spmv_split_plan_bytes", "cmrs_spmv_split_plan", "cmrs_spmv_split",
            "cmrs_spmm", "cmrs_spmm_plan_bytes", "cmrs_spmm_plan", "cmrs_spmm_batched",
            "cmrs_padded_bits", "cmrs_padded_plan_workspace", "cmrs_padded_plan", "cmrs_padded_from_csr",
            "cmrs_padded_spmv",
            "cmrs_calib_stream_read", "cmrs_calib_gather", "cmrs_features", "cmrs_mlp_forward", "cmrs_mlp_backward",
            "cmrs_mse_grad", "cmrs_adam_step", "cmrs_status_string", "cmrs_last_error"]


class CmrsError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        name = lib.cmrs_status_string(status).decode()
        detail = lib.cmrs_last_error().decode()
        super().__init__(f"{where}: {name}: {detail}")


def _check(status: int, where: str):
    if status != CMRS_OK:
        raise CmrsError(status, where)


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptr(t: torch.Tensor | None) -> int | None:
    if t is None or t.numel() == 0:
        return None
    return t.data_ptr()


def _dev(t: torch.Tensor, name: str, dtype=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    return t


# ----------------------------------------------------------------- API
def abi_version() -> int:
    return int(lib.cmrs_abi_version())


def num_strips(rows: int, height: int) -> int:
    return int(lib.cmrs_num_strips(rows, height))


def bits_for_height(height: int) -> int:
    return int(lib.cmrs_bits_for_height(height))


@dataclass
class CmrsMatrix:
    """A CMRS matrix on the GPU: strip_ptr int32[strips+1], col_word int32
    [nnz] holding the uint32 packed words, val [nnz]."""
    rows: int
    cols: int
    height: int
    bits: int
    sorted: bool
    strip_ptr: torch.Tensor
    col_word: torch.Tensor
    val: torch.Tensor

    @property
    def nnz(self) -> int:
        return int(self.col_word.numel())

    @property
    def strips(self) -> int:
        return int(self.strip_ptr.numel()) - 1

    def desc(self) -> CmrsMatDesc:
        return CmrsMatDesc(self.rows, self.cols, self.nnz, self.height, self.bits, int(self.sorted),
                           _DT[self.val.dtype], _ptr(self.strip_ptr), _ptr(self.col_word), _ptr(self.val))


def from_csr_workspace_bytes(rows: int, nnz: int, height: int, sort: bool) -> int:
    return int(lib.cmrs_from_csr_workspace(rows, nnz, height, CMRS_SORT if sort else 0))


def from_csr(row_ptr: torch.Tensor, col_ind: torch.Tensor, val: torch.Tensor, cols: int, height: int,
             sort: bool = False, in_place: bool = False, workspace: torch.Tensor | None = None,
             out: CmrsMatrix | None = None, stream=None) -> CmrsMatrix:
    """CSR -> CMRS on the GPU.  in_place (unsorted only) packs the column words
    into col_ind's storage and keeps val's storage.  ``out`` reuses the arrays
    of an existing matrix of the same shape."""
    _dev(row_ptr, "row_ptr", torch.int32)
    _dev(col_ind, "col_ind", torch.int32)
    _dev(val, "val")
    if val.dtype not in _DT:
        raise TypeError(f"unsupported value dtype {val.dtype}")
    rows = row_ptr.numel() - 1
    nnz = col_ind.numel()
    if val.numel() != nnz:
        raise ValueError("val and col_ind differ in length")
    if in_place and sort:
        raise ValueError("the sorted conversion cannot run in place")
    strips = num_strips(rows, height)
    if strips < 0 or bits_for_height(height) < 0:
        raise ValueError(f"bad height {height}")
    dev = row_ptr.device
    if out is not None:
        sp, cw, vo = out.strip_ptr, out.col_word, out.val
    else:
        sp = torch.empty(strips + 1, dtype=torch.int32, device=dev)
        cw = col_ind if in_place else torch.empty(nnz, dtype=torch.int32, device=dev)
        vo = val if in_place else torch.empty_like(val)
    wsb = from_csr_workspace_bytes(rows, nnz, height, sort)
    if wsb and (workspace is None or workspace.numel() * workspace.element_size() < wsb):
        workspace = torch.empty(wsb, dtype=torch.uint8, device=dev)
    st = lib.cmrs_from_csr(rows, cols, nnz, _ptr(row_ptr), _ptr(col_ind), _ptr(val), _DT[val.dtype], height,
                           CMRS_SORT if sort else 0, _ptr(sp), _ptr(cw), _ptr(vo),
                           _ptr(workspace) if wsb else None, wsb, _stream(stream))
    _check(st, "cmrs_from_csr")
    return CmrsMatrix(rows, cols, height, bits_for_height(height), bool(sort), sp, cw, vo)


def to_csr(A: CmrsMatrix, out=None, stream=None):
    """CMRS -> CSR on the GPU; returns (row_ptr, col_ind, val)."""
    dev = A.col_word.device
    if out is None:
        rp = torch.empty(A.rows + 1, dtype=torch.int32, device=dev)
        ci = torch.empty(A.nnz, dtype=torch.int32, device=dev)
        vo = torch.empty_like(A.val)
    else:
        rp, ci, vo = out
    d = A.desc()
    st = lib.cmrs_to_csr(ctypes.byref(d), _ptr(rp), _ptr(ci), _ptr(vo), None, 0, _stream(stream))
    _check(st, "cmrs_to_csr")
    return rp, ci, vo


def spmv(A: CmrsMatrix, x: torch.Tensor, out: torch.Tensor | None = None, variant: int | str = SPMV_AUTO,
         stream=None) -> torch.Tensor:
    """y = A x.  fp64 values take fp64 x/y; fp32 and bf16 values take fp32 x/y."""
    if isinstance(variant, str):
        variant = VARIANTS[variant]
    xdt = torch.float64 if A.val.dtype == torch.float64 else torch.float32
    _dev(x, "x", xdt)
    if x.numel() != A.cols:
        raise ValueError(f"x has {x.numel()} entries, the matrix {A.cols} columns")
    y = out if out is not None else torch.empty(A.rows, dtype=xdt, device=x.device)
    _dev(y, "y", xdt)
    if y.numel() != A.rows:
        raise ValueError("y has the wrong length")
    d = A.desc()
    st = lib.cmrs_spmv(ctypes.byref(d), _ptr(x), _ptr(y), _DT[xdt], int(variant), _stream(stream))
    _check(st, "cmrs_spmv")
    return y


@dataclass
class ColblockPlan:
    """Split points of the column-blocked schedule (int32 [strips, nb-1])."""
    col_blocks: int
    split: torch.Tensor | None

    @property
    def nbytes(self) -> int:
        return 0 if self.split is None else self.split.numel() * 4


def colblock_plan(A: CmrsMatrix, col_blocks: int, stream=None) -> ColblockPlan:
    d = A.desc()
    nbytes = int(lib.cmrs_colblock_plan_bytes(ctypes.byref(d), col_blocks))
    split = torch.empty(max(nbytes // 4, 1), dtype=torch.int32, device=A.col_word.device) if nbytes else None
    st = lib.cmrs_colblock_plan(ctypes.byref(d), col_blocks, _ptr(split), nbytes, _stream(stream))
    _check(st, "cmrs_colblock_plan")
    return ColblockPlan(col_blocks, split)


COLBLOCK_SCHEDULES = {"passes": 0, "concurrent": 1, "phased": 2}


def spmv_colblock_workspace_bytes(A: CmrsMatrix, col_blocks: int, schedule: str = "passes") -> int:
    d = A.desc()
    return int(lib.cmrs_spmv_colblock_workspace(ctypes.byref(d), col_blocks, COLBLOCK_SCHEDULES[schedule]))


def spmv_colblock(A: CmrsMatrix, plan: ColblockPlan, x: torch.Tensor, out: torch.Tensor | None = None,
                  variant: int | str = SPMV_AUTO, schedule: str = "passes", workspace: torch.Tensor | None = None,
                  stream=None) -> torch.Tensor:
    """y = A x with the column-blocked schedule (A sorted)."""
    if isinstance(variant, str):
        variant = VARIANTS[variant]
    xdt = torch.float64 if A.val.dtype == torch.float64 else torch.float32
    _dev(x, "x", xdt)
    if x.numel() != A.cols:
        raise ValueError(f"x has {x.numel()} entries, the matrix {A.cols} columns")
    y = out if out is not None else torch.empty(A.rows, dtype=xdt, device=x.device)
    _dev(y, "y", xdt)
    if y.numel() != A.rows:
        raise ValueError("y has the wrong length")
    wsb = spmv_colblock_workspace_bytes(A, plan.col_blocks, schedule)
    if wsb and (workspace is None or workspace.numel() * workspace.element_size() < wsb):
        workspace = torch.empty(wsb, dtype=torch.uint8, device=x.device)
    d = A.desc()
    st = lib.cmrs_spmv_colblock(ctypes.byref(d), _ptr(x), _ptr(y), _DT[xdt], int(variant), plan.col_blocks,
                                _ptr(plan.split), plan.nbytes, COLBLOCK_SCHEDULES[schedule],
                                _ptr(workspace) if wsb else None, wsb, _stream(stream))
    _check(st, "cmrs_spmv_colblock")
    return y


def spmv_colblock_noalloc(A: CmrsMatrix, plan: ColblockPlan, x: torch.Tensor, out: torch.Tensor | None = None,
                          variant: int | str = SPMV_AUTO, stream=None) -> torch.Tensor:
    """The concurrent column-blocked y = A x with its partial sums in the
    library's static device scratch (cmrs_spmv_colblock_noalloc): allocates
    nothing when ``out`` is given."""
    if isinstance(variant, str):
        variant = VARIANTS[variant]
    xdt = torch.float64 if A.val.dtype == torch.float64 else torch.float32
    _dev(x, "x", xdt)
    if x.numel() != A.cols:
        raise ValueError(f"x has {x.numel()} entries, the matrix {A.cols} columns")
    y = out if out is not None else torch.empty(A.rows, dtype=xdt, device=x.device)
    _dev(y, "y", xdt)
    if y.numel() != A.rows:
        raise ValueError("y has the wrong length")
    d = A.desc()
    st = lib.cmrs_spmv_colblock_noalloc(ctypes.byref(d), _ptr(x), _ptr(y), _DT[xdt], int(variant), plan.col_blocks,
                                        _ptr(plan.split), plan.nbytes, _stream(stream))
    _check(st, "cmrs_spmv_colblock_noalloc")
    return y


class SplitPlan:
    """Plan of the split schedule: the device buffer and the filled struct."""

    def __init__(self, buf: torch.Tensor, plan: SplitPlanStruct):
        self.buf = buf
        self.plan = plan


def split_plan(A: CmrsMatrix, long_len: int = 0, chunk_len: int = 0, out: SplitPlan | None = None,
               stream=None) -> SplitPlan:
    """Heavy-strip plan of the split schedule (asynchronous; reads A's
    strip_ptr).  ``out`` reuses the buffer of an earlier plan of A."""
    d = A.desc()
    nbytes = int(lib.cmrs_spmv_split_plan_bytes(ctypes.byref(d), long_len, chunk_len))
    if nbytes == 0:
        raise ValueError("invalid matrix or lengths (cmrs_spmv_split_plan_bytes returned 0)")
    if out is not None and out.buf.numel() >= nbytes:
        buf = out.buf
    else:
        buf = torch.empty(nbytes, dtype=torch.uint8, device=A.col_word.device)
    plan = SplitPlanStruct()
    st = lib.cmrs_spmv_split_plan(ctypes.byref(d), long_len, chunk_len, buf.data_ptr(), buf.numel(),
                                  ctypes.byref(plan), _stream(stream))
    _check(st, "cmrs_spmv_split_plan")
    return SplitPlan(buf, plan)


def spmv_split(A: CmrsMatrix, plan: SplitPlan, x: torch.Tensor, out: torch.Tensor | None = None,
               stream=None) -> torch.Tensor:
    """y = A x with the split schedule."""
    xdt = torch.float64 if A.val.dtype == torch.float64 else torch.float32
    _dev(x, "x", xdt)
    if x.numel() != A.cols:
        raise ValueError(f"x has {x.numel()} entries, the matrix {A.cols} columns")
    y = out if out is not None else torch.empty(A.rows, dtype=xdt, device=x.device)
    _dev(y, "y", xdt)
    if y.numel() != A.rows:
        raise ValueError("y has the wrong length")
    d = A.desc()
    st = lib.cmrs_spmv_split(ctypes.byref(d), ctypes.byref(plan.plan), _ptr(x), _ptr(y), _DT[xdt], _stream(stream))
    _check(st, "cmrs_spmv_split")
    return y


def _rhs_block(t: torch.Tensor, name: str, n: int, dtype) -> int:
    """Check a row-major (n, nrhs) block with unit column stride; returns ld."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() != 2 or t.shape[0] != n:
        raise ValueError(f"{name} must have shape ({n}, nrhs), got {tuple(t.shape)}")
    if t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError(f"{name} needs unit stride along the right-hand sides")
    if t.shape[0] > 1 and t.stride(0) < t.shape[1]:
        raise ValueError(f"{name} has a leading dimension below nrhs")
    return max(int(t.stride(0)), int(t.shape[1])) if t.shape[0] > 1 else int(t.shape[1])


def spmm(A: CmrsMatrix, X: torch.Tensor, out: torch.Tensor | None = None, group: int = 0,
         stream=None) -> torch.Tensor:
    """Y = A X for X of shape (cols, nrhs), nrhs <= 8, row-major (one launch)."""
    xdt = torch.float64 if A.val.dtype == torch.float64 else torch.float32
    ldx = _rhs_block(X, "X", A.cols, xdt)
    nrhs = int(X.shape[1])
    Y = out if out is not None else torch.empty(A.rows, nrhs, dtype=xdt, device=X.device)
    ldy = _rhs_block(Y, "Y", A.rows, xdt)
    if Y.shape[1] != nrhs:
        raise ValueError("X and Y differ in the number of right-hand sides")
    d = A.desc()
    st = lib.cmrs_spmm(ctypes.byref(d), nrhs, _ptr(X), ldx, _ptr(Y), ldy, _DT[xdt], group, _stream(stream))
    _check(st, "cmrs_spmm")
    return Y


class SpmmPlan:
    """A batch plan: the device descriptor buffer, the filled plan struct and
    references that keep every bound tensor alive while the plan exists."""

    def __init__(self, desc: torch.Tensor, plan: SpmmPlanStruct, keep):
        self.desc = desc
        self.plan = plan
        self._keep = keep

    @property
    def tiles(self) -> int:
        return int(self.plan.tiles)

    @property
    def grid(self) -> int:
        return int(self.plan.grid)


def spmm_plan(mats, Xs, Ys, tile_nnz: int = 0, group: int = 0, blocks_per_cu: int = 0, stream=None) -> SpmmPlan:
    """Plan Y_i = A_i X_i for lists of matrices and (cols_i, nrhs_i) / (rows_i,
    nrhs_i) row-major blocks.  Synchronises the stream (set-up call)."""
    n = len(mats)
    if len(Xs) != n or len(Ys) != n:
        raise ValueError("mats, Xs and Ys differ in length")
    if n == 0:
        raise ValueError("empty batch")
    xdt = torch.float64 if mats[0].val.dtype == torch.float64 else torch.float32
    descs = (CmrsMatDesc * n)(*[A.desc() for A in mats])
    nrhs = (ctypes.c_int32 * n)()
    ldx = (ctypes.c_int32 * n)()
    ldy = (ctypes.c_int32 * n)()
    xp = (ctypes.c_void_p * n)()
    yp = (ctypes.c_void_p * n)()
    for i, (A, X, Y) in enumerate(zip(mats, Xs, Ys)):
        ldx[i] = _rhs_block(X, f"X[{i}]", A.cols, xdt)
        ldy[i] = _rhs_block(Y, f"Y[{i}]", A.rows, xdt)
        if X.shape[1] != Y.shape[1]:
            raise ValueError(f"X[{i}] and Y[{i}] differ in the number of right-hand sides")
        nrhs[i] = int(X.shape[1])
        xp[i] = _ptr(X)
        yp[i] = _ptr(Y)
    tun = SpmmTuning(tile_nnz, group, blocks_per_cu, 0)
    nbytes = int(lib.cmrs_spmm_plan_bytes(n, descs, nrhs, ctypes.byref(tun)))
    if nbytes == 0:
        raise ValueError("invalid batch (cmrs_spmm_plan_bytes returned 0)")
    desc = torch.empty(nbytes, dtype=torch.uint8, device=mats[0].val.device)
    plan = SpmmPlanStruct()
    st = lib.cmrs_spmm_plan(n, descs, nrhs, xp, ldx, yp, ldy, _DT[xdt], ctypes.byref(tun), desc.data_ptr(), nbytes,
                            ctypes.byref(plan), _stream(stream))
    _check(st, "cmrs_spmm_plan")
    return SpmmPlan(desc, plan, (list(mats), list(Xs), list(Ys)))


def spmm_batched(plan: SpmmPlan, stream=None) -> None:
    """Run a batch plan: one persistent launch."""
    st = lib.cmrs_spmm_batched(ctypes.byref(plan.plan), _stream(stream))
    _check(st, "cmrs_spmm_batched")


def padded_bits(height: int) -> int:
    return int(lib.cmrs_padded_bits(height))


def padded_from_csr(row_ptr: torch.Tensor, col_ind: torch.Tensor, val: torch.Tensor, cols: int, height: int,
                    stream=None) -> CmrsMatrix:
    """CSR -> the padded CMRS of Sec. 6.7 (chunks of 64, <= 8 entries of a
    row per chunk).  Synchronises the stream once (to size the output);
    the result's nnz is the padded size, ``real_nnz`` the CSR's."""
    _dev(row_ptr, "row_ptr", torch.int32)
    _dev(col_ind, "col_ind", torch.int32)
    _dev(val, "val")
    if val.dtype not in _DT:
        raise TypeError(f"unsupported value dtype {val.dtype}")
    rows = row_ptr.numel() - 1
    nnz = col_ind.numel()
    strips = num_strips(rows, height)
    if strips < 0 or padded_bits(height) < 0:
        raise ValueError(f"bad height {height}")
    dev = row_ptr.device
    sp = torch.empty(strips + 1, dtype=torch.int32, device=dev)
    wsb = int(lib.cmrs_padded_plan_workspace(rows, height))
    ws = torch.empty(max(wsb, 8), dtype=torch.uint8, device=dev)
    total = ctypes.c_int64(0)
    st = lib.cmrs_padded_plan(rows, nnz, _ptr(row_ptr), height, _ptr(sp), ctypes.byref(total), ws.data_ptr(), wsb,
                              _stream(stream))
    _check(st, "cmrs_padded_plan")
    pn = int(total.value)
    cw = torch.empty(pn, dtype=torch.int32, device=dev)
    vo = torch.empty(pn, dtype=val.dtype, device=dev)
    st = lib.cmrs_padded_from_csr(rows, cols, nnz, _ptr(row_ptr), _ptr(col_ind), _ptr(val), _DT[val.dtype], height,
                                  _ptr(sp), pn, _ptr(cw), _ptr(vo), _stream(stream))
    _check(st, "cmrs_padded_from_csr")
    M = CmrsMatrix(rows, cols, height, padded_bits(height), False, sp, cw, vo)
    M.real_nnz = nnz
    return M


def padded_spmv(A: CmrsMatrix, x: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """y = A x for a matrix from padded_from_csr."""
    xdt = torch.float64 if A.val.dtype == torch.float64 else torch.float32
    _dev(x, "x", xdt)
    if x.numel() != A.cols:
        raise ValueError(f"x has {x.numel()} entries, the matrix {A.cols} columns")
    y = out if out is not None else torch.empty(A.rows, dtype=xdt, device=x.device)
    _dev(y, "y", xdt)
    d = A.desc()
    st = lib.cmrs_padded_spmv(ctypes.byref(d), _ptr(x), _ptr(y), _DT[xdt], _stream(stream))
    _check(st, "cmrs_padded_spmv")
    return y


def validate_csr(row_ptr: torch.Tensor, col_ind: torch.Tensor, cols: int, stream=None) -> int:
    """Device CSR check; returns the flag (0 = valid).  Synchronises the stream."""
    _dev(row_ptr, "row_ptr", torch.int32)
    _dev(col_ind, "col_ind", torch.int32)
    flag = torch.empty(1, dtype=torch.int32, device=row_ptr.device)
    st = lib.cmrs_validate_csr(row_ptr.numel() - 1, cols, col_ind.numel(), _ptr(row_ptr), _ptr(col_ind),
                               flag.data_ptr(), _stream(stream))
    _check(st, "cmrs_validate_csr")
    return int(flag.item())


def calib_stream_read(A: CmrsMatrix, lds_words_per_lane: int, sink: torch.Tensor, stream=None) -> None:
    """Read-only pass over A's word and value streams (Sec. 6.3 calibration)."""
    st = lib.cmrs_calib_stream_read(_ptr(A.col_word), _ptr(A.val), A.nnz, _DT[A.val.dtype], lds_words_per_lane,
                                    sink.data_ptr(), _stream(stream))
    _check(st, "cmrs_calib_stream_read")


def calib_gather(idx: torch.Tensor, x: torch.Tensor, sink: torch.Tensor, stream=None) -> None:
    """sum of x[idx[i]]: random single-element read rate."""
    _dev(idx, "idx", torch.int32)
    st = lib.cmrs_calib_gather(_ptr(idx), idx.numel(), _ptr(x), _DT[x.dtype], sink.data_ptr(), _stream(stream))
    _check(st, "cmrs_calib_gather")
