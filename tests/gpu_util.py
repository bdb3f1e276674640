"""Helpers for the GPU parity tests: move seeded CSR matrices to the device
in each storage precision, and fetch results back as numpy arrays."""
import numpy as np
import torch

import synth


def dev():
    return torch.device("cuda:0")


def host_vals(A_val: np.ndarray, dtype: str) -> np.ndarray:
    """Stored values as the GPU sees them: fp64, fp32 (RNE) or bf16 bit patterns."""
    if dtype == "f64":
        return np.ascontiguousarray(A_val, dtype=np.float64)
    if dtype == "f32":
        return synth.round_to_f32(A_val)
    if dtype == "bf16":
        return synth.round_to_bf16_bits(A_val)
    raise ValueError(dtype)


def vals_as_f64(v: np.ndarray, dtype: str) -> np.ndarray:
    if dtype == "bf16":
        return synth.bf16_bits_to_f64(v)
    return v.astype(np.float64)


def to_torch_vals(v: np.ndarray, dtype: str) -> torch.Tensor:
    if dtype == "bf16":
        return torch.from_numpy(v.view(np.int16).copy()).view(torch.bfloat16).to(dev())
    return torch.from_numpy(np.ascontiguousarray(v)).to(dev())


def upload(A: synth.Csr, dtype: str = "f64"):
    hv = host_vals(A.val, dtype)
    rp = torch.from_numpy(A.row_ptr).to(dev())
    ci = torch.from_numpy(A.col_ind).to(dev())
    return rp, ci, to_torch_vals(hv, dtype), hv


def val_bits(t: torch.Tensor) -> np.ndarray:
    """Raw bit patterns of a value tensor (for bit-exact comparisons)."""
    t = t.detach().cpu()
    if t.dtype == torch.float64:
        return t.numpy().view(np.uint64)
    if t.dtype == torch.float32:
        return t.numpy().view(np.uint32)
    return t.view(torch.int16).numpy().view(np.uint16)


def np_bits(v: np.ndarray) -> np.ndarray:
    return v.view({8: np.uint64, 4: np.uint32, 2: np.uint16}[v.dtype.itemsize])


def words(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)


def xy_vector(x64: np.ndarray, dtype: str) -> tuple[torch.Tensor, np.ndarray]:
    """x on the device in the path's x/y type, and the same values as fp64."""
    if dtype == "f64":
        xs = np.ascontiguousarray(x64, dtype=np.float64)
    else:
        xs = synth.round_to_f32(x64)
    return torch.from_numpy(xs).to(dev()), xs.astype(np.float64)
