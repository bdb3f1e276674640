"""Seeded synthetic CSR matrices generated directly on the GPU with torch.

Used for the configuration-selection data set, which needs thousands of
matrices of up to millions of rows (numpy generation would dominate the time).
Five families: 3-D 27-point stencils, band matrices (bandwidth 8..64, 60 %
fill), Poisson row lengths with uniform columns, Zipf row lengths with columns
clustered around the diagonal, and block-sparse matrices of dense 32x32
tiles.  Every generator takes a torch.Generator on the device and returns
(row_ptr int32, col_ind int32, val float64, cols) with columns ascending and
distinct inside each row.  No CMRS arithmetic here.
"""
from __future__ import annotations

import math

import torch

FAMILIES = ("stencil", "banded", "poisson", "zipf", "dblock")


def _csr_from_pairs(rows, cols, r, c, g):
    """Sort (row, col) pairs, drop repeats, build CSR with N(0,1) values."""
    key = r.to(torch.int64) * cols + c.to(torch.int64)
    key = torch.unique(key, sorted=True)
    r = (key // cols).to(torch.int64)
    c = (key % cols).to(torch.int32)
    counts = torch.bincount(r, minlength=rows)
    row_ptr = torch.zeros(rows + 1, dtype=torch.int64, device=key.device)
    row_ptr[1:] = torch.cumsum(counts, 0)
    val = torch.randn(c.numel(), generator=g, dtype=torch.float64, device=key.device)
    return row_ptr.to(torch.int32), c, val, cols


def stencil(n, g):
    nx = max(2, round(n ** (1 / 3)))
    ny = nx
    nz = max(2, n // (nx * ny))
    n = nx * ny * nz
    dev = g.device
    i = torch.arange(n, device=dev)
    x, y, z = i % nx, (i // nx) % ny, i // (nx * ny)
    rs, cs = [], []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                ok = (x + dx >= 0) & (x + dx < nx) & (y + dy >= 0) & (y + dy < ny) & (z + dz >= 0) & (z + dz < nz)
                rs.append(i[ok])
                cs.append((i + dx + dy * nx + dz * nx * ny)[ok])
    return _csr_from_pairs(n, n, torch.cat(rs), torch.cat(cs), g)


def banded(n, g, bandwidth=None, fill=0.6):
    dev = g.device
    if bandwidth is None:
        bandwidth = int(torch.randint(8, 65, (1,), generator=g, device=dev).item())
    offs = torch.arange(-bandwidth, bandwidth + 1, device=dev)
    rs, cs = [], []
    chunk = max(1, (1 << 24) // offs.numel())
    for a in range(0, n, chunk):
        i = torch.arange(a, min(n, a + chunk), device=dev)
        c = i[:, None] + offs[None, :]
        keep = (c >= 0) & (c < n) & ((torch.rand(c.shape, generator=g, device=dev) < fill) | (offs[None, :] == 0))
        rs.append(i[:, None].expand_as(c)[keep])
        cs.append(c[keep])
    return _csr_from_pairs(n, n, torch.cat(rs), torch.cat(cs), g)


def poisson(n, g, mean=None):
    dev = g.device
    if mean is None:
        mean = float(torch.exp(torch.empty(1, device=dev).uniform_(math.log(2), math.log(64), generator=g)).item())
    k = torch.clamp(torch.poisson(torch.full((n,), mean, device=dev), generator=g), min=1).to(torch.int64)
    r = torch.repeat_interleave(torch.arange(n, device=dev), k)
    c = torch.randint(0, n, (r.numel(),), generator=g, device=dev)
    return _csr_from_pairs(n, n, r, c, g)


def zipf(n, g, a=None, kmax=10000, near=0.7, half_window=512):
    dev = g.device
    if a is None:
        a = float(torch.empty(1, device=dev).uniform_(1.8, 2.6, generator=g).item())
    ks = torch.arange(1, kmax + 1, dtype=torch.float64, device=dev)
    cdf = torch.cumsum(ks ** (-a), 0)
    cdf = cdf / cdf[-1]
    u = torch.rand(n, generator=g, dtype=torch.float64, device=dev)
    k = (torch.searchsorted(cdf, u) + 1).clamp(max=kmax)
    r = torch.repeat_interleave(torch.arange(n, device=dev), k)
    m = r.numel()
    is_near = torch.rand(m, generator=g, device=dev) < near
    off = torch.randint(-half_window, half_window + 1, (m,), generator=g, device=dev)
    c = torch.where(is_near, (r + off).clamp(0, n - 1), torch.randint(0, n, (m,), generator=g, device=dev))
    return _csr_from_pairs(n, n, r, c, g)


def dblock(n, g, block=32, per_row=None):
    dev = g.device
    nb = max(1, n // block)
    n = nb * block
    if per_row is None:
        per_row = int(torch.randint(1, 5, (1,), generator=g, device=dev).item())
    bc = torch.randint(0, nb, (nb, per_row), generator=g, device=dev)
    bc[:, 0] = torch.arange(nb, device=dev)
    br = torch.arange(nb, device=dev)[:, None].expand_as(bc)
    tr = torch.arange(block, device=dev)
    r = (br.reshape(-1, 1, 1) * block + tr[None, :, None]).expand(-1, block, block)
    c = (bc.reshape(-1, 1, 1) * block + tr[None, None, :]).expand(-1, block, block)
    return _csr_from_pairs(n, n, r.reshape(-1), c.reshape(-1), g)


def generate(family, n, g):
    return {"stencil": stencil, "banded": banded, "poisson": poisson, "zipf": zipf, "dblock": dblock}[family](n, g)


def batched_workload(seed: int = 0, count: int = 256, lo: int = 10_000, hi: int = 500_000, dev="cuda"):
    """The uneven batch: `count` matrices with rows log-uniform in [lo, hi],
    alternately 3-D 27-point stencils and band matrices (bandwidth uniform in
    8..64, 60 % fill), values N(0,1), each with 1..8 right-hand sides.
    Returns a list of (family, row_ptr, col_ind, val, cols, nrhs)."""
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    out = []
    for i in range(count):
        u = torch.rand(2, generator=g, device=dev).tolist()
        n = int(round(math.exp(math.log(lo) + u[0] * (math.log(hi) - math.log(lo)))))
        nrhs = 1 + min(7, int(u[1] * 8))
        if i % 2 == 0:
            rp, ci, val, cols = stencil(n, g)
            fam = "stencil"
        else:
            rp, ci, val, cols = banded(n, g)
            fam = "banded"
        out.append((fam, rp, ci, val, cols, nrhs))
    return out
