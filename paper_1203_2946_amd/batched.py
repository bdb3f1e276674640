"""Batched uneven multi-right-hand-side products: autotuner and graph runner.

A batch is many CMRS matrices of different sizes, each with its own 1..8
right-hand sides.  `tune()` times candidate plans (work-tile size, entry
slots per strip, resident workgroups per CU) of the one persistent launch
(cmrs_spmm_batched) on the actual batch and keeps the fastest; `Graph`
captures that launch into a HIP graph and replays it.  `run_separate()` is
the baseline: one cmrs_spmm launch per matrix.  Every product runs in the
library's kernels; torch provides memory, streams, events and the graph.
"""
from __future__ import annotations

import itertools

import numpy as np
import torch

from . import cmrs

DEFAULT_CANDIDATES = {
    "tile_nnz": (4_096, 8_192, 32_768),
    "group": (0, 8, 16),
    "blocks_per_cu": (2, 4, 8),
}


def batch_bytes(mats, nrhs) -> int:
    """Algorithmic bytes of one batch: per matrix the value and word streams,
    the strip pointers, X read once and Y written once per right-hand side."""
    tot = 0
    for A, r in zip(mats, nrhs):
        sv = A.val.element_size()
        sx = 8 if A.val.dtype == torch.float64 else 4
        tot += (sv + 4) * A.nnz + 4 * (A.strips + 1) + sx * r * (A.cols + A.rows)
    return tot


def batch_flops(mats, nrhs) -> int:
    return sum(2 * A.nnz * r for A, r in zip(mats, nrhs))


def _time(fn, reps: int, warmup: int = 2) -> list[float]:
    for _ in range(warmup):
        fn()
    evs = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        evs.append((a, b))
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in evs]


def run_separate(mats, Xs, Ys, group: int = 0) -> None:
    for A, X, Y in zip(mats, Xs, Ys):
        cmrs.spmm(A, X, out=Y, group=group)


def tune(mats, Xs, Ys, candidates=None, reps: int = 5):
    """Time every candidate plan; returns (best_plan, best_tuning, table)
    with table rows (tuning dict, median ms)."""
    cand = dict(DEFAULT_CANDIDATES)
    if candidates:
        cand.update(candidates)
    keys = list(cand)
    table = []
    best = None
    for values in itertools.product(*(cand[k] for k in keys)):
        tun = dict(zip(keys, values))
        plan = cmrs.spmm_plan(mats, Xs, Ys, **tun)
        ms = float(np.median(_time(lambda: cmrs.spmm_batched(plan), reps)))
        table.append((tun, ms))
        if best is None or ms < best[2]:
            best = (plan, tun, ms)
        else:
            del plan
    return best[0], best[1], table


class Graph:
    """One persistent batched launch captured in a HIP graph."""

    def __init__(self, plan):
        self.plan = plan
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(side):
            with torch.cuda.graph(self.graph, stream=side):
                cmrs.spmm_batched(plan)
        torch.cuda.synchronize()

    def replay(self) -> None:
        self.graph.replay()
