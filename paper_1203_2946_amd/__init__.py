"""CMRS sparse matrix-vector product for AMD MI355X (gfx950).

Compressed Multi-Row Storage (Koza et al., arXiv:1203.2946): CSR rows grouped
into strips of ``height`` rows, one strip pointer per strip, the row-in-strip
id packed into the low bits of each column word.  The HIP kernels and the
C ABI live in ``csrc/`` and build into ``libcmrs.so`` in this directory; the
Python API in :mod:`paper_1203_2946_amd.cmrs` only marshals torch tensors
through that ABI.

Modules: ``cmrs`` (the binding: conversions, SpMV schedules, several
right-hand sides, batched persistent launches, the padded layout of
Sec. 6.7), ``batched`` (batch autotuner and HIP-graph runner), ``selector``
(learned choice of height and schedule, trained with the library's own MLP
kernels), ``model`` (the paper's byte and performance models), ``build``.

Importing this package does not load the library; importing ``.cmrs`` does,
and raises if it is not built.
"""
__all__ = ["cmrs", "model", "batched", "selector"]
