"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This package only *generates* matrices and vectors (numpy PCG64 streams) and
rounds fp64 data to the storage precisions.  It holds none of the CMRS
method's arithmetic: no strip partition, no packing, no products.
"""
from .matrices import (  # noqa: F401
    Csr,
    banded,
    dense_as_sparse,
    identity,
    laplace2d,
    permutation,
    poisson_rows,
    random_csr,
    round_to_bf16_bits,
    bf16_bits_to_f64,
    round_to_f32,
    stencil27,
    dense_blocks,
    uniform_vector,
    normal_vector,
    zipf_clustered,
)
