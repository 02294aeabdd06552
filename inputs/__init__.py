"""Seeded synthetic workloads shared by the oracle tests and the HIP path.

This package builds problem inputs only: sparsity patterns, matrix values,
right-hand sides and dense vectors, all from a counter-based generator
(SplitMix64).  It holds none of the method's arithmetic (no SpMV, no
format conversion, no solver), so that neither side of a parity test can
lean on the other through it.
"""
from .rng import splitmix64, u64_stream, uniform, normal
from .generators import (
    Problem,
    hpcg27,
    hpcg27_rank,
    hpcg27_levels,
    aniso7,
    zipf,
    banded,
    banded_spd,
    random_sparse,
    uniform_vector,
    serving_stream,
    ZIPF_EXPONENT,
)

__all__ = [
    "splitmix64", "u64_stream", "uniform", "normal",
    "Problem", "hpcg27", "hpcg27_rank", "hpcg27_levels", "aniso7", "zipf", "banded", "banded_spd",
    "random_sparse", "uniform_vector", "serving_stream", "ZIPF_EXPONENT",
]
