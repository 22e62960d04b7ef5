"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This package generates coordinates, values and initial factor matrices only.
It holds no part of the ALTO method (no encoding, ordering, partitioning or
MTTKRP arithmetic), so that the two sides it feeds stay independent.
"""

from .tensors import (  # noqa: F401
    CONFIGS,
    SparseTensor,
    make_config,
    make_factors,
    uniform_distinct_tensor,
    zipf_tensor,
    random_small_tensor,
)
