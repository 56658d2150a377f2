"""Seeded synthetic LASSO inputs shared by the oracle, the tests and the benchmark.

This package only builds inputs (sparse matrices, right-hand sides, planted
solutions, regularisation weights).  It holds none of the coordinate-descent
arithmetic: no sampling, no step, no objective.
"""

from .lasso import (  # noqa: F401
    CSC,
    LassoInstance,
    random_csc,
    random_csc_ragged,
    planted_lasso,
    tightness_matrix,
    biregular_matrix,
    separable_matrix,
    orthonormal_block_hadamard,
    dense_to_csc,
    csc_to_dense,
)
from .configs import CONFIGS, make_config  # noqa: F401
