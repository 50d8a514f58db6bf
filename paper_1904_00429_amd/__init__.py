"""MI355X (gfx950) library for the multilevel Monte Carlo estimator of E[AB]
and E[x^T y] by uniform-probability sketching (Wu & Polydorides,
arXiv:1904.00429).  The compute path is the HIP library libmlmc.so (C ABI in
include/mlmc.h); this package is its thin binding."""
from .mlmc import (FLAG_SHARED_SAMPLES, PREC, SHARED_LEVEL_FIELD, BatchedEstimate, BatchProblem,  # noqa: F401
                   Func, InnerProductGraph, Law, Result,
                   gather_columns, inner_product_estimate, inner_product_estimate_noalloc, matmul_adjoint_reparam,
                   matmul_estimate, matmul_workspace_size, optimal_index_weights, philox, sample_indices,
                   sample_indices_weighted)
from .autograd import MLMCMatmul, mlmc_matmul  # noqa: F401
from ._lib import MLMCError  # noqa: F401
