"""MI355X (gfx950) sparse-covariance exact Gaussian process.

Python binding of ``libgpsparse.so`` (the C ABI in ``include/gpsparse.h``).
This module only marshals arguments: every step of the hot path runs in the
library's HIP kernels.  PyTorch supplies device memory (its caching
allocator is handed to the library) and streams.

The library must be built first (``python -m paper_2411_05869_amd.build``);
nothing here falls back to a CPU implementation.
"""
from __future__ import annotations

from ._lib import (  # noqa: F401
    CORE_MATERN,
    CORE_NONE,
    CORE_PACIOREK,
    FP64,
    MIXED,
    LOGDET_EXACT,
    LOGDET_NONE,
    LOGDET_SLQ_REORTH,
    LOGDET_SLQ,
    PRECOND_BLOCK_JACOBI,
    PRECOND_JACOBI,
    SOLVER_AUTO,
    SOLVER_CG,
    SOLVER_MINRES,
    Context,
    Dataset,
    GPError,
    Matrix,
    Predictor,
    lib,
    library_path,
)
