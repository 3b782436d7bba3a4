"""Python binding of libgep (dense generalized symmetric-definite eigensolver on
an MI355X GPU).

Argument marshalling only: every step of the solve runs in the HIP kernels of
libgep.so.  There is no CPU fallback: if the library is missing, every call
raises.

Matrices are torch.float64 CUDA tensors.  libgep works in column-major storage;
for a symmetric matrix the bytes of a contiguous torch tensor are the same in
either order, so symmetric inputs are passed without a copy (libgep reads the
triangle that is lower in column-major order, i.e. the upper triangle of the
row-major torch view).  Outputs that are not symmetric (eigenvectors) are
returned as the transpose view of a column-major buffer.
"""
from __future__ import annotations

import ctypes
import os

from ._binding import (GEPError, JOB_VALUES, JOB_VECTORS, PREC_FP64, PREC_MIXED, lib, lib_path,
                       workspace_size)
from .api import (BatchedGraph, BatchedSolver, GEPFunction, band_reduce, backward, dgemm, reduce,
                  solve, solve_batched, solve_cholfree, solve_explicit_inverse, solve_jacobi, solve_lowest, tridiag_eig, tridiagonalize, profile_enable, profile_read, PHASES, PROBE_KERNELS,
                  probe_enable, probe_read)

__all__ = [
    "GEPError", "JOB_VALUES", "JOB_VECTORS", "PREC_FP64", "PREC_MIXED", "lib", "lib_path",
    "workspace_size", "BatchedGraph", "BatchedSolver", "GEPFunction", "band_reduce", "backward",
    "dgemm", "reduce", "solve", "solve_cholfree", "solve_explicit_inverse", "solve_jacobi",
    "solve_lowest",
    "solve_batched", "tridiag_eig", "tridiagonalize", "profile_enable", "profile_read", "PHASES",
    "PROBE_KERNELS", "probe_enable", "probe_read",
]
