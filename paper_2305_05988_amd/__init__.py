"""MI355X iterative sparse solvers: Jacobi, symmetric Gauss-Seidel, CG and
BiCGStab on CSR or matrix-free 7/27-point stencils, with a mixed-precision
refined CG.  Every step runs in the HIP library libitsolve.so (C ABI in
include/itsolve.h); this package only marshals torch tensors to it.
"""
from .api import (CSRMatrix, SolveInfo, StencilMatrix, cast_values, dot, solve, spmv,  # noqa: F401
                  stream_copy)
from ._lib import ItsError  # noqa: F401
