"""MI355X iterative sparse solvers: Jacobi, symmetric Gauss-Seidel, CG and
BiCGStab on CSR or matrix-free 7/27-point stencils, with a mixed-precision
refined CG, a CG-NB variant, and differentiable solves (adjoint gradients
with respect to the right-hand side and to per-cell diffusion
coefficients, and to the stored values of a CSR matrix).  Every step runs
in the HIP library libitsolve.so (C ABI in
include/itsolve.h); this package only marshals torch tensors to it.
"""
from .api import (Batch, CSRMatrix, SolveInfo, StencilMatrix, VarCoefMatrix, cast_values,  # noqa: F401
                  csr_solve, diffusion_solve, dot, solve, solve_noalloc, spmv, stencil_solve,
                  stream_copy, varcoef_grad)
from ._lib import ItsError  # noqa: F401
