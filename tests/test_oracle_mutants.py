"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake into a copy of oracle.c (on the CPU, in a
temporary directory), builds it, swaps it in and checks that the named pin
tests fail.  The real oracle is restored afterwards.
"""
import os

import pytest

import oracle
from oracle import build as obuild

from . import test_oracle_kernels as K
from . import test_oracle_solvers as S
from . import test_oracle_varcoef as V

SRC = os.path.join(os.path.dirname(obuild.__file__), "oracle.c")

# (name, exact source fragment, replacement, pins expected to fail)
MUTANTS = [
    ("cg residual sign", "r[i] = fma(-alpha, q[i], r[i]);", "r[i] = fma(alpha, q[i], r[i]);",
     [lambda: S.test_cg_matches_dense_lu(S.inputs.poisson7_csr, (6, 5, 4))]),
    ("cg beta inverted", "beta = rho_new / rho;", "beta = rho / rho_new;",
     [lambda: S.test_cg_matches_dense_lu(S.inputs.poisson7_csr, (6, 5, 4))]),
    ("cg direction update drops r", "for (i = 0; i < n; i++) p[i] = fma(beta, p[i], r[i]);",
     "for (i = 0; i < n; i++) p[i] = beta * p[i];",
     [lambda: S.test_cg_finite_termination(3, 7)]),
    ("cgnb update sign as printed", "x[i] = fma(gamma, p[i], fma(-gamma, r[i], x[i]));",
     "x[i] = fma(-gamma, p[i], fma(gamma, r[i], x[i]));",
     [lambda: S.test_cgnb_matches_dense_lu(S.inputs.poisson7_csr, (6, 5, 4))]),
    ("cgnb recurrence drops beta", "ap[i] = fma(beta, ap[i], w[i]);", "ap[i] = w[i];",
     [lambda: S.test_cgnb_finite_termination(3, 7)]),
    ("bicgstab omega term dropped", "x[i] = fma(omega, s[i], fma(alpha, p[i], x[i]));",
     "x[i] = fma(alpha, p[i], x[i]);",
     [lambda: S.test_bicgstab_matches_dense_lu_upwind((5, 5, 5))]),
    ("bicgstab beta missing omega", "double bet = an_new / (alpha_d * omega);",
     "double bet = an_new / alpha_d;",
     [lambda: S.test_bicgstab_finite_termination_upwind(3, 7)]),
    ("bicgstab shadow not renormalised on restart", "rs[i] = r[i] / rnorm;\n      }\n      alpha_n = rnorm;",
     "}\n      alpha_n = rnorm;",
     [S.test_bicgstab_restart_paths]),
    ("jacobi updates in place", "xb[i] = relax_row(rp, col, val, b, xa, i, dpos[i]);",
     "xa[i] = relax_row(rp, col, val, b, xa, i, dpos[i]); xb[i] = xa[i];",
     [lambda: S.test_jacobi_damps_slowest_mode_by_cos_pi_h(7)]),
    ("sgs backward sweep runs forward", "for (c = ncolors - 1; c >= 0; c--) /* backward sweep */",
     "for (c = 0; c < ncolors; c++) /* backward sweep */",
     [lambda: S.test_redblack_sgs_mode_closed_form(2)]),
    ("dot drops product error", "acc_add(&a, fma(x[i], y[i], -p));", "(void)0;",
     [K.test_dot_products_split_exactly]),
    ("dot without tie correction", "if (y == x - hi) hi = x;", "(void)x;",
     [K.test_dot_half_way_cases]),
    ("spmv reversed order", "for (k = rp[i]; k < rp[i + 1]; k++) acc = fma(val[k], x[col[k]], acc);",
     "for (k = rp[i + 1] - 1; k >= rp[i]; k--) acc = fma(val[k], x[col[k]], acc);",
     [K.test_spmv_is_an_fma_chain_in_stored_order]),
    ("spmv_f32 accumulates in double",
     "    float acc = 0.0f;\n    for (k = rp[i]; k < rp[i + 1]; k++) acc = fmaf(val[k], x[col[k]], acc);\n    y[i] = acc;",
     "    double acc = 0.0;\n    for (k = rp[i]; k < rp[i + 1]; k++) acc = fma((double)val[k], (double)x[col[k]], acc);\n    y[i] = (float)acc;",
     [K.test_spmv_f32_is_an_fp32_fma_chain_in_stored_order]),
    ("spmv_f32 rounds each product",
     "for (k = rp[i]; k < rp[i + 1]; k++) acc = fmaf(val[k], x[col[k]], acc);",
     "for (k = rp[i]; k < rp[i + 1]; k++) acc = val[k] * x[col[k]] + acc;",
     [K.test_spmv_f32_is_an_fp32_fma_chain_in_stored_order]),
    ("spmv_f32 reversed order",
     "for (k = rp[i]; k < rp[i + 1]; k++) acc = fmaf(val[k], x[col[k]], acc);",
     "for (k = rp[i + 1] - 1; k >= rp[i]; k--) acc = fmaf(val[k], x[col[k]], acc);",
     [K.test_spmv_f32_is_an_fp32_fma_chain_in_stored_order]),
    ("ir update unscaled", "x[i] = fma(rn, (double)d[i], x[i]);", "x[i] = x[i] + (double)d[i];",
     [lambda: S.test_ir_cg_reaches_fp64_accuracy(S.np.float32)]),
    ("varcoef face arithmetic mean", "return (2.0 * a * b) / (a + b);", "return 0.5 * (a + b);",
     [lambda: V.test_operator_matches_face_flux_assembly((3, 3, 3))]),
    ("varcoef boundary face doubled", "        f[o] = k[i];\n", "        f[o] = 2.0 * k[i];\n",
     [V.test_unit_coefficients_give_the_poisson_matrix,
      lambda: V.test_operator_matches_face_flux_assembly((4, 3, 2))]),
    ("varcoef gradient drops the square", "const double d = (2.0 * k[m] * k[m]) / (s * s);",
     "const double d = (2.0 * k[m]) / s;",
     [lambda: V.test_gradient_matches_central_differences((3, 3, 2))]),
    ("varcoef gradient drops boundary faces", "term = lam[i] * x[i];", "term = 0.0;",
     [lambda: V.test_gradient_matches_central_differences((3, 3, 2))]),
    ("varcoef gradient sign", "dk[i] = -acc;", "dk[i] = acc;",
     [lambda: V.test_gradient_matches_central_differences((4, 2, 3))]),
]


@pytest.mark.parametrize("name,old,new,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_catches_mutant(tmp_path, name, old, new, pins):
    src = open(SRC).read()
    assert src.count(old) == 1, f"fragment for '{name}' not found exactly once"
    mut = tmp_path / "oracle_mut.c"
    mut.write_text(src.replace(old, new))
    so = obuild.build(source=str(mut), out=str(tmp_path / "liboracle_mut.so"))
    prev = oracle.use_library(oracle.load(so))
    try:
        for pin in pins:
            with pytest.raises(AssertionError):
                pin()
    finally:
        oracle.use_library(prev)
