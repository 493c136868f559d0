"""The paper's one-node iteration counts (Sec. 4.1: a 128 x 128 x 6144 grid,
b = A 1, x0 = 0, stop when ||r||_2 < 1e-6, BiCGStab restart threshold 1e-5)
reproduced under the reading that its matrix carries 27 on the diagonal and
-1 on every neighbour, for the 7- and the 27-point stencil alike.

CG and BiCGStab land two iterations below the printed counts on both
stencils (the paper does not say how it counts; its loops test at the top
of an iteration); Jacobi and symmetric Gauss-Seidel match exactly on the
7-point stencil.  The 27-point
Jacobi and Gauss-Seidel counts are not asserted: the paper's Gauss-Seidel
ordering is not the eight-colour one used here, and its Jacobi test is not
stated.  HPCG's (26, -1) operator, the other reading, needs several times
the printed CG count, which is what rules it out."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GRID = (128, 128, 6144)


def its():
    import paper_2305_05988_amd as m
    return m


def counts(npts, diag, methods):
    from paper_2305_05988_amd import inputs
    print(f"paper counts: {npts}-point stencil, diagonal {diag:g}, {GRID}", flush=True)
    offs = inputs.OFFSETS7 if npts == 7 else inputs.OFFSETS27
    S = its().StencilMatrix(*GRID, [diag if o == (0, 0, 0) else -1.0 for o in offs])
    b = its().spmv(S, torch.ones(S.n, dtype=torch.float64, device="cuda"))
    rtol = 1e-6 / its().dot(b, b) ** 0.5
    out = {}
    for m in methods:
        kw = dict(method=m, rtol=rtol, max_iter=2000)
        if m == "bicgstab":
            kw.update(restart_mode="paper", restart_tol=1e-5)
        x, info = its().solve(S, b, **kw)
        assert info.status == "ok", (m, info)
        out[m] = info.iters
    return out


def test_paper_counts_7pt():
    c = counts(7, 27.0, ("cg", "bicgstab", "sgs", "jacobi"))
    assert c["jacobi"] == 18 and c["sgs"] == 9, c
    assert 12 - 2 <= c["cg"] <= 12 and 8 - 2 <= c["bicgstab"] <= 8, c


def test_paper_counts_27pt():
    c = counts(27, 27.0, ("cg", "bicgstab"))
    assert 72 - 2 <= c["cg"] <= 72 and 45 - 2 <= c["bicgstab"] <= 45, c


def test_hpcg_operator_does_not_fit_the_counts():
    c = counts(27, 26.0, ("cg",))
    assert c["cg"] > 5 * 72, c
