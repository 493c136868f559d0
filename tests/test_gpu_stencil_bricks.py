"""The matrix-free stencil sweep at the brick plans its full-size workloads
run: several 64-point x tiles (halos between tiles), bricks of many z planes
(the z+2 prefetch and the four rotating LDS plane slots), and a last brick
shorter than the others.  Each test asserts the plan first, so it provably
reaches those paths, then compares with the oracle on the CSR form of the
same operator: SpMV, Jacobi and Gauss-Seidel bit for bit, CG and BiCGStab
iterates to 0 ulps (the scalars are correctly rounded dots).  Each case
prints its name before it starts."""
import numpy as np
import pytest

import oracle
from paper_2305_05988_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def its():
    import paper_2305_05988_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def say(msg):
    print(f"stencil bricks: {msg}", flush=True)


def expected_plan(nx, ny, nz, target_first=4096, target_second=2048, min_planes=16):
    """The sweep's plan restated: 64 x 4 tiles; z cut into chunks for about
    4096 bricks while a chunk keeps at least 16 planes, else about 2048."""
    nbx, nby = -(-nx // 64), -(-ny // 4)
    nxy = nbx * nby

    def zb_for(target):
        chunks = max(1, min(nz, -(-target // nxy)))
        return max(1, -(-nz // chunks))
    zb = zb_for(target_first)
    if zb < min_planes:
        zb = zb_for(target_second)
    return nbx, nby, -(-nz // zb), zb


# ---------------------------------------------------------------- 256^3, 7 points

@pytest.fixture(scope="module")
def poisson256():
    say("building the 256^3 Poisson CSR matrix and the matrix-free operator")
    g = (256, 256, 256)
    Acsr = inputs.poisson7_csr(*g)
    S = its().StencilMatrix(*g, inputs.POISSON7)
    xs = inputs.uniform_vector(S.n, 1)
    b = oracle.spmv(Acsr, xs)
    return Acsr, S, xs, b


def test_plan_256_poisson(poisson256):
    _, S, _, _ = poisson256
    assert S.plan == (4, 64, 16, 16) == expected_plan(256, 256, 256)


def test_spmv_256_poisson(poisson256):
    Acsr, S, xs, b = poisson256
    say("SpMV, 256^3 7-point (4 x tiles, 16-plane bricks)")
    assert np.array_equal(host(its().spmv(S, dev(xs))), b)


def test_cg_256_poisson(poisson256):
    Acsr, S, _, b = poisson256
    say("CG, 3 iterations, 256^3 7-point")
    ref, rr = oracle.cg(Acsr, b, rtol=0.0, max_iter=3)
    x, info = its().solve(S, dev(b), method="cg", rtol=0.0, max_iter=3)
    assert info.iters == rr.iters == 3
    assert np.array_equal(host(x), ref)
    assert abs(info.rel_res - rr.rel_res) <= 1e-12 * rr.rel_res


def test_jacobi_256_poisson(poisson256):
    Acsr, S, _, b = poisson256
    say("Jacobi, 2 sweeps, 256^3 7-point")
    ref, rr = oracle.jacobi(Acsr, b, rtol=0.0, max_iter=2)
    x, info = its().solve(S, dev(b), method="jacobi", rtol=0.0, max_iter=2)
    assert info.iters == rr.iters == 2
    assert np.array_equal(host(x), ref)
    assert abs(info.rel_res - rr.rel_res) <= 1e-12 * rr.rel_res


def test_redblack_sgs_256_poisson(poisson256):
    Acsr, S, _, b = poisson256
    say("red-black SGS, 2 iterations, 256^3 7-point (residual pass on the bricks)")
    col = inputs.redblack_colors(256, 256, 256)
    ref, rr = oracle.sgs(Acsr, col, 2, b, rtol=0.0, max_iter=2)
    x, info = its().solve(S, dev(b), method="sgs", rtol=0.0, max_iter=2)
    assert info.iters == rr.iters == 2
    assert np.array_equal(host(x), ref)
    assert abs(info.rel_res - rr.rel_res) <= 1e-12 * rr.rel_res


# ------------------------------------------------------------- 192^3, 27 points

def test_stencil27_192():
    g = (192, 192, 192)
    S = its().StencilMatrix(*g, inputs.STENCIL27)
    assert S.plan == (3, 48, 15, 13) == expected_plan(*g)  # last chunk: 10 planes
    say("building the 192^3 27-point CSR matrix")
    Acsr = inputs.stencil27_csr(*g)
    xs = inputs.uniform_vector(S.n, 1)
    b = oracle.spmv(Acsr, xs)
    say("SpMV and CG (2 iterations), 192^3 27-point (3 x tiles, 13-plane bricks)")
    assert np.array_equal(host(its().spmv(S, dev(xs))), b)
    ref, rr = oracle.cg(Acsr, b, rtol=0.0, max_iter=2)
    x, info = its().solve(S, dev(b), method="cg", rtol=0.0, max_iter=2)
    assert info.iters == rr.iters == 2
    assert np.array_equal(host(x), ref)


# --------------------------------------------- 96^3 upwind, transposed BiCGStab

def test_transposed_bicgstab_96_upwind():
    g = (96, 96, 96)
    c = inputs.convdiff7()
    S = its().StencilMatrix(*g, c)
    assert S.plan == (2, 24, 32, 3) == expected_plan(*g)
    At = inputs.stencil_csr(*g, tuple(reversed(c)))
    b = inputs.uniform_vector(S.n, 2)
    say("BiCGStab with A^T, 3 iterations, 96^3 upwind (2 x tiles, 3-plane bricks)")
    ref, rr = oracle.bicgstab(At, b, rtol=0.0, max_iter=3)
    x, info = its().solve(S, dev(b), method="bicgstab", rtol=0.0, max_iter=3, transpose=True)
    assert info.iters == rr.iters == 3
    assert np.array_equal(host(x), ref)


# ------------------------------------------- ragged tiles and a one-plane brick

RAGGED = (130, 64, 100)  # 3 x tiles (the last 2 points wide), last brick 1 plane


@pytest.mark.parametrize("kind", ["poisson7", "stencil27", "convdiff7"])
def test_ragged_bricks_spmv_and_jacobi(kind):
    coef = {"poisson7": inputs.POISSON7, "stencil27": inputs.STENCIL27,
            "convdiff7": inputs.convdiff7()}[kind]
    S = its().StencilMatrix(*RAGGED, coef)
    assert S.plan == (3, 16, 34, 3) == expected_plan(*RAGGED)
    Acsr = inputs.stencil_csr(*RAGGED, coef)
    x = inputs.uniform_vector(S.n, 7)
    say(f"SpMV and Jacobi (2 sweeps), {RAGGED} {kind}")
    assert np.array_equal(host(its().spmv(S, dev(x))), oracle.spmv(Acsr, x))
    b = oracle.spmv(Acsr, inputs.uniform_vector(S.n, 1))
    ref, rr = oracle.jacobi(Acsr, b, rtol=0.0, max_iter=2)
    xj, info = its().solve(S, dev(b), method="jacobi", rtol=0.0, max_iter=2)
    assert info.iters == rr.iters == 2 and np.array_equal(host(xj), ref)


@pytest.mark.parametrize("kind,method,k", [("poisson7", "cg", 3), ("stencil27", "cg", 3),
                                           ("poisson7", "cgnb", 3), ("convdiff7", "bicgstab", 3),
                                           ("poisson7", "sgs", 2), ("stencil27", "sgs", 2)])
def test_ragged_bricks_solvers(kind, method, k):
    coef = {"poisson7": inputs.POISSON7, "stencil27": inputs.STENCIL27,
            "convdiff7": inputs.convdiff7()}[kind]
    S = its().StencilMatrix(*RAGGED, coef)
    Acsr = inputs.stencil_csr(*RAGGED, coef)
    b = oracle.spmv(Acsr, inputs.uniform_vector(S.n, 1))
    say(f"{method}, {k} iterations, {RAGGED} {kind}")
    if method == "sgs":
        if kind == "poisson7":
            col, nc = inputs.redblack_colors(*RAGGED), 2
        else:
            col, nc = inputs.octant_colors(*RAGGED), 8
        ref, rr = oracle.sgs(Acsr, col, nc, b, rtol=0.0, max_iter=k)
    else:
        ref, rr = getattr(oracle, method)(Acsr, b, rtol=0.0, max_iter=k)
    x, info = its().solve(S, dev(b), method=method, rtol=0.0, max_iter=k)
    assert info.iters == rr.iters == k
    assert np.array_equal(host(x), ref)
    assert abs(info.rel_res - rr.rel_res) <= 1e-12 * rr.rel_res


# ------------------------------------------ converged BiCGStab with restarts

@pytest.mark.parametrize("form", ["stencil", "packed_csr"])
def test_converged_bicgstab_64_upwind_with_restarts(form):
    g = (64, 64, 64)
    Acsr = inputs.convdiff7_csr(*g)
    if form == "stencil":
        A = its().StencilMatrix(*g, inputs.convdiff7())
        assert A.plan == expected_plan(*g)
    else:
        A = its().CSRMatrix.from_numpy(*Acsr, pack=True)
    b = oracle.spmv(Acsr, inputs.uniform_vector(A.n, 1))
    say(f"BiCGStab to 1e-8, 64^3 upwind ({form}); the oracle restarts several times")
    ref, rr = oracle.bicgstab(Acsr, b, rtol=1e-8, max_iter=2000)
    assert rr.restarts >= 3
    x, info = its().solve(A, dev(b), method="bicgstab", rtol=1e-8, max_iter=2000)
    assert info.status == "ok"
    assert info.iters == rr.iters and info.restarts == rr.restarts
    assert np.array_equal(host(x), ref)
