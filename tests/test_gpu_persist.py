"""The persistent solver kernels (one cooperative launch per solve, grid
barriers instead of kernel boundaries; CG, the paper's CG-NB and BiCGStab
with B1's split-phase barriers) against the oracle: iterates bit for bit at
fixed iteration counts and converged, on every operator form; identical to
the launch-per-pass schedule; status paths (breakdowns, b = 0, max_iter 0);
and a barrier wait forced to give up from the host, after which every block
has left the kernel and the next solve is normal."""
import os

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
    print(f"persistent: {msg}", flush=True)


def _matrix(kind, g):
    if kind == "csr7":
        Acsr = inputs.poisson7_csr(*g)
        return Acsr, its().CSRMatrix.from_numpy(*Acsr)
    if kind == "csr7p":
        Acsr = inputs.poisson7_csr(*g)
        return Acsr, its().CSRMatrix.from_numpy(*Acsr, pack=True, max_fill=2.0)
    if kind == "csr27p":
        Acsr = inputs.stencil27_csr(*g)
        return Acsr, its().CSRMatrix.from_numpy(*Acsr, pack=True, max_fill=2.0)
    if kind == "sten7":
        return inputs.poisson7_csr(*g), its().StencilMatrix(*g, inputs.POISSON7)
    if kind == "sten27":
        return inputs.stencil27_csr(*g), its().StencilMatrix(*g, inputs.STENCIL27)
    if kind == "csrcdp":
        Acsr = inputs.convdiff7_csr(*g)
        return Acsr, its().CSRMatrix.from_numpy(*Acsr, pack=True, max_fill=2.0)
    if kind == "stencd":
        return inputs.convdiff7_csr(*g), its().StencilMatrix(*g, inputs.convdiff7())
    if kind == "var7":
        n = int(np.prod(g))
        k = inputs.diffusion_coefficients(inputs.gaussian_field(n, 21))
        return oracle.varcoef_csr(*g, k), its().VarCoefMatrix(*g, dev(k))
    raise KeyError(kind)


def _rhs(Acsr, seed=1):
    return oracle.spmv(Acsr, inputs.uniform_vector(Acsr[0].size - 1, seed))


SYMMETRIC = ["csr7", "csr7p", "csr27p", "sten7", "sten27", "var7"]
NONSYMMETRIC = ["csrcdp", "stencd"]
GRID = (19, 13, 11)


@pytest.mark.parametrize("kind", SYMMETRIC)
@pytest.mark.parametrize("method", ["cg", "cgnb"])
@pytest.mark.parametrize("k", [1, 2, 9])
def test_fixed_k_bit_exact(kind, method, k):
    Acsr, A = _matrix(kind, GRID)
    b = _rhs(Acsr)
    ref, rr = getattr(oracle, method)(Acsr, b, rtol=0.0, max_iter=k)
    x, info = its().solve(A, dev(b), method=method, rtol=0.0, max_iter=k, persistent=True)
    assert info.status == "not_converged" and info.iters == rr.iters == k
    assert np.array_equal(host(x), ref)
    assert abs(info.rel_res - rr.rel_res) <= 1e-12 * rr.rel_res


@pytest.mark.parametrize("kind", NONSYMMETRIC + ["sten7"])
@pytest.mark.parametrize("k", [1, 2, 9])
def test_bicgstab_fixed_k_bit_exact(kind, k):
    Acsr, A = _matrix(kind, GRID)
    b = _rhs(Acsr)
    ref, rr = oracle.bicgstab(Acsr, b, rtol=0.0, max_iter=k)
    x, info = its().solve(A, dev(b), method="bicgstab", rtol=0.0, max_iter=k, persistent=True)
    assert info.iters == rr.iters == k
    assert np.array_equal(host(x), ref)


@pytest.mark.parametrize("kind", ["csr7p", "sten7", "csr7"])
@pytest.mark.parametrize("method", ["cg", "cgnb", "bicgstab"])
def test_converged_32cube(kind, method):
    say(f"{method} to 1e-8, 32^3 {kind}")
    Acsr, A = _matrix(kind, (32, 32, 32))
    b = _rhs(Acsr)
    ref, rr = getattr(oracle, method)(Acsr, b, rtol=1e-8, max_iter=5000)
    x, info = its().solve(A, dev(b), method=method, rtol=1e-8, max_iter=5000, persistent=True)
    assert rr.status == oracle.OK and info.status == "ok"
    assert info.iters == rr.iters
    assert np.array_equal(host(x), ref)
    assert abs(info.true_rel_res - rr.true_rel_res) <= 1e-6 * rr.true_rel_res


@pytest.mark.parametrize("method", ["cg", "cgnb", "bicgstab"])
def test_same_bits_as_launch_per_pass(method):
    Acsr, A = _matrix("csr27p", (40, 36, 30))  # several tiles per block
    b = _rhs(Acsr, seed=3)
    x1, i1 = its().solve(A, dev(b), method=method, rtol=1e-9, max_iter=3000)
    x2, i2 = its().solve(A, dev(b), method=method, rtol=1e-9, max_iter=3000, persistent=True)
    assert i1.status == i2.status == "ok" and i1.iters == i2.iters
    assert torch.equal(x1, x2)


@pytest.mark.parametrize("split", ["1", "0"])
@pytest.mark.parametrize("mode,tol", [("cosine", 0.9), ("paper", 30.0)])
def test_bicgstab_restarts_both_schedules(monkeypatch, split, mode, tol):
    monkeypatch.setenv("ITS_BICGSTAB_SPLIT", split)
    Acsr, A = _matrix("csrcdp", (14, 12, 10))
    b = _rhs(Acsr, seed=8)
    rm = oracle.RESTART_COSINE if mode == "cosine" else oracle.RESTART_PAPER
    ref, rr = oracle.bicgstab(Acsr, b, rtol=1e-10, max_iter=2000, restart_tol=tol, restart_mode=rm)
    x, info = its().solve(A, dev(b), method="bicgstab", rtol=1e-10, max_iter=2000,
                          restart_tol=tol, restart_mode=mode, persistent=True)
    assert rr.restarts > 0 and info.restarts == rr.restarts and info.iters == rr.iters
    assert np.array_equal(host(x), ref)


def test_transposed_bicgstab():
    g = (18, 11, 9)
    c = inputs.convdiff7()
    At = inputs.stencil_csr(*g, tuple(reversed(c)))
    S = its().StencilMatrix(*g, c)
    b = inputs.uniform_vector(S.n, 2)
    ref, rr = oracle.bicgstab(At, b, rtol=0.0, max_iter=6)
    x, info = its().solve(S, dev(b), method="bicgstab", rtol=0.0, max_iter=6, transpose=True,
                          persistent=True)
    assert info.iters == rr.iters == 6 and np.array_equal(host(x), ref)


@pytest.mark.parametrize("method", ["cg", "cgnb", "bicgstab"])
def test_status_paths(method):
    S = its().StencilMatrix(5, 4, 3, inputs.POISSON7)
    z = torch.zeros(60, dtype=torch.float64, device="cuda")
    x, info = its().solve(S, z, x0=torch.ones_like(z), method=method, persistent=True)
    assert info.status == "ok" and info.iters == 0 and not host(x).any()
    Acsr, A = _matrix("sten7", (6, 5, 4))
    x, info = its().solve(A, dev(_rhs(Acsr)), method=method, max_iter=0, persistent=True)
    assert info.status == "not_converged" and info.iters == 0 and not host(x).any()
    A1 = its().CSRMatrix.from_numpy(np.array([0, 1]), np.array([0]), np.array([4.0]), pack=True)
    x, info = its().solve(A1, dev(np.array([3.0])), method=method, rtol=1e-14, max_iter=10,
                          persistent=True)
    assert info.status == "ok" and host(x)[0] == 0.75


def test_breakdowns():
    A = its().CSRMatrix.from_numpy(np.array([0, 1, 2]), np.array([0, 1]), np.array([1.0, -1.0]))
    x, info = its().solve(A, dev(np.array([1.0, 1.0])), method="cg", persistent=True)
    assert info.status == "breakdown" and info.iters == 0
    B = its().CSRMatrix.from_numpy(np.array([0, 1, 2]), np.array([1, 0]), np.array([1.0, 1.0]))
    x, info = its().solve(B, dev(np.array([1.0, 0.0])), method="bicgstab", persistent=True)
    assert info.status == "breakdown" and info.iters == 0


def test_other_methods_refuse_persistent():
    S = its().StencilMatrix(5, 4, 3, inputs.POISSON7)
    b = torch.ones(60, dtype=torch.float64, device="cuda")
    for kw in (dict(method="jacobi"), dict(method="sgs"), dict(method="cg", inner_dtype="f32")):
        with pytest.raises(its().ItsError) as e:
            its().solve(S, b, persistent=True, **kw)
        assert e.value.status == -4


def test_barrier_give_up_forced_from_host(monkeypatch):
    # every barrier waits for one more block than was launched, so no wait
    # can complete: each block polls 2000 times, gives up and leaves
    Acsr, A = _matrix("sten7", (24, 24, 24))
    b = dev(_rhs(Acsr))
    monkeypatch.setenv("ITS_BARRIER_TEST_EXTRA", "1")
    monkeypatch.setenv("ITS_BARRIER_SPIN_LIMIT", "2000")
    for method in ("cg", "cgnb", "bicgstab"):
        with pytest.raises(its().ItsError) as e:
            its().solve(A, b, method=method, rtol=1e-8, max_iter=100, persistent=True)
        assert e.value.status == -2 and "gave up" in str(e.value)
    monkeypatch.delenv("ITS_BARRIER_TEST_EXTRA")
    monkeypatch.delenv("ITS_BARRIER_SPIN_LIMIT")
    ref, rr = oracle.cg(Acsr, host(b), rtol=1e-8, max_iter=100)
    x, info = its().solve(A, b, method="cg", rtol=1e-8, max_iter=100, persistent=True)
    assert info.status == "ok" and info.iters == rr.iters and np.array_equal(host(x), ref)


@pytest.mark.parametrize("blocks", ["8", "64", "1000"])
def test_block_counts(monkeypatch, blocks):
    monkeypatch.setenv("ITS_PERSISTENT_BLOCKS", blocks)
    Acsr, A = _matrix("csr7p", (40, 40, 40))
    b = _rhs(Acsr)
    ref, rr = oracle.cgnb(Acsr, b, rtol=0.0, max_iter=5)
    x, info = its().solve(A, dev(b), method="cgnb", rtol=0.0, max_iter=5, persistent=True)
    assert info.iters == 5 and np.array_equal(host(x), ref)
