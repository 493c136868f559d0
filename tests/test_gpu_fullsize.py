"""GPU parity at the benchmark workloads' full sizes and launch
configurations: a few fixed iterations of each method on the full-size
matrix, compared with the oracle over every row (or, for the batch, over
sampled systems).  The iterates are expected bit for bit, as at small
sizes; each case prints its name before it starts."""
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
    print(f"full size: {msg}", flush=True)


@pytest.fixture(scope="module")
def poisson256():
    say("building the 256^3 Poisson CSR matrix")
    Acsr = inputs.poisson7_csr(256)
    A = its().CSRMatrix.from_numpy(*Acsr, validate=False, pack=True)
    xs = inputs.uniform_vector(Acsr[0].size - 1, 1)
    b = oracle.spmv(Acsr, xs)
    return Acsr, A, b


def test_full_size_jacobi_256(poisson256):
    Acsr, A, b = poisson256
    say("Jacobi, 2 sweeps, 256^3 packed CSR")
    ref, rr = oracle.jacobi(Acsr, b, rtol=0.0, max_iter=2)
    x, info = its().solve(A, dev(b), method="jacobi", rtol=0.0, max_iter=2)
    assert info.iters == rr.iters == 2
    assert np.array_equal(host(x), ref)
    assert abs(info.rel_res - rr.rel_res) <= 1e-12 * rr.rel_res


def test_full_size_redblack_sgs_256(poisson256):
    Acsr, A, b = poisson256
    say("red-black SGS, 2 iterations, 256^3 packed CSR with colour packs")
    col = inputs.redblack_colors(256, 256, 256)
    A.set_colors(col, 2)
    ref, rr = oracle.sgs(Acsr, col, 2, b, rtol=0.0, max_iter=2)
    x, info = its().solve(A, dev(b), method="sgs", rtol=0.0, max_iter=2)
    assert info.iters == rr.iters == 2
    assert np.array_equal(host(x), ref)
    assert abs(info.rel_res - rr.rel_res) <= 1e-12 * rr.rel_res


def test_full_size_bicgstab_192_convdiff():
    say("BiCGStab, 3 iterations, 192^3 upwind convection-diffusion, packed CSR")
    Acsr = inputs.convdiff7_csr(192)
    A = its().CSRMatrix.from_numpy(*Acsr, validate=False, pack=True)
    b = oracle.spmv(Acsr, inputs.uniform_vector(Acsr[0].size - 1, 1))
    ref, rr = oracle.bicgstab(Acsr, b, rtol=0.0, max_iter=3)
    x, info = its().solve(A, dev(b), method="bicgstab", rtol=0.0, max_iter=3)
    assert info.iters == rr.iters == 3
    assert np.array_equal(host(x), ref)


@pytest.mark.parametrize("lowp", ["f32", "f16"])
def test_full_size_ir_27pt_192(lowp):
    say(f"mixed-precision refinement ({lowp} values), 3 inner iterations, 27-point 192^3")
    Acsr = inputs.stencil27_csr(192)
    A = its().CSRMatrix.from_numpy(*Acsr, validate=False, lowp=(lowp,), pack=True)
    b = oracle.spmv(Acsr, inputs.uniform_vector(Acsr[0].size - 1, 1))
    lo = Acsr[2].astype(np.float32 if lowp == "f32" else np.float16)
    ref, rr = oracle.ir_cg(Acsr, lo, b, rtol=1e-10, max_iter=3, inner_rtol=1e-4)
    x, info = its().solve(A, dev(b), method="cg", rtol=1e-10, max_iter=3, inner_dtype=lowp,
                          inner_rtol=1e-4)
    assert info.status == "not_converged" and rr.status == oracle.NOT_CONVERGED
    assert info.iters == rr.iters and info.inner_iters == rr.inner_iters == 3
    assert np.array_equal(host(x), ref)


@pytest.mark.parametrize("lowp", ["f32", "f16"])
def test_ir_7pt_blocks_walk_several_tiles(lowp):
    # 128 x 151 x 211 rows: x-lines of two whole slices, so every slice is an
    # offset slice; 15931 tiles over 4096 blocks, so blocks walk three or
    # four tiles (both ends of the two-tile loop), and the last tile holds
    # two slices (the other two lie past the last row)
    g = (128, 151, 211)
    say(f"mixed-precision refinement ({lowp} values), 3 inner iterations, 7-point {g}")
    Acsr = inputs.poisson7_csr(*g)
    A = its().CSRMatrix.from_numpy(*Acsr, validate=False, lowp=(lowp,), pack=True)
    assert A.packed_column_slots == 0  # every slice an offset slice
    b = oracle.spmv(Acsr, inputs.uniform_vector(Acsr[0].size - 1, 4))
    lo = Acsr[2].astype(np.float32 if lowp == "f32" else np.float16)
    for k in (1, 3):
        ref, rr = oracle.ir_cg(Acsr, lo, b, rtol=1e-10, max_iter=k, inner_rtol=1e-4)
        x, info = its().solve(A, dev(b), method="cg", rtol=1e-10, max_iter=k, inner_dtype=lowp,
                              inner_rtol=1e-4)
        assert info.inner_iters == rr.inner_iters == k
        assert np.array_equal(host(x), ref)


def test_full_size_varcoef_128():
    say("variable-coefficient CG, 2 iterations, and the gradient kernel, 128^3")
    g = (128, 128, 128)
    n = 128 ** 3
    k = inputs.diffusion_coefficients(inputs.gaussian_field(n, 3))
    A = its().VarCoefMatrix(*g, dev(k))
    Acsr = oracle.varcoef_csr(*g, k)
    b = inputs.uniform_vector(n, 1)
    ref, rr = oracle.cg(Acsr, b, rtol=0.0, max_iter=2)
    x, info = its().solve(A, dev(b), method="cg", rtol=0.0, max_iter=2)
    xg = host(x)
    assert info.iters == rr.iters == 2 and np.array_equal(xg, ref)
    lam = inputs.uniform_vector(n, 2)
    dk = its().varcoef_grad(A, dev(xg), dev(lam))
    assert np.array_equal(host(dk), oracle.varcoef_grad(*g, k, xg, lam))


def test_full_size_batch_512x8_sampled():
    say("batched CG, 512 systems x 8 right-hand sides, 2 iterations; systems 0, 137, 511 "
        "against the oracle")
    nsys, nrhs = 512, 8
    dims, k, b = inputs.batch_systems(nsys, nrhs, seed=4)
    B = its().Batch(dims, dev(k), nrhs)
    x, info = B.solve(dev(b.ravel()), rtol=0.0, max_iter=2)
    assert np.all(info.iters == 2)
    xg = host(x).reshape(-1, nrhs)
    n_s = np.prod(dims.astype(np.int64), axis=1)
    off = np.concatenate([[0], np.cumsum(n_s)])
    for s in (0, 137, 511):
        Acsr = oracle.varcoef_csr(*[int(v) for v in dims[s]], k[off[s]:off[s + 1]])
        for r in range(nrhs):
            ref, rr = oracle.cg(Acsr, b[off[s]:off[s + 1], r], rtol=0.0, max_iter=2)
            assert np.array_equal(xg[off[s]:off[s + 1], r], ref), (s, r)
