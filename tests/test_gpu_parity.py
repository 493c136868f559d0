"""GPU parity: the HIP path through the C ABI against the oracle on the same
seeded inputs.

Bars: SpMV, Jacobi and Gauss-Seidel iterates bit-exact (identical fma chains
and IEEE division); dot products equal to the correctly rounded value
(double-double accumulation); CG and BiCGStab iterates within 1e-10
relative of the oracle with iteration counts within +-1 (the scalars come
from the same correctly rounded dots, so the iterates are expected to match
bit for bit, and the tests report the largest difference in ulps).
"""
import numpy as np
import pytest

import oracle
from paper_2305_05988_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def its():
    import paper_2305_05988_amd as m
    return m


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def ulps(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    ia = a.view(np.int64)
    ib = b.view(np.int64)
    ia = np.where(ia < 0, np.int64(-2 ** 63) - ia, ia)
    ib = np.where(ib < 0, np.int64(-2 ** 63) - ib, ib)
    return int(np.max(np.abs(ia - ib))) if a.size else 0


def rel(a, b):
    d = np.max(np.abs(np.asarray(a) - np.asarray(b)))
    s = np.max(np.abs(b))
    return d / s if s > 0 else d


GRIDS7 = [(1, 1, 1), (5, 3, 2), (17, 9, 5), (32, 32, 32), (33, 20, 7)]


# ------------------------------------------------------------------ kernels

@pytest.mark.parametrize("n", [1, 63, 256, 257, 4099, 65536 * 3 + 17, 1 << 21])
def test_dot_is_correctly_rounded(n):
    x = inputs.uniform_vector(n, 10)
    y = inputs.uniform_vector(n, 11) * 1e3
    got = its().dot(dev(x), dev(y))
    assert got == oracle.dot(x, y)


def test_dot_under_cancellation():
    rng = np.random.default_rng(5)
    x = rng.standard_normal(100000) * 2.0 ** rng.integers(-40, 40, 100000)
    y = rng.standard_normal(100000)
    x2 = np.concatenate([x, -x, [1e-20]])
    y2 = np.concatenate([y, y, [1.0]])
    # a condition number ~1e31 is beyond double-double: the documented bound
    # n 2^-104 sum|x_i y_i| + half an ulp of the exact value applies
    got, exact = its().dot(dev(x2), dev(y2)), oracle.dot(x2, y2)
    bound = x2.size * 2.0 ** -104 * np.sum(np.abs(x2 * y2)) + 2.0 ** -53 * abs(exact)
    assert abs(got - exact) <= bound


@pytest.mark.parametrize("g", GRIDS7)
@pytest.mark.parametrize("kind", ["poisson7", "convdiff7", "stencil27"])
def test_spmv_bit_exact_csr_and_stencil(g, kind):
    gen = {"poisson7": inputs.poisson7_csr, "convdiff7": inputs.convdiff7_csr,
           "stencil27": inputs.stencil27_csr}[kind]
    coef = {"poisson7": inputs.POISSON7, "convdiff7": inputs.convdiff7(),
            "stencil27": inputs.STENCIL27}[kind]
    Acsr = gen(*g)
    n = Acsr[0].size - 1
    x = inputs.uniform_vector(n, 3)
    ref = oracle.spmv(Acsr, x)
    A = its().CSRMatrix.from_numpy(*Acsr)
    assert np.array_equal(host(its().spmv(A, dev(x))), ref)
    A.pack(max_fill=2.0)
    assert np.array_equal(host(its().spmv(A, dev(x))), ref)
    S = its().StencilMatrix(*g, coef)
    assert np.array_equal(host(its().spmv(S, dev(x))), ref)


def test_csr_int64_row_pointers_narrowed_on_device():
    import ctypes as C
    from paper_2305_05988_amd import _lib as L
    rp, col, val = inputs.poisson7_csr(17, 9, 5)
    assert rp.dtype == np.int64
    n, nnz = rp.size - 1, col.size
    x = inputs.uniform_vector(n, 3)
    ref = oracle.spmv((rp, col, val), x)
    t_col, t_val = dev(col), dev(val)
    t_rp64 = dev(rp)
    h = C.c_void_p()
    lib = L.lib()
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.its_csr_create64(n, nnz, C.c_void_p(t_rp64.data_ptr()), C.c_void_p(t_col.data_ptr()),
                                C.c_void_p(t_val.data_ptr()), s, C.byref(h)) == L.ITS_OK
    del t_rp64  # the handle holds its own narrowed copy
    torch.cuda.synchronize()
    try:
        assert lib.its_csr_validate(h, 1, s) == L.ITS_OK
        xd, yd = dev(x), torch.empty(n, dtype=torch.float64, device="cuda")
        assert lib.its_spmv(h, C.c_void_p(xd.data_ptr()), C.c_void_p(yd.data_ptr()), s) == L.ITS_OK
        assert np.array_equal(host(yd), ref)
    finally:
        lib.its_matrix_destroy(h)
    # through the binding, packed, and a row pointer out of range refused
    A = its().CSRMatrix(dev(rp), t_col, t_val)
    A.pack(max_fill=2.0)
    assert np.array_equal(host(its().spmv(A, dev(x))), ref)
    bad = rp.copy()
    bad[3] = nnz + 1
    with pytest.raises(its().ItsError) as e:
        its().CSRMatrix(dev(bad), t_col, t_val)
    assert e.value.status == L.ITS_E_INVALID


def test_spmv_empty_and_ragged_rows():
    # rows 1 and 3 empty, ragged lengths
    rp = np.array([0, 3, 3, 4, 4, 7], np.int64)
    col = np.array([0, 2, 4, 1, 0, 3, 4], np.int32)
    val = np.array([1.5, -2.0, 0.25, 3.0, -1.0, 2.0, 0.5])
    x = inputs.uniform_vector(5, 4)
    A = its().CSRMatrix.from_numpy(rp, col, val)
    assert np.array_equal(host(its().spmv(A, dev(x))), oracle.spmv((rp, col, val), x))


def _ragged_csr(n, seed, max_len=13):
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, max_len + 1, n)
    lens[::17] = 0
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    col = np.concatenate([np.sort(rng.choice(n, size=k, replace=False)) for k in lens]
                         ).astype(np.int32) if rp[-1] else np.zeros(0, np.int32)
    val = rng.uniform(-2.0, 2.0, rp[-1])
    return rp, col, val


def _column_slots(rp, col):
    """Slots of the packed layout that keep column indices: a 64-row slice
    of width w stores none when its rows have strictly ascending columns
    whose offsets (column - row) form a set of exactly w values (w <= 32)."""
    n = rp.size - 1
    total = 0
    for s in range(0, n, 64):
        rows = range(s, min(n, s + 64))
        w = max(int(rp[i + 1] - rp[i]) for i in rows)
        if w == 0:
            continue
        offs, ok = set(), w <= 32
        for i in rows:
            c = col[rp[i]:rp[i + 1]].astype(np.int64)
            ok = ok and bool(np.all(np.diff(c) > 0))
            offs |= set((c - i).tolist())
        if not ok or len(offs) != w:
            total += 64 * w
    return total


@pytest.mark.parametrize("n,max_len", [(1, 3), (63, 9), (64, 4), (200, 13), (1000, 5), (4099, 30)])
def test_packed_layout_ragged_rows(n, max_len):
    # empty rows, rows longer than a gather group, a partial last slice
    Acsr = _ragged_csr(n, n + max_len, max_len)
    rp = Acsr[0]
    x = inputs.uniform_vector(n, 9)
    ref = oracle.spmv(Acsr, x)
    A = its().CSRMatrix.from_numpy(*Acsr)
    slots = A.pack(max_fill=4.0)
    lens = np.diff(rp)
    widths = [lens[s:s + 64].max() for s in range(0, n, 64)]
    assert slots == 64 * int(np.sum(widths))
    assert A.packed_column_slots == _column_slots(*Acsr[:2])
    assert np.array_equal(host(its().spmv(A, dev(x))), ref)


def _mixed_slices_csr():
    """A 7-point Poisson CSR on 40 x 8 x 4 (20 slices) with a few rows
    edited: rows 70 and 700 trade a neighbour for an offset no other row of
    their slice has (those slices keep columns), row 300 loses one entry and
    row 1279 (the last) loses its diagonal (both slices stay offset slices)."""
    rp, col, val = inputs.poisson7_csr(40, 8, 4)
    rows = [list(zip(col[rp[i]:rp[i + 1]].tolist(), val[rp[i]:rp[i + 1]].tolist()))
            for i in range(rp.size - 1)]

    def swap(i, old, new, v):
        r = [e for e in rows[i] if e[0] != old] + [(new, v)]
        rows[i] = sorted(r)

    swap(70, 71, 73, -0.75)
    swap(700, 699, 698, 0.5)
    rows[300] = [e for e in rows[300] if e[0] != 301]
    rows[1279] = [e for e in rows[1279] if e[0] != 1279]
    rp2 = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    col2 = np.array([c for r in rows for c, _ in r], np.int32)
    val2 = np.array([v for r in rows for _, v in r])
    return rp2, col2, val2


def test_packed_offset_and_column_slices_mixed():
    Acsr = _mixed_slices_csr()
    n = Acsr[0].size - 1
    x = inputs.uniform_vector(n, 5)
    A = its().CSRMatrix.from_numpy(*Acsr, validate=False, pack=True, max_fill=2.0)
    expect = _column_slots(*Acsr[:2])
    # the slices of row 70 (on the z = 0 face: width 6) and row 700 (width 7)
    assert 0 < expect < A.packed_slots and expect == 64 * (6 + 7)
    assert A.packed_column_slots == expect
    assert np.array_equal(host(its().spmv(A, dev(x))), oracle.spmv(Acsr, x))
    S = its().CSRMatrix.from_numpy(*inputs.poisson7_csr(40, 8, 4), pack=True, max_fill=2.0)
    assert S.packed_column_slots == 0


@pytest.mark.parametrize("lo,hi", [(15, 15), (16, 15), (16, 16)])
def test_packed_band_widths_around_offset_limit(lo, hi):
    # band rows of 31, 32 and 33 entries: offset slices hold at most 32
    n = 300
    rows = [np.arange(max(0, i - lo), min(n, i + hi + 1)) for i in range(n)]
    rp = np.concatenate([[0], np.cumsum([r.size for r in rows])]).astype(np.int64)
    col = np.concatenate(rows).astype(np.int32)
    val = inputs.uniform_vector(col.size, lo + hi)
    A = its().CSRMatrix.from_numpy(rp, col, val, pack=True, max_fill=2.0)
    expect = _column_slots(rp, col)
    assert A.packed_column_slots == expect
    assert (expect == 0) == (lo + hi + 1 <= 32)
    x = inputs.uniform_vector(n, 7)
    assert np.array_equal(host(its().spmv(A, dev(x))), oracle.spmv((rp, col, val), x))


def test_packed_mixed_slices_cg_and_bicgstab():
    Acsr = _mixed_slices_csr()
    b = oracle.spmv(Acsr, inputs.uniform_vector(Acsr[0].size - 1, 6))
    A = its().CSRMatrix.from_numpy(*Acsr, validate=False, pack=True, max_fill=2.0)
    for method, ref in (("cg", oracle.cg), ("bicgstab", oracle.bicgstab)):
        xr, rr = ref(Acsr, b, rtol=0.0, max_iter=5)
        x, info = its().solve(A, dev(b), method=method, rtol=0.0, max_iter=5)
        assert info.iters == rr.iters == 5
        assert np.array_equal(host(x), xr), method


def test_packed_layout_all_rows_empty():
    A = its().CSRMatrix.from_numpy(np.zeros(101, np.int64), np.zeros(0, np.int32), np.zeros(0))
    assert A.pack() == 0
    assert not host(its().spmv(A, dev(inputs.uniform_vector(100, 2)))).any()


def test_pack_refuses_excess_padding():
    # one dense row in the first slice: 64 * 640 slots for 1279 entries
    n = 640
    rp = np.concatenate([[0, n], n + np.arange(1, n)]).astype(np.int64)
    col = np.concatenate([np.arange(n), np.arange(1, n)]).astype(np.int32)
    val = inputs.uniform_vector(col.size, 3)
    A = its().CSRMatrix.from_numpy(rp, col, val)
    with pytest.raises(its().ItsError) as e:
        A.pack(max_fill=16.0)
    assert e.value.status == -4 and A.packed_slots == 0
    with pytest.raises(its().ItsError) as e:
        A.pack(max_fill=0.5)
    assert e.value.status == -1
    x = inputs.uniform_vector(n, 4)
    assert np.array_equal(host(its().spmv(A, dev(x))), oracle.spmv((rp, col, val), x))


def test_lowp_values_must_precede_packing():
    Acsr = inputs.poisson7_csr(4, 4, 4)
    A = its().CSRMatrix.from_numpy(*Acsr, pack=True, max_fill=2.0)
    with pytest.raises(its().ItsError):
        A.set_lowp(its().cast_values(A.val, "f32"))


def test_cast_values_round_to_nearest():
    v = np.concatenate([inputs.uniform_vector(10000, 5) * 100, [26.0, -1.0, 1 + 2 ** -11 + 2 ** -30]])
    t = dev(v)
    assert np.array_equal(host(its().cast_values(t, "f32")), v.astype(np.float32))
    assert np.array_equal(host(its().cast_values(t, "f16")), v.astype(np.float16))


def test_stream_copy():
    v = inputs.uniform_vector(1000001, 6)
    src = dev(v)
    dst = torch.empty_like(src)
    its().stream_copy(src, dst)
    assert np.array_equal(host(dst), v)


# ---------------------------------------------------------------------- CG

def _system(Acsr, seed=1):
    n = Acsr[0].size - 1
    xs = inputs.uniform_vector(n, seed)
    return xs, oracle.spmv(Acsr, xs)


def _matrix(kind, g):
    if kind.endswith("p"):  # the same CSR matrix in the packed device layout
        Acsr, A = _matrix(kind[:-1], g)
        assert A.pack(max_fill=2.0) >= Acsr[1].size
        return Acsr, A
    if kind == "csr7":
        Acsr = inputs.poisson7_csr(*g)
        return Acsr, its().CSRMatrix.from_numpy(*Acsr, lowp=("f32", "f16"))
    if kind == "sten7":
        return inputs.poisson7_csr(*g), its().StencilMatrix(*g, inputs.POISSON7)
    if kind == "csr27":
        Acsr = inputs.stencil27_csr(*g)
        return Acsr, its().CSRMatrix.from_numpy(*Acsr, lowp=("f32", "f16"))
    if kind == "sten27":
        return inputs.stencil27_csr(*g), its().StencilMatrix(*g, inputs.STENCIL27)
    if kind == "csrcd":
        Acsr = inputs.convdiff7_csr(*g)
        return Acsr, its().CSRMatrix.from_numpy(*Acsr)
    if kind == "stencd":
        return inputs.convdiff7_csr(*g), its().StencilMatrix(*g, inputs.convdiff7())
    raise KeyError(kind)


@pytest.mark.parametrize("kind", ["csr7", "sten7", "csr27", "csr7p", "csr27p"])
@pytest.mark.parametrize("k", [1, 2, 7, 40])
def test_cg_fixed_k_iterates(kind, k):
    Acsr, A = _matrix(kind, (19, 13, 11))
    xs, b = _system(Acsr)
    ref, rr = oracle.cg(Acsr, b, rtol=0.0, max_iter=k)
    x, info = its().solve(A, dev(b), method="cg", rtol=0.0, max_iter=k)
    xg = host(x)
    assert info.status == "not_converged" and info.iters == k == rr.iters
    assert rel(xg, ref) <= 1e-10, f"max ulps {ulps(xg, ref)}"
    assert ulps(xg, ref) == 0


@pytest.mark.parametrize("kind", ["csr7", "sten7", "csr7p"])
def test_cg_converged_32cube(kind):
    Acsr, A = _matrix(kind, (32, 32, 32))
    xs, b = _system(Acsr, seed=1)
    ref, rr = oracle.cg(Acsr, b, rtol=1e-8, max_iter=5000)
    x, info = its().solve(A, dev(b), method="cg", rtol=1e-8, max_iter=5000)
    xg = host(x)
    assert rr.status == oracle.OK and info.status == "ok"
    assert abs(info.iters - rr.iters) <= 1
    assert rel(xg, ref) <= 1e-10
    assert info.true_rel_res <= 1.01e-8
    print(f"CG 32^3 {kind}: iters {info.iters} (oracle {rr.iters}), max ulps {ulps(xg, ref)}")


@pytest.mark.parametrize("check_every", [1, 3, 64])
def test_cg_polling_interval_does_not_change_result(check_every):
    Acsr, A = _matrix("csr7", (16, 16, 16))
    xs, b = _system(Acsr)
    ref, rr = oracle.cg(Acsr, b, rtol=1e-9, max_iter=1000)
    x, info = its().solve(A, dev(b), method="cg", rtol=1e-9, max_iter=1000, check_every=check_every)
    assert info.iters == rr.iters and ulps(host(x), ref) == 0


def test_cg_nonzero_initial_guess():
    Acsr, A = _matrix("csr7", (12, 12, 12))
    xs, b = _system(Acsr)
    x0 = inputs.uniform_vector(xs.size, 77)
    ref, rr = oracle.cg(Acsr, b, x0=x0, rtol=1e-9, max_iter=1000)
    x, info = its().solve(A, dev(b), x0=dev(x0), method="cg", rtol=1e-9, max_iter=1000)
    assert info.iters == rr.iters and rel(host(x), ref) <= 1e-10


# ------------------------------------------------------------------ CG-NB

@pytest.mark.parametrize("kind", ["csr7", "sten7", "csr27", "csr7p"])
@pytest.mark.parametrize("k", [1, 2, 7, 40])
def test_cgnb_fixed_k_iterates(kind, k):
    Acsr, A = _matrix(kind, (19, 13, 11))
    xs, b = _system(Acsr)
    ref, rr = oracle.cgnb(Acsr, b, rtol=0.0, max_iter=k)
    x, info = its().solve(A, dev(b), method="cgnb", rtol=0.0, max_iter=k)
    xg = host(x)
    assert info.status == "not_converged" and info.iters == k == rr.iters
    assert rel(xg, ref) <= 1e-10, f"max ulps {ulps(xg, ref)}"
    assert ulps(xg, ref) == 0


@pytest.mark.parametrize("kind", ["csr7", "sten7"])
def test_cgnb_converged_32cube(kind):
    Acsr, A = _matrix(kind, (32, 32, 32))
    xs, b = _system(Acsr, seed=1)
    ref, rr = oracle.cgnb(Acsr, b, rtol=1e-8, max_iter=5000)
    x, info = its().solve(A, dev(b), method="cgnb", rtol=1e-8, max_iter=5000)
    xg = host(x)
    assert rr.status == oracle.OK and info.status == "ok"
    assert abs(info.iters - rr.iters) <= 1 and rel(xg, ref) <= 1e-10
    assert info.true_rel_res <= 1.01e-8


# ------------------------------------------------------------------ Jacobi

@pytest.mark.parametrize("kind", ["csr7", "sten7", "csrcd", "sten27", "csrcdp", "csr27p"])
@pytest.mark.parametrize("k", [0, 1, 2, 25])
def test_jacobi_fixed_k_bit_exact(kind, k):
    Acsr, A = _matrix(kind, (17, 9, 6))
    xs, b = _system(Acsr)
    ref, rr = oracle.jacobi(Acsr, b, rtol=0.0, max_iter=k)
    x, info = its().solve(A, dev(b), method="jacobi", rtol=0.0, max_iter=k)
    assert info.iters == rr.iters == k
    assert np.array_equal(host(x), ref)


def test_jacobi_32cube_cap_binds():
    # rho_J = cos(pi/33) = 0.99547: 1e-8 needs ~4000 sweeps, so the cap of
    # 2000 binds and parity is at exactly 2000 sweeps
    Acsr, A = _matrix("csr7", (32, 32, 32))
    xs, b = _system(Acsr)
    ref, rr = oracle.jacobi(Acsr, b, rtol=1e-8, max_iter=2000)
    x, info = its().solve(A, dev(b), method="jacobi", rtol=1e-8, max_iter=2000)
    assert rr.status == oracle.NOT_CONVERGED and info.status == "not_converged"
    assert info.iters == rr.iters == 2000
    assert np.array_equal(host(x), ref)


def test_jacobi_converges_upwind():
    Acsr, A = _matrix("stencd", (20, 20, 20))
    xs, b = _system(Acsr)
    ref, rr = oracle.jacobi(Acsr, b, rtol=1e-8, max_iter=500)
    x, info = its().solve(A, dev(b), method="jacobi", rtol=1e-8, max_iter=500)
    assert rr.status == oracle.OK and info.status == "ok" and info.iters == rr.iters
    assert np.array_equal(host(x), ref)


# ------------------------------------------------------------ Gauss-Seidel

@pytest.mark.parametrize("k", [1, 2, 9])
@pytest.mark.parametrize("kind", ["csr7", "sten7", "csr27", "sten27", "csr7p", "csr27p"])
def test_sgs_fixed_k_bit_exact(kind, k):
    g = (11, 7, 6)
    Acsr, A = _matrix(kind, g)
    xs, b = _system(Acsr)
    nc = 8 if "27" in kind else 2
    col = inputs.redblack_colors(*g) if nc == 2 else inputs.octant_colors(*g)
    if kind.startswith("csr"):
        A.set_colors(col, nc)
    ref, rr = oracle.sgs(Acsr, col, nc, b, rtol=0.0, max_iter=k)
    x, info = its().solve(A, dev(b), method="sgs", rtol=0.0, max_iter=k)
    assert info.iters == rr.iters == k
    assert np.array_equal(host(x), ref)
    # the residual of the returned iterate (two colours: formed inside the sweeps)
    assert abs(info.rel_res - rr.rel_res) <= 1e-12 * rr.rel_res


def test_sgs_converged_32cube_redblack():
    g = (32, 32, 32)
    Acsr, A = _matrix("csr7", g)
    xs, b = _system(Acsr)
    col = inputs.redblack_colors(*g)
    A.set_colors(col, 2)
    ref, rr = oracle.sgs(Acsr, col, 2, b, rtol=1e-8, max_iter=5000)
    x, info = its().solve(A, dev(b), method="sgs", rtol=1e-8, max_iter=5000)
    assert rr.status == oracle.OK and info.status == "ok" and info.iters == rr.iters
    assert np.array_equal(host(x), ref)
    assert abs(info.rel_res - rr.rel_res) <= 1e-12 * rr.rel_res
    S = its().StencilMatrix(*g, inputs.POISSON7)
    x2, info2 = its().solve(S, dev(b), method="sgs", rtol=1e-8, max_iter=5000)
    assert info2.iters == rr.iters and np.array_equal(host(x2), ref)


@pytest.mark.parametrize("pack_first", [False, True])
def test_sgs_packed_colours_in_either_order(pack_first):
    g = (13, 9, 7)
    Acsr = inputs.poisson7_csr(*g)
    col = inputs.redblack_colors(*g)
    A = its().CSRMatrix.from_numpy(*Acsr)
    if pack_first:
        A.pack(max_fill=2.0)
        A.set_colors(col, 2)
    else:
        A.set_colors(col, 2)
        A.pack(max_fill=2.0)
    xs, b = _system(Acsr)
    ref, rr = oracle.sgs(Acsr, col, 2, b, rtol=1e-8, max_iter=2000)
    x, info = its().solve(A, dev(b), method="sgs", rtol=1e-8, max_iter=2000)
    assert rr.status == oracle.OK and info.iters == rr.iters
    assert np.array_equal(host(x), ref)


@pytest.mark.parametrize("pack", [False, True])
@pytest.mark.parametrize("n", [1, 2, 3])
def test_sgs_two_colours_tiny(pack, n):
    """Two colours with one row, or an empty black colour: the test inside
    the sweeps and the restore of the tested black rows at the edges."""
    rows, cols, vals = [0], [], []
    for i in range(n):  # tridiagonal (4, -1)
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                cols.append(j)
                vals.append(4.0 if j == i else -1.0)
        rows.append(len(cols))
    Acsr = (np.array(rows), np.array(cols, dtype=np.int32), np.array(vals))
    col = (np.arange(n) % 2).astype(np.uint8)
    A = its().CSRMatrix.from_numpy(*Acsr, pack=pack)
    A.set_colors(col, 2)
    b = inputs.uniform_vector(n, 3)
    for rtol, cap in ((0.0, 3), (1e-12, 50)):
        ref, rr = oracle.sgs(Acsr, col, 2, b, rtol=rtol, max_iter=cap)
        x, info = its().solve(A, dev(b), method="sgs", rtol=rtol, max_iter=cap)
        assert info.iters == rr.iters and np.array_equal(host(x), ref), (rtol, cap)


@pytest.mark.parametrize("g", [(1, 1, 1), (2, 1, 1), (3, 1, 1), (1, 1, 2), (2, 2, 1), (3, 3, 3),
                               (13, 9, 7)])
def test_sgs_two_colours_stencil_edges(g):
    """The 7-point matrix-free half-sweeps on their compact colour index:
    grids with one cell, an empty black colour, odd sides (lines whose red
    cells start at x = 1), at a fixed count and converged."""
    Acsr = inputs.poisson7_csr(*g)
    S = its().StencilMatrix(*g, inputs.POISSON7)
    col = inputs.redblack_colors(*g)
    b = inputs.uniform_vector(S.n, 5)
    for rtol, cap in ((0.0, 3), (1e-12, 400)):
        ref, rr = oracle.sgs(Acsr, col, 2, b, rtol=rtol, max_iter=cap)
        x, info = its().solve(S, dev(b), method="sgs", rtol=rtol, max_iter=cap)
        assert info.iters == rr.iters and np.array_equal(host(x), ref), (rtol, cap)
        assert abs(info.rel_res - rr.rel_res) <= 1e-12 * rr.rel_res


def test_sgs_rejects_bad_colouring():
    g = (6, 6, 6)
    Acsr, A = _matrix("csr27", g)
    with pytest.raises(its().ItsError):
        A.set_colors(inputs.redblack_colors(*g), 2)


# --------------------------------------------------------------- BiCGStab

@pytest.mark.parametrize("kind", ["csrcd", "stencd", "csr7", "csrcdp"])
@pytest.mark.parametrize("k", [1, 3, 12])
def test_bicgstab_fixed_k(kind, k):
    Acsr, A = _matrix(kind, (18, 11, 9))
    xs, b = _system(Acsr, seed=2)
    ref, rr = oracle.bicgstab(Acsr, b, rtol=0.0, max_iter=k)
    x, info = its().solve(A, dev(b), method="bicgstab", rtol=0.0, max_iter=k)
    xg = host(x)
    assert info.iters == rr.iters == k
    assert rel(xg, ref) <= 1e-10, f"max ulps {ulps(xg, ref)}"
    assert ulps(xg, ref) == 0


@pytest.mark.parametrize("kind", ["csrcd", "stencd", "csrcdp"])
def test_bicgstab_converged(kind):
    Acsr, A = _matrix(kind, (40, 36, 30))
    xs, b = _system(Acsr, seed=1)
    ref, rr = oracle.bicgstab(Acsr, b, rtol=1e-8, max_iter=1000)
    x, info = its().solve(A, dev(b), method="bicgstab", rtol=1e-8, max_iter=1000)
    assert rr.status == oracle.OK and info.status == "ok"
    assert abs(info.iters - rr.iters) <= 1 and rel(host(x), ref) <= 1e-10
    assert info.true_rel_res <= 1.01e-8


@pytest.mark.parametrize("mode,tol", [("cosine", 0.9), ("paper", 30.0)])
def test_bicgstab_restart_paths(mode, tol):
    Acsr, A = _matrix("csrcd", (14, 12, 10))
    xs, b = _system(Acsr, seed=8)
    rm = oracle.RESTART_COSINE if mode == "cosine" else oracle.RESTART_PAPER
    ref, rr = oracle.bicgstab(Acsr, b, rtol=1e-10, max_iter=2000, restart_tol=tol, restart_mode=rm)
    x, info = its().solve(A, dev(b), method="bicgstab", rtol=1e-10, max_iter=2000,
                          restart_tol=tol, restart_mode=mode)
    assert rr.restarts > 0 and info.restarts == rr.restarts
    assert info.iters == rr.iters and rel(host(x), ref) <= 1e-10


# ---------------------------------------------------- mixed precision (IR)

@pytest.mark.parametrize("kind", ["csr27", "sten27", "csr7", "csr7p", "csr27p"])
@pytest.mark.parametrize("lowp", ["f32", "f16"])
@pytest.mark.parametrize("g", [(24, 20, 18), (23, 19, 17)])  # the second: a partial last slice
def test_ir_cg_matches_oracle(kind, lowp, g):
    Acsr, A = _matrix(kind, g)
    xs, b = _system(Acsr, seed=1)
    lo = Acsr[2].astype(np.float32 if lowp == "f32" else np.float16)
    ref, rr = oracle.ir_cg(Acsr, lo, b, rtol=1e-10, max_iter=5000, inner_rtol=1e-4)
    x, info = its().solve(A, dev(b), method="cg", rtol=1e-10, max_iter=5000,
                          inner_dtype=lowp, inner_rtol=1e-4)
    xg = host(x)
    assert rr.status == oracle.OK and info.status == "ok"
    assert info.iters == rr.iters and info.inner_iters == rr.inner_iters
    assert rel(xg, ref) <= 1e-10
    x64, r64 = oracle.cg(Acsr, b, rtol=1e-12, max_iter=5000)
    err = np.linalg.norm(xg - x64) / np.linalg.norm(x64)
    print(f"IR {kind} {lowp}: outer {info.iters} inner {info.inner_iters}, "
          f"error vs FP64 oracle {err:.2e}, ulps vs IR oracle {ulps(xg, ref)}")
    assert err <= 1e-8


@pytest.mark.parametrize("lowp", ["f32", "f16"])
@pytest.mark.parametrize("g", [(1, 1, 1), (2, 1, 1), (63, 1, 1), (65, 1, 1), (129, 1, 1),
                               (200, 1, 1), (65, 3, 1), (70, 2, 3)])
def test_ir_small_and_ragged_slices(lowp, g):
    """The refinement on packed offset-slice matrices whose slices pair up
    unevenly: one row, a lone partial slice, a last slice narrower than the
    one it pairs with (the tile falls back to one row per lane), partial
    slices inside a pair; iterates bit for bit."""
    print(f"IR edge: {g} {lowp}", flush=True)
    Acsr, A = _matrix("csr7p", g)
    xs, b = _system(Acsr, seed=5)
    lo = Acsr[2].astype(np.float32 if lowp == "f32" else np.float16)
    ref, rr = oracle.ir_cg(Acsr, lo, b, rtol=1e-10, max_iter=500, inner_rtol=1e-4)
    x, info = its().solve(A, dev(b), method="cg", rtol=1e-10, max_iter=500, inner_dtype=lowp,
                          inner_rtol=1e-4)
    assert rr.status == oracle.OK and info.status == "ok"
    assert info.iters == rr.iters and info.inner_iters == rr.inner_iters
    assert np.array_equal(host(x), ref)


# ------------------------------------------------------- edge cases / status

@pytest.mark.parametrize("method", ["jacobi", "sgs", "cg", "bicgstab", "cgnb"])
def test_zero_rhs(method):
    A = its().StencilMatrix(5, 4, 3, inputs.POISSON7)
    x, info = its().solve(A, torch.zeros(60, dtype=torch.float64, device="cuda"),
                          x0=torch.ones(60, dtype=torch.float64, device="cuda"), method=method)
    assert info.status == "ok" and info.iters == 0 and not host(x).any()


@pytest.mark.parametrize("method", ["jacobi", "cg", "bicgstab", "cgnb"])
def test_nan_rhs_is_invalid(method):
    A = its().StencilMatrix(5, 4, 3, inputs.POISSON7)
    b = np.ones(60)
    b[7] = np.nan
    with pytest.raises(its().ItsError) as e:
        its().solve(A, dev(b), method=method)
    assert e.value.status == -1


@pytest.mark.parametrize("method", ["jacobi", "sgs", "cg", "bicgstab", "cgnb"])
def test_max_iter_zero(method):
    Acsr, A = _matrix("sten7", (6, 5, 4))
    xs, b = _system(Acsr)
    x, info = its().solve(A, dev(b), method=method, rtol=1e-8, max_iter=0)
    assert info.status == "not_converged" and info.iters == 0 and not host(x).any()


@pytest.mark.parametrize("pack", [False, True])
def test_single_unknown(pack):
    A = its().CSRMatrix.from_numpy(np.array([0, 1]), np.array([0]), np.array([4.0]), pack=pack)
    for method in ("jacobi", "cg", "bicgstab", "cgnb"):
        x, info = its().solve(A, dev(np.array([3.0])), method=method, rtol=1e-14, max_iter=10)
        assert info.status == "ok" and host(x)[0] == 0.75, method


def test_cg_breakdown_on_indefinite():
    A = its().CSRMatrix.from_numpy(np.array([0, 1, 2]), np.array([0, 1]), np.array([1.0, -1.0]))
    x, info = its().solve(A, dev(np.array([1.0, 1.0])), method="cg")
    assert info.status == "breakdown" and info.iters == 0


def test_bicgstab_breakdown_alpha_d_zero():
    A = its().CSRMatrix.from_numpy(np.array([0, 1, 2]), np.array([1, 0]), np.array([1.0, 1.0]))
    x, info = its().solve(A, dev(np.array([1.0, 0.0])), method="bicgstab")
    assert info.status == "breakdown" and info.iters == 0


def test_jacobi_rejects_missing_diagonal():
    A = its().CSRMatrix.from_numpy(np.array([0, 1, 2]), np.array([1, 0]), np.array([1.0, 1.0]))
    with pytest.raises(its().ItsError):
        its().solve(A, dev(np.array([1.0, 0.0])), method="jacobi")


def test_invalid_csr_rejected():
    with pytest.raises(its().ItsError):
        its().CSRMatrix.from_numpy(np.array([0, 2, 3]), np.array([1, 0, 5]), np.ones(3))


def test_empty_system():
    A = its().StencilMatrix(0, 4, 4, inputs.POISSON7)
    x, info = its().solve(A, torch.zeros(0, dtype=torch.float64, device="cuda"))
    assert info.status == "ok" and x.numel() == 0


def test_workspace_too_small():
    A = its().StencilMatrix(8, 8, 8, inputs.POISSON7)
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    from paper_2305_05988_amd import api
    with pytest.raises(its().ItsError) as e:
        import ctypes as C
        r = api.L.Result()
        o = api.options()
        b = torch.ones(512, dtype=torch.float64, device="cuda")
        x = torch.zeros_like(b)
        api.L.check(api.L.lib().its_solve(A.handle, C.byref(o), api._ptr(b), api._ptr(x),
                                          api._ptr(ws), 1024, api._stream(), C.byref(r)), "solve")
    assert e.value.status == -3


# ------------------------------------------------------------- full size

def test_full_size_poisson256_packed_cg():
    """The timed workload's matrix and launch configuration (256^3 Poisson,
    packed CSR, FP64 CG): SpMV and two CG iterations compared with the
    oracle over every row."""
    g = (256, 256, 256)
    print("full size: building 256^3 Poisson CSR", flush=True)
    Acsr = inputs.poisson7_csr(*g)
    n = Acsr[0].size - 1
    A = its().CSRMatrix.from_numpy(*Acsr, validate=False, pack=True)
    xs = inputs.uniform_vector(n, 1)
    b = oracle.spmv(Acsr, xs)
    bg = its().spmv(A, dev(xs))
    assert np.array_equal(host(bg), b)
    print("full size: SpMV bit-exact; oracle CG, 2 iterations", flush=True)
    ref, rr = oracle.cg(Acsr, b, rtol=0.0, max_iter=2)
    x, info = its().solve(A, bg, method="cg", rtol=0.0, max_iter=2)
    xg = host(x)
    assert info.iters == rr.iters == 2
    assert ulps(xg, ref) == 0
    assert abs(info.rel_res - rr.rel_res) <= 1e-12 * rr.rel_res
    # an odd count: the last iteration's x update is applied after the loop
    print("full size: oracle CG, 3 iterations", flush=True)
    ref, rr = oracle.cg(Acsr, b, rtol=0.0, max_iter=3)
    x, info = its().solve(A, bg, method="cg", rtol=0.0, max_iter=3)
    assert info.iters == rr.iters == 3
    assert ulps(host(x), ref) == 0


# ------------------------------------------------------------ mid size

@pytest.mark.parametrize("pack", [True, False])
def test_mid_size_blocks_take_several_tiles(pack):
    """128^3 Poisson (8192 tiles of 256 rows): the grid is capped at 4096
    blocks so one finishing kernel suffices, and each block walks two tiles.
    SpMV, two CG iterations and two Jacobi sweeps against the oracle."""
    g = (128, 128, 128)
    print(f"mid size: 128^3 Poisson CSR, pack={pack}", flush=True)
    Acsr = inputs.poisson7_csr(*g)
    n = Acsr[0].size - 1
    A = its().CSRMatrix.from_numpy(*Acsr, validate=False, pack=pack)
    xs = inputs.uniform_vector(n, 3)
    b = oracle.spmv(Acsr, xs)
    bg = its().spmv(A, dev(xs))
    assert np.array_equal(host(bg), b)
    ref, rr = oracle.cg(Acsr, b, rtol=0.0, max_iter=2)
    x, info = its().solve(A, bg, method="cg", rtol=0.0, max_iter=2)
    assert info.iters == rr.iters == 2 and ulps(host(x), ref) == 0
    ref, rr = oracle.jacobi(Acsr, b, rtol=0.0, max_iter=2)
    x, info = its().solve(A, bg, method="jacobi", rtol=0.0, max_iter=2)
    assert info.iters == rr.iters == 2 and ulps(host(x), ref) == 0


# ------------------------------------------------------------ graph replays

@pytest.mark.parametrize("method,kind,extra", [
    ("cg", "csr7p", {}), ("cg", "sten7", {}), ("cgnb", "csr7p", {}), ("bicgstab", "csrcdp", {}),
    ("jacobi", "csrcdp", {}), ("sgs", "csr7p", {}), ("sgs", "sten27", {}),
    ("cg", "csr27p", {"inner_dtype": "f16", "inner_rtol": 1e-3}), ("bicgstab", "stencd", {"transpose": True})])
def test_graph_replays_match_eager_launches(method, kind, extra):
    """The iteration loop runs as a captured HIP graph (graph=True) or launch
    by launch; both must give the same bits, over repeated solves and with a
    new right-hand side through the cached graph."""
    g = (13, 11, 9)
    Acsr, A = _matrix(kind, g)
    if method == "sgs" and kind.startswith("csr"):
        A.set_colors(inputs.redblack_colors(*g), 2)
    cap = 60 if method in ("jacobi", "sgs") else 400
    for seed in (1, 2):
        xs, b = _system(Acsr, seed=seed)
        bt = dev(b)
        ref, ri = its().solve(A, bt, method=method, rtol=1e-9, max_iter=cap, **extra)
        for _ in range(2):
            x, info = its().solve(A, bt, method=method, rtol=1e-9, max_iter=cap, check_every=4,
                                  graph=True, **extra)
            assert info.iters == ri.iters and info.status == ri.status
            assert np.array_equal(host(x), host(ref))
