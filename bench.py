"""Benchmark: FP64 CG on the 256^3 Poisson 7-point CSR system to relative
residual 1e-8 (x* ~ U[-1,1) seed 1, b = A x*, x0 = 0), one MI355X.  The CSR
matrix is handed to the library, which packs it into its device layout
(sliced ELLPACK, its_csr_pack) during setup; --layout csr keeps the CSR
arrays instead.

A step is one complete solve.  The JSON line reports CG iterations per
second over the timed steps, the roofline of the dominant kernel (the fused
SpMV + dot pass) from HIP events recorded around every launch inside the
timed region, the oracle timed on the host, and -- beside the metric -- the
mixed-precision refinement against FP64 CG at 1e-8 plus the other methods of
the library on their workloads.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-extras] [--no-cpu]
                    [--layout packed|csr]
    python bench.py --extra-only batched|small32|differentiation|paper_counts|kernels|footprint

paper_counts is not part of the default run: it reproduces the paper's
one-node iteration counts (Sec. 4.1) for candidate readings of its matrix.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "CG iters/s + achieved HBM GB/s, 256^3 Poisson; mixed-prec vs FP64 at 1e-8"
# the sources that define the CSR SpMV pass of CG (its traffic counters are
# tied to their hash)
KERNEL_SOURCES = ["paper_2305_05988_amd/csrc/common.hpp", "paper_2305_05988_amd/csrc/rowops.hpp",
                  "paper_2305_05988_amd/csrc/csr.hpp", "paper_2305_05988_amd/csrc/sell.hpp",
                  "paper_2305_05988_amd/csrc/kernels_cg.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "cg_pass1_poisson256_traffic.txt")
# Inside the timed region every PROFILE_EVERY-th launch of each kernel is
# bracketed by HIP events: enough samples for the per-launch average, few
# enough markers not to perturb the iteration rate.  Odd, so that the samples
# alternate between even iterations (whose update pass defers x) and odd ones.
PROFILE_EVERY = 7


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def csr_bytes(n, nnz, val_bytes=8):
    """Matrix bytes read per application: values, int32 columns, int32 row_ptr."""
    return val_bytes * nnz + 4 * nnz + 4 * (n + 1)


def packed_matrix_bytes(A, n):
    """Bytes of the matrix representation one SpMV pass reads: for the packed
    layout the padded value slots (8 B), the column indices of the slices
    that keep them (4 B), the per-position offset (4 B) and lane mask (8 B)
    of the offset slices and the int64 slice offsets -- no row pointers; for
    an unpacked matrix the CSR arrays."""
    slots, col_slots = A.packed_slots, A.packed_column_slots
    if not slots:
        return csr_bytes(n, A.nnz)
    return (8 * slots + 4 * col_slots + 12 * ((slots - col_slots) // 64)
            + 8 * ((n + 63) // 64 + 1))


def host_cpu():
    """Model name of the host CPU and the cores this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count()
    return model, avail


def measured_traffic(sha):
    """HBM bytes per launch of the SpMV pass from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    for line in open(TRAFFIC_FILE):
        m = re.match(r"TRAFFIC\s+(.*)", line.strip())
        if m:
            kv = dict(t.split("=", 1) for t in m.group(1).split())
            if kv.get("src_sha") == sha:
                return float(kv["bytes_per_launch"])
    return None


def cpu_baseline(steps_small=3, steps_large=13):
    """The oracle's CG on the same 256^3 system, single-threaded and pinned to
    one host core, timed as the difference of two runs so the per-iteration
    rate excludes setup."""
    import oracle
    from paper_2305_05988_amd import inputs
    model, avail = host_cpu()
    A = inputs.poisson7_csr(256)
    xs = inputs.uniform_vector(A[0].size - 1, 1)
    b = oracle.spmv(A, xs)
    saved = os.sched_getaffinity(0) if hasattr(os, "sched_getaffinity") else None
    core = min(saved) if saved else None
    if core is not None:
        os.sched_setaffinity(0, {core})
    try:
        times = {}
        for k in (steps_small, steps_large):
            t0 = time.perf_counter()
            oracle.cg(A, b, rtol=0.0, max_iter=k)
            times[k] = time.perf_counter() - t0
    finally:
        if saved:
            os.sched_setaffinity(0, saved)
    per_it = (times[steps_large] - times[steps_small]) / (steps_large - steps_small)
    return {"value": 1.0 / per_it, "unit": "iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps_large - steps_small} FP64 CG iterations of the 256^3 Poisson CSR "
                      f"system (difference of {steps_large}- and {steps_small}-iteration runs, "
                      f"single thread pinned to core {core})",
            "host_cpu": model, "host_cores_available": avail, "pinned_core": core,
            "seconds": times[steps_small] + times[steps_large]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--fixed-iters", type=int, default=0,
                    help="profiling: solve with rtol=0 for exactly this many iterations")
    ap.add_argument("--layout", choices=("packed", "csr"), default="packed",
                    help="device layout of the CSR matrix (packed: its_csr_pack)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="profiling: one 1 GiB stream copy first (HBM counter calibration)")
    ap.add_argument("--extra-only",
                    choices=("batched", "small32", "differentiation", "paper_counts", "kernels",
                             "footprint"),
                    help="profiling: run only this secondary workload and print its figures "
                         "(kernels: a few fixed iterations of every benchmark workload, one "
                         "after the other, with each kernel's bytes per launch; footprint: "
                         "streaming rates below and above the 256 MB Infinity Cache)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the solver "
              f"runs one GPU's whole subdomain; multi-GPU sharding is design-only)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2305_05988_amd as its
    from paper_2305_05988_amd import _lib, inputs

    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    torch.cuda.set_device(0)
    if args.copy_probe:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        its.stream_copy(src, dst)
        torch.cuda.synchronize()
        log(f"copy probe: {src.numel() * 8} bytes read, {dst.numel() * 8} bytes written")
        del src, dst
    if args.extra_only:
        fn = {"batched": batched, "small32": small32, "differentiation": differentiation,
              "paper_counts": paper_counts, "kernels": kernel_suite, "footprint": footprint}
        print(json.dumps({args.extra_only: fn[args.extra_only](its, inputs)}), flush=True)
        return
    N = args.n
    t0 = time.perf_counter()
    rp, col, val = inputs.poisson7_csr(N)
    n, nnz = rp.size - 1, col.size
    # low-precision copies of the values (mixed-precision refinement) are
    # attached first, so packing covers them too
    A = its.CSRMatrix.from_numpy(rp, col, val, lowp=("f32", "f16"),
                                 pack=args.layout == "packed")
    del rp, col, val
    xs = torch.from_numpy(inputs.uniform_vector(n, 1)).cuda()
    b = its.spmv(A, xs)
    torch.cuda.synchronize()
    slots = A.packed_slots
    log(f"setup {N}^3 CSR n={n} nnz={nnz} layout {args.layout} (slots {slots}) in "
        f"{time.perf_counter() - t0:.1f}s")

    V = 8 * n
    # Bytes per launch and per iteration are those of the matrix
    # representation the pass actually reads (packed layout: no row pointers,
    # no columns in offset slices) plus the vector touches:
    #   pass 1: matrix + gathered {r, p} pairs (2V) + q written (V);
    #   pass 2: r, p, q read and r, p written every iteration, x read and
    #           written every other iteration (its update is deferred by one
    #           iteration): 6V on average.
    # The CSR-equivalent figure (int32 columns and row pointers, as if the CSR
    # arrays were streamed) is kept under its own keys.
    M_csr = csr_bytes(n, nnz)
    M = packed_matrix_bytes(A, n)
    col_slots = A.packed_column_slots
    bytes_pass1 = M + 3 * V
    bytes_pass2 = 6 * V
    bytes_iter = bytes_pass1 + bytes_pass2
    csr_bytes_iter = M_csr + 10 * V

    opts = dict(method="cg", rtol=args.rtol, max_iter=20000)
    if args.fixed_iters:
        opts = dict(method="cg", rtol=0.0, max_iter=args.fixed_iters)
    ws = torch.empty(its.api.workspace_bytes(A, **opts), dtype=torch.uint8, device="cuda")
    for _ in range(args.warmup):
        x, info = its.solve(A, b, workspace=ws, profile=PROFILE_EVERY, **opts)
    torch.cuda.synchronize()
    iters = 0
    ms1 = ms2 = 0.0
    l1 = l2 = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x, info = its.solve(A, b, workspace=ws, profile=PROFILE_EVERY, **opts)
        iters += info.iters
        ms1 += info.kernel_ms[0]
        ms2 += info.kernel_ms[1]
        l1 += info.kernel_launches[0]
        l2 += info.kernel_launches[1]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert info.status == ("not_converged" if args.fixed_iters else "ok"), info
    its_per_s = iters / dt
    avg1 = ms1 / max(l1, 1) * 1e-3
    avg2 = ms2 / max(l2, 1) * 1e-3
    sha = kernel_source_sha()
    traffic = measured_traffic(sha)
    kname = "packed CSR" if slots else "CSR"
    roof = {"bound": "hbm", "kernel": f"k_cg_pass1 ({kname} SpMV + p.q)",
            "achieved": bytes_pass1 / avg1 / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": bytes_pass1 / avg1 / 1e9 / HBM_PEAK_GBS, "traffic": traffic,
            "algorithmic_bytes_per_launch": bytes_pass1, "avg_launch_us": avg1 * 1e6,
            "launches": l1, "kernel_src_sha": sha,
            "layout_column_slots": col_slots, "layout_slots": slots,
            "csr_equivalent_bytes_per_launch": M_csr + 3 * V,
            "csr_equivalent_gbs": (M_csr + 3 * V) / avg1 / 1e9,
            "update_pass": {"kernel": "k_cg_pass2", "avg_launch_us": avg2 * 1e6,
                            "bytes_per_launch_avg": bytes_pass2,
                            "achieved": bytes_pass2 / avg2 / 1e9,
                            "frac": bytes_pass2 / avg2 / 1e9 / HBM_PEAK_GBS}}
    xerr = (x - xs).norm().item() / xs.norm().item()
    result = {
        "metric": METRIC, "value": its_per_s, "unit": "iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"poisson7_{N}^3_csr_fp64_cg_rtol{args.rtol:g}", "n": n,
                   "nnz": nnz, "x_star": "U[-1,1) seed 1", "b": "A x*", "x0": 0,
                   "iters_per_solve": info.iters,
                   "device_layout": ("sliced ELLPACK, 64-row slices (its_csr_pack), "
                                     f"{slots} slots, {col_slots} of them with column "
                                     "indices" if slots else "CSR")},
        "achieved_gbs": its_per_s * bytes_iter / 1e9,
        "hbm_frac": its_per_s * bytes_iter / 1e9 / HBM_PEAK_GBS,
        "algorithmic_bytes_per_iter": bytes_iter,
        "csr_equivalent_bytes_per_iter": csr_bytes_iter,
        "csr_equivalent_gbs": its_per_s * csr_bytes_iter / 1e9,
        "true_rel_res": info.true_rel_res, "rel_err_vs_xstar": xerr,
        "roofline": roof,
    }
    log(f"CG {N}^3: {info.iters} it/solve, {its_per_s:.1f} it/s, "
        f"{result['achieved_gbs']:.0f} GB/s ({result['hbm_frac']:.3f} of peak); pass1 "
        f"{avg1 * 1e6:.1f} us ({roof['achieved']:.0f} GB/s), pass2 {avg2 * 1e6:.1f} us")

    if not args.no_extras:
        result["extras"] = extras(its, inputs, A, b, xs, n, nnz, N, args, ws, float(dt / iters))
    del ws
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline()
        log(f"cpu baseline {result['cpu_baseline']['value']:.3f} it/s")
    print(json.dumps(result), flush=True)


def timed(fn, reps=1):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, out


def ir_27pt(its, inputs, args, N=192):
    """Mixed precision on the SPD 27-point (26, -1) CSR system at 192^3: values
    stored in FP32 and separately in FP16, refinement to 1e-10 (error against
    an FP64 CG solution to 1e-12 and against x*) and to 1e-8 (wall time
    against FP64 CG to 1e-8)."""
    import torch
    t0 = time.perf_counter()
    rp, col, val = inputs.stencil27_csr(N)
    n, nnz = rp.size - 1, col.size
    A = its.CSRMatrix.from_numpy(rp, col, val, lowp=("f32", "f16"), validate=False,
                                 pack=args.layout == "packed")
    del rp, col, val
    xs = torch.from_numpy(inputs.uniform_vector(n, 1)).cuda()
    b = its.spmv(A, xs)
    torch.cuda.synchronize()
    out = {"n": n, "nnz": nnz, "setup_s": time.perf_counter() - t0}
    xref, iref = its.solve(A, b, method="cg", rtol=1e-12, max_iter=20000)
    out["fp64_cg_1e-12_iters"] = iref.iters
    its.solve(A, b, method="cg", rtol=1e-8, max_iter=20000)
    t64, (x64, i64) = timed(lambda: its.solve(A, b, method="cg", rtol=1e-8, max_iter=20000))
    out.update({"fp64_cg_1e-8_s": t64, "fp64_cg_1e-8_iters": i64.iters,
                "fp64_cg_1e-8_iters_per_s": i64.iters / t64})
    xn = xref.norm().item()
    for lowp in ("f32", "f16"):
        for rtol in (1e-8, 1e-10):
            kw = dict(method="cg", rtol=rtol, max_iter=20000, inner_dtype=lowp, inner_rtol=1e-4)
            its.solve(A, b, **kw)
            t, (xl, il) = timed(lambda: its.solve(A, b, **kw))
            key = f"ir_{lowp}_{rtol:g}"
            out[f"{key}_s"] = t
            out[f"{key}_outer"] = il.iters
            out[f"{key}_inner"] = il.inner_iters
            out[f"{key}_true_rel_res"] = il.true_rel_res
            out[f"{key}_err_vs_fp64"] = (xl - xref).norm().item() / xn
            out[f"{key}_err_vs_xstar"] = (xl - xs).norm().item() / xs.norm().item()
            if rtol == 1e-8:
                out[f"{key}_speedup_vs_fp64"] = t64 / t
    log(f"ir 27-point {N}^3: {json.dumps(out)}")
    del A, xs, b, xref, x64
    return out


def small32(its, inputs, N=32):
    """The 32^3 Poisson CSR system (packed), where launches and reductions
    rather than HBM set the pace: time to solution of each method to 1e-8
    (Jacobi capped at 2000 sweeps), median of 5."""
    import statistics
    import torch
    rp, col, val = inputs.poisson7_csr(N)
    n = rp.size - 1
    A = its.CSRMatrix.from_numpy(rp, col, val, pack=True, max_fill=2.0)
    A.set_colors(inputs.redblack_colors(N, N, N), 2)
    b = its.spmv(A, torch.from_numpy(inputs.uniform_vector(n, 1)).cuda())
    out = {}

    def med(kw, env=None):
        saved = {k: os.environ.get(k) for k in (env or {})}
        os.environ.update(env or {})
        try:
            its.solve(A, b, rtol=1e-8, **kw)
            ts = []
            for _ in range(5):
                t, (x, info) = timed(lambda: its.solve(A, b, rtol=1e-8, **kw))
                ts.append(t)
        finally:
            for k, v in saved.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v
        t = statistics.median(ts)
        return {"iters": info.iters, "status": info.status, "s": t, "iters_per_s": info.iters / t}

    for method, cap in (("cg", 5000), ("bicgstab", 5000), ("cgnb", 5000), ("jacobi", 2000),
                        ("sgs", 5000)):
        for graph in (False, True):
            out[method + ("_graph" if graph else "")] = med(dict(method=method, max_iter=cap,
                                                                 graph=graph))
    # one persistent cooperative kernel per solve (grid barriers); BiCGStab
    # with B1's split-phase barriers and, for comparison, with all three
    # barriers blocking
    for method in ("cg", "cgnb", "bicgstab"):
        out[method + "_persistent"] = med(dict(method=method, max_iter=5000, persistent=True))
    out["bicgstab_persistent_blocking"] = med(dict(method="bicgstab", max_iter=5000,
                                                   persistent=True),
                                              env={"ITS_BICGSTAB_SPLIT": "0"})
    log(f"32^3: {json.dumps(out)}")
    return out


def batched(its, inputs, nsys=512, nrhs=8):
    """512 variable-coefficient 7-point systems, sides U{16..64} per axis,
    g ~ N(0, 1) per cell, k = exp(g), 8 right-hand sides U[-1, 1) each
    (default_rng([4, s]) per system), FP64 CG to 1e-8 per (system, rhs) in
    one graph-captured batch.  The first solve includes the autotuning; the
    second is timed."""
    import numpy as np
    import torch
    t0 = time.perf_counter()
    dims, k, b = inputs.batch_systems(nsys, nrhs, seed=4)
    n_s = np.prod(dims.astype(np.int64), axis=1)
    B = its.Batch(dims, torch.from_numpy(k).cuda(), nrhs)
    bt = torch.from_numpy(b.ravel()).cuda()
    del b, k
    setup = time.perf_counter() - t0
    x, first = B.solve(bt, rtol=1e-8, max_iter=20000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, info = B.solve(bt, rtol=1e-8, max_iter=20000)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    it = info.iters
    # bytes actually needed: per (system, rhs) iteration 9 vector touches of 8 B per cell on
    # average (x is read and written every other iteration);
    # per system iteration the operator once for all right-hand sides: the diagonal and the
    # three upper face coefficients (32 B per cell; a lower face is the neighbour's upper one)
    vec_bytes = float(np.sum(it * n_s[:, None]) * 72)
    coef_bytes = float(np.sum(it.max(axis=1) * n_s) * 32)
    out = {"systems": nsys, "rhs": nrhs, "cells": int(n_s.sum()), "setup_s": setup,
           "status": info.status, "solve_s": dt, "first_solve_s": first.solve_ms / 1e3,
           "tune_ms": first.tune_ms, "tiles_per_item": info.tiles_per_item,
           "planes_per_brick": info.planes_per_brick,
           "graph_iters": info.graph_iters, "replays": info.replays,
           "iters_max": int(it.max()), "iters_mean": float(it.mean()), "iters_min": int(it.min()),
           "solves_per_s": nsys * nrhs / dt,
           "cell_rhs_iters_per_s": float(np.sum(it * n_s[:, None])) / dt,
           "achieved_gbs": (vec_bytes + coef_bytes) / dt / 1e9}
    log(f"batched: {json.dumps(out)}")
    del B, bt, x
    return out


def differentiation(its, inputs):
    """Variable-coefficient diffusion on 128^3 (theta ~ N(0,1) seed 3, k =
    exp(theta), x_target U[-1,1) seed 2, b U[-1,1) seed 1): CG forward to
    1e-10, loss 0.5 ||x - x_target||^2, backward = adjoint CG to 1e-10 plus
    the gradient kernel.  And the BiCGStab adjoint (solve with A^T) on 96^3
    upwind convection-diffusion, Peclet 10."""
    import torch
    out = {}
    N = 128
    n = N ** 3
    theta = torch.from_numpy(inputs.gaussian_field(n, 3)).cuda().requires_grad_(True)
    xt = torch.from_numpy(inputs.uniform_vector(n, 2)).cuda()
    b = torch.from_numpy(inputs.uniform_vector(n, 1)).cuda().requires_grad_(True)
    A = its.VarCoefMatrix(N, N, N, torch.exp(theta.detach()))
    x, fi = its.solve(A, b.detach(), method="cg", rtol=1e-10, max_iter=20000)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, fi = its.solve(A, b.detach(), method="cg", rtol=1e-10, max_iter=20000)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    lam, ai = its.solve(A, (x - xt).contiguous(), method="cg", rtol=1e-10, max_iter=20000)
    dk = its.varcoef_grad(A, x, lam)
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    # the same through torch.autograd (forward + backward)
    t0 = time.perf_counter()
    xa = its.diffusion_solve(torch.exp(theta), b, (N, N, N), rtol=1e-10)
    L = 0.5 * ((xa - xt) ** 2).sum()
    L.backward()
    torch.cuda.synchronize()
    t_auto = time.perf_counter() - t0
    V = 8 * n
    out["diff_varcoef_128"] = {
        "forward_iters": fi.iters, "forward_s": t_fwd, "forward_iters_per_s": fi.iters / t_fwd,
        "forward_achieved_gbs": fi.iters / t_fwd * 11 * V / 1e9,
        "adjoint_iters": ai.iters, "backward_s": t_bwd, "autograd_forward_backward_s": t_auto,
        "loss": L.item(), "grad_theta_norm": theta.grad.norm().item(),
        "grad_b_norm": b.grad.norm().item(),
        "grad_matches_direct": bool(torch.allclose(theta.grad, dk * torch.exp(theta.detach()),
                                                   rtol=1e-12, atol=0.0))}
    del A, x, lam, dk, xa, theta, b, xt
    # BiCGStab adjoint on upwind convection-diffusion
    M = 96
    S = its.StencilMatrix(M, M, M, inputs.convdiff7())
    bb = torch.from_numpy(inputs.uniform_vector(M ** 3, 1)).cuda().requires_grad_(True)
    w = torch.from_numpy(inputs.uniform_vector(M ** 3, 2)).cuda()
    its.solve(S, bb.detach(), method="bicgstab", rtol=1e-10, max_iter=5000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xb = its.stencil_solve(S, bb, rtol=1e-10)
    torch.cuda.synchronize()
    t_f = time.perf_counter() - t0
    t0 = time.perf_counter()
    (xb * w).sum().backward()
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    _, fi = its.solve(S, bb.detach(), method="bicgstab", rtol=1e-10, max_iter=5000)
    _, ai = its.solve(S, w, method="bicgstab", rtol=1e-10, max_iter=5000, transpose=True)
    out["adjoint_bicgstab_96_upwind"] = {"forward_iters": fi.iters, "forward_s": t_f,
                                         "adjoint_iters": ai.iters, "backward_s": t_b,
                                         "adjoint_true_rel_res": ai.true_rel_res}
    log(f"differentiation: {json.dumps(out)}")
    return out


# Iteration counts the paper prints for one node (Sec. 4.1): 128 x 128 x 6144
# cells, b = A 1, x0 = 0, stop when ||r||_2 < 1e-6, BiCGStab restart
# threshold 1e-5 on sqrt|alpha_n|.
PAPER_COUNTS = {7: {"bicgstab": 8, "cg": 12, "sgs": 9, "jacobi": 18},
                27: {"bicgstab": 45, "cg": 72, "sgs": 142, "jacobi": 515}}


def paper_counts(its, inputs, grid=(128, 128, 6144)):
    """Iterations to the paper's absolute criterion on its one-node grid for
    candidate readings of its matrix (a centred 7- or 27-point stencil with
    -1 off the diagonal): diagonal 27 on both stencils, 26 on the 27-point
    one, 6 on the 7-point one (capped).  Matrix-free stencils; the absolute
    test ||r|| < 1e-6 is the relative one with rtol = 1e-6 / ||b||."""
    import torch
    out = {}
    cases = [(7, 27.0), (7, 6.0), (27, 27.0), (27, 26.0)]
    for npts, diag in cases:
        offs = inputs.OFFSETS7 if npts == 7 else inputs.OFFSETS27
        coef = [diag if o == (0, 0, 0) else -1.0 for o in offs]
        S = its.StencilMatrix(*grid, coef)
        b = its.spmv(S, torch.ones(S.n, dtype=torch.float64, device="cuda"))
        bn = its.dot(b, b) ** 0.5
        row = {"b_norm": bn, "paper": PAPER_COUNTS[npts]}
        for method in ("cg", "cgnb", "bicgstab", "sgs", "jacobi"):
            kw = dict(method=method, rtol=1e-6 / bn, max_iter=2000)
            if method == "bicgstab":
                kw.update(restart_mode="paper", restart_tol=1e-5)
            t, (x, info) = timed(lambda: its.solve(S, b, **kw))
            row[method] = {"iters": info.iters, "status": info.status, "s": t,
                           "true_res": info.true_rel_res * bn}
            del x
        log(f"paper counts {npts}-point diagonal {diag:g}: {json.dumps(row)}")
        out[f"{npts}pt_diag{diag:g}"] = row
        del S, b
        torch.cuda.empty_cache()
    return out


def kernel_suite(its, inputs, iters=10):
    """A few fixed iterations of each benchmark workload, one after the other
    in one process, for per-kernel profiles (rocprofv3 kernel trace and HBM
    counters): for every workload the bytes per launch each of its kernels
    needs -- the matrix representation it reads (packed layout: no row
    pointers, no columns in offset slices) plus its vector touches.  V = 8n,
    V32 = 4n.  Kernels shared by two workloads of different sizes are told
    apart by their grid."""
    import torch
    out = {}

    def run(A, b, **kw):
        its.solve(A, b, **kw)
        torch.cuda.synchronize()

    def packed_lowp_bytes(A, n, vb):
        slots, cs = A.packed_slots, A.packed_column_slots
        return vb * slots + 4 * cs + 12 * ((slots - cs) // 64) + 8 * ((n + 63) // 64 + 1)

    # 256^3 Poisson, packed CSR with FP32 and FP16 value copies
    N = 256
    rp, col, val = inputs.poisson7_csr(N)
    n = rp.size - 1
    A = its.CSRMatrix.from_numpy(rp, col, val, lowp=("f32", "f16"), validate=False, pack=True)
    del rp, col, val
    b = its.spmv(A, torch.from_numpy(inputs.uniform_vector(n, 1)).cuda())
    V, V32 = 8 * n, 4 * n
    M, M32, M16 = packed_matrix_bytes(A, n), packed_lowp_bytes(A, n, 4), packed_lowp_bytes(A, n, 2)
    log(f"kernels: cg 256^3 ({iters} iterations)")
    run(A, b, method="cg", rtol=0.0, max_iter=iters)
    log(f"kernels: jacobi 256^3 ({iters} sweeps)")
    run(A, b, method="jacobi", rtol=0.0, max_iter=iters)
    for lowp, Ml in (("f32", M32), ("f16", M16)):
        log(f"kernels: refinement ({lowp} values) 256^3 ({iters} inner iterations)")
        run(A, b, method="cg", rtol=1e-12, max_iter=iters, inner_dtype=lowp, inner_rtol=1e-30)
    out["poisson256_packed"] = {
        "n": n, "grid_spmv": (n + 255) // 256,
        "k_cg_pass1<SellOp<double": M + 3 * V, "k_cg_pass2<double, true": 6 * V,
        "k_jacobi<SellOp<double": M + 3 * V,
        "k_cg_pass1<SellOp<float": M32 + 3 * V32, "k_cg_pass1_pairs<SellOp<__half": M16 + 3 * V32,
        "k_cg_pass2_f32x2": 6 * V32, "k_residual<SellOp<double": M + 3 * V}
    del A, b
    torch.cuda.empty_cache()
    # 256^3 matrix-free 7-point stencil
    S = its.StencilMatrix(N, N, N, inputs.POISSON7)
    b = torch.from_numpy(inputs.uniform_vector(n, 1)).cuda()
    log(f"kernels: matrix-free cg 256^3 ({iters} iterations)")
    run(S, b, method="cg", rtol=0.0, max_iter=iters)
    log(f"kernels: matrix-free red-black sgs 256^3 ({iters} iterations)")
    run(S, b, method="sgs", rtol=0.0, max_iter=iters)
    out["poisson256_stencil"] = {"n": n, "k_cg_pass1<StencilOp<7, double": 3 * V,
                                 "k_gs_stencil<7>": 3 * V // 2 + V // 2,
                                 "k_gs_check<StencilOp<7, double": 2 * V}
    del S, b
    torch.cuda.empty_cache()
    # 192^3 upwind convection-diffusion, packed CSR
    rp, col, val = inputs.convdiff7_csr(192)
    n2 = rp.size - 1
    C2 = its.CSRMatrix.from_numpy(rp, col, val, validate=False, pack=True)
    del rp, col, val
    b2 = its.spmv(C2, torch.from_numpy(inputs.uniform_vector(n2, 1)).cuda())
    log(f"kernels: bicgstab 192^3 upwind ({iters} iterations)")
    run(C2, b2, method="bicgstab", rtol=0.0, max_iter=iters)
    M2, V2 = packed_matrix_bytes(C2, n2), 8 * n2
    out["convdiff192_packed"] = {"n": n2, "k_bicg_a<": M2 + 6 * V2, "k_bicg_b<": M2 + 3 * V2,
                                 "k_bicg_c": 9 * V2}
    del C2, b2
    torch.cuda.empty_cache()
    # 192^3 27-point, packed CSR with FP32 and FP16 value copies
    rp, col, val = inputs.stencil27_csr(192)
    A3 = its.CSRMatrix.from_numpy(rp, col, val, lowp=("f32", "f16"), validate=False, pack=True)
    del rp, col, val
    b3 = its.spmv(A3, torch.from_numpy(inputs.uniform_vector(n2, 1)).cuda())
    log(f"kernels: cg 27-point 192^3 ({iters} iterations)")
    run(A3, b3, method="cg", rtol=0.0, max_iter=iters)
    for lowp in ("f32", "f16"):
        log(f"kernels: refinement ({lowp} values) 27-point 192^3 ({iters} inner iterations)")
        run(A3, b3, method="cg", rtol=1e-12, max_iter=iters, inner_dtype=lowp, inner_rtol=1e-30)
    V3, V3_32 = 8 * n2, 4 * n2
    out["stencil27_192_packed"] = {
        "n": n2, "k_cg_pass1<SellOp<double": packed_matrix_bytes(A3, n2) + 3 * V3,
        "k_cg_pass2<double, true": 6 * V3,
        "k_cg_pass1_pairs<SellOp<float": packed_lowp_bytes(A3, n2, 4) + 3 * V3_32,
        "k_cg_pass1_pairs<SellOp<__half": packed_lowp_bytes(A3, n2, 2) + 3 * V3_32,
        "k_cg_pass2_f32x2": 6 * V3_32}
    del A3, b3
    torch.cuda.empty_cache()
    return out


def footprint(its, inputs, iters=10):
    """Streaming rate against working-set size.  MI355X keeps a 256 MB
    memory-side Infinity Cache in front of HBM, so a pass whose vectors were
    just written by the previous pass can stream faster than HBM alone allows
    while they fit.  Measured: the stream copy (footprint 2x the bytes
    copied), and the single-system CG passes on the matrix-free 7-point
    stencil at 256^3 (16.8M rows: 0.5 GB of vectors) and at 640 x 640 x 670
    (274M rows: about the 512 x 8 batch's 275.5M values), fixed iterations.
    The wall-clock rates printed here include launch gaps (they dominate the
    small copies); per-launch durations come from a rocprofv3 kernel trace
    of this leg (the copies run in ascending size, 21 launches each)."""
    import torch
    out = {"copy_gbs": {}}
    for mib in (32, 64, 128, 256, 512, 1024, 4096):
        src = torch.ones(mib << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        its.stream_copy(src, dst)
        t, _ = timed(lambda: its.stream_copy(src, dst), reps=20)
        out["copy_gbs"][f"{mib}MiB"] = 2 * src.numel() * 8 / t / 1e9
        del src, dst
        torch.cuda.empty_cache()
    log(f"footprint: copy {json.dumps(out['copy_gbs'])}")
    for dims in ((256, 256, 256), (640, 640, 670)):
        S = its.StencilMatrix(*dims, inputs.POISSON7)
        n = S.n
        b = torch.ones(n, dtype=torch.float64, device="cuda")
        its.solve(S, b, method="cg", rtol=0.0, max_iter=iters)
        t, (x, info) = timed(lambda: its.solve(S, b, method="cg", rtol=0.0, max_iter=iters))
        key = "x".join(str(d) for d in dims)
        # pass 1 moves 3V (the {r, p} pairs and q), pass 2 5V on even and 7V
        # on odd iterations (x every other one)
        out[key] = {"n": n, "iters": info.iters, "s": t, "ms_per_iter": t / info.iters * 1e3,
                    "bytes_per_iter": 9 * 8 * n, "gbs": info.iters * 9 * 8 * n / t / 1e9}
        log(f"footprint: stencil cg {key}: {json.dumps(out[key])}")
        del S, b, x
        torch.cuda.empty_cache()
    return out


def extras(its, inputs, A, b, xs, n, nnz, N, args, ws, s_per_it):
    import torch
    ex = {}
    V = 8 * n
    # mixed-precision refinement vs FP64 CG, same system, same tolerance
    t64, (x64, i64) = timed(lambda: its.solve(A, b, method="cg", rtol=args.rtol, max_iter=20000))
    mp = {"fp64_cg_s": t64, "fp64_iters": i64.iters}
    for lowp in ("f32", "f16"):
        its.solve(A, b, method="cg", rtol=args.rtol, max_iter=20000, inner_dtype=lowp,
                  inner_rtol=1e-4)
        t, (xl, il) = timed(lambda: its.solve(A, b, method="cg", rtol=args.rtol, max_iter=20000,
                                              inner_dtype=lowp, inner_rtol=1e-4))
        mp[f"ir_{lowp}_s"] = t
        mp[f"ir_{lowp}_outer"] = il.iters
        mp[f"ir_{lowp}_inner"] = il.inner_iters
        mp[f"ir_{lowp}_true_rel_res"] = il.true_rel_res
        mp[f"ir_{lowp}_speedup_vs_fp64"] = t64 / t
        mp[f"ir_{lowp}_rel_diff_vs_fp64_cg"] = (xl - x64).norm().item() / x64.norm().item()
    ex["mixed_precision_256"] = mp
    log(f"mixed precision: {json.dumps(mp)}")
    # the paper's CG-NB (Algorithm 1) on the same CSR system
    its.solve(A, b, method="cgnb", rtol=args.rtol, max_iter=20000)
    t, (xn, info) = timed(lambda: its.solve(A, b, method="cgnb", rtol=args.rtol, max_iter=20000))
    Mp = packed_matrix_bytes(A, n)
    # CG-NB: SpMV pass on r (matrix + {r, Ap} pairs gathered 2V + w written V),
    # update pass (reads pairs 2V, p, w, x; writes pairs 2V, p, x): M + 12V
    ex["cgnb_256_csr"] = {"iters": info.iters, "s": t, "iters_per_s": info.iters / t,
                          "bytes_per_iter": Mp + 12 * V,
                          "achieved_gbs": info.iters / t * (Mp + 12 * V) / 1e9,
                          "true_rel_res": info.true_rel_res, "vs_cg_time": t / t64}
    # matrix-free stencil CG on the same grid
    S = its.StencilMatrix(N, N, N, inputs.POISSON7)
    its.solve(S, b, method="cg", rtol=args.rtol, max_iter=20000)
    t, (xs_, info) = timed(lambda: its.solve(S, b, method="cg", rtol=args.rtol, max_iter=20000))
    # matrix-free: pass 1 gathers the {r, p} pairs (2V) and writes q (V);
    # pass 2 moves 6V on average (x every other iteration): 9V
    ex["stencil_cg_256"] = {"iters": info.iters, "s": t, "iters_per_s": info.iters / t,
                            "bytes_per_iter": 9 * V,
                            "achieved_gbs": info.iters / t * 9 * V / 1e9}
    # Jacobi: 2000 capped sweeps on the CSR system
    its.solve(A, b, method="jacobi", rtol=args.rtol, max_iter=50)
    t, (xj, info) = timed(lambda: its.solve(A, b, method="jacobi", rtol=args.rtol, max_iter=500))
    # the sweep reads the matrix, gathers x_k, reads b and writes x_{k+1}
    ex["jacobi_256_csr"] = {"sweeps": info.iters, "s": t, "sweeps_per_s": info.iters / t,
                            "bytes_per_sweep": Mp + 3 * V,
                            "achieved_gbs": info.iters / t * (Mp + 3 * V) / 1e9}
    # red-black symmetric Gauss-Seidel, matrix-free
    its.solve(S, b, method="sgs", rtol=args.rtol, max_iter=5)
    t, (xg, info) = timed(lambda: its.solve(S, b, method="sgs", rtol=args.rtol, max_iter=200))
    ex["rbsgs_256_stencil"] = {"iters": info.iters, "s": t, "iters_per_s": info.iters / t}
    # red-black symmetric Gauss-Seidel on the CSR matrix (colour-packed half-sweeps)
    A.set_colors(inputs.redblack_colors(N, N, N), 2)
    its.solve(A, b, method="sgs", rtol=args.rtol, max_iter=5)
    t, (xg, info) = timed(lambda: its.solve(A, b, method="sgs", rtol=args.rtol, max_iter=100))
    ex["rbsgs_256_csr"] = {"iters": info.iters, "s": t, "iters_per_s": info.iters / t}
    # stream copy: achievable bandwidth
    src = torch.empty(n * 8, dtype=torch.float64, device="cuda").uniform_()
    dst = torch.empty_like(src)
    its.stream_copy(src, dst)
    t, _ = timed(lambda: its.stream_copy(src, dst), reps=20)
    ex["stream_copy_gbs"] = 2 * src.numel() * 8 / t / 1e9
    del src, dst
    # BiCGStab on 192^3 upwind convection-diffusion (Peclet 10)
    rp, col, val = inputs.convdiff7_csr(192)
    n2, nnz2 = rp.size - 1, col.size
    C = its.CSRMatrix.from_numpy(rp, col, val, pack=args.layout == "packed")
    del rp, col, val
    x2 = torch.from_numpy(inputs.uniform_vector(n2, 1)).cuda()
    b2 = its.spmv(C, x2)
    its.solve(C, b2, method="bicgstab", rtol=args.rtol, max_iter=2000)
    reps = 10
    t, (xb, info) = timed(lambda: its.solve(C, b2, method="bicgstab", rtol=args.rtol, max_iter=2000),
                          reps=reps)
    # two SpMV passes over the matrix; the pair layout of the vectors moves
    # 18V per iteration (one more than the fused minimum of 17V)
    M2 = packed_matrix_bytes(C, n2)
    ex["bicgstab_192_convdiff_csr"] = {"iters": info.iters, "restarts": info.restarts,
                                       "s_per_solve": t, "iters_per_s": info.iters / t,
                                       "solves_per_s": 1.0 / t,
                                       "bytes_per_iter": 2 * M2 + 18 * 8 * n2,
                                       "achieved_gbs": info.iters / t * (2 * M2 + 18 * 8 * n2) / 1e9,
                                       "true_rel_res": info.true_rel_res}
    del C, x2, b2, xb
    ex["ir_27pt_192"] = ir_27pt(its, inputs, args)
    ex.update(differentiation(its, inputs))
    ex["batched_512x8_varcoef"] = batched(its, inputs)
    ex["small_32"] = small32(its, inputs)
    if args.layout == "packed":
        # the same CG solve with the matrix left in CSR (LDS-staged tiles)
        rp, col, val = inputs.poisson7_csr(N)
        U = its.CSRMatrix.from_numpy(rp, col, val, validate=False)
        del rp, col, val
        its.solve(U, b, method="cg", rtol=args.rtol, max_iter=20000)
        t, (xu, info) = timed(lambda: its.solve(U, b, method="cg", rtol=args.rtol, max_iter=20000))
        ex["cg_256_csr_unpacked"] = {"iters": info.iters, "iters_per_s": info.iters / t,
                                     "identical_to_packed": bool(torch.equal(xu, x64))}
        del U, xu
    log(f"extras: {json.dumps(ex)}")
    return ex


if __name__ == "__main__":
    main()
