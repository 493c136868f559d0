// Relaxation kernels: Jacobi sweep and colour-ordered symmetric Gauss-Seidel.
#pragma once

#include "common.hpp"
#include "csr.hpp"
#include "sell.hpp"
#include "stencil.hpp"

namespace its {

// ------------------------------------------------------------------ Jacobi
// One fused sweep: the residual of x_k (full chain) and x_{k+1} = (b - off)/d.
// The test applies to x_k, so a converged solve returns x_k from xo.
template <class Op>
__global__ void __launch_bounds__(kBlock) k_jacobi(Op A, const double *__restrict__ b,
                                                   const double *__restrict__ xo,
                                                   double *__restrict__ xn, const State *st,
                                                   Reduce *R) {
  __shared__ typename Op::Smem sm;
  if (st->flag != kRunning) return;
  auto xj = [&](int32_t j) { return xo[j]; };
  auto same = [](double v) { return v; };
  Dot2 a;
  A.rows(sm, xj, same, [&](int32_t i, bool valid, auto &&entries, auto &&) {
    double full = 0.0, off = 0.0, diag = 0.0;
    entries([&](int32_t j, double av, double v) {
      full = fma(av, v, full);
      if (j == i)
        diag = av;
      else
        off = fma(av, v, off);
    });
    if (valid) {
      const double bi = ld_nt(b + i);
      const double ri = bi - full;
      a.add(ri, ri);
      st_pairs<GathersPairs<Op>::value>(xn + i, (bi - off) / diag);
    }
  });
  DD v[1] = {a.get()};
  block_partial<1>(v, R, rev_of(A));
}

// The sweep's residual belongs to x_k: test it; if it fails, x_{k+1} is the
// new iterate.
struct FinJacobi {
  State *st;
  __device__ bool active() const { return st->flag == kRunning; }
  __device__ void operator()(DD (&v)[1]) const {
    const double rr = dd_round(v[0]);
    const int64_t k = st->k;
    st->rho = rr;
    if (rr <= st->thr2)
      st->flag = kConverged;
    else if (!finite(rr))
      st->flag = kBreakdown;
    else if (k >= st->max_iter)
      st->flag = kMaxIter;
    else
      st->k = k + 1;
  }
};

// ------------------------------------------------------------ Gauss-Seidel
// Half-sweep over the rows of one colour, in place.  Rows of one colour do
// not couple, so their updates are independent and the order within the
// colour does not change any bit.
//
// With two colours (red 0, black 1) on a CSR matrix an iteration after the
// first sweeps black then red, and the residual of the iterate it leaves
// comes from the sweeps themselves instead of a separate SpMV pass:
//   kGsFinal  (red sweep): after a row's update, its full chain again with
//             the new value -- the red residual of the new iterate (slot 0);
//   kGsLagged (next black sweep): before a row's update, the full chain over
//             the values it reads anyway -- the black residual of that same
//             iterate (slot 1) -- and the old value saved to xs, so a solve
//             that stops on this test can put the tested iterate back.
// Every chain is the SpMV chain (ascending columns, diagonal in place), so
// r.r equals the separate pass's bit for bit.  (The matrix-free sweeps keep
// the separate pass: its LDS-tiled stencil SpMV costs less than the extra
// chains in the sweeps.)
enum : int32_t { kGsPlain = 0, kGsFinal = 1, kGsLagged = 2 };

// One dot's block partial into slot d; the other slots are left alone (the
// red and black residual partials of one test come from two kernels).
__device__ __forceinline__ void block_partial_at(DD v, int d, Reduce *R, bool rev = false) {
  DD t[1] = {v};
  block_reduce<1>(t);
  if (threadIdx.x == 0) R->p1[d][sched_place(rev)] = t[0];
}

template <int Mode>
__global__ void __launch_bounds__(kBlock) k_gs_rows_csr(CsrOp<double, double> A,
                                                        const int32_t *__restrict__ rows,
                                                        int32_t count, const double *__restrict__ b,
                                                        double *x, double *__restrict__ xs,
                                                        const State *st, Reduce *R) {
  if (st->flag != kRunning) return;
  Dot2 a;
  for_rows(count, [&](int32_t t) {
    const int32_t i = rows[t];
    const double bi = b[i];
    double full, off, diag;
    A.relax(i, [&](int32_t j) { return x[j]; }, full, off, diag);
    if (Mode == kGsLagged) {
      const double ri = bi - full;
      a.add(ri, ri);
      xs[t] = x[i];
    }
    x[i] = (bi - off) / diag;
    if (Mode == kGsFinal) {
      A.relax(i, [&](int32_t j) { return x[j]; }, full, off, diag);
      const double ri = bi - full;
      a.add(ri, ri);
    }
  });
  if (Mode != kGsPlain) block_partial_at(a.get(), Mode == kGsFinal ? 0 : 1, R);
}

// The same half-sweep over a colour's rows in their own packed layout (row p
// of the layout is rows[p]), so the entries stream coalesced.
template <int Mode, class Op>
__global__ void __launch_bounds__(kBlock) k_gs_rows_packed(Op A, const int32_t *__restrict__ rows,
                                                           const double *__restrict__ b, double *x,
                                                           double *__restrict__ xs,
                                                           const State *st, Reduce *R) {
  __shared__ typename Op::Smem sm;
  if (st->flag != kRunning) return;
  auto xj = [&](int32_t j) { return x[j]; };
  Dot2 a;
  for_tiles(A.n, [&](int32_t r0, int32_t r1) {
    const int32_t p = r0 + int32_t(threadIdx.x);
    const int32_t i = p < r1 ? rows[p] : -1;
    double full = 0.0, off = 0.0, diag = 0.0, xi = 0.0;
    A.tile_entries(r0, r1, sm, xj, [&](int32_t j, double av, double v) {
      if (Mode == kGsLagged) full = fma(av, v, full);
      if (j != i) {
        off = fma(av, v, off);
      } else {
        diag = av;
        xi = v;
      }
    });
    const double bi = p < r1 ? b[i] : 0.0;
    if (p < r1) {
      if (Mode == kGsLagged) {
        const double ri = bi - full;
        a.add(ri, ri);
        xs[p] = xi;
      }
      x[i] = (bi - off) / diag;
    }
    if (Mode == kGsFinal) {
      double f2 = 0.0;
      A.tile_entries(r0, r1, sm, xj, [&](int32_t, double av, double v) { f2 = fma(av, v, f2); });
      if (p < r1) {
        const double ri = bi - f2;
        a.add(ri, ri);
      }
    }
  }, rev_of(A));
  if (Mode != kGsPlain) block_partial_at(a.get(), Mode == kGsFinal ? 0 : 1, R, rev_of(A));
}

// Matrix-free half-sweep over one colour's cells, walked on a compact index
// so that every thread updates a cell: with two colours (7 points) every
// other cell of each x line, with eight (27 points) every other cell along
// each axis.
template <int NPTS>
__host__ __device__ inline int64_t gs_colour_cells(int32_t nx, int32_t ny, int32_t nz) {
  const int64_t hx = (nx + 1) / 2;
  return NPTS == 7 ? hx * ny * nz : hx * ((ny + 1) / 2) * ((nz + 1) / 2);
}

template <int NPTS>
__global__ void __launch_bounds__(kBlock) k_gs_stencil(StencilOp<NPTS, double> A, int32_t color,
                                                       const double *__restrict__ b, double *x,
                                                       const State *st) {
  if (st->flag != kRunning) return;
  const int32_t hx = (A.nx + 1) / 2;
  const int32_t hy = NPTS == 7 ? A.ny : (A.ny + 1) / 2;
  const int32_t cells = int32_t(gs_colour_cells<NPTS>(A.nx, A.ny, A.nz));
  for_rows(cells, [&](int32_t t) {
    const int32_t line = t / hx, k = t - line * hx;
    const int32_t qz = line / hy, qy = line - qz * hy;
    int32_t ix, iy, iz;
    if (NPTS == 7) {
      iy = qy;
      iz = qz;
      ix = 2 * k + ((color + iy + iz) & 1);
    } else {
      ix = 2 * k + (color & 1);
      iy = 2 * qy + ((color >> 1) & 1);
      iz = 2 * qz + (color >> 2);
    }
    if (ix >= A.nx || iy >= A.ny || iz >= A.nz) return;
    const int32_t i = ix + A.nx * (iy + A.ny * iz);
    double off = 0.0;
    A.row_entries_at(i, ix, iy, iz, [&](int32_t j) { return x[j]; },
                     [&](int32_t j, double av, double v) {
                       if (j != i) off = fma(av, v, off);
                     });
    x[i] = (b[i] - off) / A.c[NPTS / 2];
  });
}

// Puts the black rows of the tested iterate back: x[rows[p]] = xs[p] over the
// black colour's row list.
__global__ void __launch_bounds__(kBlock) k_gs_restore_rows(const int32_t *__restrict__ rows,
                                                            int32_t count, const double *__restrict__ xs,
                                                            double *__restrict__ x) {
  for_rows(count, [&](int32_t p) { x[rows[p]] = xs[p]; });
}

// The test after a lagged black sweep: r.r of the iterate = red part (slot 0,
// from the red sweep that made it) + black part (slot 1).
struct FinGs2 {
  State *st;
  __device__ bool active() const { return st->flag == kRunning; }
  __device__ void operator()(DD (&v)[2]) const {
    const double rr = dd_round(dd_add(v[0], v[1]));
    const int64_t k = st->k + 1;
    st->k = k;
    st->rho = rr;
    if (rr <= st->thr2)
      st->flag = kConverged;
    else if (!finite(rr))
      st->flag = kBreakdown;
    else if (k >= st->max_iter)
      st->flag = kMaxIter;
  }
};

// Residual of the iterate after a full symmetric iteration, and the test.
template <class Op>
__global__ void __launch_bounds__(kBlock) k_gs_check(Op A, const double *__restrict__ b,
                                                     const double *__restrict__ x, const State *st,
                                                     Reduce *R) {
  __shared__ typename Op::Smem sm;
  if (st->flag != kRunning) return;
  auto xj = [&](int32_t j) { return x[j]; };
  auto same = [](double v) { return v; };
  Dot2 a;
  A.rows(sm, xj, same, [&](int32_t i, bool valid, auto &&entries, auto &&) {
    double acc = 0.0;
    entries([&](int32_t, double av, double v) { acc = fma(av, v, acc); });
    if (valid) {
      const double ri = b[i] - acc;
      a.add(ri, ri);
    }
  });
  DD v[1] = {a.get()};
  block_partial<1>(v, R, rev_of(A));
}

// Residual of x_{k+1} after a symmetric iteration, and the test.
struct FinGs {
  State *st;
  __device__ bool active() const { return st->flag == kRunning; }
  __device__ void operator()(DD (&v)[1]) const {
    const double rr = dd_round(v[0]);
    const int64_t k = st->k + 1;
    st->k = k;
    st->rho = rr;
    if (rr <= st->thr2)
      st->flag = kConverged;
    else if (!finite(rr))
      st->flag = kBreakdown;
    else if (k >= st->max_iter)
      st->flag = kMaxIter;
  }
};

}  // namespace its
