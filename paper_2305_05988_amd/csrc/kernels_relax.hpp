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
      st_nt(xn + i, (bi - off) / diag);
    }
  });
  DD v[1] = {a.get()};
  block_partial<1>(v, R);
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

__global__ void __launch_bounds__(kBlock) k_gs_rows_csr(CsrOp<double, double> A,
                                                        const int32_t *__restrict__ rows,
                                                        int32_t count, const double *__restrict__ b,
                                                        double *x, const State *st) {
  if (st->flag != kRunning) return;
  for_rows(count, [&](int32_t t) {
    const int32_t i = rows[t];
    double full, off, diag;
    A.relax(i, [&](int32_t j) { return x[j]; }, full, off, diag);
    x[i] = (b[i] - off) / diag;
  });
}

// The same half-sweep over a colour's rows in their own packed layout (row p
// of the layout is rows[p]), so the entries stream coalesced.
__global__ void __launch_bounds__(kBlock) k_gs_rows_packed(SellOp<double, double> A,
                                                           const int32_t *__restrict__ rows,
                                                           const double *__restrict__ b, double *x,
                                                           const State *st) {
  __shared__ SellOp<double, double>::Smem sm;
  if (st->flag != kRunning) return;
  auto xj = [&](int32_t j) { return x[j]; };
  for_tiles(A.n, [&](int32_t r0, int32_t r1) {
    const int32_t p = r0 + int32_t(threadIdx.x);
    const int32_t i = p < r1 ? rows[p] : -1;
    double off = 0.0, diag = 0.0;
    A.tile_entries(r0, r1, sm, xj, [&](int32_t j, double av, double v) {
      if (j != i)
        off = fma(av, v, off);
      else
        diag = av;
    });
    if (p < r1) x[i] = (b[i] - off) / diag;
  });
}

template <int NPTS>
__global__ void __launch_bounds__(kBlock) k_gs_stencil(StencilOp<NPTS, double> A, int32_t color,
                                                       const double *__restrict__ b, double *x,
                                                       const State *st) {
  if (st->flag != kRunning) return;
  for_rows(A.n, [&](int32_t i) {
    int32_t ix, iy, iz;
    A.coords(i, ix, iy, iz);
    const int32_t c = (NPTS == 7) ? ((ix + iy + iz) & 1) : ((ix & 1) + 2 * (iy & 1) + 4 * (iz & 1));
    if (c != color) return;
    double off = 0.0;
    A.row_entries_at(i, ix, iy, iz, [&](int32_t j) { return x[j]; },
                     [&](int32_t j, double av, double v) {
                       if (j != i) off = fma(av, v, off);
                     });
    x[i] = (b[i] - off) / A.c[NPTS / 2];
  });
}

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
  block_partial<1>(v, R);
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
