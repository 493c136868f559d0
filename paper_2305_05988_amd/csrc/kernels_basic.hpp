// Basic kernels: state reset, dot product, SpMV, residual, fill.
#pragma once

#include "common.hpp"
#include "rowops.hpp"

namespace its {

// ------------------------------------------------------------------ basics

// Zero nstates consecutive States.
__global__ void k_reset(State *st, int nstates, Reduce *R) {
  uint32_t *w = reinterpret_cast<uint32_t *>(st);
  const int words = int(sizeof(State) / 4) * nstates;
  for (int i = threadIdx.x; i < words; i += blockDim.x) w[i] = 0u;
}

// Zero `count` 64-bit words (one block).
__global__ void k_zero_words(unsigned long long *w, int count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) w[i] = 0ull;
}

// ------------------------------------------------------ scalar updates
// Each reducing pass stores per-block partials; the finishing kernel that
// follows it on the stream reduces them and applies one of these.

// Stores a plain dot product into st->dot[out].
struct FinDot {
  State *st;
  int out;
  __device__ bool active() const { return true; }
  __device__ void operator()(DD (&v)[1]) const { st->dot[out] = dd_round(v[0]); }
};

// Start of an iteration loop; the stopping threshold and the iteration cap
// live in the State so that a captured graph of iterations serves any
// right-hand side.
__global__ void k_begin(State *st, int32_t flag, double rho, double thr2, int64_t max_iter) {
  if (threadIdx.x != 0) return;
  st->thr2 = thr2;
  st->max_iter = max_iter;
  st->flag = flag;
  st->k = 0;
  st->restart = 0;
  st->restarts = 0;
  st->rho = rho;
  st->alpha = st->beta = st->omega = 0.0;
  st->alpha_x = 0.0;
}

// Dot product x.y (finished by FinDot).
__global__ void __launch_bounds__(kBlock) k_dot(int32_t n, const double *__restrict__ x,
                                                const double *__restrict__ y, Reduce *R) {
  Dot2 a;
  for_rows(n, [&](int32_t i) { a.add(ld_nt(x + i), ld_nt(y + i)); });
  DD v[1] = {a.get()};
  block_partial<1>(v, R);
}

template <class Op>
__global__ void __launch_bounds__(kBlock) k_spmv(Op A, const double *__restrict__ x,
                                                 double *__restrict__ y) {
  __shared__ typename Op::Smem sm;
  auto xj = [&](int32_t j) { return x[j]; };
  auto same = [](double v) { return v; };
  A.rows(sm, xj, same, [&](int32_t i, bool valid, auto &&entries, auto &&) {
    double acc = 0.0;
    entries([&](int32_t, double a, double v) { acc = fma(a, v, acc); });
    if (valid) st_nt(y + i, acc);
  });
}

// r = b - A x (r may be null; entry i stored at r[i * rstride]) and r.r
// (finished by FinDot).
template <class Op>
__global__ void __launch_bounds__(kBlock) k_residual(Op A, const double *__restrict__ b,
                                                     const double *__restrict__ x, double *r,
                                                     int rstride, Reduce *R) {
  __shared__ typename Op::Smem sm;
  auto xj = [&](int32_t j) { return x[j]; };
  auto same = [](double v) { return v; };
  Dot2 a;
  A.rows(sm, xj, same, [&](int32_t i, bool valid, auto &&entries, auto &&) {
    double acc = 0.0;
    entries([&](int32_t, double av, double v) { acc = fma(av, v, acc); });
    if (valid) {
      const double ri = ld_nt(b + i) - acc;
      if (r) st_nt(r + int64_t(i) * rstride, ri);
      a.add(ri, ri);
    }
  });
  DD v[1] = {a.get()};
  block_partial<1>(v, R, rev_of(A));
}

__global__ void __launch_bounds__(kBlock) k_fill(int32_t n, double *x, double v) {
  for_rows(n, [&](int32_t i) { x[i] = v; });
}

}  // namespace its
