// HIP kernels of the solver hot path.  Each iteration of a method is a short
// sequence of fused streaming passes; the scalars of the method live in a
// device State and are produced by the block that finishes each pass's
// grid reduction, so an iteration needs no host round trip.
#pragma once

#include "common.hpp"
#include "ops.hpp"

namespace its {

// ------------------------------------------------------------------ basics

// Zero nstates consecutive States.
__global__ void k_reset(State *st, int nstates, Reduce *R) {
  uint32_t *w = reinterpret_cast<uint32_t *>(st);
  const int words = int(sizeof(State) / 4) * nstates;
  for (int i = threadIdx.x; i < words; i += blockDim.x) w[i] = 0u;
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

__global__ void k_begin(State *st, int32_t flag, double rho) {
  if (threadIdx.x != 0) return;
  st->flag = flag;
  st->k = 0;
  st->restart = 0;
  st->restarts = 0;
  st->rho = rho;
  st->alpha = st->beta = st->omega = 0.0;
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
  for_tiles(A.n, [&](int32_t r0, int32_t r1) {
    double acc = 0.0;
    A.tile_entries(r0, r1, sm, xj, [&](int32_t, double a, double v) { acc = fma(a, v, acc); });
    const int32_t i = r0 + int32_t(threadIdx.x);
    if (i < r1) st_nt(y + i, acc);
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
  Dot2 a;
  for_tiles(A.n, [&](int32_t r0, int32_t r1) {
    double acc = 0.0;
    A.tile_entries(r0, r1, sm, xj, [&](int32_t, double av, double v) { acc = fma(av, v, acc); });
    const int32_t i = r0 + int32_t(threadIdx.x);
    if (i < r1) {
      const double ri = ld_nt(b + i) - acc;
      if (r) st_nt(r + int64_t(i) * rstride, ri);
      a.add(ri, ri);
    }
  });
  DD v[1] = {a.get()};
  block_partial<1>(v, R);
}

__global__ void __launch_bounds__(kBlock) k_fill(int32_t n, double *x, double v) {
  for_rows(n, [&](int32_t i) { x[i] = v; });
}

// ---------------------------------------------------------------------- CG
// Classical CG, two fused passes per iteration (T = double, or float for the
// inner solve of the mixed-precision refinement):
//   pass 1: p = r + beta p formed on the fly for every gathered column,
//           q = A p, alpha = rho / (p.q)
//   pass 2: p = r + beta p stored, x += alpha p, r -= alpha q, rho' = r.r,
//           convergence test, beta = rho'/rho
// At the first iteration p = r.  r and p are stored interleaved as pairs
// {r_i, p_i}, so pass 1 gathers both with one access per column.

template <class Op, class T>
__global__ void __launch_bounds__(kBlock) k_cg_pass1(Op A,
                                                     const typename Pair<T>::type *__restrict__ rp,
                                                     T *__restrict__ q, const State *st,
                                                     Reduce *R) {
  __shared__ typename Op::Smem sm;
  if (st->flag != kRunning) return;
  const bool first = st->k == 0;
  const T beta = T(st->beta);
  auto pj = [&](int32_t j) -> T {
    const typename Pair<T>::type v = rp[j];
    return first ? v.x : fmaT(beta, v.y, v.x);
  };
  Dot2 a;
  for_tiles(A.n, [&](int32_t r0, int32_t r1) {
    T acc = T(0);
    A.tile_entries(r0, r1, sm, pj, [&](int32_t, T av, T v) { acc = fmaT(av, v, acc); });
    const int32_t i = r0 + int32_t(threadIdx.x);
    if (i < r1) {
      st_nt(q + i, acc);
      a.add(double(pj(i)), double(acc));
    }
  });
  DD v[1] = {a.get()};
  block_partial<1>(v, R);
}

// alpha = rho / (p.q); p.q = 0 or non-finite is a breakdown.
struct FinCg1 {
  State *st;
  __device__ bool active() const { return st->flag == kRunning; }
  __device__ void operator()(DD (&v)[1]) const {
    const double pq = dd_round(v[0]);
    if (pq == 0.0 || !finite(pq))
      st->flag = kBreakdown;
    else
      st->alpha = st->rho / pq;
  }
};

template <class T>
__global__ void __launch_bounds__(kBlock) k_cg_pass2(int32_t n, T *__restrict__ x,
                                                     typename Pair<T>::type *__restrict__ rp,
                                                     const T *__restrict__ q, const State *st,
                                                     Reduce *R) {
  using P2 = typename Pair<T>::type;
  if (st->flag != kRunning) return;
  const bool first = st->k == 0;
  const T beta = T(st->beta), alpha = T(st->alpha);
  Dot2 a;
  for_rows(n, [&](int32_t i) {
    const P2 v = ld_nt(rp + i);
    const T r0 = v.x;
    const T pi = first ? r0 : fmaT(beta, v.y, r0);
    const T xi = ld_nt(x + i);
    const T qi = ld_nt(q + i);
    st_nt(x + i, fmaT(alpha, pi, xi));
    const T ri = fmaT(-alpha, qi, r0);
    P2 o;
    o.x = ri;
    o.y = pi;
    st_nt(rp + i, o);
    a.add(double(ri), double(ri));
  });
  DD v[1] = {a.get()};
  block_partial<1>(v, R);
}

// rho' = r.r, one more iteration, beta = rho'/rho, convergence test.
struct FinCg2 {
  State *st;
  double thr2;
  int64_t max_iter;
  __device__ bool active() const { return st->flag == kRunning; }
  __device__ void operator()(DD (&v)[1]) const {
    const double rho_new = dd_round(v[0]);
    const int64_t k = st->k + 1;
    st->k = k;
    st->beta = rho_new / st->rho;
    st->rho = rho_new;
    if (rho_new <= thr2)
      st->flag = kConverged;
    else if (!finite(rho_new))
      st->flag = kBreakdown;
    else if (k >= max_iter)
      st->flag = kMaxIter;
  }
};

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
  Dot2 a;
  for_tiles(A.n, [&](int32_t r0, int32_t r1) {
    const int32_t i = r0 + int32_t(threadIdx.x);
    double full = 0.0, off = 0.0, diag = 0.0;
    A.tile_entries(r0, r1, sm, xj, [&](int32_t j, double av, double v) {
      full = fma(av, v, full);
      if (j == i)
        diag = av;
      else
        off = fma(av, v, off);
    });
    if (i < r1) {
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
  double thr2;
  int64_t max_iter;
  __device__ bool active() const { return st->flag == kRunning; }
  __device__ void operator()(DD (&v)[1]) const {
    const double rr = dd_round(v[0]);
    const int64_t k = st->k;
    st->rho = rr;
    if (rr <= thr2)
      st->flag = kConverged;
    else if (!finite(rr))
      st->flag = kBreakdown;
    else if (k >= max_iter)
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
  Dot2 a;
  for_tiles(A.n, [&](int32_t r0, int32_t r1) {
    double acc = 0.0;
    A.tile_entries(r0, r1, sm, xj, [&](int32_t, double av, double v) { acc = fma(av, v, acc); });
    const int32_t i = r0 + int32_t(threadIdx.x);
    if (i < r1) {
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
  double thr2;
  int64_t max_iter;
  __device__ bool active() const { return st->flag == kRunning; }
  __device__ void operator()(DD (&v)[1]) const {
    const double rr = dd_round(v[0]);
    const int64_t k = st->k + 1;
    st->k = k;
    st->rho = rr;
    if (rr <= thr2)
      st->flag = kConverged;
    else if (!finite(rr))
      st->flag = kBreakdown;
    else if (k >= max_iter)
      st->flag = kMaxIter;
  }
};

// --------------------------------------------------------------- BiCGStab
// Algorithm 2's arithmetic in three fused passes per iteration:
//   A: p = r + beta (p - omega v) on the fly (p = r after a restart or at the
//      start), r' = r/||r|| after a restart, v = A p, alpha_d = v.r'
//   B: s = r - alpha v on the fly, t = A s, t.s, t.t, omega
//   C: x = (x + alpha p) + omega s, r = s - omega t, alpha_n' = r.r',
//      beta = r.r, restart test, convergence test
// p and v are double-buffered (pass A gathers the old ones).

__global__ void __launch_bounds__(kBlock) k_bicg_init(int32_t n, const double *__restrict__ r,
                                                      double *__restrict__ rs, Reduce *R,
                                                      double rnorm) {
  Dot2 a;
  for_rows(n, [&](int32_t i) {
    const double rsi = r[i] / rnorm;
    rs[i] = rsi;
    a.add(r[i], rsi);
  });
  DD v[1] = {a.get()};
  block_partial<1>(v, R);
}

struct FinBicgInit {  // alpha_n = r.r'
  State *st;
  __device__ bool active() const { return true; }
  __device__ void operator()(DD (&v)[1]) const { st->alpha_n = dd_round(v[0]); }
};

template <class Op>
__global__ void __launch_bounds__(kBlock) k_bicg_a(Op A, const double *__restrict__ r, double *rs,
                                                   const double *__restrict__ po,
                                                   const double *__restrict__ vo,
                                                   double *__restrict__ pn, double *__restrict__ vn,
                                                   const State *st, Reduce *R) {
  __shared__ typename Op::Smem sm;
  if (st->flag != kRunning) return;
  const bool plain = st->k == 0 || st->restart;
  const bool restart = st->restart;
  const double bet = st->beta, om = st->omega;
  const double rn = restart ? __builtin_sqrt(st->rho) : 1.0;
  auto pj = [&](int32_t j) -> double {
    return plain ? r[j] : fma(bet, fma(-om, vo[j], po[j]), r[j]);
  };
  Dot2 a;
  for_tiles(A.n, [&](int32_t r0, int32_t r1) {
    double acc = 0.0;
    A.tile_entries(r0, r1, sm, pj, [&](int32_t, double av, double v) { acc = fma(av, v, acc); });
    const int32_t i = r0 + int32_t(threadIdx.x);
    if (i < r1) {
      st_nt(pn + i, pj(i));
      st_nt(vn + i, acc);
      double rsi;
      if (restart) {
        rsi = r[i] / rn;
        rs[i] = rsi;
      } else {
        rsi = rs[i];
      }
      a.add(acc, rsi);
    }
  });
  DD v[1] = {a.get()};
  block_partial<1>(v, R);
}

// alpha_d = v.r', alpha = alpha_n / alpha_d; the restart (if any) is consumed.
struct FinBicgA {
  State *st;
  __device__ bool active() const { return st->flag == kRunning; }
  __device__ void operator()(DD (&v)[1]) const {
    const double ad = dd_round(v[0]);
    st->restart = 0;
    if (ad == 0.0 || !finite(ad)) {
      st->flag = kBreakdown;
    } else {
      st->alpha_d = ad;
      st->alpha = st->alpha_n / ad;
    }
  }
};

template <class Op>
__global__ void __launch_bounds__(kBlock) k_bicg_b(Op A, const double *__restrict__ r,
                                                   const double *__restrict__ v,
                                                   double *__restrict__ t, const State *st,
                                                   Reduce *R) {
  __shared__ typename Op::Smem sm;
  if (st->flag != kRunning) return;
  const double alpha = st->alpha;
  auto sj = [&](int32_t j) -> double { return fma(-alpha, v[j], r[j]); };
  Dot2 a0, a1;
  for_tiles(A.n, [&](int32_t r0, int32_t r1) {
    double acc = 0.0;
    A.tile_entries(r0, r1, sm, sj, [&](int32_t, double av, double x) { acc = fma(av, x, acc); });
    const int32_t i = r0 + int32_t(threadIdx.x);
    if (i < r1) {
      st_nt(t + i, acc);
      a0.add(acc, sj(i));
      a1.add(acc, acc);
    }
  });
  DD d[2] = {a0.get(), a1.get()};
  block_partial<2>(d, R);
}

// omega = (t.s) / (t.t), 0 if t.t = 0.
struct FinBicgB {
  State *st;
  __device__ bool active() const { return st->flag == kRunning; }
  __device__ void operator()(DD (&d)[2]) const {
    const double ts = dd_round(d[0]), tt = dd_round(d[1]);
    st->ts = ts;
    st->tt = tt;
    st->omega = (tt == 0.0) ? 0.0 : ts / tt;
  }
};

__global__ void __launch_bounds__(kBlock) k_bicg_c(int32_t n, double *__restrict__ x, double *r,
                                                   const double *__restrict__ rs,
                                                   const double *__restrict__ p,
                                                   const double *__restrict__ v,
                                                   const double *__restrict__ t, const State *st,
                                                   Reduce *R) {
  if (st->flag != kRunning) return;
  const double alpha = st->alpha, om = st->omega;
  const bool half = (om == 0.0);
  Dot2 a0, a1;
  for_rows(n, [&](int32_t i) {
    const double si = fma(-alpha, ld_nt(v + i), ld_nt(r + i));
    const double xi = ld_nt(x + i), pi = ld_nt(p + i), rsi = ld_nt(rs + i);
    double ri;
    if (half) {
      st_nt(x + i, fma(alpha, pi, xi));
      ri = si;
    } else {
      st_nt(x + i, fma(om, si, fma(alpha, pi, xi)));
      ri = fma(-om, ld_nt(t + i), si);
    }
    st_nt(r + i, ri);
    a0.add(ri, rsi);
    a1.add(ri, ri);
  });
  DD d[2] = {a0.get(), a1.get()};
  block_partial<2>(d, R);
}

// alpha_n' = r.r', beta = r.r; the restart test, then the convergence test
// (in that order, as the restart count of the returned iterate includes a
// restart decided in its last iteration).
struct FinBicgC {
  State *st;
  double thr2;
  int64_t max_iter;
  double restart_tol2;
  int32_t paper_mode;
  __device__ bool active() const { return st->flag == kRunning; }
  __device__ void operator()(DD (&d)[2]) const {
    const double om = st->omega;
    const bool half = (om == 0.0);
    const double an = dd_round(d[0]), beta = dd_round(d[1]);
    const int64_t k = st->k + 1;
    st->k = k;
    st->rho = beta;
    if (half) {
      st->flag = (beta <= thr2) ? kConverged : kBreakdown;
      return;
    }
    const bool want = paper_mode ? (__builtin_fabs(an) < restart_tol2)
                                 : (an * an < restart_tol2 * beta);
    if (want && beta > 0.0 && finite(beta)) {
      st->restart = 1;
      st->alpha_n = __builtin_sqrt(beta);
      st->restarts += 1;
    } else {
      st->beta = an / (st->alpha_d * om);
      st->alpha_n = an;
    }
    if (beta <= thr2)
      st->flag = kConverged;
    else if (!finite(beta))
      st->flag = kBreakdown;
    else if (k >= max_iter)
      st->flag = kMaxIter;
  }
};

// ------------------------------------------------- mixed-precision refinement
// Outer step: rh = (float)(r/rn), d = 0, rh.rh; then (after the inner CG)
// x += rn * d in double.

// rh is the first member of the inner {r, p} pairs (stride 2).
__global__ void __launch_bounds__(kBlock) k_ir_scale(int32_t n, const double *__restrict__ r,
                                                     float *__restrict__ rh, float *__restrict__ d,
                                                     Reduce *R, double rn) {
  Dot2 a;
  for_rows(n, [&](int32_t i) {
    const float v = float(r[i] / rn);
    rh[2 * int64_t(i)] = v;
    d[i] = 0.0f;
    a.add(double(v), double(v));
  });
  DD v[1] = {a.get()};
  block_partial<1>(v, R);
}

__global__ void __launch_bounds__(kBlock) k_ir_update(int32_t n, double *__restrict__ x,
                                                      const float *__restrict__ d, double rn) {
  for_rows(n, [&](int32_t i) { st_nt(x + i, fma(rn, double(ld_nt(d + i)), ld_nt(x + i))); });
}

// ----------------------------------------------------------------- utilities

__global__ void __launch_bounds__(kBlock) k_cast_f32(int64_t n, const double *src, float *dst) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    dst[i] = float(src[i]);
}

// double -> IEEE half in one rounding (nearest-even), no float intermediate
__global__ void __launch_bounds__(kBlock) k_cast_f16(int64_t n, const double *src, _Float16 *dst) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    dst[i] = static_cast<_Float16>(src[i]);
}

// Streaming copy, 16 bytes per lane.
__global__ void __launch_bounds__(kBlock) k_copy(int64_t n, const double *__restrict__ src,
                                                 double *__restrict__ dst) {
  const int64_t n2 = n / 2;
  const double2 *s2 = reinterpret_cast<const double2 *>(src);
  double2 *d2 = reinterpret_cast<double2 *>(dst);
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n2; i += stride) d2[i] = s2[i];
  if (blockIdx.x == 0 && threadIdx.x == 0 && (n & 1)) dst[n - 1] = src[n - 1];
}

// CSR structure check: counts bad rows into *bad.
__global__ void __launch_bounds__(kBlock) k_csr_check(int32_t n, int32_t nnz,
                                                      const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ col,
                                                      const double *__restrict__ val,
                                                      int32_t need_diag, uint32_t *bad) {
  for_rows(n, [&](int32_t i) {
    const int32_t b = rp[i], e = rp[i + 1];
    bool ok = (b <= e) && (b >= 0) && (e <= nnz) && (i != 0 || b == 0) && (i != n - 1 || e == nnz);
    bool diag = false;
    if (ok) {
      int32_t last = -1;
      for (int32_t k = b; k < e; ++k) {
        const int32_t c = col[k];
        if (c < 0 || c >= n || c <= last) ok = false;
        last = c;
        if (c == i && val[k] != 0.0) diag = true;
      }
    }
    if (!ok || (need_diag && !diag)) atomicAdd(bad, 1u);
  });
}

// Colouring check: colour in range, no off-diagonal entry couples two rows
// of the same colour.
__global__ void __launch_bounds__(kBlock) k_color_check(int32_t n, const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ col,
                                                        const uint8_t *__restrict__ color,
                                                        int32_t ncolors, uint32_t *bad) {
  for_rows(n, [&](int32_t i) {
    const int32_t ci = color[i];
    bool ok = ci < ncolors;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
      const int32_t c = col[k];
      if (c != i && color[c] == ci) ok = false;
    }
    if (!ok) atomicAdd(bad, 1u);
  });
}

}  // namespace its
