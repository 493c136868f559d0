// Conjugate gradient passes (FP64, and FP32 for the refinement's inner solve).
#pragma once

#include "common.hpp"
#include "rowops.hpp"

namespace its {

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
  using P2 = typename Pair<T>::type;
  const bool first = st->k == 0;
  const T beta = T(st->beta);
  auto load = [&](int32_t j) -> P2 { return rp[j]; };
  auto pv = [&](const P2 &v) -> T { return first ? v.x : fmaT(beta, v.y, v.x); };
  Dot2 a;
  A.rows(sm, load, pv, [&](int32_t i, bool valid, auto &&entries, auto &&own) {
    T acc = T(0), pi = T(0);
    bool have = false;  // p_i taken from the row's diagonal entry
    entries([&](int32_t j, T av, T pj) {
      acc = fmaT(av, pj, acc);
      if (j == i) {
        pi = pj;
        have = true;
      }
    });
    if (valid) {
      st_nt(q + i, acc);
      if (!have) pi = own();
      a.add(double(pi), double(acc));
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

// Pass 2 of the FP32 inner solve with two rows per thread: the rows' {r, p}
// pairs move as one 16-byte access and x, q as 8-byte ones, so a wave moves
// as many bytes per memory instruction as the FP64 pass (one row per thread
// would halve that and leave the pass instruction-bound).  Row arithmetic is
// that of k_cg_pass2<float>; the dot partial is exact before its final
// rounding, so the pairing of rows does not change it.
__global__ void __launch_bounds__(kBlock) k_cg_pass2_f32x2(int32_t n, float *__restrict__ x,
                                                           float2_t *__restrict__ rp,
                                                           const float *__restrict__ q,
                                                           const State *st, Reduce *R) {
  if (st->flag != kRunning) return;
  const bool first = st->k == 0;
  const float beta = float(st->beta), alpha = float(st->alpha);
  Dot2 a;
  // row with r_i, the old p_i, x_i, q_i: returns the new {r_i, p_i}, updates x_i
  auto row = [&](float r0, float pold, float &xi, float qi) -> float2_t {
    const float pi = first ? r0 : fmaT(beta, pold, r0);
    xi = fmaT(alpha, pi, xi);
    float2_t o;
    o.x = fmaT(-alpha, qi, r0);
    o.y = pi;
    a.add(double(o.x), double(o.x));
    return o;
  };
  for_rows(n >> 1, [&](int32_t i) {  // rows 2i, 2i + 1
    const float4_t v = ld_nt(reinterpret_cast<const float4_t *>(rp) + i);
    const float2_t xv = ld_nt(reinterpret_cast<const float2_t *>(x) + i);
    const float2_t qv = ld_nt(reinterpret_cast<const float2_t *>(q) + i);
    float x0 = xv.x, x1 = xv.y;
    const float2_t o0 = row(v.x, v.y, x0, qv.x);
    const float2_t o1 = row(v.z, v.w, x1, qv.y);
    float2_t xo;
    xo.x = x0;
    xo.y = x1;
    float4_t o;
    o.x = o0.x;
    o.y = o0.y;
    o.z = o1.x;
    o.w = o1.y;
    st_nt(reinterpret_cast<float2_t *>(x) + i, xo);
    st_nt(reinterpret_cast<float4_t *>(rp) + i, o);
  });
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {  // the last row of an odd n
    const int32_t i = n - 1;
    const float2_t v = rp[i];
    float xi = x[i];
    const float2_t o = row(v.x, v.y, xi, q[i]);
    x[i] = xi;
    rp[i] = o;
  }
  DD v[1] = {a.get()};
  block_partial<1>(v, R);
}

// rho' = r.r, one more iteration, beta = rho'/rho, convergence test.
struct FinCg2 {
  State *st;
  __device__ bool active() const { return st->flag == kRunning; }
  __device__ void operator()(DD (&v)[1]) const {
    const double rho_new = dd_round(v[0]);
    const int64_t k = st->k + 1;
    st->k = k;
    st->beta = rho_new / st->rho;
    st->rho = rho_new;
    if (rho_new <= st->thr2)
      st->flag = kConverged;
    else if (!finite(rho_new))
      st->flag = kBreakdown;
    else if (k >= st->max_iter)
      st->flag = kMaxIter;
  }
};

}  // namespace its
