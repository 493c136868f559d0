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
//
// x is read and written every other iteration (both pass 2 kernels): an even
// iteration k leaves x_k as it is and keeps alpha_k; the odd iteration k + 1,
// which reads p_k from the pairs anyway, forms
// x_{k+2} = fma(alpha_{k+1}, p_{k+1}, fma(alpha_k, p_k, x_k)), the same two
// roundings in the same order as updating x at each iteration.  A solve that
// stops after an even iteration applies the pending update with k_cg_flush_x
// (k_cg_flush_x32 for the FP32 inner solve).

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
  block_partial<1>(v, R, rev_of(A));
}

// Pass 1 of the refinement's FP32 inner CG on an FP32/FP16 offset-slice
// layout, two rows per lane (SellOp::walk_pairs): for each row the
// arithmetic of k_cg_pass1.  rp must be readable at indices -1 and n.
template <class Op>
__global__ void __launch_bounds__(kBlock) k_cg_pass1_pairs(Op A, const float2_t *rp, float *q,
                                                           const State *st, Reduce *R) {
  if (st->flag != kRunning) return;
  const bool first = st->k == 0;
  const float beta = float(st->beta);
  auto pv = [&](const float2_t &v) -> float { return first ? v.x : fmaT(beta, v.y, v.x); };
  Dot2 a;
  A.walk_pairs(rp, [&](int32_t i0, int32_t i1, bool valid0, bool valid1, auto &&entries) {
    float acc0 = 0.0f, acc1 = 0.0f, p0 = 0.0f, p1 = 0.0f;
    bool have0 = false, have1 = false;  // p_i taken from the row's diagonal entry
    entries(
        [&](int32_t j, float av, const float2_t &raw) {
          const float pj = pv(raw);
          acc0 = fmaT(av, pj, acc0);
          if (j == i0) {
            p0 = pj;
            have0 = true;
          }
        },
        [&](int32_t j, float av, const float2_t &raw) {
          const float pj = pv(raw);
          acc1 = fmaT(av, pj, acc1);
          if (j == i1) {
            p1 = pj;
            have1 = true;
          }
        });
    if (valid0) {
      st_nt(q + i0, acc0);
      if (!have0) p0 = pv(rp[i0]);
      a.add(double(p0), double(acc0));
    }
    if (valid1) {
      st_nt(q + i1, acc1);
      if (!have1) p1 = pv(rp[i1]);
      a.add(double(p1), double(acc1));
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

// pq, pq_count: when pq is not null, the SpMV pass's p.q as second-level
// (group) sums, at most kGroup, which every block reduces itself in the
// finishing kernel's order (finish_in_block) and turns into alpha as FinCg1
// does -- block 0 records alpha, or the breakdown, in the State -- so no
// finishing kernel runs between the two passes.  They must not be
// first-level partials: this pass writes its own partials there.
template <class T, bool Keep>
__global__ void __launch_bounds__(kBlock) k_cg_pass2(int32_t n, T *__restrict__ x,
                                                     typename Pair<T>::type *__restrict__ rp,
                                                     const T *__restrict__ q, State *st,
                                                     Reduce *R, const DD *pq, int32_t pq_count) {
  using P2 = typename Pair<T>::type;
  if (st->flag != kRunning) return;
  T alpha;
  if (pq) {
    __shared__ double s_alpha;
    __shared__ int s_ok;
    const double rho = st->rho;
    const DD *src[1] = {pq};
    finish_in_block<1>(src, pq_count, [&](DD (&v)[1]) {
      const double pqv = dd_round(v[0]);
      const bool ok = pqv != 0.0 && finite(pqv);
      s_ok = ok;
      s_alpha = ok ? rho / pqv : 0.0;
      if (blockIdx.x == 0) {
        if (ok)
          st->alpha = s_alpha;
        else
          st->flag = kBreakdown;
      }
    });
    __syncthreads();
    if (!s_ok) return;  // block-uniform
    alpha = T(s_alpha);
  } else {
    alpha = T(st->alpha);
  }
  const bool first = st->k == 0;
  const bool defer = (st->k & 1) == 0;  // x waits for the next iteration
  const T beta = T(st->beta), alpha_x = T(st->alpha_x);
  Dot2 a;
  // rows i and i + kBlock of each tile of 2 kBlock rows, the loads of both in
  // flight together (a row past n re-reads row n - 1 and stores nothing)
  const int64_t ntiles = (int64_t(n) + 2 * kBlock - 1) / (2 * kBlock);
  const Sched sc = my_tiles(ntiles);
  // the tiles are walked from the end of each XCD's chunk, where the SpMV
  // pass that ran just before finished, so the start of this pass finds
  // some of the lines that pass touched last still in the memory-side cache
  // (the partial slots and the rows of each block are those of a forward
  // walk; only the order in which a block's Dot2 takes its tiles differs)
  const int64_t last = sc.begin < sc.end ? sc.begin + (sc.end - 1 - sc.begin) / sc.stride * sc.stride
                                         : sc.begin - sc.stride;
  for (int64_t t = last; t >= sc.begin; t -= sc.stride) {
    int32_t i[2];
    i[0] = int32_t(t * 2 * kBlock + threadIdx.x);
    i[1] = i[0] + kBlock;
    P2 v[2];
    T qi[2], xi[2] = {T(0), T(0)};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int32_t j = min(i[h], n - 1);
      v[h] = ld_nt(rp + j);
      qi[h] = ld_nt(q + j);
      if (!defer) xi[h] = ld_nt(x + j);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (i[h] >= n) continue;
      const T r0 = v[h].x;
      const T pi = first ? r0 : fmaT(beta, v[h].y, r0);
      // on odd iterations v.y is p of the deferred even iteration
      if (!defer) st_nt(x + i[h], fmaT(alpha, pi, fmaT(alpha_x, v[h].y, xi[h])));
      const T ri = fmaT(-alpha, qi[h], r0);
      P2 o;
      o.x = ri;
      o.y = pi;
      st_pairs<Keep>(rp + i[h], o);
      a.add(double(ri), double(ri));
    }
  }
  DD v[1] = {a.get()};
  block_partial<1>(v, R);
}

// After the iterations of an FP64 CG solve: an odd count of completed
// iterations leaves the last one's x update pending (p is still in the
// pairs); apply it.
__global__ void __launch_bounds__(kBlock) k_cg_flush_x(int32_t n, double *__restrict__ x,
                                                       const double2_t *__restrict__ rp,
                                                       const State *st) {
  if ((st->k & 1) == 0) return;
  const double alpha_x = st->alpha_x;
  for_rows(n, [&](int32_t i) { x[i] = fma(alpha_x, rp[i].y, x[i]); });
}

// The same for the FP32 inner solve's correction d.
__global__ void __launch_bounds__(kBlock) k_cg_flush_x32(int32_t n, float *__restrict__ x,
                                                         const float2_t *__restrict__ rp,
                                                         const State *st) {
  if ((st->k & 1) == 0) return;
  const float alpha_x = float(st->alpha_x);
  for_rows(n, [&](int32_t i) { x[i] = fmaT(alpha_x, rp[i].y, x[i]); });
}

// Pass 2 of the FP32 inner solve with two rows per thread: the rows' {r, p}
// pairs move as one 16-byte access and x, q as 8-byte ones, so a wave moves
// as many bytes per memory instruction as the FP64 pass (one row per thread
// would halve that and leave the pass instruction-bound).  Row arithmetic is
// that of k_cg_pass2<float>; the dot partial is exact before its final
// rounding, so the pairing of rows does not change it.
template <bool Keep>
__global__ void __launch_bounds__(kBlock) k_cg_pass2_f32x2(int32_t n, float *__restrict__ x,
                                                           float2_t *__restrict__ rp,
                                                           const float *__restrict__ q,
                                                           const State *st, Reduce *R) {
  if (st->flag != kRunning) return;
  const bool first = st->k == 0;
  const bool defer = (st->k & 1) == 0;  // x waits for the next iteration, as in k_cg_pass2
  const float beta = float(st->beta), alpha = float(st->alpha), alpha_x = float(st->alpha_x);
  Dot2 a;
  // row with r_i, the old p_i, x_i, q_i: returns the new {r_i, p_i}, updates x_i
  // (on odd iterations, with the deferred step of the even one first)
  auto row = [&](float r0, float pold, float &xi, float qi) -> float2_t {
    const float pi = first ? r0 : fmaT(beta, pold, r0);
    if (!defer) xi = fmaT(alpha, pi, fmaT(alpha_x, pold, xi));
    float2_t o;
    o.x = fmaT(-alpha, qi, r0);
    o.y = pi;
    a.add(double(o.x), double(o.x));
    return o;
  };
  for_rows(n >> 1, [&](int32_t i) {  // rows 2i, 2i + 1
    const float4_t v = ld_nt(reinterpret_cast<const float4_t *>(rp) + i);
    float2_t xv = {0.0f, 0.0f};
    if (!defer) xv = ld_nt(reinterpret_cast<const float2_t *>(x) + i);
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
    if (!defer) st_nt(reinterpret_cast<float2_t *>(x) + i, xo);
    st_pairs<Keep>(reinterpret_cast<float4_t *>(rp) + i, o);
  });
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {  // the last row of an odd n
    const int32_t i = n - 1;
    const float2_t v = rp[i];
    float xi = defer ? 0.0f : x[i];
    const float2_t o = row(v.x, v.y, xi, q[i]);
    if (!defer) x[i] = xi;
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
    if (k & 1) st->alpha_x = st->alpha;  // iteration k - 1 (even) deferred its x update
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
