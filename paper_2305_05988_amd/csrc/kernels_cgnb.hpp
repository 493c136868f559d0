// CG-NB, the paper's nonblocking CG (Algorithm 1), in two fused passes per
// iteration.  The SpMV is applied to r; A p is carried by the recurrence
// A p_j = A r_j + beta_j A p_{j-1}; r and A p are stored interleaved as pairs
// {r_i, (Ap)_i} so the SpMV pass gathers both with one access.
//   pass X: r_j = r_{j-1} - alpha_{j-1} (Ap)_{j-1} formed on the fly for every
//           gathered column, w = A r_j, alpha_n,j = r_j.r_j
//   pass Y: r_j again (same fma), (Ap)_j = fma(beta, (Ap)_{j-1}, w),
//           p_j = fma(beta, p_{j-1}, r_j),
//           x_j = x_{j-1} + gamma (p_j - r_j) as the three-term update
//           fma(gamma, p_j, fma(-gamma, r_j, x_{j-1})),
//           alpha_d,j = (Ap)_j.p_j
// with beta = alpha_n,j / alpha_n,j-1 and
// gamma = alpha_n,j-1^2 / (alpha_d,j-1 alpha_n,j).  (Algorithm 1 prints the x
// update with a minus sign; gamma (p_j - r_j) = alpha_{j-1} p_{j-1}, so it is
// an addition.)  If alpha_n,j is exactly 0, gamma divides by zero and the
// update takes its exact value alpha_{j-1} p_{j-1}.
#pragma once

#include "common.hpp"
#include "rowops.hpp"

namespace its {

// Start: w = A r0 (stored as (Ap)_0), p0 = r0, alpha_d,0 = (Ap)_0.p0.
template <class Op>
__global__ void __launch_bounds__(kBlock) k_cgnb_init(Op A, double2_t *__restrict__ ra,
                                                      double *__restrict__ p, Reduce *R) {
  __shared__ typename Op::Smem sm;
  auto rj = [&](int32_t j) -> double { return ra[j].x; };
  auto same = [](double v) { return v; };
  Dot2 a;
  A.rows(sm, rj, same, [&](int32_t i, bool valid, auto &&entries, auto &&) {
    double acc = 0.0;
    entries([&](int32_t, double av, double v) { acc = fma(av, v, acc); });
    if (valid) {
      const double ri = ra[i].x;
      st_nt(p + i, ri);
      a.add(acc, ri);
      // own pair only: other rows gather the .x member, never .y
      ra[i].y = acc;
    }
  });
  DD v[1] = {a.get()};
  block_partial<1>(v, R, rev_of(A));
}

struct FinCgnbInit {  // alpha_d,0 and alpha_0
  State *st;
  __device__ bool active() const { return st->flag == kRunning; }
  __device__ void operator()(DD (&v)[1]) const {
    const double ad = dd_round(v[0]);
    if (ad == 0.0 || !finite(ad)) {
      st->flag = kBreakdown;
    } else {
      st->alpha_d = ad;
      st->alpha = st->rho / ad;
    }
  }
};

template <class Op>
__global__ void __launch_bounds__(kBlock) k_cgnb_x(Op A, const double2_t *__restrict__ ra,
                                                   double *__restrict__ w, const State *st,
                                                   Reduce *R) {
  __shared__ typename Op::Smem sm;
  if (st->flag != kRunning) return;
  const double alpha = st->alpha;
  auto load = [&](int32_t j) -> double2_t { return ra[j]; };
  auto rv = [&](const double2_t &v) -> double { return fma(-alpha, v.y, v.x); };
  Dot2 a;
  A.rows(sm, load, rv, [&](int32_t i, bool valid, auto &&entries, auto &&own) {
    double acc = 0.0, ri = 0.0;
    bool have = false;  // r_i taken from the row's diagonal entry
    entries([&](int32_t j, double av, double rj) {
      acc = fma(av, rj, acc);
      if (j == i) {
        ri = rj;
        have = true;
      }
    });
    if (valid) {
      st_nt(w + i, acc);
      if (!have) ri = own();
      a.add(ri, ri);
    }
  });
  DD v[1] = {a.get()};
  block_partial<1>(v, R, rev_of(A));
}

// alpha_n,j; beta and gamma for pass Y.
struct FinCgnbX {
  State *st;
  __device__ bool active() const { return st->flag == kRunning; }
  __device__ void operator()(DD (&v)[1]) const {
    const double an_new = dd_round(v[0]), an = st->rho;
    st->alpha_n = an_new;
    st->beta = an_new / an;
    st->gamma = (an * an) / (st->alpha_d * an_new);
  }
};

template <bool Keep>
__global__ void __launch_bounds__(kBlock) k_cgnb_y(int32_t n, double *__restrict__ x,
                                                   double2_t *__restrict__ ra,
                                                   double *__restrict__ p,
                                                   const double *__restrict__ w, const State *st,
                                                   Reduce *R) {
  if (st->flag != kRunning) return;
  const double alpha = st->alpha, beta = st->beta, gamma = st->gamma;
  const bool exact = st->alpha_n == 0.0;  // gamma = 1/0: use the limit alpha p_{j-1}
  Dot2 a;
  for_rows(n, [&](int32_t i) {
    const double2_t v = ld_nt(ra + i);
    const double ri = fma(-alpha, v.y, v.x);
    const double api = fma(beta, v.y, ld_nt(w + i));
    const double p_old = ld_nt(p + i);
    const double pi = fma(beta, p_old, ri);
    const double xi = ld_nt(x + i);
    st_nt(x + i, exact ? fma(alpha, p_old, xi) : fma(gamma, pi, fma(-gamma, ri, xi)));
    st_nt(p + i, pi);
    double2_t o;
    o.x = ri;
    o.y = api;
    st_pairs<Keep>(ra + i, o);
    a.add(api, pi);
  }, Keep);  // backwards with kept pairs: k_cgnb_x starts where this ends
  DD v[1] = {a.get()};
  block_partial<1>(v, R, Keep);
}

// alpha_d,j; one more iteration; the test on alpha_n,j (the residual of the
// x_j just formed); alpha_j for the next pass X.
struct FinCgnbY {
  State *st;
  __device__ bool active() const { return st->flag == kRunning; }
  __device__ void operator()(DD (&v)[1]) const {
    const double ad = dd_round(v[0]), an = st->alpha_n;
    const int64_t k = st->k + 1;
    st->k = k;
    st->rho = an;
    if (an <= st->thr2)
      st->flag = kConverged;
    else if (!finite(an))
      st->flag = kBreakdown;
    else if (k >= st->max_iter)
      st->flag = kMaxIter;
    else if (ad == 0.0 || !finite(ad))
      st->flag = kBreakdown;
    else {
      st->alpha_d = ad;
      st->alpha = an / ad;
    }
  }
};

}  // namespace its
