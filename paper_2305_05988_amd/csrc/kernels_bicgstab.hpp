// BiCGStab passes (arithmetic of the paper's Algorithm 2, with restart).
#pragma once

#include "common.hpp"
#include "rowops.hpp"

namespace its {

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
  // p_j from the loaded {r_j, p_j, v_j} (only r_j when p = r)
  struct RPV {
    double r, p, v;
  };
  auto load = [&](int32_t j) -> RPV {
    if (plain) return RPV{r[j], 0.0, 0.0};  // block-uniform
    return RPV{r[j], po[j], vo[j]};
  };
  auto pv = [&](const RPV &e) -> double { return plain ? e.r : fma(bet, fma(-om, e.v, e.p), e.r); };
  Dot2 a;
  A.rows(sm, load, pv, [&](int32_t i, bool valid, auto &&entries, auto &&own) {
    double acc = 0.0, pi = 0.0;
    bool have = false;  // p_i taken from the row's diagonal entry
    entries([&](int32_t j, double av, double p) {
      acc = fma(av, p, acc);
      if (j == i) {
        pi = p;
        have = true;
      }
    });
    if (valid) {
      if (!have) pi = own();
      st_nt(pn + i, pi);
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
  auto load = [&](int32_t j) -> double2_t {
    double2_t e;
    e.x = r[j];
    e.y = v[j];
    return e;
  };
  auto sv = [&](const double2_t &e) -> double { return fma(-alpha, e.y, e.x); };
  Dot2 a0, a1;
  A.rows(sm, load, sv, [&](int32_t i, bool valid, auto &&entries, auto &&own) {
    double acc = 0.0, si = 0.0;
    bool have = false;  // s_i taken from the row's diagonal entry
    entries([&](int32_t j, double av, double sv_j) {
      acc = fma(av, sv_j, acc);
      if (j == i) {
        si = sv_j;
        have = true;
      }
    });
    if (valid) {
      if (!have) si = own();
      st_nt(t + i, acc);
      a0.add(acc, si);
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
      st->flag = (beta <= st->thr2) ? kConverged : kBreakdown;
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
    if (beta <= st->thr2)
      st->flag = kConverged;
    else if (!finite(beta))
      st->flag = kBreakdown;
    else if (k >= st->max_iter)
      st->flag = kMaxIter;
  }
};

}  // namespace its
