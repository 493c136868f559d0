// BiCGStab passes (arithmetic of the paper's Algorithm 2, with restart).
#pragma once

#include "common.hpp"
#include "rowops.hpp"

namespace its {

// --------------------------------------------------------------- BiCGStab
// Algorithm 2's arithmetic in three fused passes per iteration:
//   A: p = r + beta u on the fly (p = r after a restart or at the start),
//      r' = r/||r|| after a restart, v = A p, alpha_d = v.r'
//   B: s = r - alpha v on the fly, t = A s, t.s, t.t, omega
//   C: x = (x + alpha p) + omega s, r = s - omega t, u = p - omega v,
//      alpha_n' = r.r', beta = r.r, restart test, convergence test
// u = p - omega v is formed in pass C, where omega is already known, so
// pass A forms p = fma(beta, u, r) -- the same roundings as forming
// fma(beta, fma(-omega, v, p), r) there.  What the SpMV passes gather is
// stored as interleaved pairs, one 16-byte access per column: {r, u} for
// pass A (written by pass C), {r, v} for pass B (written by pass A).

// r' = r / ||r||, alpha_n = r.r' (r: the first members of the {r, u} pairs)
__global__ void __launch_bounds__(kBlock) k_bicg_init(int32_t n, const double2_t *__restrict__ ru,
                                                      double *__restrict__ rs, Reduce *R,
                                                      double rnorm) {
  Dot2 a;
  for_rows(n, [&](int32_t i) {
    const double ri = ru[i].x;
    const double rsi = ri / rnorm;
    rs[i] = rsi;
    a.add(ri, rsi);
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
__global__ void __launch_bounds__(kBlock) k_bicg_a(Op A, const double2_t *__restrict__ ru,
                                                   double *__restrict__ rs, double *__restrict__ p,
                                                   double2_t *__restrict__ rv, const State *st,
                                                   Reduce *R) {
  __shared__ typename Op::Smem sm;
  if (st->flag != kRunning) return;
  const bool plain = st->k == 0 || st->restart;
  const bool restart = st->restart;
  const double bet = st->beta;
  const double rn = restart ? __builtin_sqrt(st->rho) : 1.0;
  auto load = [&](int32_t j) -> double2_t { return ru[j]; };
  auto pv = [&](const double2_t &e) -> double { return plain ? e.x : fma(bet, e.y, e.x); };
  Dot2 a;
  A.rows(sm, load, pv, [&](int32_t i, bool valid, auto &&entries, auto &&own) {
    double acc = 0.0, pi = 0.0;
    bool have = false;  // p_i taken from the row's diagonal entry
    entries([&](int32_t j, double av, double pj) {
      acc = fma(av, pj, acc);
      if (j == i) {
        pi = pj;
        have = true;
      }
    });
    if (valid) {
      if (!have) pi = own();
      const double ri = ru[i].x;
      st_nt(p + i, pi);
      double2_t o;
      o.x = ri;
      o.y = acc;
      st_pairs<GathersPairs<Op>::value>(rv + i, o);
      double rsi;
      if (restart) {
        rsi = ri / rn;
        rs[i] = rsi;
      } else {
        rsi = rs[i];
      }
      a.add(acc, rsi);
    }
  });
  DD v[1] = {a.get()};
  block_partial<1>(v, R, rev_of(A));
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
__global__ void __launch_bounds__(kBlock) k_bicg_b(Op A, const double2_t *__restrict__ rv,
                                                   double *__restrict__ t, const State *st,
                                                   Reduce *R) {
  __shared__ typename Op::Smem sm;
  if (st->flag != kRunning) return;
  const double alpha = st->alpha;
  auto load = [&](int32_t j) -> double2_t { return rv[j]; };
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
  block_partial<2>(d, R, rev_of(A));
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

template <bool Keep>
__global__ void __launch_bounds__(kBlock) k_bicg_c(int32_t n, double *__restrict__ x,
                                                   double2_t *__restrict__ ru,
                                                   const double *__restrict__ rs,
                                                   const double *__restrict__ p,
                                                   const double2_t *__restrict__ rv,
                                                   const double *__restrict__ t, const State *st,
                                                   Reduce *R) {
  if (st->flag != kRunning) return;
  const double alpha = st->alpha, om = st->omega;
  const bool half = (om == 0.0);
  Dot2 a0, a1;
  // rows i and i + kBlock of each tile of 2 kBlock rows, the loads of both in
  // flight together (a row past n re-reads row n - 1 and stores nothing)
  const int64_t ntiles = (int64_t(n) + 2 * kBlock - 1) / (2 * kBlock);
  const Sched sc = my_tiles(ntiles);
  for (int64_t k = sc.begin; k < sc.end; k += sc.stride) {
    int32_t i[2];
    i[0] = int32_t(k * 2 * kBlock + threadIdx.x);
    i[1] = i[0] + kBlock;
    double2_t e[2];
    double xi[2], pi[2], rsi[2], ti[2] = {0.0, 0.0};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int32_t j = min(i[h], n - 1);
      e[h] = ld_nt(rv + j);  // {r_j, v_j}
      xi[h] = ld_nt(x + j);
      pi[h] = ld_nt(p + j);
      rsi[h] = ld_nt(rs + j);
      if (!half) ti[h] = ld_nt(t + j);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (i[h] >= n) continue;
      const double si = fma(-alpha, e[h].y, e[h].x);
      double ri;
      if (half) {
        st_nt(x + i[h], fma(alpha, pi[h], xi[h]));
        ri = si;
      } else {
        st_nt(x + i[h], fma(om, si, fma(alpha, pi[h], xi[h])));
        ri = fma(-om, ti[h], si);
      }
      double2_t o;
      o.x = ri;
      o.y = fma(-om, e[h].y, pi[h]);  // u = p - omega v
      st_pairs<Keep>(ru + i[h], o);
      a0.add(ri, rsi[h]);
      a1.add(ri, ri);
    }
  }
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
