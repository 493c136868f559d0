// Persistent solver kernels: the whole iteration loop of CG, CG-NB or
// BiCGStab in one cooperative launch whose blocks are all co-resident and
// meet at grid barriers (common.hpp) instead of kernel boundaries.  Where a
// launch costs more than a pass's work (small systems: the loop is bound by
// launch and reduction latency, not HBM), each reduction point then costs
// one barrier instead of a pass kernel plus one or two finishing kernels.
//
// The row arithmetic is that of the streaming passes (kernels_cg.hpp,
// kernels_cgnb.hpp, kernels_bicgstab.hpp): the same fma chains, roundings
// and double-double dot products, so the iterates are the same bit for bit.
// Every block reduces the partials of every reduction itself, in one fixed
// order (finish_half), so all blocks hold the same scalars (a State copy in
// LDS), take the same decisions and leave the loop together; block 0 stores
// the final State for the host.
//
// The reduced-synchronisation forms of the paper (Section 3.1, Algorithms
// 1-2) become split-phase barriers: a block arrives as soon as its partial of
// a reduction is stored, does the work that does not need the reduced value,
// and only then waits.
//   CG (classical): the SpMV pass needs beta, the update needs alpha: both
//     barriers block; only the x update (read by no other block) runs between
//     arrive and wait of the r.r barrier.
//   CG-NB (Algorithm 1): alpha_n = r.r is arrived at before the SpMV on r
//     (r formed on the fly from the previous iterate's {r, A p} pairs), so the
//     SpMV overlaps that reduction; alpha_d blocks.  The pairs alternate
//     between two buffers, as a fast block's update pass may start while a
//     slow block's SpMV still gathers the previous iterate's pairs.
//   BiCGStab-B1 (Algorithm 2): alpha_d blocks; the omega reduction overlaps
//     the update x_{j+1/2} = x_j + alpha p_j, and the alpha_n, beta reduction
//     overlaps x_{j+1} = x_{j+1/2} + omega s_j (the B1 ordering; its other
//     overlapped update, p_{j+1/2}, is gathered by the next SpMV pass right
//     after that barrier, so it is formed before arriving).  With split =
//     false the same updates run after the waits (classical BiCGStab's three
//     blocking points), for comparison.
//
// Work that runs between arrive and wait touches only rows the block owns
// (own_rows(), the rows() mapping of the thread), which no other block reads
// before the next barrier.
#pragma once

#include "common.hpp"
#include "kernels_basic.hpp"
#include "kernels_bicgstab.hpp"
#include "kernels_cg.hpp"
#include "kernels_cgnb.hpp"
#include "rowops.hpp"

namespace its {

// Copies the State into the block's LDS copy.
__device__ __forceinline__ void load_state(State &ls, const State *gst) {
  if (threadIdx.x == 0) ls = *gst;
  __syncthreads();
}

// After the loop: one barrier (the last iteration's own-row updates of x
// become visible), then r = b - A x, its r.r into dot[2], and block 0 stores
// the State.
template <class Op>
__device__ __forceinline__ void persist_epilogue(const Op &A, typename Op::Smem &sm, const double *b,
                                                 const double *x, State &ls, State *gst, Reduce *R,
                                                 const GridSync &gs, SyncState &ss, int &buf) {
  grid_arrive(gs, ss);
  if (!grid_wait(gs, ss)) return;
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
  block_partial_half<1>(v, R, buf);
  grid_arrive(gs, ss);
  if (!grid_wait(gs, ss)) return;
  finish_half<1>(R, buf, FinDot{&ls, 2});
  buf ^= 1;
  if (blockIdx.x == 0 && threadIdx.x == 0) *gst = ls;
}

// ------------------------------------------------------------------- CG

template <class Op>
__global__ void __launch_bounds__(kBlock) k_cg_persist(Op A, double *x,
                                                       double2_t *rp,
                                                       double *q,
                                                       const double *b, State *gst,
                                                       Reduce *R, GridSync gs) {
  __shared__ typename Op::Smem sm;
  __shared__ State ls;
  load_state(ls, gst);
  SyncState ss;
  if (!grid_init(gs, ss)) return;
  int buf = 0;
  while (ls.flag == kRunning) {
    // SpMV pass: p = r + beta p on the fly, q = A p, p.q
    {
      const bool first = ls.k == 0;
      const double beta = ls.beta;
      auto load = [&](int32_t j) -> double2_t { return rp[j]; };
      auto pv = [&](const double2_t &v) -> double { return first ? v.x : fma(beta, v.y, v.x); };
      Dot2 a;
      A.rows(sm, load, pv, [&](int32_t i, bool valid, auto &&entries, auto &&own) {
        double acc = 0.0, pi = 0.0;
        bool have = false;
        entries([&](int32_t j, double av, double pj) {
          acc = fma(av, pj, acc);
          if (j == i) {
            pi = pj;
            have = true;
          }
        });
        if (valid) {
          q[i] = acc;
          if (!have) pi = own();
          a.add(pi, acc);
        }
      });
      DD v[1] = {a.get()};
      block_partial_half<1>(v, R, buf);
    }
    grid_arrive(gs, ss);
    if (!grid_wait(gs, ss)) return;
    finish_half<1>(R, buf, FinCg1{&ls});
    buf ^= 1;
    if (ls.flag != kRunning) break;
    // update pass (own rows): p = r + beta p, r -= alpha q, r.r
    const bool first = ls.k == 0;
    const double beta = ls.beta, alpha = ls.alpha;
    {
      Dot2 a;
      A.own_rows([&](int32_t i) {
        const double2_t v = rp[i];
        const double pi = first ? v.x : fma(beta, v.y, v.x);
        const double ri = fma(-alpha, q[i], v.x);
        double2_t o;
        o.x = ri;
        o.y = pi;
        rp[i] = o;
        a.add(ri, ri);
      });
      DD v[1] = {a.get()};
      block_partial_half<1>(v, R, buf);
    }
    grid_arrive(gs, ss);
    // split phase: x += alpha p for the own rows while the others arrive
    A.own_rows([&](int32_t i) { x[i] = fma(alpha, rp[i].y, x[i]); });
    if (!grid_wait(gs, ss)) return;
    finish_half<1>(R, buf, FinCg2{&ls});
    buf ^= 1;
  }
  persist_epilogue(A, sm, b, x, ls, gst, R, gs, ss, buf);
}

// ---------------------------------------------------------------- CG-NB
// ra[0], ra[1]: the {r, A p} pair buffers; iteration j reads ra[j & 1] and
// writes ra[(j + 1) & 1] (k_cgnb_init filled ra[0]).

template <class Op>
__global__ void __launch_bounds__(kBlock) k_cgnb_persist(Op A, double *x,
                                                         double2_t *ra0, double2_t *ra1,
                                                         double *p,
                                                         double *w,
                                                         const double *b, State *gst,
                                                         Reduce *R, GridSync gs) {
  __shared__ typename Op::Smem sm;
  __shared__ State ls;
  load_state(ls, gst);
  SyncState ss;
  if (!grid_init(gs, ss)) return;
  int buf = 0;
  while (ls.flag == kRunning) {
    const double2_t *cur = (ls.k & 1) ? ra1 : ra0;
    double2_t *nxt = (ls.k & 1) ? ra0 : ra1;
    const double alpha = ls.alpha;
    // r_j = r_{j-1} - alpha A p_{j-1} of the own rows and alpha_n,j = r_j.r_j
    {
      Dot2 a;
      A.own_rows([&](int32_t i) {
        const double2_t v = cur[i];
        const double ri = fma(-alpha, v.y, v.x);
        a.add(ri, ri);
      });
      DD v[1] = {a.get()};
      block_partial_half<1>(v, R, buf);
    }
    grid_arrive(gs, ss);
    // split phase: the SpMV on r_j (r_j formed on the fly for every gathered
    // column) overlaps the alpha_n reduction
    {
      auto load = [&](int32_t j) -> double2_t { return cur[j]; };
      auto rv = [&](const double2_t &v) -> double { return fma(-alpha, v.y, v.x); };
      A.rows(sm, load, rv, [&](int32_t i, bool valid, auto &&entries, auto &&) {
        double acc = 0.0;
        entries([&](int32_t, double av, double rj) { acc = fma(av, rj, acc); });
        if (valid) w[i] = acc;
      });
    }
    if (!grid_wait(gs, ss)) return;
    finish_half<1>(R, buf, FinCgnbX{&ls});
    buf ^= 1;
    // update pass (own rows): A p_j, p_j, x_j, alpha_d,j = (A p_j).p_j
    {
      const double beta = ls.beta, gamma = ls.gamma;
      const bool exact = ls.alpha_n == 0.0;
      Dot2 a;
      A.own_rows([&](int32_t i) {
        const double2_t v = cur[i];
        const double ri = fma(-alpha, v.y, v.x);
        const double api = fma(beta, v.y, w[i]);
        const double p_old = p[i];
        const double pi = fma(beta, p_old, ri);
        const double xi = x[i];
        x[i] = exact ? fma(alpha, p_old, xi) : fma(gamma, pi, fma(-gamma, ri, xi));
        p[i] = pi;
        double2_t o;
        o.x = ri;
        o.y = api;
        nxt[i] = o;
        a.add(api, pi);
      });
      DD v[1] = {a.get()};
      block_partial_half<1>(v, R, buf);
    }
    grid_arrive(gs, ss);
    if (!grid_wait(gs, ss)) return;
    finish_half<1>(R, buf, FinCgnbY{&ls});
    buf ^= 1;
  }
  persist_epilogue(A, sm, b, x, ls, gst, R, gs, ss, buf);
}

// ------------------------------------------------------------- BiCGStab
// Workspace as the streaming passes: {r, u} pairs, r', p, {r, v} pairs, t.

template <class Op, bool Split>
__global__ void __launch_bounds__(kBlock) k_bicg_persist(Op A, double *x,
                                                         double2_t *ru,
                                                         double *rs,
                                                         double *p,
                                                         double2_t *rv,
                                                         double *t,
                                                         const double *b, State *gst,
                                                         Reduce *R, double restart_tol2,
                                                         int32_t paper_mode, GridSync gs) {
  __shared__ typename Op::Smem sm;
  __shared__ State ls;
  load_state(ls, gst);
  SyncState ss;
  if (!grid_init(gs, ss)) return;
  int buf = 0;
  while (ls.flag == kRunning) {
    // pass A: p = r + beta u on the fly (p = r at the start and after a
    // restart; r' = r/||r|| after a restart), v = A p, alpha_d = v.r'
    {
      const bool plain = ls.k == 0 || ls.restart;
      const bool restart = ls.restart;
      const double bet = ls.beta;
      const double rn = restart ? __builtin_sqrt(ls.rho) : 1.0;
      auto load = [&](int32_t j) -> double2_t { return ru[j]; };
      auto pv = [&](const double2_t &e) -> double { return plain ? e.x : fma(bet, e.y, e.x); };
      Dot2 a;
      A.rows(sm, load, pv, [&](int32_t i, bool valid, auto &&entries, auto &&own) {
        double acc = 0.0, pi = 0.0;
        bool have = false;
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
          p[i] = pi;
          double2_t o;
          o.x = ri;
          o.y = acc;
          rv[i] = o;
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
      block_partial_half<1>(v, R, buf);
    }
    grid_arrive(gs, ss);
    if (!grid_wait(gs, ss)) return;
    finish_half<1>(R, buf, FinBicgA{&ls});
    buf ^= 1;
    if (ls.flag != kRunning) break;
    const double alpha = ls.alpha;
    // pass B: s = r - alpha v on the fly, t = A s, t.s and t.t
    {
      auto load = [&](int32_t j) -> double2_t { return rv[j]; };
      auto sv = [&](const double2_t &e) -> double { return fma(-alpha, e.y, e.x); };
      Dot2 a0, a1;
      A.rows(sm, load, sv, [&](int32_t i, bool valid, auto &&entries, auto &&own) {
        double acc = 0.0, si = 0.0;
        bool have = false;
        entries([&](int32_t j, double av, double sj) {
          acc = fma(av, sj, acc);
          if (j == i) {
            si = sj;
            have = true;
          }
        });
        if (valid) {
          if (!have) si = own();
          t[i] = acc;
          a0.add(acc, si);
          a1.add(acc, acc);
        }
      });
      DD d[2] = {a0.get(), a1.get()};
      block_partial_half<2>(d, R, buf);
    }
    grid_arrive(gs, ss);
    // x_{j+1/2} = x_j + alpha p_j: overlaps the omega reduction (B1)
    auto half_step = [&]() { A.own_rows([&](int32_t i) { x[i] = fma(alpha, p[i], x[i]); }); };
    if (Split) half_step();
    if (!grid_wait(gs, ss)) return;
    if (!Split) half_step();
    finish_half<2>(R, buf, FinBicgB{&ls});
    buf ^= 1;
    // pass C (own rows): s, r = s - omega t, u = p - omega v, r.r', r.r
    const double om = ls.omega;
    const bool half = (om == 0.0);
    {
      Dot2 a0, a1;
      A.own_rows([&](int32_t i) {
        const double2_t e = rv[i];
        const double si = fma(-alpha, e.y, e.x);
        const double ri = half ? si : fma(-om, t[i], si);
        double2_t o;
        o.x = ri;
        o.y = fma(-om, e.y, p[i]);
        ru[i] = o;
        a0.add(ri, rs[i]);
        a1.add(ri, ri);
      });
      DD d[2] = {a0.get(), a1.get()};
      block_partial_half<2>(d, R, buf);
    }
    grid_arrive(gs, ss);
    // x_{j+1} = x_{j+1/2} + omega s_j: overlaps the alpha_n, beta reduction
    auto full_step = [&]() {
      if (half) return;
      A.own_rows([&](int32_t i) {
        const double2_t e = rv[i];
        x[i] = fma(om, fma(-alpha, e.y, e.x), x[i]);
      });
    };
    if (Split) full_step();
    if (!grid_wait(gs, ss)) return;
    if (!Split) full_step();
    finish_half<2>(R, buf, FinBicgC{&ls, restart_tol2, paper_mode});
    buf ^= 1;
  }
  persist_epilogue(A, sm, b, x, ls, gst, R, gs, ss, buf);
}

}  // namespace its
