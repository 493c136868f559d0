// Batched CG: many independent variable-coefficient diffusion systems, each
// with several right-hand sides, advanced together.
#pragma once

#include "common.hpp"

namespace its {

// Layout.  The systems' cells are concatenated (system s owns global cells
// [off_s, off_s + n_s), rows numbered i + nx(j + ny k) inside it).  Vectors
// interleave the right-hand sides: value (cell g, rhs r) sits at g R + r, so
// a block's 256 threads cover 256/R consecutive cells x R right-hand sides
// and every access is coalesced.  The operator is stored once per cell as
// its 7 coefficients in chain order (z-1, y-1, x-1, diagonal, x+1, y+1, z+1;
// 0 outside the grid), coef[o * ncell + g], and reused by all R right-hand
// sides.  Work items are runs of 256/R-cell tiles inside one system; each
// item leaves one double-double partial per right-hand side, and one block
// per system finishes the reductions in a fixed order.  After every
// iteration the items of the systems still running are gathered, with all
// a block needs to start loading, into a dense list that the two CG passes
// walk, so stopped systems cost nothing and the work stays spread evenly.
constexpr int kBatchMaxRhs = 8;

// Division of an unsigned 32-bit value by a fixed divisor d >= 1 as a
// multiply-high and shifts (Granlund and Montgomery, 1994: m = floor(2^32
// (2^l - d) / d) + 1 with l = ceil(log2 d)), exact for every 32-bit value.
struct Divisor {
  uint32_t m, s1, s2;
  __device__ __forceinline__ uint32_t div(uint32_t n) const {
    const uint32_t t = __umulhi(m, n);
    return (t + ((n - t) >> s1)) >> s2;
  }
};

inline Divisor make_divisor(uint32_t d) {
  uint32_t l = 0;
  while ((uint64_t(1) << l) < d) ++l;
  Divisor v;
  v.m = uint32_t(((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1);
  v.s1 = l < 1 ? l : 1;
  v.s2 = l > 1 ? l - 1 : 0;
  return v;
}

struct BatchSys {
  int64_t off;           // first global cell
  int32_t nx, ny, nz;
  int32_t tiles;         // ceil(n / cells per tile)
  int32_t item0, item1;  // its work items
  Divisor dx, dy;        // by nx and by ny
  int32_t pad;
};

struct BatchItem {
  int32_t sys, t0, t1;   // tiles [t0, t1) of system sys
  int32_t pad;
};

// An item of a running system, as the CG passes read it.
struct BatchAct {
  BatchSys sy;
  int32_t w;             // the item's index (its partial slot)
  int32_t sys, t0, t1;
};

// CG scalars of one (system, right-hand side).
struct BatchCg {
  double rho, alpha, beta, bb, thr2;
  int64_t k;
  int32_t flag;
  int32_t zero_b;
};

struct BatchView {
  int32_t nsys, nrhs, cells;  // cells per tile = kBlock / nrhs
  int32_t nitems;
  int64_t ncell;
  const BatchSys *sys;
  const BatchItem *items;
  const double *coef;
  BatchCg *st;
  int32_t *sys_run;  // per system: 1 while any of its right-hand sides runs
  int32_t *sys_base; // per system: its first slot in act (running systems)
  int32_t *nact;     // items of the running systems
  BatchAct *act;     // those items, in system and item order
  DD *part;          // [item][rhs][2]
};

__device__ __forceinline__ void batch_coords(const BatchSys &sy, int64_t lc, int32_t &ix,
                                             int32_t &iy, int32_t &iz) {
  const int32_t t = int32_t(lc / sy.nx);
  ix = int32_t(lc - int64_t(t) * sy.nx);
  iz = t / sy.ny;
  iy = t - iz * sy.ny;
}

// Per-cell coefficients of the variable-coefficient operator (the roundings
// of VarCoefOp: harmonic faces ((2 a) b) / (a + b) with a the lower row,
// boundary face = the cell's k, diagonal summed from 0 in face order).
__global__ void __launch_bounds__(kBlock) k_batch_coef(BatchView V, const double *__restrict__ k,
                                                       double *__restrict__ coef) {
  for (int32_t s = blockIdx.x; s < V.nsys; s += gridDim.x) {
    const BatchSys sy = V.sys[s];
    const int64_t n = int64_t(sy.nx) * sy.ny * sy.nz;
    const int64_t nxy = int64_t(sy.nx) * sy.ny;
    for (int64_t lc = threadIdx.x; lc < n; lc += kBlock) {
      int32_t ix, iy, iz;
      batch_coords(sy, lc, ix, iy, iz);
      const int64_t g = sy.off + lc;
      const bool in[6] = {iz > 0, iy > 0, ix > 0, ix < sy.nx - 1, iy < sy.ny - 1, iz < sy.nz - 1};
      const int64_t off[6] = {-nxy, -sy.nx, -1, 1, sy.nx, nxy};
      const double kc = k[g];
      double f[6], diag = 0.0;
#pragma unroll
      for (int o = 0; o < 6; ++o) {
        if (!in[o]) {
          f[o] = kc;
        } else {
          const double kn = k[g + off[o]];
          f[o] = o < 3 ? (2.0 * kn * kc) / (kn + kc) : (2.0 * kc * kn) / (kc + kn);
        }
        diag = diag + f[o];
      }
      const int64_t N = V.ncell;
      coef[0 * N + g] = in[0] ? -f[0] : 0.0;
      coef[1 * N + g] = in[1] ? -f[1] : 0.0;
      coef[2 * N + g] = in[2] ? -f[2] : 0.0;
      coef[3 * N + g] = diag;
      coef[4 * N + g] = in[3] ? -f[3] : 0.0;
      coef[5 * N + g] = in[4] ? -f[4] : 0.0;
      coef[6 * N + g] = in[5] ? -f[5] : 0.0;
    }
  }
}

// Sums of the threads that share a right-hand side (lane % R), valid in
// threads 0..R-1; fixed order: butterfly within the wave, then waves 0..3.
template <int ND>
__device__ __forceinline__ void batch_block_reduce(DD (&v)[ND], int R) {
  __shared__ DD sm[ND][kWaves][kBatchMaxRhs];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int off = 32; off >= R; off >>= 1) {
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      DD o;
      o.hi = __shfl_xor(v[d].hi, off);
      o.lo = __shfl_xor(v[d].lo, off);
      v[d] = dd_add(v[d], o);
    }
  }
  if (lane < R) {
#pragma unroll
    for (int d = 0; d < ND; ++d) sm[d][w][lane] = v[d];
  }
  __syncthreads();
  if (int(threadIdx.x) < R) {
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      DD t = sm[d][0][threadIdx.x];
      for (int j = 1; j < kWaves; ++j) t = dd_add(t, sm[d][j][threadIdx.x]);
      v[d] = t;
    }
  }
  __syncthreads();
}

// One row of the operator for (cell g, rhs r): the chain over the 7
// coefficients in order, neighbours outside the grid skipped; value(raw)
// forms x_j from the gathered entry.  Gathers are unconditional (outside the
// grid: the cell itself, not consumed).
template <class Load, class Value>
__device__ __forceinline__ double batch_row(const BatchView &V, const BatchSys &sy, int64_t lc,
                                            int r, Load &&load, Value &&value, double &own) {
  int32_t ix, iy, iz;
  batch_coords(sy, lc, ix, iy, iz);
  const int64_t g = sy.off + lc;
  const int64_t nxy = int64_t(sy.nx) * sy.ny;
  const bool in[7] = {iz > 0, iy > 0, ix > 0, true, ix < sy.nx - 1, iy < sy.ny - 1, iz < sy.nz - 1};
  const int64_t off[7] = {-nxy, -sy.nx, -1, 0, 1, sy.nx, nxy};
  decltype(load(0)) raw[7];
#pragma unroll
  for (int o = 0; o < 7; ++o) raw[o] = load((in[o] ? g + off[o] : g) * V.nrhs + r);
  double a[7];
#pragma unroll
  for (int o = 0; o < 7; ++o) a[o] = V.coef[o * V.ncell + g];
  double acc = 0.0;
#pragma unroll
  for (int o = 0; o < 7; ++o) {
    const double xj = value(raw[o]);
    if (o == 3) own = xj;
    if (in[o]) acc = fma(a[o], xj, acc);
  }
  return acc;
}

// Prologue: r = b - A x (stored as the first member of the {r, p} pairs),
// partials of r.r and b.b per (item, rhs).
__global__ void __launch_bounds__(kBlock) k_batch_residual(BatchView V, const double *__restrict__ b,
                                                           const double *__restrict__ x,
                                                           double2_t *__restrict__ rp) {
  const int R = V.nrhs, cl = threadIdx.x / R, r = threadIdx.x % R;
  const Sched sc = my_tiles(V.nitems);
  for (int64_t w = sc.begin; w < sc.end; w += sc.stride) {
    const BatchItem it = V.items[w];
    const BatchSys sy = V.sys[it.sys];
    const int64_t n = int64_t(sy.nx) * sy.ny * sy.nz;
    Dot2 arr, abb;
    for (int32_t t = it.t0; t < it.t1; ++t) {
      const int64_t lc = int64_t(t) * V.cells + cl;
      if (lc < n) {
        double own;
        const double ax = batch_row(V, sy, lc, r, [&](int64_t e) { return x[e]; },
                                    [](double v) { return v; }, own);
        const int64_t e = (sy.off + lc) * R + r;
        const double bi = b[e];
        const double ri = bi - ax;
        double2_t o;
        o.x = ri;
        o.y = 0.0;
        rp[e] = o;
        arr.add(ri, ri);
        abb.add(bi, bi);
      }
    }
    DD v[2] = {arr.get(), abb.get()};
    batch_block_reduce<2>(v, R);
    if (int(threadIdx.x) < R) {
      V.part[(int64_t(w) * R + threadIdx.x) * 2 + 0] = v[0];
      V.part[(int64_t(w) * R + threadIdx.x) * 2 + 1] = v[1];
    }
  }
}

// Totals of dots 0..ND-1 over system s's items, per rhs, valid in threads
// 0..R-1 (called by the whole block).  Thread t adds items item0 + t/R,
// item0 + t/R + 256/R, ... of rhs t % R in that order, then the fixed
// block reduction combines them.
template <int ND>
__device__ __forceinline__ void batch_sums(const BatchView &V, const BatchSys &sy, double (&out)[ND]) {
  const int R = V.nrhs, r = threadIdx.x % R, j0 = threadIdx.x / R, step = kBlock / R;
  DD v[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) v[d] = DD{0.0, 0.0};
  for (int32_t w = sy.item0 + j0; w < sy.item1; w += step) {
#pragma unroll
    for (int d = 0; d < ND; ++d) v[d] = dd_add(v[d], V.part[(int64_t(w) * R + r) * 2 + d]);
  }
  batch_block_reduce<ND>(v, R);
#pragma unroll
  for (int d = 0; d < ND; ++d) out[d] = dd_round(v[d]);
}

// After the prologue: rho = r.r and bb = b.b of every (system, rhs).
__global__ void __launch_bounds__(kBlock) k_batch_sums(BatchView V) {
  const int s = blockIdx.x;
  double t[2];
  batch_sums<2>(V, V.sys[s], t);
  if (int(threadIdx.x) < V.nrhs) {
    BatchCg &c = V.st[s * V.nrhs + threadIdx.x];
    c.rho = t[0];
    c.bb = t[1];
  }
}

// Start: thresholds (computed on the host) in thr2; the first test, as the
// single-system CG does it.
__global__ void __launch_bounds__(kBlock) k_batch_begin(BatchView V, int64_t max_iter) {
  const int s = blockIdx.x;
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  if (int(threadIdx.x) < V.nrhs) {
    BatchCg &c = V.st[s * V.nrhs + threadIdx.x];
    c.k = 0;
    c.alpha = c.beta = 0.0;
    c.zero_b = c.bb == 0.0;
    if (c.zero_b)
      c.flag = kConverged;
    else if (c.rho <= c.thr2)
      c.flag = kConverged;
    else if (!finite(c.rho))
      c.flag = kBreakdown;
    else if (max_iter <= 0)
      c.flag = kMaxIter;
    else
      c.flag = kRunning;
    if (c.flag == kRunning) atomicOr(&any, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) V.sys_run[s] = any;
}

// x = 0 where b = 0 (the single-system solve returns x = 0 for b = 0).
__global__ void __launch_bounds__(kBlock) k_batch_zero(BatchView V, double *__restrict__ x) {
  const int R = V.nrhs, cl = threadIdx.x / R, r = threadIdx.x % R;
  const Sched sc = my_tiles(V.nitems);
  for (int64_t w = sc.begin; w < sc.end; w += sc.stride) {
    const BatchItem it = V.items[w];
    const BatchSys sy = V.sys[it.sys];
    if (!V.st[it.sys * R + r].zero_b) continue;
    const int64_t n = int64_t(sy.nx) * sy.ny * sy.nz;
    for (int32_t t = it.t0; t < it.t1; ++t) {
      const int64_t lc = int64_t(t) * V.cells + cl;
      if (lc < n) x[(sy.off + lc) * R + r] = 0.0;
    }
  }
}

// CG pass 1: p = r + beta p formed on the fly, q = A p, partial p.q.
//
// Rows of one work item are consecutive cells, so the x and y neighbours of
// a tile of C = 256/R cells all lie in the cell window [L - nx, L + C + nx).
// The block keeps that window, as formed p values, in an LDS ring of S cells
// and slides it by one tile per step: each step loads only the C cells that
// enter the window (one coalesced load per thread, two steps ahead) and
// gathers just the two z neighbours (one step ahead), so a step's loads are
// in flight while earlier tiles are computed.  The 7 coefficients of a cell
// are read once by the R lanes that share it (lane r takes coefficients r,
// r + R, ...) and passed between those lanes.  Systems with nx too large
// for the ring (2 C + 2 nx > S) take the gather path.  Both paths run the
// same chain.
constexpr int kRingVals = 2048;  // doubles: 16 KB of LDS

template <int R>
__global__ void __launch_bounds__(kBlock) k_batch_pass1(BatchView V, const double2_t *__restrict__ rp,
                                                        double *__restrict__ q) {
  constexpr int C = kBlock / R, S = kRingVals / R, kL = (7 + R - 1) / R;
  __shared__ double ring[kRingVals];
  const int cl = threadIdx.x / R, r = threadIdx.x % R;
  const Sched sc = my_tiles(*V.nact);
  for (int64_t w = sc.begin; w < sc.end; w += sc.stride) {
    const BatchAct it = V.act[w];
    const BatchSys &sy = it.sy;
    const BatchCg &c = V.st[it.sys * R + r];
    const bool first = c.k == 0;
    const double beta = c.beta;
    auto value = [&](const double2_t &v) { return first ? v.x : fma(beta, v.y, v.x); };
    const int32_t nx = sy.nx;
    const int64_t n = int64_t(nx) * sy.ny * sy.nz;
    Dot2 a;
    if (2 * C + 2 * nx <= S && n * R < (int64_t(1) << 31)) {
      // cell and element indices of this system fit 32 bits here
      const int32_t nn = int32_t(n), nxy = nx * sy.ny;
      const double2_t *rs = rp + sy.off * R + r;  // (cell 0, rhs r) of this system
      const double *cf = V.coef + sy.off;          // coefficient o of cell c: cf[o ncell + c]
      auto slot = [&](int32_t cell) -> double & { return ring[(cell & (S - 1)) * R + r]; };
      // what a tile gathers besides the window: its z neighbours and this
      // lane's share of the coefficients
      struct Ahead {
        int32_t lc, ix, iy, iz;
        double2_t zm, zp;
        double cv[kL];
      };
      auto gather = [&](int32_t t, Ahead &g) {
        const int32_t lc = t * C + cl;
        g.lc = lc < nn ? lc : 0;
        const int32_t tq = int32_t(sy.dx.div(uint32_t(g.lc)));
        g.ix = g.lc - tq * nx;
        g.iz = int32_t(sy.dy.div(uint32_t(tq)));
        g.iy = tq - g.iz * sy.ny;
        g.zm = rs[(g.iz > 0 ? g.lc - nxy : g.lc) * R];
        g.zp = rs[(g.iz < sy.nz - 1 ? g.lc + nxy : g.lc) * R];
#pragma unroll
        for (int j = 0; j < kL; ++j) {
          const int o = r + j * R;
          g.cv[j] = cf[int64_t(o < 7 ? o : 6) * V.ncell + g.lc];
        }
        g.lc = lc;
      };
      Ahead cur;
      gather(it.t0, cur);
      // the window of the first tile, loaded in rounds of C cells, four
      // rounds in flight at a time
      const int32_t A = it.t0 * C;
      const int32_t lo = A - nx > 0 ? A - nx : 0;
      const int32_t hi = A + C + nx < nn ? A + C + nx : nn;
      // the cells entering the window of the second tile
      int32_t pc = A + C + nx + cl;
      bool pf = it.t0 + 1 < it.t1 && pc < nn;
      double2_t pv = rs[(pf ? pc : 0) * R];
      for (int32_t u0 = lo; u0 < hi; u0 += 4 * C) {  // block-uniform
        double2_t pre[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int32_t cc = u0 + u * C + cl;
          pre[u] = rs[(cc < hi ? cc : lo) * R];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int32_t cc = u0 + u * C + cl;
          if (cc < hi) slot(cc) = value(pre[u]);
        }
      }
      __syncthreads();
      for (int32_t t = it.t0; t < it.t1; ++t) {
        // loads for later steps: the cells entering the window of tile
        // t + 2, the gathers of tile t + 1
        const int32_t pc2 = pc + C;
        const bool pf2 = t + 2 < it.t1 && pc2 < nn;
        const double2_t pv2 = rs[(pf2 ? pc2 : 0) * R];
        const bool more = t + 1 < it.t1;  // block-uniform
        Ahead nxt;
        if (more) gather(t + 1, nxt);
        double co[7];
        if constexpr (R == 1) {
#pragma unroll
          for (int o = 0; o < 7; ++o) co[o] = cur.cv[o];
        } else {
          const int base = int(threadIdx.x & 63) & ~(R - 1);
#pragma unroll
          for (int o = 0; o < 7; ++o) co[o] = __shfl(cur.cv[o / R], base | (o % R), 64);
        }
        const bool valid = cur.lc < nn;
        const int32_t lcs = valid ? cur.lc : 0;
        const bool in[7] = {cur.iz > 0,      cur.iy > 0,          cur.ix > 0,         true,
                            cur.ix < nx - 1, cur.iy < sy.ny - 1, cur.iz < sy.nz - 1};
        const double xv[7] = {value(cur.zm),  slot(lcs - nx), slot(lcs - 1), slot(lcs),
                              slot(lcs + 1),  slot(lcs + nx), value(cur.zp)};
        double acc = 0.0;
#pragma unroll
        for (int o = 0; o < 7; ++o)
          if (in[o]) acc = fma(co[o], xv[o], acc);
        if (valid) {
          st_nt(q + (sy.off + cur.lc) * R + r, acc);
          a.add(xv[3], acc);
        }
        // the window of tile t + 1 is complete after this write
        if (pf) slot(pc) = value(pv);
        __syncthreads();
        pc = pc2;
        pf = pf2;
        pv = pv2;
        if (more) cur = nxt;
      }
    } else {
      for (int32_t t = it.t0; t < it.t1; ++t) {
        const int64_t lc = int64_t(t) * C + cl;
        if (lc < n) {
          double pi;
          const double acc = batch_row(V, sy, lc, r, [&](int64_t e) { return rp[e]; }, value, pi);
          st_nt(q + (sy.off + lc) * R + r, acc);
          a.add(pi, acc);
        }
      }
    }
    DD v[2] = {a.get(), DD{0.0, 0.0}};
    batch_block_reduce<2>(v, R);
    if (int(threadIdx.x) < R) V.part[(int64_t(it.w) * R + threadIdx.x) * 2] = v[0];
  }
}

// alpha = rho / (p.q) per running (system, rhs); p.q = 0 or non-finite is a
// breakdown.
__global__ void __launch_bounds__(kBlock) k_batch_fin1(BatchView V) {
  const int s = blockIdx.x;
  if (!V.sys_run[s]) return;  // block-uniform
  double t[1];
  batch_sums<1>(V, V.sys[s], t);
  if (int(threadIdx.x) >= V.nrhs) return;
  BatchCg &c = V.st[s * V.nrhs + threadIdx.x];
  if (c.flag != kRunning) return;
  const double pq = t[0];
  if (pq == 0.0 || !finite(pq))
    c.flag = kBreakdown;
  else
    c.alpha = c.rho / pq;
}

// CG pass 2: p = r + beta p stored, x += alpha p, r -= alpha q, partial r.r.
// Pass 2 has no neighbours, so the P items of a system take its tiles
// round-robin (item j: tiles j, j + P, j + 2P, ...): the blocks that run
// side by side then stream through neighbouring tiles.  Four tiles per
// step, their loads issued together (index clamped to the system's first
// cell where a tile runs past the system).
template <int R>
__global__ void __launch_bounds__(kBlock) k_batch_pass2(BatchView V, double *__restrict__ x,
                                                        double2_t *__restrict__ rp,
                                                        const double *__restrict__ q) {
  constexpr int C = kBlock / R, U = 4;
  const int cl = threadIdx.x / R, r = threadIdx.x % R;
  const Sched sc = my_tiles(*V.nact);
  for (int64_t w = sc.begin; w < sc.end; w += sc.stride) {
    const BatchAct it = V.act[w];
    const BatchSys &sy = it.sy;
    const BatchCg &c = V.st[it.sys * R + r];
    const bool run = c.flag == kRunning;
    const bool first = c.k == 0;
    const double beta = c.beta, alpha = c.alpha;
    const int64_t n = int64_t(sy.nx) * sy.ny * sy.nz;
    const int64_t e0 = sy.off * R + r;
    const int32_t P = sy.item1 - sy.item0, j = it.w - sy.item0;
    Dot2 a;
    for (int32_t t = j; t < sy.tiles; t += U * P) {
      bool ok[U];
      int64_t e[U];
      double2_t v[U];
      double xo[U], qo[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t tt = t + u * P;
        const int64_t lc = int64_t(tt) * C + cl;
        ok[u] = run && tt < sy.tiles && lc < n;
        e[u] = e0 + (ok[u] ? lc : 0) * R;
        v[u] = ld_nt(rp + e[u]);
        xo[u] = ld_nt(x + e[u]);
        qo[u] = ld_nt(q + e[u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (!ok[u]) continue;
        const double pi = first ? v[u].x : fma(beta, v[u].y, v[u].x);
        st_nt(x + e[u], fma(alpha, pi, xo[u]));
        const double ri = fma(-alpha, qo[u], v[u].x);
        double2_t o;
        o.x = ri;
        o.y = pi;
        st_nt(rp + e[u], o);
        a.add(ri, ri);
      }
    }
    DD v[2] = {a.get(), DD{0.0, 0.0}};
    batch_block_reduce<2>(v, R);
    if (int(threadIdx.x) < R) V.part[(int64_t(it.w) * R + threadIdx.x) * 2] = v[0];
  }
}

// rho' = r.r, one more iteration, beta = rho'/rho, test; the system stays
// running while any of its right-hand sides does.
__global__ void __launch_bounds__(kBlock) k_batch_fin2(BatchView V, int64_t max_iter) {
  const int s = blockIdx.x;
  if (!V.sys_run[s]) return;  // block-uniform
  double t[1];
  batch_sums<1>(V, V.sys[s], t);
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  if (int(threadIdx.x) < V.nrhs) {
    BatchCg &c = V.st[s * V.nrhs + threadIdx.x];
    if (c.flag == kRunning) {
      const double rho_new = t[0];
      const int64_t k = c.k + 1;
      c.k = k;
      c.beta = rho_new / c.rho;
      c.rho = rho_new;
      if (rho_new <= c.thr2)
        c.flag = kConverged;
      else if (!finite(rho_new))
        c.flag = kBreakdown;
      else if (k >= max_iter)
        c.flag = kMaxIter;
    }
    if (c.flag == kRunning) atomicOr(&any, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) V.sys_run[s] = any;
}

// Items of the running systems: exclusive prefix over the systems (one
// block; thread t takes a contiguous run of systems) and the total, which
// the host also polls (0 once every system has stopped).
__global__ void __launch_bounds__(kBlock) k_batch_scan(BatchView V) {
  __shared__ int32_t part[kBlock];
  const int t = threadIdx.x;
  const int32_t lo = int32_t(int64_t(V.nsys) * t / kBlock), hi = int32_t(int64_t(V.nsys) * (t + 1) / kBlock);
  int32_t sum = 0;
  for (int32_t u = lo; u < hi; ++u)
    if (V.sys_run[u]) sum += V.sys[u].item1 - V.sys[u].item0;
  part[t] = sum;
  __syncthreads();
  if (t == 0) {
    int32_t acc = 0;
    for (int j = 0; j < kBlock; ++j) {
      const int32_t v = part[j];
      part[j] = acc;
      acc += v;
    }
    *V.nact = acc;
  }
  __syncthreads();
  int32_t acc = part[t];
  for (int32_t u = lo; u < hi; ++u) {
    V.sys_base[u] = acc;
    if (V.sys_run[u]) acc += V.sys[u].item1 - V.sys[u].item0;
  }
}

// The records of the running systems' items (one block per system).
__global__ void __launch_bounds__(kBlock) k_batch_compact(BatchView V) {
  const int s = blockIdx.x;
  if (!V.sys_run[s]) return;  // block-uniform
  const BatchSys sy = V.sys[s];
  const int32_t base = V.sys_base[s];
  for (int32_t j = threadIdx.x; j < sy.item1 - sy.item0; j += kBlock) {
    const BatchItem it = V.items[sy.item0 + j];
    BatchAct a;
    a.sy = sy;
    a.w = sy.item0 + j;
    a.sys = s;
    a.t0 = it.t0;
    a.t1 = it.t1;
    V.act[base + j] = a;
  }
}

}  // namespace its
