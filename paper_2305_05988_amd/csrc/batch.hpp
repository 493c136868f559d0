// Batched CG: many independent variable-coefficient diffusion systems, each
// with several right-hand sides, advanced together.
#pragma once

#include "common.hpp"

namespace its {

// Layout.  The systems' cells are concatenated (system s owns global cells
// [off_s, off_s + n_s), rows numbered i + nx(j + ny k) inside it).  Vectors
// interleave the right-hand sides: value (cell g, rhs r) sits at g R + r, so
// a block's 256 threads cover 256/R consecutive cells x R right-hand sides
// and every access is coalesced.  The operator is stored once per cell and
// reused by all R right-hand sides: its diagonal and its three upper face
// coefficients (x+1, y+1, z+1; 0 outside the grid), coef[a * ncell + g] for
// a = 0 (diagonal), 1 (x+1), 2 (y+1), 3 (z+1).  A lower face's coefficient
// is the upper one of the neighbour across it, the same value bit for bit
// (the harmonic mean 2 k k' / (k + k') of the two cells, formed from the
// same operands in either order), so 32 bytes per cell hold the operator's
// 7 coefficients in chain order (z-1, y-1, x-1, diagonal, x+1, y+1, z+1):
// coef_at(o) below.  The SpMV pass works on bricks (an x-y tile of a system marched
// through a run of z planes), the other passes on work items (runs of
// 256/R-cell tiles inside one system); each brick or item leaves one
// double-double partial per right-hand side, and one block per system
// finishes the reductions in a fixed order.  After every iteration the
// bricks and items of the systems still running are gathered, with all a
// block needs to start loading, into dense lists that the two CG passes
// walk, so stopped systems cost nothing and the work stays spread evenly.
constexpr int kBatchMaxRhs = 8;

struct BatchSys {
  int64_t off;             // first global cell
  int32_t nx, ny, nz;
  int32_t tiles;           // ceil(n / cells per tile)
  int32_t item0, item1;    // its work items
  int32_t brick0, brick1;  // its bricks
};

// Brick of the SpMV pass: cells [x0, x0 + TX) x [y0, y0 + TY) x [z0, z1) of
// system sys (clipped to the grid), with TX x TY = 2 * 256/R cells.
struct BatchBrick {
  int32_t sys, x0, y0, z0, z1, pad;
};

// A brick of a running system, as the SpMV pass reads it.
struct BatchActB {
  int64_t off;
  int32_t b;             // the brick's index (its partial slot)
  int32_t sys, nx, ny, nz, x0, y0, z0, z1, pad;
};

struct BatchItem {
  int32_t sys, t0, t1;   // tiles [t0, t1) of system sys
  int32_t pad;
};

// An item of a running system, as the update pass reads it.
struct BatchAct {
  BatchSys sy;
  int32_t w;             // the item's index (its partial slot)
  int32_t sys, t0, t1;
};

// CG scalars of one (system, right-hand side).
struct BatchCg {
  double rho, alpha, beta, bb, thr2;
  double alpha_x;  // step of the x update deferred from an even iteration
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
  int32_t *sys_base; // [2 s], [2 s + 1]: system s's first slots in act and act1
  int32_t *nact;     // [0] items, [1] bricks of the running systems
  BatchAct *act;     // those items, in system and item order
  BatchActB *act1;   // those bricks, in system and brick order
  const BatchBrick *bricks;
  DD *part;          // [item][rhs][2]
  DD *part1;         // [brick][rhs][2]
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
// Where coefficient o of the chain (z-1, y-1, x-1, diagonal, x+1, y+1, z+1)
// of a cell is stored: array kCoefArray[o], at the cell itself or, for a
// lower face, at the neighbour across it (cell - nxy, - nx, - 1).
constexpr int kCoefs = 4;
constexpr int kCoefArray[7] = {3, 2, 1, 0, 1, 2, 3};

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
      // the lower faces' values are the lower neighbours' upper ones
      const int64_t N = V.ncell;
      coef[0 * N + g] = diag;
      coef[1 * N + g] = in[3] ? -f[3] : 0.0;
      coef[2 * N + g] = in[4] ? -f[4] : 0.0;
      coef[3 * N + g] = in[5] ? -f[5] : 0.0;
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
      v[d] = dd_cascade(v[d], o);
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
      for (int j = 1; j < kWaves; ++j) t = dd_cascade(t, sm[d][j][threadIdx.x]);
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
  for (int o = 0; o < 7; ++o) a[o] = V.coef[kCoefArray[o] * V.ncell + (o < 3 && in[o] ? g + off[o] : g)];
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

// Totals of dots 0..ND-1 over the partial slots [w0, w1) of one system, per
// rhs, valid in threads 0..R-1 (called by the whole block).  Thread t adds
// slots w0 + t/R, w0 + t/R + 256/R, ... of rhs t % R in that order, then
// the fixed block reduction combines them.
template <int ND>
__device__ __forceinline__ void batch_sums(const BatchView &V, const DD *part, int32_t w0, int32_t w1,
                                           double (&out)[ND]) {
  const int R = V.nrhs, r = threadIdx.x % R, j0 = threadIdx.x / R, step = kBlock / R;
  DD v[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) v[d] = DD{0.0, 0.0};
  for (int32_t w = w0 + j0; w < w1; w += step) {
#pragma unroll
    for (int d = 0; d < ND; ++d) v[d] = dd_add(v[d], part[(int64_t(w) * R + r) * 2 + d]);
  }
  batch_block_reduce<ND>(v, R);
#pragma unroll
  for (int d = 0; d < ND; ++d) out[d] = dd_round(v[d]);
}

// After the prologue: rho = r.r and bb = b.b of every (system, rhs).
__global__ void __launch_bounds__(kBlock) k_batch_sums(BatchView V) {
  const int s = blockIdx.x;
  double t[2];
  const BatchSys sy = V.sys[s];
  batch_sums<2>(V, V.part, sy.item0, sy.item1, t);
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
    c.alpha = c.beta = c.alpha_x = 0.0;
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
// A block marches one brick through its z planes.  Each plane of the brick's
// tile, with a one-cell halo in x and y, is loaded once with coalesced loads
// (the R right-hand sides of a cell are adjacent), formed into p values and
// kept in LDS; four plane slots rotate, so planes z-1, z, z+1 are read from
// LDS while plane z+2 is in flight.  Every neighbour of a row then comes from
// LDS, and each value is read from memory once per brick plus its halo.  The
// 7 coefficients of a cell are read once by the R lanes that share it (lane
// r takes coefficients r, r + R, ...; a lower face's from the neighbour's
// upper face, whose line the neighbouring cell or the previous plane already
// brought in), one plane ahead, and passed between those lanes.  The chain
// is the single-system one.
template <int R>
struct BrickShape;
template <>
struct BrickShape<1> {
  static constexpr int TX = 64, TY = 8;
};
template <>
struct BrickShape<2> {
  static constexpr int TX = 32, TY = 8;
};
template <>
struct BrickShape<4> {
  static constexpr int TX = 32, TY = 4;
};
template <>
struct BrickShape<8> {
  static constexpr int TX = 16, TY = 4;
};

template <int R>
__global__ void __launch_bounds__(kBlock) k_batch_pass1(BatchView V, const double2_t *__restrict__ rp,
                                                        double *__restrict__ q) {
  constexpr int TX = BrickShape<R>::TX, TY = BrickShape<R>::TY;
  constexpr int C = kBlock / R;                   // cells per layer of the block
  constexpr int CPT = TX * TY / C;                // cells per thread per plane
  constexpr int HX = TX + 2, HS = HX * (TY + 2);  // halo tile
  constexpr int NV = HS * R, NR = (NV + kBlock - 1) / kBlock;
  constexpr int kL = (7 + R - 1) / R;
  static_assert(CPT * C == TX * TY, "brick tile must fill whole layers");
  __shared__ double slot[4][NV];  // value (halo cell h, rhs r) at h R + r
  const int t = threadIdx.x, r = t % R, cl = t / R;
  const Sched sc = my_tiles(V.nact[1]);
  for (int64_t w = sc.begin; w < sc.end; w += sc.stride) {
    const BatchActB bk = V.act1[w];
    const BatchCg &c = V.st[bk.sys * R + r];
    const bool first = c.k == 0;
    const double beta = c.beta;
    auto value = [&](const double2_t &v) { return first ? v.x : fma(beta, v.y, v.x); };
    const int32_t nx = bk.nx, ny = bk.ny, nz = bk.nz;
    const int64_t nxy = int64_t(nx) * ny;
    const double2_t *rs = rp + bk.off * R + r;  // (cell 0, rhs r) of this system
    const double *cf = V.coef + bk.off;          // array a of cell c: cf[a ncell + c]
    // The parts of this thread's addresses that do not change from plane to
    // plane, formed once per brick: the in-plane cell of each halo value it
    // loads (-1 outside the grid) and of each of its cells, and its cells'
    // neighbour flags (bit 0 y-1, 1 x-1, 2 x+1, 3 y+1, 4 inside the grid).
    int32_t hoff[NR];
#pragma unroll
    for (int u = 0; u < NR; ++u) {
      const int v = t + u * kBlock, h = v / R;
      const int32_t gx = bk.x0 - 1 + h % HX, gy = bk.y0 - 1 + h / HX;
      const bool in = v < NV && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
      hoff[u] = in ? gx + nx * gy : -1;  // a plane has fewer than 2^31 cells
    }
    int32_t coff[CPT];
    uint32_t nb[CPT];
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const int k = cl + u * C;
      const int32_t gx = bk.x0 + k % TX, gy = bk.y0 + k / TX;
      const bool inside = gx < nx && gy < ny;
      coff[u] = inside ? gx + nx * gy : -1;
      nb[u] = uint32_t(gy > 0) | uint32_t(gx > 0) << 1 | uint32_t(gx < nx - 1) << 2 |
              uint32_t(gy < ny - 1) << 3 | uint32_t(inside) << 4;
    }
    // loads are unconditional (halo cells outside the grid load cell 0,
    // never consumed) so a plane's loads stay in flight together
    double2_t hv[NR];
    auto issue = [&](int32_t z) {
      const int64_t zo = nxy * z;
#pragma unroll
      for (int u = 0; u < NR; ++u) hv[u] = rs[(hoff[u] >= 0 ? int64_t(hoff[u]) + zo : 0) * R];
    };
    auto put = [&](int32_t z) {
      double *d = slot[z & 3];
#pragma unroll
      for (int u = 0; u < NR; ++u)
        if (t + u * kBlock < NV) d[t + u * kBlock] = value(hv[u]);
    };
    // this thread's cells of the tile: k = cl + u C.  Lane r's coefficient
    // j is chain entry o = r + j R (entries past 6 load the diagonal, never
    // used): array kCoefArray[o], and for a lower face the neighbour's cell
    // when that neighbour exists (its flag: z > 0, nb bit 0 or bit 1).
    const double *ca[kL];
#pragma unroll
    for (int j = 0; j < kL; ++j) {
      const int o = r + j * R;
      ca[j] = cf + int64_t(o < 7 ? kCoefArray[o] : 0) * V.ncell;
    }
    // lower faces are the chain entries o = r + j R < 3, so only the first
    // kLow entries of a lane can be one; such an entry is read at the
    // neighbour across the face (a plane back for z-1, where z > 0; a row
    // back for y-1 and a cell back for x-1, where the cell's flags have them)
    constexpr int kLow = R == 1 ? 3 : R == 2 ? 2 : 1;
    auto coefs = [&](int32_t z, double (&cv)[CPT][kL]) {
      const int64_t zo = nxy * z;
#pragma unroll
      for (int u = 0; u < CPT; ++u) {
        const int64_t cell = coff[u] >= 0 ? int64_t(coff[u]) + zo : 0;
#pragma unroll
        for (int j = 0; j < kL; ++j) {
          int64_t at = cell;
          if (j < kLow && coff[u] >= 0) {
            const int o = r + j * R;
            at -= o == 0 ? (z > 0 ? nxy : 0)
                         : o == 1 ? ((nb[u] & 1u) ? nx : 0) : o == 2 ? ((nb[u] & 2u) ? 1 : 0) : 0;
          }
          cv[u][j] = ca[j][at];
        }
      }
    };
    Dot2 a;
    for (int32_t z = max(bk.z0 - 1, 0); z <= min(bk.z0 + 1, nz - 1); ++z) {
      issue(z);
      put(z);
    }
    double cv[CPT][kL];
    coefs(bk.z0, cv);
    __syncthreads();
    for (int32_t z = bk.z0; z < bk.z1; ++z) {
      const int32_t zn = z + 2;
      const bool pf = zn <= bk.z1 && zn < nz;  // block-uniform
      if (pf) issue(zn);
      const bool more = z + 1 < bk.z1;         // block-uniform
      double cn[CPT][kL];
      if (more) coefs(z + 1, cn);
      const double *pm = slot[(z - 1) & 3], *pc = slot[z & 3], *pp = slot[(z + 1) & 3];
#pragma unroll
      for (int u = 0; u < CPT; ++u) {
        const int k = cl + u * C;
        const int hc = ((k / TX) + 1) * HX + k % TX + 1;  // the cell in the halo tile
        double co[7];
        if constexpr (R == 1) {
#pragma unroll
          for (int o = 0; o < 7; ++o) co[o] = cv[u][o];
        } else {
          const int base = int(threadIdx.x & 63) & ~(R - 1);
#pragma unroll
          for (int o = 0; o < 7; ++o) co[o] = __shfl(cv[u][o / R], base | (o % R), 64);
        }
        const double xv[7] = {pm[hc * R + r],        pc[(hc - HX) * R + r], pc[(hc - 1) * R + r],
                              pc[hc * R + r],        pc[(hc + 1) * R + r],  pc[(hc + HX) * R + r],
                              pp[hc * R + r]};
        const bool in[7] = {z > 0, bool(nb[u] & 1u), bool(nb[u] & 2u), true, bool(nb[u] & 4u),
                            bool(nb[u] & 8u), z < nz - 1};
        double acc = 0.0;
#pragma unroll
        for (int o = 0; o < 7; ++o)
          if (in[o]) acc = fma(co[o], xv[o], acc);
        if (nb[u] & 16u) {
          st_nt(q + (bk.off + int64_t(coff[u]) + nxy * z) * R + r, acc);
          a.add(xv[3], acc);
        }
      }
      if (pf) put(zn);
      __syncthreads();
      if (more) {
#pragma unroll
        for (int u = 0; u < CPT; ++u)
#pragma unroll
          for (int j = 0; j < kL; ++j) cv[u][j] = cn[u][j];
      }
    }
    DD v[1] = {a.get()};
    batch_block_reduce<1>(v, R);
    if (int(threadIdx.x) < R) V.part1[(int64_t(bk.b) * R + threadIdx.x) * 2] = v[0];
  }
}

// alpha = rho / (p.q) per running (system, rhs); p.q = 0 or non-finite is a
// breakdown.
__global__ void __launch_bounds__(kBlock) k_batch_fin1(BatchView V) {
  const int s = blockIdx.x;
  if (!V.sys_run[s]) return;  // block-uniform
  double t[1];
  const BatchSys sy = V.sys[s];
  batch_sums<1>(V, V.part1, sy.brick0, sy.brick1, t);
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
// An item walks its own run of tiles [t0, t1), four adjacent tiles per step
// with their loads issued together (index clamped to the system's first cell
// where a tile runs past the item or the system).  Measured on the 512 x 8
// batch: 2.4 % faster than dealing a system's tiles to its items round-robin.
template <int R>
__global__ void __launch_bounds__(kBlock) k_batch_pass2(BatchView V, double *__restrict__ x,
                                                        double2_t *__restrict__ rp,
                                                        const double *__restrict__ q) {
  constexpr int C = kBlock / R, U = 4;
  const int cl = threadIdx.x / R, r = threadIdx.x % R;
  const Sched sc = my_tiles(V.nact[0]);
  for (int64_t w = sc.begin; w < sc.end; w += sc.stride) {
    const BatchAct it = V.act[w];
    const BatchSys &sy = it.sy;
    const BatchCg &c = V.st[it.sys * R + r];
    const bool run = c.flag == kRunning;
    const bool first = c.k == 0;
    // x is read and written on odd iterations only, with the deferred update
    // of the even one first (the same roundings as updating it every time)
    const bool defer = (c.k & 1) == 0;
    const double beta = c.beta, alpha = c.alpha, alpha_x = c.alpha_x;
    const int64_t n = int64_t(sy.nx) * sy.ny * sy.nz;
    const int64_t e0 = sy.off * R + r;
    Dot2 a;
    for (int32_t t = it.t0; t < it.t1; t += U) {
      bool ok[U];
      int64_t e[U];
      double2_t v[U];
      double xo[U], qo[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t tt = t + u;
        const int64_t lc = int64_t(tt) * C + cl;
        ok[u] = run && tt < it.t1 && lc < n;
        e[u] = e0 + (ok[u] ? lc : 0) * R;
        v[u] = ld_nt(rp + e[u]);
        xo[u] = defer ? 0.0 : ld_nt(x + e[u]);
        qo[u] = ld_nt(q + e[u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (!ok[u]) continue;
        const double pi = first ? v[u].x : fma(beta, v[u].y, v[u].x);
        if (!defer) st_nt(x + e[u], fma(alpha, pi, fma(alpha_x, v[u].y, xo[u])));
        const double ri = fma(-alpha, qo[u], v[u].x);
        double2_t o;
        o.x = ri;
        o.y = pi;
        st_nt(rp + e[u], o);
        a.add(ri, ri);
      }
    }
    DD v[1] = {a.get()};
    batch_block_reduce<1>(v, R);
    if (int(threadIdx.x) < R) V.part[(int64_t(it.w) * R + threadIdx.x) * 2] = v[0];
  }
}

// After the iterations: a (system, rhs) that stopped after an odd count of
// iterations still owes the x update of its last (even) iteration, whose p
// is in the pairs.  Grid: (systems, kFlushParts) blocks; the stride of a
// thread is a multiple of the rhs count, so each thread serves one rhs.
constexpr int kFlushParts = 32;
__global__ void __launch_bounds__(kBlock) k_batch_flush_x(BatchView V, double *__restrict__ x,
                                                          const double2_t *__restrict__ rp) {
  const int s = blockIdx.x;
  const BatchSys sy = V.sys[s];
  const int R = V.nrhs;
  const BatchCg &c = V.st[int64_t(s) * R + int(threadIdx.x) % R];
  if ((c.k & 1) == 0) return;
  const double alpha_x = c.alpha_x;
  const int64_t e0 = sy.off * R, e1 = (sy.off + int64_t(sy.nx) * sy.ny * sy.nz) * R;
  for (int64_t e = e0 + int64_t(blockIdx.y) * kBlock + threadIdx.x; e < e1;
       e += int64_t(kBlock) * kFlushParts)
    x[e] = fma(alpha_x, rp[e].y, x[e]);
}

// rho' = r.r, one more iteration, beta = rho'/rho, test; the system stays
// running while any of its right-hand sides does.
__global__ void __launch_bounds__(kBlock) k_batch_fin2(BatchView V, int64_t max_iter) {
  const int s = blockIdx.x;
  if (!V.sys_run[s]) return;  // block-uniform
  double t[1];
  const BatchSys sy = V.sys[s];
  batch_sums<1>(V, V.part, sy.item0, sy.item1, t);
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  if (int(threadIdx.x) < V.nrhs) {
    BatchCg &c = V.st[s * V.nrhs + threadIdx.x];
    if (c.flag == kRunning) {
      const double rho_new = t[0];
      const int64_t k = c.k + 1;
      if (k & 1) c.alpha_x = c.alpha;  // iteration k - 1 (even) deferred its x update
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

// Items and bricks of the running systems: exclusive prefixes over the
// systems (one block; thread t takes a contiguous run of systems) and the
// totals; the host polls the item total (0 once every system has stopped).
__global__ void __launch_bounds__(kBlock) k_batch_scan(BatchView V) {
  __shared__ int32_t part[2][kBlock];
  const int t = threadIdx.x;
  const int32_t lo = int32_t(int64_t(V.nsys) * t / kBlock), hi = int32_t(int64_t(V.nsys) * (t + 1) / kBlock);
  int32_t si = 0, sb = 0;
  for (int32_t u = lo; u < hi; ++u)
    if (V.sys_run[u]) {
      si += V.sys[u].item1 - V.sys[u].item0;
      sb += V.sys[u].brick1 - V.sys[u].brick0;
    }
  part[0][t] = si;
  part[1][t] = sb;
  __syncthreads();
  if (t < 2) {
    int32_t acc = 0;
    for (int j = 0; j < kBlock; ++j) {
      const int32_t v = part[t][j];
      part[t][j] = acc;
      acc += v;
    }
    V.nact[t] = acc;
  }
  __syncthreads();
  int32_t ai = part[0][t], ab = part[1][t];
  for (int32_t u = lo; u < hi; ++u) {
    V.sys_base[2 * u] = ai;
    V.sys_base[2 * u + 1] = ab;
    if (V.sys_run[u]) {
      ai += V.sys[u].item1 - V.sys[u].item0;
      ab += V.sys[u].brick1 - V.sys[u].brick0;
    }
  }
}

// The records of the running systems' items and bricks (one block per
// system).
__global__ void __launch_bounds__(kBlock) k_batch_compact(BatchView V) {
  const int s = blockIdx.x;
  if (!V.sys_run[s]) return;  // block-uniform
  const BatchSys sy = V.sys[s];
  const int32_t base = V.sys_base[2 * s], base1 = V.sys_base[2 * s + 1];
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
  for (int32_t j = threadIdx.x; j < sy.brick1 - sy.brick0; j += kBlock) {
    const BatchBrick br = V.bricks[sy.brick0 + j];
    BatchActB a;
    a.off = sy.off;
    a.b = sy.brick0 + j;
    a.sys = s;
    a.nx = sy.nx;
    a.ny = sy.ny;
    a.nz = sy.nz;
    a.x0 = br.x0;
    a.y0 = br.y0;
    a.z0 = br.z0;
    a.z1 = br.z1;
    a.pad = 0;
    V.act1[base1 + j] = a;
  }
}

}  // namespace its
