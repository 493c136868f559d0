// Matrix-free stencil operator (see rowops.hpp for the row-walk contract).
#pragma once

#include "rowops.hpp"

namespace its {

// Matrix-free constant-coefficient stencil on nx*ny*nz, row = i + nx(j + ny k).
// Neighbours outside the grid are skipped, exactly as the CSR rows of the
// same operator omit them, so both give bit-identical chains.  NPTS = 7:
// offsets (k-1, j-1, i-1, centre, i+1, j+1, k+1); NPTS = 27: dk outer, dj, di
// inner.  Coefficients in that (ascending column) order.
//
// The SpMV passes sweep the grid in bricks: a block owns a 64 x 4 (x, y) tile
// and marches it through zb planes.  Each plane of the tile, with a one-point
// halo in x and y (66 x 6 points), is loaded once with coalesced row loads,
// turned into x_j by the pass's value functor and kept in LDS; four plane
// slots rotate, so planes z-1, z, z+1 are read from LDS while plane z+2 is
// being loaded.  Every neighbour value then comes from LDS instead of a
// gather through the vector-memory path.  Rows keep the CSR chain order.
template <int NPTS, class T>
struct StencilOp {
  int32_t nx, ny, nz, n;
  T c[NPTS];
  int32_t nbx = 0, nby = 0, nbz = 0, zb = 1;  // brick grid (plan())

  static constexpr int kTX = 64, kTY = kBlock / 64;  // one point per thread per plane
  static constexpr int kCols = kTX + 2, kTileRows = kTY + 2, kPlane = kCols * kTileRows;
  static constexpr int kSlots = 4;
  struct Smem {
    T v[kSlots][kPlane];
  };

  // Brick plan, cutting z into chunks of zb planes: about 4096 bricks where
  // each still marches at least 16 planes (measured at 256^3: 83 us per CG
  // SpMV pass against 87 us with 2048 bricks and 90 us with 8192), else
  // about 2048 (8 resident blocks on each of 256 CUs).
  void plan() {
    nbx = (nx + kTX - 1) / kTX;
    nby = (ny + kTY - 1) / kTY;
    const int64_t nxy = int64_t(nbx) * nby;
    auto zb_for = [&](int64_t target) {
      int64_t chunks = nxy > 0 ? (target + nxy - 1) / nxy : 1;
      if (chunks > nz) chunks = nz;
      if (chunks < 1) chunks = 1;
      const int64_t z = (nz + chunks - 1) / chunks;
      return int32_t(z < 1 ? 1 : z);
    };
    zb = zb_for(4096);
    if (zb < 16) zb = zb_for(2048);
    nbz = (nz + zb - 1) / zb;
  }
  int grid() const {
    int64_t b = int64_t(nbx) * nby * nbz;
    if (b < 1) b = 1;
    int g = int(b < kMaxGrid ? b : kMaxGrid);
    if (g >= 64) g -= g % kXcds;
    return g;
  }

  __device__ __forceinline__ void coords(int32_t i, int32_t &ix, int32_t &iy, int32_t &iz) const {
    const int32_t t = i / nx;
    ix = i - t * nx;
    iz = t / ny;
    iy = t - iz * ny;
  }

  // ------------------------------------------------------ row at a time
  // (used by the Gauss-Seidel colour sweeps, which update in place)
  template <class Fetch, class Consume>
  __device__ __forceinline__ void row_entries_at(int32_t i, int32_t ix, int32_t iy, int32_t iz,
                                                 Fetch &&fetch, Consume &&consume) const {
    const int32_t nxy = nx * ny;
    if constexpr (NPTS == 7) {
      const bool has[7] = {iz > 0, iy > 0, ix > 0, true, ix < nx - 1, iy < ny - 1, iz < nz - 1};
      const int32_t d[7] = {-nxy, -nx, -1, 0, 1, nx, nxy};
      // neighbours outside the grid fetch the row itself (not consumed)
      decltype(fetch(0)) xv[7];
#pragma unroll
      for (int o = 0; o < 7; ++o) xv[o] = fetch(has[o] ? i + d[o] : i);
#pragma unroll
      for (int o = 0; o < 7; ++o)
        if (has[o]) consume(i + d[o], c[o], xv[o]);
    } else {
#pragma unroll
      for (int dk = -1; dk <= 1; ++dk) {
        // one plane (9 entries) of gathers in flight at a time
        decltype(fetch(0)) xv[9];
        bool in[9];
#pragma unroll
        for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
          for (int di = -1; di <= 1; ++di) {
            const int u = (dj + 1) * 3 + (di + 1);
            in[u] = (iz + dk >= 0) && (iz + dk < nz) && (iy + dj >= 0) && (iy + dj < ny) &&
                    (ix + di >= 0) && (ix + di < nx);
            xv[u] = fetch(in[u] ? i + dk * nxy + dj * nx + di : i);
          }
#pragma unroll
        for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
          for (int di = -1; di <= 1; ++di) {
            const int u = (dj + 1) * 3 + (di + 1);
            if (in[u]) consume(i + dk * nxy + dj * nx + di, c[(dk + 1) * 9 + u], xv[u]);
          }
      }
    }
  }

  // The rows a thread owns in rows(), in the same order: body(i).
  template <class Body>
  __device__ __forceinline__ void own_rows(Body &&body) const {
    const int64_t nbricks = int64_t(nbx) * nby * nbz;
    const Sched sc = my_tiles(nbricks);
    const int t = threadIdx.x, lane = t & 63, wy = t >> 6;
    const int32_t nxy = nx * ny;
    for (int64_t bi = sc.begin; bi < sc.end; bi += sc.stride) {
      const int32_t bx = int32_t(bi % nbx), by = int32_t((bi / nbx) % nby);
      const int32_t bz = int32_t(bi / (int64_t(nbx) * nby));
      const int32_t gx = bx * kTX + lane, gy = by * kTY + wy;
      if (gx >= nx || gy >= ny) continue;
      const int32_t z0 = bz * zb, z1 = min(nz, z0 + zb);
      for (int32_t z = z0; z < z1; ++z) body(gx + nx * gy + nxy * z);
    }
  }

  // ------------------------------------------------------ 2.5-D row sweep
  template <class Load, class Value, class Body>
  __device__ __forceinline__ void rows(Smem &sm, Load &&load, Value &&value, Body &&body) const {
    using Raw = decltype(load(0));
    constexpr int kPer = (kPlane + kBlock - 1) / kBlock;  // halo-tile points per thread
    const int64_t nbricks = int64_t(nbx) * nby * nbz;
    const Sched sc = my_tiles(nbricks);
    const int t = threadIdx.x, lane = t & 63, wy = t >> 6;
    const int32_t nxy = nx * ny;
    for (int64_t bi = sc.begin; bi < sc.end; bi += sc.stride) {
      const int32_t bx = int32_t(bi % nbx), by = int32_t((bi / nbx) % nby);
      const int32_t bz = int32_t(bi / (int64_t(nbx) * nby));
      const int32_t x0 = bx * kTX, y0 = by * kTY, z0 = bz * zb, z1 = min(nz, z0 + zb);
      // point k of the halo tile of plane z: its row, or -1 outside the grid
      auto tile_row = [&](int k, int32_t z) -> int32_t {
        const int32_t gy = y0 - 1 + k / kCols, gx = x0 - 1 + k % kCols;
        if (k >= kPlane || z < 0 || z >= nz || gx < 0 || gx >= nx || gy < 0 || gy >= ny) return -1;
        return gx + nx * gy + nxy * z;
      };
      // loads are unconditional (points outside the grid load row 0, whose
      // value is never consumed) so they stay in flight together
      Raw rv[kPer];
      auto issue = [&](int32_t z) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
          const int32_t r = tile_row(t + u * kBlock, z);
          rv[u] = load(r >= 0 ? r : 0);
        }
      };
      auto put = [&](int32_t z) {
        T *dst = sm.v[z & (kSlots - 1)];
#pragma unroll
        for (int u = 0; u < kPer; ++u)
          if (t + u * kBlock < kPlane) dst[t + u * kBlock] = value(rv[u]);
      };
      for (int32_t z = max(z0 - 1, 0); z <= min(z0 + 1, nz - 1); ++z) {
        issue(z);
        put(z);
      }
      __syncthreads();
      const int32_t gx = x0 + lane, gy = y0 + wy;
      const bool valid = gx < nx && gy < ny;
      const int c0 = (wy + 1) * kCols + lane + 1;  // the thread's point in the halo tile
      for (int32_t z = z0; z < z1; ++z) {
        const int32_t zn = z + 2;
        const bool pf = zn <= z1 && zn < nz;  // block-uniform
        if (pf) issue(zn);
        const T *pm = sm.v[(z - 1) & (kSlots - 1)];
        const T *pc = sm.v[z & (kSlots - 1)];
        const T *pp = sm.v[(z + 1) & (kSlots - 1)];
        const int32_t i = gx + nx * gy + nxy * z;
        auto entries = [&](auto &&consume) {
          if (!valid) return;
          if constexpr (NPTS == 7) {
            const T xv[7] = {pm[c0], pc[c0 - kCols], pc[c0 - 1], pc[c0], pc[c0 + 1], pc[c0 + kCols], pp[c0]};
            if (z > 0) consume(i - nxy, c[0], xv[0]);
            if (gy > 0) consume(i - nx, c[1], xv[1]);
            if (gx > 0) consume(i - 1, c[2], xv[2]);
            consume(i, c[3], xv[3]);
            if (gx < nx - 1) consume(i + 1, c[4], xv[4]);
            if (gy < ny - 1) consume(i + nx, c[5], xv[5]);
            if (z < nz - 1) consume(i + nxy, c[6], xv[6]);
          } else {
#pragma unroll
            for (int dk = -1; dk <= 1; ++dk) {
              const T *pl = dk < 0 ? pm : (dk == 0 ? pc : pp);
              T xv[9];
#pragma unroll
              for (int u = 0; u < 9; ++u) xv[u] = pl[c0 + (u / 3 - 1) * kCols + (u % 3 - 1)];
#pragma unroll
              for (int u = 0; u < 9; ++u) {
                const int dj = u / 3 - 1, di = u % 3 - 1;
                if (z + dk >= 0 && z + dk < nz && gy + dj >= 0 && gy + dj < ny && gx + di >= 0 &&
                    gx + di < nx)
                  consume(i + dk * nxy + dj * nx + di, c[(dk + 1) * 9 + u], xv[u]);
              }
            }
          }
        };
        auto own = [&]() -> T { return pc[c0]; };
        body(i, valid, entries, own);
        if (pf) put(zn);
        __syncthreads();
      }
    }
  }
};

// Operators of a 3-D grid get their brick plan on the host.
template <class Op>
inline void plan_op(Op &) {}
template <int NPTS, class T>
inline void plan_op(StencilOp<NPTS, T> &op) {
  op.plan();
}

}  // namespace its
