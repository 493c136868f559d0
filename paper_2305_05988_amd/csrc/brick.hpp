// The 2.5-D brick sweep of the matrix-free operators (the constant stencils
// of stencil.hpp and the variable-coefficient operator of varcoef.hpp).
#pragma once

#include "common.hpp"

namespace its {

// A block owns a 64 x 4 (x, y) tile of an nx*ny*nz grid (row = i + nx(j +
// ny k)) and marches it through a chunk of zb planes.  Each plane of the
// tile, with a one-point halo in x and y (66 x 6 points), is loaded once
// with coalesced row loads and stored in LDS by the operator; four plane
// slots rotate, so planes z-1, z, z+1 are read from LDS while plane z+2 is
// being loaded.  Every neighbour value then comes from LDS instead of a
// gather through the vector-memory path.
constexpr int kBrickTX = 64, kBrickTY = kBlock / 64;  // one point per thread per plane
constexpr int kBrickCols = kBrickTX + 2, kBrickRows = kBrickTY + 2;
constexpr int kBrickPlane = kBrickCols * kBrickRows;
constexpr int kBrickSlots = 4;

struct BrickGeom {
  int32_t nx, ny, nz;
  int32_t nbx, nby, nbz, zb;  // x tiles, y tiles, z chunks, planes per chunk
};

// Cutting z into chunks of zb planes: about 4096 bricks where each still
// marches at least 16 planes (measured at 256^3: 83 us per CG SpMV pass
// against 87 us with 2048 bricks and 90 us with 8192), else about 2048 (8
// resident blocks on each of 256 CUs).
inline BrickGeom brick_plan(int32_t nx, int32_t ny, int32_t nz) {
  BrickGeom g{nx, ny, nz, 0, 0, 0, 1};
  g.nbx = (nx + kBrickTX - 1) / kBrickTX;
  g.nby = (ny + kBrickTY - 1) / kBrickTY;
  const int64_t nxy = int64_t(g.nbx) * g.nby;
  auto zb_for = [&](int64_t target) {
    int64_t chunks = nxy > 0 ? (target + nxy - 1) / nxy : 1;
    if (chunks > nz) chunks = nz;
    if (chunks < 1) chunks = 1;
    const int64_t z = (nz + chunks - 1) / chunks;
    return int32_t(z < 1 ? 1 : z);
  };
  g.zb = zb_for(4096);
  if (g.zb < 16) g.zb = zb_for(2048);
  g.nbz = (nz + g.zb - 1) / g.zb;
  return g;
}

inline int brick_grid(const BrickGeom &g) {
  int64_t b = int64_t(g.nbx) * g.nby * g.nbz;
  if (b < 1) b = 1;
  int grid = int(b < kMaxGrid ? b : kMaxGrid);
  if (grid >= 64) grid -= grid % kXcds;
  return grid;
}

// The rows a thread owns in brick_march(), in the same order: body(i).
template <class Body>
__device__ __forceinline__ void brick_own_rows(const BrickGeom &g, Body &&body) {
  const int64_t nbricks = int64_t(g.nbx) * g.nby * g.nbz;
  const Sched sc = my_tiles(nbricks);
  const int t = threadIdx.x, lane = t & 63, wy = t >> 6;
  const int32_t nxy = g.nx * g.ny;
  for (int64_t bi = sc.begin; bi < sc.end; bi += sc.stride) {
    const int32_t bx = int32_t(bi % g.nbx), by = int32_t((bi / g.nbx) % g.nby);
    const int32_t bz = int32_t(bi / (int64_t(g.nbx) * g.nby));
    const int32_t gx = bx * kBrickTX + lane, gy = by * kBrickTY + wy;
    if (gx >= g.nx || gy >= g.ny) continue;
    const int32_t z0 = bz * g.zb, z1 = min(g.nz, z0 + g.zb);
    for (int32_t z = z0; z < z1; ++z) body(gx + g.nx * gy + nxy * z);
  }
}

// The march.  issue(r) loads what the operator stages for grid row r (a
// point outside the grid passes row 0, whose values are never consumed);
// put(slot, k, raw) stores it as point k of the halo tile in plane slot
// `slot`.  Loads are unconditional so they stay in flight together.  For
// every row of every plane, called by every thread of the block:
// row_fn(i, valid, gx, gy, z, slot of z - 1, slot of z, slot of z + 1, c0)
// with c0 the thread's point in the halo tile (valid = false past the grid).
template <class Issue, class Put, class RowFn>
__device__ __forceinline__ void brick_march(const BrickGeom &g, Issue &&issue, Put &&put, RowFn &&row_fn) {
  using Raw = decltype(issue(0));
  constexpr int kPer = (kBrickPlane + kBlock - 1) / kBlock;  // halo-tile points per thread
  const int64_t nbricks = int64_t(g.nbx) * g.nby * g.nbz;
  const Sched sc = my_tiles(nbricks);
  const int t = threadIdx.x, lane = t & 63, wy = t >> 6;
  const int32_t nx = g.nx, ny = g.ny, nz = g.nz, nxy = nx * ny;
  for (int64_t bi = sc.begin; bi < sc.end; bi += sc.stride) {
    const int32_t bx = int32_t(bi % g.nbx), by = int32_t((bi / g.nbx) % g.nby);
    const int32_t bz = int32_t(bi / (int64_t(g.nbx) * g.nby));
    const int32_t x0 = bx * kBrickTX, y0 = by * kBrickTY, z0 = bz * g.zb, z1 = min(nz, z0 + g.zb);
    // the in-plane part of the row of each halo-tile point this thread
    // loads (the same for every plane), or -1 outside the grid
    int32_t pin[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int k = t + u * kBlock;
      const int32_t py = y0 - 1 + k / kBrickCols, px = x0 - 1 + k % kBrickCols;
      pin[u] = k < kBrickPlane && px >= 0 && px < nx && py >= 0 && py < ny ? px + nx * py : -1;
    }
    Raw rv[kPer];
    auto load_plane = [&](int32_t z) {
      // callers pass planes inside the grid
      const int32_t zo = nxy * z;
#pragma unroll
      for (int u = 0; u < kPer; ++u) rv[u] = issue(pin[u] >= 0 ? pin[u] + zo : 0);
    };
    auto store_plane = [&](int32_t z) {
      const int slot = z & (kBrickSlots - 1);
#pragma unroll
      for (int u = 0; u < kPer; ++u)
        if (t + u * kBlock < kBrickPlane) put(slot, t + u * kBlock, rv[u]);
    };
    for (int32_t z = max(z0 - 1, 0); z <= min(z0 + 1, nz - 1); ++z) {
      load_plane(z);
      store_plane(z);
    }
    __syncthreads();
    const int32_t gx = x0 + lane, gy = y0 + wy;
    const bool valid = gx < nx && gy < ny;
    const int c0 = (wy + 1) * kBrickCols + lane + 1;
    for (int32_t z = z0; z < z1; ++z) {
      const int32_t zn = z + 2;
      const bool pf = zn <= z1 && zn < nz;  // block-uniform
      if (pf) load_plane(zn);
      row_fn(gx + nx * gy + nxy * z, valid, gx, gy, z, (z - 1) & (kBrickSlots - 1), z & (kBrickSlots - 1),
             (z + 1) & (kBrickSlots - 1), c0);
      if (pf) store_plane(zn);
      __syncthreads();
    }
  }
}

}  // namespace its
