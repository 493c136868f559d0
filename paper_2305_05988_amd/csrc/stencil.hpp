// Matrix-free stencil operator (see rowops.hpp for the row-walk contract).
#pragma once

#include "brick.hpp"
#include "rowops.hpp"

namespace its {

// Matrix-free constant-coefficient stencil on nx*ny*nz, row = i + nx(j + ny k).
// Neighbours outside the grid are skipped, exactly as the CSR rows of the
// same operator omit them, so both give bit-identical chains.  NPTS = 7:
// offsets (k-1, j-1, i-1, centre, i+1, j+1, k+1); NPTS = 27: dk outer, dj, di
// inner.  Coefficients in that (ascending column) order.
//
// The SpMV passes sweep the grid in bricks (brick.hpp): the plane slots in
// LDS hold x_j (the pass's value of what it loads for row j), and each row
// reads its neighbours from them.  Rows keep the CSR chain order.
template <int NPTS, class T>
struct StencilOp;
template <int NPTS, class T> struct GathersPairs<StencilOp<NPTS, T>> : std::false_type {};

template <int NPTS, class T>
struct StencilOp {
  int32_t nx, ny, nz, n;
  T c[NPTS];
  int32_t nbx = 0, nby = 0, nbz = 0, zb = 1;  // brick plan (plan())

  struct Smem {
    T v[kBrickSlots][kBrickPlane];
  };

  void plan() {
    const BrickGeom g = brick_plan(nx, ny, nz);
    nbx = g.nbx;
    nby = g.nby;
    nbz = g.nbz;
    zb = g.zb;
  }
  __host__ __device__ BrickGeom geom() const { return {nx, ny, nz, nbx, nby, nbz, zb}; }
  int grid() const { return brick_grid(geom()); }

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
    brick_own_rows(geom(), body);
  }

  // ------------------------------------------------------ 2.5-D row sweep
  template <class Load, class Value, class Body>
  __device__ __forceinline__ void rows(Smem &sm, Load &&load, Value &&value, Body &&body) const {
    const int32_t nxy = nx * ny;
    brick_march(
        geom(), [&](int32_t r) { return load(r); },
        [&](int slot, int k, const auto &raw) { sm.v[slot][k] = value(raw); },
        [&](int32_t i, bool valid, int32_t gx, int32_t gy, int32_t z, int sm1, int s0, int sp1, int c0) {
          const T *pm = sm.v[sm1];
          const T *pc = sm.v[s0];
          const T *pp = sm.v[sp1];
          auto entries = [&](auto &&consume) {
            if (!valid) return;
            if constexpr (NPTS == 7) {
              const T xv[7] = {pm[c0],     pc[c0 - kBrickCols], pc[c0 - 1], pc[c0],
                               pc[c0 + 1], pc[c0 + kBrickCols], pp[c0]};
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
                for (int u = 0; u < 9; ++u) xv[u] = pl[c0 + (u / 3 - 1) * kBrickCols + (u % 3 - 1)];
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
        });
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
