// Matrix-free stencil operator (see rowops.hpp for the row-walk contract).
#pragma once

#include "rowops.hpp"

namespace its {

// Matrix-free constant-coefficient stencil on nx*ny*nz, row = i + nx(j + ny k).
// Neighbours outside the grid are skipped, exactly as the CSR rows of the
// same operator omit them, so both give bit-identical chains.  NPTS = 7:
// offsets (k-1, j-1, i-1, centre, i+1, j+1, k+1); NPTS = 27: dk outer, dj, di
// inner.  Coefficients in that (ascending column) order.
template <int NPTS, class T>
struct StencilOp {
  int32_t nx, ny, nz, n;
  T c[NPTS];

  static constexpr int kMaxBlocks = kMaxGrid;
  struct Smem {};

  __device__ __forceinline__ void coords(int32_t i, int32_t &ix, int32_t &iy, int32_t &iz) const {
    const int32_t t = i / nx;
    ix = i - t * nx;
    iz = t / ny;
    iy = t - iz * ny;
  }

  template <class Fetch, class Consume>
  __device__ __forceinline__ void tile_entries(int32_t r0, int32_t r1, Smem &, Fetch &&fetch,
                                               Consume &&consume) const {
    const int32_t i = r0 + int32_t(threadIdx.x);
    if (i < r1) row_entries(i, fetch, consume);
  }

  template <class Fetch, class Consume>
  __device__ __forceinline__ void row_entries(int32_t i, Fetch &&fetch, Consume &&consume) const {
    int32_t ix, iy, iz;
    coords(i, ix, iy, iz);
    row_entries_at(i, ix, iy, iz, fetch, consume);
  }

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
};

}  // namespace its
