// Matrix operators.  Every operator applies row i as a fused multiply-add
// chain over the row's entries in ascending column order, starting from +0,
// with the vector entry x_j supplied by a fetch functor f(j) -- so a kernel
// can apply A to a vector it forms on the fly (p = r + beta p, s = r - alpha v)
// without storing it first.  The SpMV of the paper (Sections 2.1-2.2) is
// the chain with f(j) = x[j].
#pragma once

#include "common.hpp"

namespace its {

__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ float widen(float v) { return v; }
__device__ __forceinline__ float widen(__half v) { return __half2float(v); }

// CSR: int32 row pointers and columns, values of type V (double, float or
// __half; half values are widened exactly to float).  T is the arithmetic
// type of the chain (double for FP64, float for the mixed-precision inner
// solve).
template <class V, class T>
struct CsrOp {
  const int32_t *__restrict__ rp;
  const int32_t *__restrict__ col;
  const V *__restrict__ val;
  int32_t n;

  template <class F>
  __device__ __forceinline__ T apply(int32_t i, F &&f) const {
    T acc = T(0);
    const int32_t e = rp[i + 1];
    for (int32_t k = rp[i]; k < e; ++k) acc = fmaT(T(widen(val[k])), f(col[k]), acc);
    return acc;
  }

  // Relaxation helpers (Jacobi / Gauss-Seidel): the off-diagonal chain (the
  // diagonal entry skipped), the full chain (b - full is the residual of the
  // fetched vector) and the diagonal value.
  template <class F>
  __device__ __forceinline__ void relax(int32_t i, F &&f, T &full, T &off, T &diag) const {
    full = T(0);
    off = T(0);
    diag = T(0);
    const int32_t e = rp[i + 1];
    for (int32_t k = rp[i]; k < e; ++k) {
      const int32_t c = col[k];
      const T a = T(widen(val[k]));
      const T xv = f(c);
      full = fmaT(a, xv, full);
      if (c == i)
        diag = a;
      else
        off = fmaT(a, xv, off);
    }
  }
};

// Matrix-free constant-coefficient stencil on nx*ny*nz, row = i + nx(j + ny k).
// Neighbours outside the grid are skipped, exactly as the CSR rows of the
// same operator omit them, so both give bit-identical chains.  NPTS = 7:
// offsets (k-1, j-1, i-1, centre, i+1, j+1, k+1); NPTS = 27: dk outer, dj, di
// inner.  Coefficients in that (ascending column) order.
template <int NPTS, class T>
struct StencilOp {
  int32_t nx, ny, nz, n;
  T c[NPTS];

  __device__ __forceinline__ void coords(int32_t i, int32_t &ix, int32_t &iy, int32_t &iz) const {
    const int32_t t = i / nx;
    ix = i - t * nx;
    iz = t / ny;
    iy = t - iz * ny;
  }

  template <class F>
  __device__ __forceinline__ T apply(int32_t i, F &&f) const {
    int32_t ix, iy, iz;
    coords(i, ix, iy, iz);
    T full, off;
    chain<false>(i, ix, iy, iz, f, full, off);
    return full;
  }

  template <class F>
  __device__ __forceinline__ void relax(int32_t i, F &&f, T &full, T &off, T &diag) const {
    int32_t ix, iy, iz;
    coords(i, ix, iy, iz);
    chain<true>(i, ix, iy, iz, f, full, off);
    diag = c[NPTS / 2];
  }

  template <bool OFF, class F>
  __device__ __forceinline__ void chain(int32_t i, int32_t ix, int32_t iy, int32_t iz, F &&f,
                                        T &full, T &off) const {
    const int32_t nxy = nx * ny;
    full = T(0);
    off = T(0);
    if constexpr (NPTS == 7) {
      const bool has[7] = {iz > 0, iy > 0, ix > 0, true, ix < nx - 1, iy < ny - 1, iz < nz - 1};
      const int32_t d[7] = {-nxy, -nx, -1, 0, 1, nx, nxy};
#pragma unroll
      for (int o = 0; o < 7; ++o) {
        if (has[o]) {
          const T xv = f(i + d[o]);
          full = fmaT(c[o], xv, full);
          if (OFF && o != 3) off = fmaT(c[o], xv, off);
        }
      }
    } else {
#pragma unroll
      for (int dk = -1; dk <= 1; ++dk) {
#pragma unroll
        for (int dj = -1; dj <= 1; ++dj) {
#pragma unroll
          for (int di = -1; di <= 1; ++di) {
            const int o = (dk + 1) * 9 + (dj + 1) * 3 + (di + 1);
            const bool in = (iz + dk >= 0) && (iz + dk < nz) && (iy + dj >= 0) && (iy + dj < ny) &&
                            (ix + di >= 0) && (ix + di < nx);
            if (in) {
              const T xv = f(i + dk * nxy + dj * nx + di);
              full = fmaT(c[o], xv, full);
              if (OFF && o != 13) off = fmaT(c[o], xv, off);
            }
          }
        }
      }
    }
  }
};

}  // namespace its
