// Matrix operators.  Every operator applies row i as a fused multiply-add
// chain over the row's entries in ascending column order, starting from +0,
// with the vector entry x_j supplied by a fetch functor f(j) -- so a kernel
// can apply A to a vector it forms on the fly (p = r + beta p, s = r - alpha v)
// without storing it first.  The SpMV of the paper (Sections 2.1-2.2) is
// the chain with f(j) = x[j].
//
// Tiles: kernels walk the rows in tiles of kBlock rows, one row per thread,
// through tile_entries(r0, r1, smem, fetch, consume): for the thread's row it
// calls consume(j, a_ij, x_j) for every entry in stored order.  Entries are
// handled in groups of kGather: all fetches of a group are issued before the
// first consume, so a thread keeps up to kGather gathers in flight while the
// chain itself stays strictly sequential.
#pragma once

#include "common.hpp"

namespace its {

constexpr int kGather = 8;

__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ float widen(float v) { return v; }
__device__ __forceinline__ float widen(__half v) { return __half2float(v); }

// Copies elements [c0, c1) of a 16-byte aligned array to LDS so that element
// k lands at dst[k - ka], ka = c0 rounded down to a 16-byte unit (returned).
// Whole 16-byte units inside [ka, c1 rounded down) go by LDS-DMA
// (global_load_lds_dwordx4: lane l of a wave writes dst_wave + 16 l); the
// remaining tail of fewer than one unit by plain loads.  Nothing outside
// [ka, c1) is read.  The caller waits (s_waitcnt) and synchronises the block
// before reading dst.
typedef __attribute__((address_space(1))) void global_void;
typedef __attribute__((address_space(3))) void lds_void;

template <class T>
__device__ __forceinline__ int32_t copy_to_lds(const T *__restrict__ src, int32_t c0, int32_t c1,
                                               T *dst) {
  constexpr int E = 16 / sizeof(T);
  const int32_t ka = c0 & ~(E - 1), kb = c1 & ~(E - 1);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int32_t units = (kb - ka) / E;
  for (int32_t u0 = w * 64; u0 < units; u0 += kBlock) {
    const int32_t u = u0 + lane;
    if (u < units)
      __builtin_amdgcn_global_load_lds((global_void *)(src + ka + u * E), (lds_void *)(dst + u0 * E),
                                       16, 0, 0);
  }
  const int32_t k = max(kb, c0) + int32_t(threadIdx.x);
  if (k < c1) dst[k - ka] = src[k];
  return ka;
}

// CSR: int32 row pointers and columns, values of type V (double, float or
// __half; half values are widened exactly to float).  col and val must be
// 16-byte aligned (checked when the matrix is created).  T is the arithmetic
// type of the chain (double for FP64, float for the mixed-precision inner
// solve).
template <class V, class T>
struct CsrOp {
  const int32_t *__restrict__ rp;
  const int32_t *__restrict__ col;
  const V *__restrict__ val;
  int32_t n;

  // A tile's entries are a contiguous slab of col/val.  It is copied to LDS
  // in chunks of kCap entries (the rows' own strided reads of col/val would
  // touch every cache line once per entry), then each thread walks its row
  // from LDS.  Rows longer than a chunk continue their chain across chunks,
  // so any row length works.  The copy goes straight from memory to LDS
  // (global_load_lds, 16 bytes per lane) without passing through registers.
  static constexpr int kCap = 2048;
  struct Smem {
    V val[kCap + 16 / sizeof(V)];
    int32_t col[kCap + 4];
    int32_t rp[kBlock + 1];
  };

  template <class Fetch, class Consume>
  __device__ __forceinline__ void tile_entries(int32_t r0, int32_t r1, Smem &sm, Fetch &&fetch,
                                               Consume &&consume) const {
    const int t = threadIdx.x, nr = r1 - r0;
    if (t < nr) sm.rp[t] = ld_nt(rp + r0 + t);
    if (t == 0) sm.rp[nr] = ld_nt(rp + r1);
    __syncthreads();
    const int32_t k0 = sm.rp[0], k1 = sm.rp[nr];
    const int32_t b = t < nr ? sm.rp[t] : 0, e = t < nr ? sm.rp[t + 1] : 0;
    if (k1 == k0) {  // no entries: keep rp readers ahead of the next tile's writes
      __syncthreads();
      return;
    }
    for (int32_t c0 = k0; c0 < k1; c0 += kCap) {
      const int32_t c1 = min(k1, c0 + kCap);
      const int32_t va = copy_to_lds(val, c0, c1, sm.val);
      const int32_t ca = copy_to_lds(col, c0, c1, sm.col);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      const int32_t kb = max(b, c0), ke = min(e, c1);
      for (int32_t k = kb; k < ke; k += kGather) {
        int32_t cj[kGather];
        T aj[kGather], xj[kGather];
#pragma unroll
        for (int u = 0; u < kGather; ++u) {
          if (k + u < ke) {
            cj[u] = sm.col[k + u - ca];
            aj[u] = T(widen(sm.val[k + u - va]));
            xj[u] = fetch(cj[u]);
          }
        }
#pragma unroll
        for (int u = 0; u < kGather; ++u)
          if (k + u < ke) consume(cj[u], aj[u], xj[u]);
      }
      __syncthreads();
    }
  }

  // Row-at-a-time forms (direct global loads) for kernels that visit rows
  // from a list rather than in tiles.
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
      T xv[7];
#pragma unroll
      for (int o = 0; o < 7; ++o)
        if (has[o]) xv[o] = fetch(i + d[o]);
#pragma unroll
      for (int o = 0; o < 7; ++o)
        if (has[o]) consume(i + d[o], c[o], xv[o]);
    } else {
#pragma unroll
      for (int dk = -1; dk <= 1; ++dk) {
        // one plane (9 entries) of gathers in flight at a time
        T xv[9];
        bool in[9];
#pragma unroll
        for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
          for (int di = -1; di <= 1; ++di) {
            const int u = (dj + 1) * 3 + (di + 1);
            in[u] = (iz + dk >= 0) && (iz + dk < nz) && (iy + dj >= 0) && (iy + dj < ny) &&
                    (ix + di >= 0) && (ix + di < nx);
            if (in[u]) xv[u] = fetch(i + dk * nxy + dj * nx + di);
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
