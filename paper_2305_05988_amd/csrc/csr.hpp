// CSR operator: LDS-DMA staged tiles of a CSR matrix (see rowops.hpp for the
// row-walk contract).
#pragma once

#include "rowops.hpp"

namespace its {

// Copies elements [c0, c1) of a 16-byte aligned array to LDS so that element
// k lands at dst[k - ka], ka = c0 rounded down to a 16-byte unit (returned).
// Whole 16-byte units inside [ka, c1 rounded down) go by LDS-DMA
// (global_load_lds_dwordx4: lane l of a wave writes dst_wave + 16 l); the
// remaining tail of fewer than one unit by plain loads.  Nothing outside
// [ka, c1) is read.  The caller waits (s_waitcnt) and synchronises the block
// before reading dst.
typedef __attribute__((address_space(1))) void global_void;
// Cache-policy operand of the LDS-DMA load: the non-temporal bit (the "nt"
// bit of the gfx94x/gfx950 cache-policy field), as for the streaming loads.
constexpr int kCachePolicyNT = 2;
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
                                       16, 0, kCachePolicyNT);
  }
  const int32_t k = max(kb, c0) + int32_t(threadIdx.x);
  if (k < c1) dst[k - ka] = ld_nt(src + k);
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

  int grid() const { return grid_for(n); }
  template <class Load, class Value, class Body>
  __device__ __forceinline__ void rows(Smem &sm, Load &&load, Value &&value, Body &&body) const {
    tiled_rows(*this, sm, load, value, body);
  }
  template <class Body>
  __device__ __forceinline__ void own_rows(Body &&body) const {
    tiled_own_rows(*this, body);
  }

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
        T aj[kGather];
        decltype(fetch(0)) xj[kGather];
#pragma unroll
        for (int u = 0; u < kGather; ++u) {
          cj[u] = r0;
          aj[u] = T(0);
          if (k + u < ke) {
            cj[u] = sm.col[k + u - ca];
            aj[u] = T(widen(sm.val[k + u - va]));
          }
        }
        // slots past the row's end fetch row r0 (not consumed)
#pragma unroll
        for (int u = 0; u < kGather; ++u) xj[u] = fetch(cj[u]);
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

}  // namespace its
