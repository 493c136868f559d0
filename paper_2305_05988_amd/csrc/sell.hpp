// Packed CSR: sliced ELLPACK with one 64-row slice per wavefront (see
// rowops.hpp for the row-walk contract).
#pragma once

#include "rowops.hpp"

namespace its {

constexpr int kSlice = 64;  // rows per slice: one wave64

// Slice s holds rows 64 s .. 64 s + 63.  Its width w_s is the longest row in
// the slice; entry j (j < w_s) of the slice's lane l (row 64 s + l) sits at
// sp[s] + 64 j + l, so the wave reads entry j of its 64 rows with one
// coalesced access and needs neither row pointers nor LDS staging.  A row
// keeps its entries in stored order; slots past its end hold column -1
// (value 0) and are skipped, so the chain is the CSR chain bit for bit.
// sp has ns + 1 entries (ns = ceil(n / 64)), sp[s + 1] - sp[s] = 64 w_s.
template <class V, class T, int NG = 4>
struct SellOp {
  const int64_t *__restrict__ sp;
  const int32_t *__restrict__ col;
  const V *__restrict__ val;
  int32_t n;

  // Entries per group whose gathers are in flight together (4 keeps the
  // passes at full occupancy, 8 waves per SIMD).
  static constexpr int kChunk = NG;
  // Grid of the packed passes: the resident capacity, 8 blocks of 4 waves
  // on each of the 256 CUs, so that all blocks run at once and the tiles
  // dealt round-robin within an XCD advance as one front (a plane of a 3-D
  // grid is gathered again one step later, from L2).  With more blocks the
  // later ones revisit neighbours long after they left L2.
  static constexpr int kMaxBlocks = 2048;

  struct Smem {};

  template <class Fetch, class Consume>
  __device__ __forceinline__ void tile_entries(int32_t r0, int32_t r1, Smem &, Fetch &&fetch,
                                               Consume &&consume) const {
    // tiles are kBlock = 4 slices long and start on a slice boundary, so
    // wave w of the block owns slice r0 / 64 + w
    const int32_t s = __builtin_amdgcn_readfirstlane((r0 >> 6) + (int32_t(threadIdx.x) >> 6));
    if (s * kSlice >= r1) return;
    const int lane = threadIdx.x & 63;
    const int64_t b = sp[s];
    const int32_t w = int32_t((sp[s + 1] - b) >> 6);
    const int32_t *c = col + b + lane;
    const V *v = val + b + lane;
    for (int32_t j0 = 0; j0 < w; j0 += kChunk) {
      int32_t cj[kChunk];
      T aj[kChunk];
      decltype(fetch(0)) xj[kChunk];
#pragma unroll
      for (int u = 0; u < kChunk; ++u) {
        cj[u] = -1;
        aj[u] = T(0);
        if (j0 + u < w) {  // wave-uniform
          cj[u] = ld_nt(c + int64_t(j0 + u) * kSlice);
          aj[u] = T(widen(ld_nt(v + int64_t(j0 + u) * kSlice)));
        }
      }
      // padding slots fetch the slice's first row (not consumed)
#pragma unroll
      for (int u = 0; u < kChunk; ++u) xj[u] = fetch(cj[u] >= 0 ? cj[u] : s * kSlice);
#pragma unroll
      for (int u = 0; u < kChunk; ++u)
        if (cj[u] >= 0) consume(cj[u], aj[u], xj[u]);
    }
  }
};

// ------------------------------------------------------------------ packing

// Width of each slice; a row whose pointers are out of order or outside
// [0, nnz] is counted in *bad and given width 0.
__global__ void __launch_bounds__(kBlock) k_sell_width(int32_t n, int32_t nnz,
                                                       const int32_t *__restrict__ rp,
                                                       int32_t *__restrict__ width, uint32_t *bad) {
  const int64_t ns = (int64_t(n) + kSlice - 1) / kSlice;
  for (int64_t s = int64_t(blockIdx.x) * kBlock + threadIdx.x; s < ns;
       s += int64_t(gridDim.x) * kBlock) {
    int32_t w = 0;
    const int32_t i1 = int32_t(min(int64_t(n), (s + 1) * kSlice));
    for (int32_t i = int32_t(s * kSlice); i < i1; ++i) {
      const int32_t b = rp[i], e = rp[i + 1];
      if (b < 0 || e < b || e > nnz) {
        atomicAdd(bad, 1u);
        continue;
      }
      w = max(w, e - b);
    }
    width[s] = w;
  }
}

// Scatters the entries of every row (and the padding of every slot past a
// row's end, including the rows of the last slice beyond n) into the
// sliced layout.  col_out may be null to pack values only.
template <class V>
__global__ void __launch_bounds__(kBlock) k_sell_scatter(int32_t n, const int32_t *__restrict__ rp,
                                                         const int32_t *__restrict__ col,
                                                         const V *__restrict__ val,
                                                         const int64_t *__restrict__ sp,
                                                         int32_t *__restrict__ col_out,
                                                         V *__restrict__ val_out) {
  const int64_t rows = (int64_t(n) + kSlice - 1) / kSlice * kSlice;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < rows;
       i += int64_t(gridDim.x) * kBlock) {
    const int64_t s = i / kSlice, l = i % kSlice;
    const int64_t base = sp[s];
    const int32_t w = int32_t((sp[s + 1] - base) / kSlice);
    int32_t b = 0, len = 0;
    if (i < n) {
      b = rp[i];
      len = min(rp[i + 1] - b, w);
      if (len < 0) len = 0;
    }
    for (int32_t j = 0; j < w; ++j) {
      const int64_t at = base + int64_t(j) * kSlice + l;
      if (col_out) col_out[at] = j < len ? col[b + j] : -1;
      val_out[at] = j < len ? val[b + j] : V(0.0f);
    }
  }
}

}  // namespace its
