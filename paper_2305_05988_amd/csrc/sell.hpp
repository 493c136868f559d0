// Packed CSR: sliced ELLPACK with one 64-row slice per wavefront, entries
// of a lane stored in pairs (see rowops.hpp for the row-walk contract).
#pragma once

#include "rowops.hpp"

namespace its {

constexpr int kSlice = 64;  // rows per slice: one wave64

// Slice s holds rows 64 s .. 64 s + 63 and has width w_s, the longest row in
// the slice; it occupies slots [sp[s], sp[s] + 64 w_s).  The slice's entries
// are cut into chunks of two consecutive entries per row (the last chunk of
// an odd width holds one): chunk c (entries 2c, 2c + 1) occupies slots
// sp[s] + 128 c + [0, 64 m) with m = min(2, w_s - 2c) entries per lane, lane l
// (row 64 s + l) at sp[s] + 128 c + m l.  A wave thus reads two entries of
// all its 64 rows with one coalesced 8-byte (columns) or 16-byte (FP64
// values) access per lane, and needs neither row pointers nor LDS staging.
// A row keeps its entries in stored order; slots past its end hold column
// -1 (value 0) and are skipped, so the chain is the CSR chain bit for bit.
// sp has ns + 1 entries (ns = ceil(n / 64)).
__host__ __device__ __forceinline__ int64_t sell_slot(int64_t base, int32_t w, int32_t j,
                                                      int32_t lane) {
  const int32_t c = j >> 1;
  const int32_t m = min(2, w - 2 * c);
  return base + 128 * int64_t(c) + int64_t(m) * lane + (j - 2 * c);
}

// Two consecutive values as one load.
typedef int32_t int2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void ld_pair(const int32_t *p, int32_t &a, int32_t &b) {
  const int2_t v = ld_nt(reinterpret_cast<const int2_t *>(p));
  a = v.x;
  b = v.y;
}
__device__ __forceinline__ void ld_pair(const double *p, double &a, double &b) {
  const double2_t v = ld_nt(reinterpret_cast<const double2_t *>(p));
  a = v.x;
  b = v.y;
}
__device__ __forceinline__ void ld_pair(const float *p, float &a, float &b) {
  const float2_t v = ld_nt(reinterpret_cast<const float2_t *>(p));
  a = v.x;
  b = v.y;
}
__device__ __forceinline__ void ld_pair(const __half *p, __half &a, __half &b) {
  const uint32_t v = ld_nt(reinterpret_cast<const uint32_t *>(p));
  a = __builtin_bit_cast(__half, static_cast<unsigned short>(v & 0xffffu));
  b = __builtin_bit_cast(__half, static_cast<unsigned short>(v >> 16));
}

template <class V, class T>
struct SellOp {
  const int64_t *__restrict__ sp;
  const int32_t *__restrict__ col;
  const V *__restrict__ val;
  int32_t n;

  struct Smem {};

  int grid() const { return grid_for(n); }
  template <class Load, class Value, class Body>
  __device__ __forceinline__ void rows(Smem &sm, Load &&load, Value &&value, Body &&body) const {
    tiled_rows(*this, sm, load, value, body);
  }

  // Entries g .. g + W - 1 of the lane's row in a slice of width w (g even):
  // all column and value loads, then all gathers, then the chain.  W is a
  // compile-time constant, so the loads and gathers are straight-line code
  // and stay in flight together.
  template <int W, class Fetch, class Consume>
  __device__ __forceinline__ void group(int64_t base, int32_t w, int32_t g, int lane,
                                        int32_t standin, Fetch &&fetch, Consume &&consume) const {
    int32_t cj[W];
    V vj[W];
#pragma unroll
    for (int c = 0; 2 * c < W; ++c) {
      const int64_t at = sell_slot(base, w, g + 2 * c, lane);
      if (2 * c + 1 < W) {
        ld_pair(col + at, cj[2 * c], cj[2 * c + 1]);
        ld_pair(val + at, vj[2 * c], vj[2 * c + 1]);
      } else {
        cj[2 * c] = ld_nt(col + at);
        vj[2 * c] = ld_nt(val + at);
      }
    }
    // padding slots fetch a stand-in row (not consumed)
    decltype(fetch(0)) xj[W];
#pragma unroll
    for (int u = 0; u < W; ++u) xj[u] = fetch(cj[u] >= 0 ? cj[u] : standin);
#pragma unroll
    for (int u = 0; u < W; ++u)
      if (cj[u] >= 0) consume(cj[u], T(widen(vj[u])), xj[u]);
  }

  template <class Fetch, class Consume>
  __device__ __forceinline__ void tile_entries(int32_t r0, int32_t r1, Smem &, Fetch &&fetch,
                                               Consume &&consume) const {
    // tiles are kBlock = 4 slices long and start on a slice boundary, so
    // wave w of the block owns slice r0 / 64 + w
    const int32_t s = __builtin_amdgcn_readfirstlane((r0 >> 6) + (int32_t(threadIdx.x) >> 6));
    if (s * kSlice >= r1) return;
    const int lane = threadIdx.x & 63;
    const int64_t base = sp[s];
    const int32_t w = int32_t((sp[s + 1] - base) >> 6);
    const int32_t standin = s * kSlice;
    // widths up to 7 (7-point stencils and the like) in one group; wider
    // slices in groups of 4, which keeps the registers of the widest group
    // within reach of 6 waves per SIMD
    switch (w) {  // wave-uniform
      case 0: return;
      case 1: group<1>(base, w, 0, lane, standin, fetch, consume); return;
      case 2: group<2>(base, w, 0, lane, standin, fetch, consume); return;
      case 3: group<3>(base, w, 0, lane, standin, fetch, consume); return;
      case 4: group<4>(base, w, 0, lane, standin, fetch, consume); return;
      case 5: group<5>(base, w, 0, lane, standin, fetch, consume); return;
      case 6: group<6>(base, w, 0, lane, standin, fetch, consume); return;
      case 7: group<7>(base, w, 0, lane, standin, fetch, consume); return;
      default: break;
    }
    int32_t g = 0;
    for (; g + 4 <= w; g += 4) group<4>(base, w, g, lane, standin, fetch, consume);
    switch (w - g) {
      case 1: group<1>(base, w, g, lane, standin, fetch, consume); break;
      case 2: group<2>(base, w, g, lane, standin, fetch, consume); break;
      case 3: group<3>(base, w, g, lane, standin, fetch, consume); break;
      default: break;
    }
  }
};

// ------------------------------------------------------------------ packing

// The packed layout covers `count` rows: row p of the layout is matrix row
// rows[p], or p itself when rows is null (a colour's rows for the
// Gauss-Seidel half-sweeps, or the whole matrix in order).
//
// Width of each slice; a row whose pointers are out of order or outside
// [0, nnz] is counted in *bad and given width 0.
__global__ void __launch_bounds__(kBlock) k_sell_width(int32_t count, int32_t nnz,
                                                       const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ rows,
                                                       int32_t *__restrict__ width, uint32_t *bad) {
  const int64_t ns = (int64_t(count) + kSlice - 1) / kSlice;
  for (int64_t s = int64_t(blockIdx.x) * kBlock + threadIdx.x; s < ns;
       s += int64_t(gridDim.x) * kBlock) {
    int32_t w = 0;
    const int32_t p1 = int32_t(min(int64_t(count), (s + 1) * kSlice));
    for (int32_t p = int32_t(s * kSlice); p < p1; ++p) {
      const int32_t i = rows ? rows[p] : p;
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
__global__ void __launch_bounds__(kBlock) k_sell_scatter(int32_t count, const int32_t *__restrict__ rp,
                                                         const int32_t *__restrict__ rows,
                                                         const int32_t *__restrict__ col,
                                                         const V *__restrict__ val,
                                                         const int64_t *__restrict__ sp,
                                                         int32_t *__restrict__ col_out,
                                                         V *__restrict__ val_out) {
  const int64_t slots = (int64_t(count) + kSlice - 1) / kSlice * kSlice;
  for (int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x; p < slots;
       p += int64_t(gridDim.x) * kBlock) {
    const int64_t s = p / kSlice;
    const int32_t l = int32_t(p % kSlice);
    const int64_t base = sp[s];
    const int32_t w = int32_t((sp[s + 1] - base) / kSlice);
    int32_t b = 0, len = 0;
    if (p < count) {
      const int32_t i = rows ? rows[p] : int32_t(p);
      b = rp[i];
      len = min(rp[i + 1] - b, w);
      if (len < 0) len = 0;
    }
    for (int32_t j = 0; j < w; ++j) {
      const int64_t at = sell_slot(base, w, j, l);
      if (col_out) col_out[at] = j < len ? col[b + j] : -1;
      val_out[at] = j < len ? val[b + j] : V(0.0f);
    }
  }
}

}  // namespace its
