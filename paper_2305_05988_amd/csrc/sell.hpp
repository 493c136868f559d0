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
//
// Offset slices store no columns.  When every row of a slice has strictly
// ascending columns and all of them draw their column offsets (column minus
// row) from one ascending list d_0 < ... < d_{w-1} of exactly w offsets, the
// slice keeps, per entry position j, the offset d_j and a 64-bit mask of the
// lanes whose row has an entry at offset d_j; a row's entries are laid out
// at the positions of their offsets (value 0 elsewhere, not consumed).
// Entry j of such a row is then column row + d_j, in the row's own order, so
// the chain is unchanged.  The descriptors of slice s sit at positions
// (sp[s] >> 6) + j of soff / smask, and the slice is flagged by bit 0 of
// sp[s] (slot bases are multiples of 64).  Structured-grid matrices (the
// stencils in CSR form) pack entirely into offset slices, which removes the
// 4-byte column index from every entry's traffic.
constexpr int64_t kOffsetSlice = 1;
constexpr int kMaxOffsetWidth = 32;
__host__ __device__ __forceinline__ int64_t slice_base(int64_t v) { return v & ~int64_t(63); }

__host__ __device__ __forceinline__ int64_t sell_slot(int64_t base, int32_t w, int32_t j,
                                                      int32_t lane) {
  const int32_t c = j >> 1;
  const int32_t m = min(2, w - 2 * c);
  return base + 128 * int64_t(c) + int64_t(m) * lane + (j - 2 * c);
}

// Low-precision values (FP32, FP16) use chunks of four entries per lane
// instead of two: within a slice of width w the entries 0 .. 4 floor(w/4) - 1
// form chunks of four (chunk c at base + 256 c + 4 l + {0..3}), a remaining
// pair sits at base + 64 f + 2 l + {0, 1} (f = 4 floor(w/4)) and a last odd
// entry at base + 64 (w - 1) + l.  A lane then reads four of its entries
// with one 16-byte (FP32) or 8-byte (FP16) access.  The FP64 values and the
// columns keep the pairs of sell_slot.
__host__ __device__ __forceinline__ int64_t sell_slot4(int64_t base, int32_t w, int32_t j,
                                                       int32_t lane) {
  const int32_t f = w / 4 * 4;
  if (j < f) return base + 64 * int64_t(j & ~3) + 4 * lane + (j & 3);
  if (w - f >= 2 && j < f + 2) return base + 64 * int64_t(f) + 2 * lane + (j - f);
  return base + 64 * int64_t(w - 1) + lane;
}
template <class V>
__host__ __device__ __forceinline__ int64_t value_slot(int64_t base, int32_t w, int32_t j,
                                                       int32_t lane) {
  return sizeof(V) < 8 ? sell_slot4(base, w, j, lane) : sell_slot(base, w, j, lane);
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

// Four consecutive values as one load.
typedef uint32_t uint2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void ld_quad(const float *p, float *v) {
  const float4_t q = ld_nt(reinterpret_cast<const float4_t *>(p));
  v[0] = q.x;
  v[1] = q.y;
  v[2] = q.z;
  v[3] = q.w;
}
__device__ __forceinline__ void ld_quad(const __half *p, __half *v) {
  const uint2_t q = ld_nt(reinterpret_cast<const uint2_t *>(p));
  v[0] = __builtin_bit_cast(__half, static_cast<unsigned short>(q.x & 0xffffu));
  v[1] = __builtin_bit_cast(__half, static_cast<unsigned short>(q.x >> 16));
  v[2] = __builtin_bit_cast(__half, static_cast<unsigned short>(q.y & 0xffffu));
  v[3] = __builtin_bit_cast(__half, static_cast<unsigned short>(q.y >> 16));
}

// N consecutive low-precision values (N = 2, 4 or 8) with the widest
// accesses that cover them (one 4-, 8- or 16-byte load for FP16; one or two
// 8- or 16-byte loads for FP32).  p must be aligned to the run's size (16
// bytes at most).
typedef uint32_t uint4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ __half half_bits(uint32_t w, int k) {
  return __builtin_bit_cast(__half, static_cast<unsigned short>(w >> (16 * k)));
}
template <int N>
__device__ __forceinline__ void ld_run(const __half *p, __half *v) {
  if constexpr (N == 8) {
    const uint4_t q = ld_nt(reinterpret_cast<const uint4_t *>(p));
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = half_bits(q[k >> 1], k & 1);
  } else if constexpr (N == 4) {
    const uint2_t q = ld_nt(reinterpret_cast<const uint2_t *>(p));
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = half_bits(q[k >> 1], k & 1);
  } else {
    static_assert(N == 2, "runs of 2, 4 or 8");
    const uint32_t q = ld_nt(reinterpret_cast<const uint32_t *>(p));
    v[0] = half_bits(q, 0);
    v[1] = half_bits(q, 1);
  }
}
template <int N>
__device__ __forceinline__ void ld_run(const float *p, float *v) {
  if constexpr (N == 2) {
    const float2_t q = ld_nt(reinterpret_cast<const float2_t *>(p));
    v[0] = q.x;
    v[1] = q.y;
  } else {
    static_assert(N == 4 || N == 8, "runs of 2, 4 or 8");
#pragma unroll
    for (int h = 0; h < N / 4; ++h) {
      const float4_t q = ld_nt(reinterpret_cast<const float4_t *>(p + 4 * h));
      v[4 * h] = q.x;
      v[4 * h + 1] = q.y;
      v[4 * h + 2] = q.z;
      v[4 * h + 3] = q.w;
    }
  }
}

// OffOnly: every non-empty slice is an offset slice (the layout stores no
// columns), so the explicit-column path is not compiled in.
template <class V, class T, bool OffOnly = false>
struct SellOp {
  using value_type = V;
  const int64_t *__restrict__ sp;
  const int32_t *__restrict__ col;
  const V *__restrict__ val;
  int32_t n;
  const int32_t *__restrict__ soff;   // offset slices: d_j per entry position
  const uint64_t *__restrict__ smask;  // offset slices: lanes with an entry at d_j
  const int32_t *__restrict__ row_of;  // layout row p is matrix row row_of[p] (null: p)

  struct Smem {};

  // FP32/FP16 passes move few bytes per tile, so per-block costs weigh more:
  // their blocks walk several tiles (and one finishing kernel suffices);
  // FP64 passes keep one tile per block
  int grid() const { return sizeof(V) < 8 ? grid_for(n, kFinishOne) : grid_for(n); }
  template <class Load, class Value, class Body>
  __device__ __forceinline__ void rows(Smem &sm, Load &&load, Value &&value, Body &&body) const {
    tiled_rows(*this, sm, load, value, body);
  }
  template <class Body>
  __device__ __forceinline__ void own_rows(Body &&body) const {
    tiled_own_rows(*this, body);
  }

  // ------------------------------------------------ two rows per lane
  // The refinement's FP32/FP16 pass moves few bytes per row, and one row per
  // lane leaves it bound by memory instructions: each entry costs a wave a
  // gather of 8-byte {r, p} pairs.  On offset-slice layouts a wave can take
  // two slices at once, lane l holding rows 2l' and 2l' + 1 (l' = l mod 32)
  // of slice 2k + l / 32: both rows have the same column offsets, so one
  // 16-byte gather at row + d brings both rows' pairs for offset d, and the
  // layout already places the two rows' values side by side (one load for
  // four entries of both rows).  Tiles are 512 rows (two slices per wave).
  // When the two slices differ in width (a grid boundary between them, or
  // the matrix's last slice) the tile takes them one row per lane instead.
  //
  // body(i0, i1, valid0, valid1, entries): the lane's two rows; inside it
  // entries(c0, c1) calls c0(j, a_ij, {r_j, p_j}) for row i0's entries and
  // c1 for row i1's, each row in stored order.  rp must be readable at
  // indices -1 and n (a lane's 16-byte gather may cover one pair past
  // either end; those halves are never consumed).  row_of must be null.
  // Slices of at most 7 entries: at most the 1536 blocks that fit at once
  // at the pass's 6 waves per SIMD (measured at 256^3, FP16 values: 8 %
  // faster than 4096 blocks); wider slices: 4096 (27-point 192^3: 3-5 %
  // faster than 1536).
  int grid_pairs(bool wide) const {
    return grid_for((int64_t(n) + 1) / 2, wide ? kFinishOne : 1536);
  }

  template <int G, class C0, class C1>
  __device__ __forceinline__ void pair_group(int64_t base, int32_t w, int32_t g, int half, int l2,
                                             int64_t ka, int64_t kb, int32_t r0, int32_t standin,
                                             const float2_t *rp, C0 &&c0, C1 &&c1) const {
    // values of entries g .. g + G - 1 of both rows (row r0: v0, r0 + 1: v1)
    V v0[G], v1[G];
    constexpr int F = G / 4 * 4;
#pragma unroll
    for (int c = 0; 4 * c < F; ++c) {
      V t[8];
      ld_run<8>(val + base + 64 * int64_t(g + 4 * c) + 8 * l2, t);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        v0[4 * c + k] = t[k];
        v1[4 * c + k] = t[4 + k];
      }
    }
    if constexpr (G - F >= 2) {
      V t[4];
      ld_run<4>(val + base + 64 * int64_t(g + F) + 4 * l2, t);
      v0[F] = t[0];
      v0[F + 1] = t[1];
      v1[F] = t[2];
      v1[F + 1] = t[3];
    }
    if constexpr ((G - F) % 2 == 1) {
      V t[2];
      ld_run<2>(val + base + 64 * int64_t(w - 1) + 2 * l2, t);
      v0[G - 1] = t[0];
      v1[G - 1] = t[1];
    }
    // the lane's slice's offsets and its two rows' entry bits
    int32_t d[G];
    uint32_t h0 = 0, h1 = 0;
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int32_t oa = soff[ka + g + u], ob = soff[kb + g + u];
      const uint64_t ma = smask[ka + g + u], mb = smask[kb + g + u];
      d[u] = half ? ob : oa;
      const uint64_t m = half ? mb : ma;
      h0 |= uint32_t((m >> (2 * l2)) & 1u) << u;
      h1 |= uint32_t((m >> (2 * l2 + 1)) & 1u) << u;
    }
    // one 16-byte gather per entry for both rows; an entry neither row has
    // gathers at the slice's first row (not consumed)
    float4_t x[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int32_t j = ((h0 | h1) >> u) & 1u ? r0 + d[u] : standin;
      __builtin_memcpy(&x[u], rp + j, sizeof(float4_t));
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      if ((h0 >> u) & 1u) c0(r0 + d[u], T(widen(v0[u])), float2_t{x[u].x, x[u].y});
      if ((h1 >> u) & 1u) c1(r0 + 1 + d[u], T(widen(v1[u])), float2_t{x[u].z, x[u].w});
    }
  }

  template <class Body>
  __device__ __forceinline__ void walk_pairs(const float2_t *rp, Body &&body) const {
    static_assert(OffOnly && sizeof(V) < 8, "two rows per lane: FP32/FP16 offset slices");
    const int64_t ntiles = (int64_t(n) + 2 * kBlock - 1) / (2 * kBlock);
    const Sched sc = my_tiles(ntiles);
    const int lane = threadIdx.x & 63, half = lane >> 5, l2 = lane & 31;
    const int32_t ns = (n + kSlice - 1) / kSlice;
    auto fetch = [&](int32_t j) { return rp[j]; };
    for (int64_t t = sc.begin; t < sc.end; t += sc.stride) {
      const int32_t sa = __builtin_amdgcn_readfirstlane(int32_t(t) * (2 * kBlock / kSlice) +
                                                        2 * (int32_t(threadIdx.x) >> 6));
      const int32_t sb = sa + 1;
      // slice bounds; a slice past the last one has width 0
      const int32_t ca = min(sa, ns - 1), cb = min(sb, ns - 1);
      const int64_t base_a = slice_base(sp[ca]), base_b = slice_base(sp[cb]);
      const int32_t wa = sa < ns ? int32_t((slice_base(sp[ca + 1]) - base_a) >> 6) : 0;
      const int32_t wb = sb < ns ? int32_t((slice_base(sp[cb + 1]) - base_b) >> 6) : 0;
      if (wa == wb) {
        const int32_t sh = half ? sb : sa;
        const int32_t r0 = sh * kSlice + 2 * l2;
        const int32_t standin = min(sh, ns - 1) * kSlice;
        const int64_t base = half ? base_b : base_a;
        const int64_t ka = base_a >> 6, kb = base_b >> 6;
        auto entries = [&](auto &&c0, auto &&c1) {
          auto grp = [&](auto G, int32_t g) {
            pair_group<decltype(G)::value>(base, wa, g, half, l2, ka, kb, r0, standin, rp, c0, c1);
          };
          // groups of four entries (a group's sixteen bytes of gathers per
          // entry keep its registers within reach of more waves per SIMD)
          int32_t g = 0;
          for (; g + 4 <= wa; g += 4) grp(std::integral_constant<int, 4>(), g);
          switch (wa - g) {
            case 1: grp(std::integral_constant<int, 1>(), g); break;
            case 2: grp(std::integral_constant<int, 2>(), g); break;
            case 3: grp(std::integral_constant<int, 3>(), g); break;
            default: break;
          }
        };
        body(r0, r0 + 1, r0 < n, r0 + 1 < n, entries);
      } else {
        // one row per lane: row 64 sa + l, then row 64 sb + l
        const int32_t i0 = sa * kSlice + lane, i1 = sb * kSlice + lane;
        auto entries = [&](auto &&c0, auto &&c1) {
          walk<true>(base_a, wa, lane, i0 < n ? i0 : ca * kSlice, ca * kSlice, fetch, c0);
          walk<true>(base_b, wb, lane, i1 < n ? i1 : cb * kSlice, cb * kSlice, fetch, c1);
        };
        body(i0, i1, i0 < n, i1 < n, entries);
      }
    }
  }

  // Entries g .. g + W - 1 of the lane's row in a slice of width w (g even):
  // all column and value loads, then all gathers, then the chain.  W is a
  // compile-time constant, so the loads and gathers are straight-line code
  // and stay in flight together.  Off: the columns come from the slice's
  // offsets (row + d_j where the lane's mask bit is set) instead of loads.
  template <int W, bool Off, class Fetch, class Consume>
  __device__ __forceinline__ void group(int64_t base, int32_t w, int32_t g, int lane, int32_t row,
                                        int32_t standin, Fetch &&fetch, Consume &&consume) const {
    int32_t cj[W];
    bool has[W];
    V vj[W];
#pragma unroll
    for (int c = 0; 2 * c < W; ++c) {
      const int64_t at = sell_slot(base, w, g + 2 * c, lane);
      if (2 * c + 1 < W) {
        if (!Off) ld_pair(col + at, cj[2 * c], cj[2 * c + 1]);
        if (sizeof(V) == 8) ld_pair(val + at, vj[2 * c], vj[2 * c + 1]);
      } else {
        if (!Off) cj[2 * c] = ld_nt(col + at);
        if (sizeof(V) == 8) vj[2 * c] = ld_nt(val + at);
      }
    }
    if constexpr (sizeof(V) < 8) {
      // groups start at multiples of 4 and a group shorter than 4 ends the
      // slice, so the group's chunks are the slice's own
      constexpr int F = W / 4 * 4;
#pragma unroll
      for (int c = 0; 4 * c < F; ++c) ld_quad(val + sell_slot4(base, w, g + 4 * c, lane), vj + 4 * c);
      if constexpr (W - F >= 2) ld_pair(val + sell_slot4(base, w, g + F, lane), vj[F], vj[F + 1]);
      if constexpr ((W - F) % 2 == 1) vj[W - 1] = ld_nt(val + sell_slot4(base, w, g + W - 1, lane));
    }
    if (Off) {
      // the group's descriptors are wave-uniform: all of them are loaded
      // before any is used, so they arrive together (a load under the
      // lane's mask test would make each wait for the previous one)
      const int64_t k = (base >> 6) + g;
      int32_t offs[W];
      uint64_t msk[W];
#pragma unroll
      for (int u = 0; u < W; ++u) {
        offs[u] = soff[k + u];
        msk[u] = smask[k + u];
      }
#pragma unroll
      for (int u = 0; u < W; ++u) cj[u] = row + offs[u];
      // the wave-uniform mask is the lane condition itself (it becomes the
      // exec mask; no per-lane bit test)
#pragma unroll
      for (int u = 0; u < W; ++u) has[u] = __builtin_amdgcn_inverse_ballot_w64(msk[u]);
    } else {
#pragma unroll
      for (int u = 0; u < W; ++u) has[u] = cj[u] >= 0;
    }
    // padding slots fetch a stand-in row (not consumed)
    decltype(fetch(0)) xj[W];
#pragma unroll
    for (int u = 0; u < W; ++u) xj[u] = fetch(has[u] ? cj[u] : standin);
#pragma unroll
    for (int u = 0; u < W; ++u)
      if (has[u]) consume(cj[u], T(widen(vj[u])), xj[u]);
  }

  template <bool Off, class Fetch, class Consume>
  __device__ __forceinline__ void walk(int64_t base, int32_t w, int lane, int32_t row,
                                       int32_t standin, Fetch &&fetch, Consume &&consume) const {
    // widths up to 7 (7-point stencils and the like) in one group; wider
    // slices in groups of 4, which keeps the registers of the widest group
    // within reach of 6 waves per SIMD
    switch (w) {  // wave-uniform
      case 0: return;
      case 1: group<1, Off>(base, w, 0, lane, row, standin, fetch, consume); return;
      case 2: group<2, Off>(base, w, 0, lane, row, standin, fetch, consume); return;
      case 3: group<3, Off>(base, w, 0, lane, row, standin, fetch, consume); return;
      case 4: group<4, Off>(base, w, 0, lane, row, standin, fetch, consume); return;
      case 5: group<5, Off>(base, w, 0, lane, row, standin, fetch, consume); return;
      case 6: group<6, Off>(base, w, 0, lane, row, standin, fetch, consume); return;
      case 7: group<7, Off>(base, w, 0, lane, row, standin, fetch, consume); return;
      default: break;
    }
    int32_t g = 0;
    for (; g + 4 <= w; g += 4) group<4, Off>(base, w, g, lane, row, standin, fetch, consume);
    switch (w - g) {
      case 1: group<1, Off>(base, w, g, lane, row, standin, fetch, consume); break;
      case 2: group<2, Off>(base, w, g, lane, row, standin, fetch, consume); break;
      case 3: group<3, Off>(base, w, g, lane, row, standin, fetch, consume); break;
      default: break;
    }
  }

  template <class Fetch, class Consume>
  __device__ __forceinline__ void tile_entries(int32_t r0, int32_t r1, Smem &, Fetch &&fetch,
                                               Consume &&consume) const {
    // tiles are kBlock = 4 slices long and start on a slice boundary, so
    // wave w of the block owns slice r0 / 64 + w
    const int32_t s = __builtin_amdgcn_readfirstlane((r0 >> 6) + (int32_t(threadIdx.x) >> 6));
    if (s * kSlice >= r1) return;
    const int lane = threadIdx.x & 63;
    const int64_t raw = sp[s];
    const int64_t base = slice_base(raw);
    const int32_t w = int32_t((slice_base(sp[s + 1]) - base) >> 6);
    const int32_t standin = s * kSlice;
    if (OffOnly || (raw & kOffsetSlice)) {
      const int32_t p = standin + lane;
      const int32_t row = p < n ? (row_of ? row_of[p] : p) : standin;
      walk<true>(base, w, lane, row, standin, fetch, consume);
    } else if (!OffOnly) {
      walk<false>(base, w, lane, 0, standin, fetch, consume);
    }
  }
};

// Operators whose refinement pass walks two rows per lane.
template <class Op> struct PairWalk : std::false_type {};
template <class V> struct PairWalk<SellOp<V, float, true>> : std::integral_constant<bool, sizeof(V) < 8> {};

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

// Decides which slices become offset slices (one thread per slice): builds
// the sorted list of the column offsets of the slice's rows, and if every
// row is strictly ascending and the list holds exactly w offsets, writes the
// offsets and lane masks at (sp[s] >> 6) + j and sets the slice's flag in
// sp[s].  The slots of the slices that keep explicit columns are added to
// *col_slots.  sp must hold the unflagged slot bases on entry.
__global__ void __launch_bounds__(kBlock) k_sell_offsets(int32_t count, const int32_t *__restrict__ rp,
                                                         const int32_t *__restrict__ rows,
                                                         const int32_t *__restrict__ col, int64_t *sp,
                                                         int32_t *__restrict__ soff,
                                                         uint64_t *__restrict__ smask,
                                                         unsigned long long *col_slots) {
  const int64_t ns = (int64_t(count) + kSlice - 1) / kSlice;
  for (int64_t s = int64_t(blockIdx.x) * kBlock + threadIdx.x; s < ns;
       s += int64_t(gridDim.x) * kBlock) {
    const int64_t base = sp[s];
    const int32_t w = int32_t((slice_base(sp[s + 1]) - base) >> 6);
    if (w == 0) continue;
    bool ok = w <= kMaxOffsetWidth;
    int32_t d[kMaxOffsetWidth];
    int32_t u = 0;
    const int32_t p0 = int32_t(s * kSlice);
    const int32_t p1 = int32_t(min(int64_t(count), (s + 1) * kSlice));
    for (int32_t p = p0; ok && p < p1; ++p) {
      const int32_t i = rows ? rows[p] : p;
      for (int32_t e = rp[i]; ok && e < rp[i + 1]; ++e) {
        if (e > rp[i] && col[e] <= col[e - 1]) {
          ok = false;
          break;
        }
        const int32_t o = col[e] - i;
        int32_t at = 0;  // insertion point in the sorted list
        while (at < u && d[at] < o) ++at;
        if (at < u && d[at] == o) continue;
        if (u == w) {
          ok = false;
          break;
        }
        for (int32_t q = u; q > at; --q) d[q] = d[q - 1];
        d[at] = o;
        ++u;
      }
    }
    if (!ok || u != w) {
      atomicAdd(col_slots, static_cast<unsigned long long>(kSlice) * unsigned(w));
      continue;
    }
    uint64_t m[kMaxOffsetWidth];
    for (int32_t j = 0; j < w; ++j) m[j] = 0;
    for (int32_t p = p0; p < p1; ++p) {
      const int32_t i = rows ? rows[p] : p;
      int32_t j = 0;
      for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
        // the row's offsets are in the list, in ascending order
        while (j < w && d[j] != col[e] - i) ++j;
        if (j < w) m[j] |= uint64_t(1) << (p - p0);
      }
    }
    const int64_t k = base >> 6;
    for (int32_t j = 0; j < w; ++j) {
      soff[k + j] = d[j];
      smask[k + j] = m[j];
    }
    sp[s] = base | kOffsetSlice;
  }
}

// Scatters the entries of every row (and the padding of every slot past a
// row's end, including the rows of the last slice beyond n) into the
// sliced layout; in an offset slice a row's entries go to the positions of
// their offsets and no columns are written.  col_out may be null to pack
// values only.
template <class V>
__global__ void __launch_bounds__(kBlock) k_sell_scatter(int32_t count, const int32_t *__restrict__ rp,
                                                         const int32_t *__restrict__ rows,
                                                         const int32_t *__restrict__ col,
                                                         const V *__restrict__ val,
                                                         const int64_t *__restrict__ sp,
                                                         const int32_t *__restrict__ soff,
                                                         int32_t *__restrict__ col_out,
                                                         V *__restrict__ val_out) {
  const int64_t slots = (int64_t(count) + kSlice - 1) / kSlice * kSlice;
  for (int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x; p < slots;
       p += int64_t(gridDim.x) * kBlock) {
    const int64_t s = p / kSlice;
    const int32_t l = int32_t(p % kSlice);
    const int64_t raw = sp[s];
    const int64_t base = slice_base(raw);
    const int32_t w = int32_t((slice_base(sp[s + 1]) - base) / kSlice);
    int32_t b = 0, len = 0, i = 0;
    if (p < count) {
      i = rows ? rows[p] : int32_t(p);
      b = rp[i];
      len = min(rp[i + 1] - b, w);
      if (len < 0) len = 0;
    }
    if (raw & kOffsetSlice) {
      const int64_t k = base >> 6;
      int32_t e = 0;
      for (int32_t j = 0; j < w; ++j) {
        const bool here = e < len && col[b + e] - i == soff[k + j];
        val_out[value_slot<V>(base, w, j, l)] = here ? val[b + e] : V(0.0f);
        e += here;
      }
      continue;
    }
    for (int32_t j = 0; j < w; ++j) {
      if (col_out) col_out[sell_slot(base, w, j, l)] = j < len ? col[b + j] : -1;
      val_out[value_slot<V>(base, w, j, l)] = j < len ? val[b + j] : V(0.0f);
    }
  }
}

}  // namespace its
