// Matrix operators.  Every operator applies row i as a fused multiply-add
// chain over the row's entries in ascending column order, starting from +0,
// with the vector entry x_j derived from what a fetch functor loads for
// column j -- so a kernel can apply A to a vector it forms on the fly
// (p = r + beta p, s = r - alpha v) without storing it first.  The SpMV of
// the paper (Sections 3.1-3.2) is the chain with x_j = x[j].
//
// Tiles: kernels walk the rows in tiles of kBlock rows, one row per thread,
// through tile_entries(r0, r1, smem, fetch, consume): for the thread's row it
// calls consume(j, a_ij, raw_j) for every entry in stored order, where
// raw_j = fetch(j) is the plain load of the vector entries column j needs
// (any type) and consume does the arithmetic, including forming x_j.
// Entries are handled in groups: all fetches of a group are issued before
// the first consume and are unconditional (slots without an entry fetch a
// valid stand-in column and are not consumed).  A fetch under a divergent
// branch, or arithmetic on its result before the group's other fetches,
// makes the compiler wait for each gather in turn; this way a thread keeps
// the group's gathers in flight together while the chain itself stays
// strictly sequential.
//
// Row sweep: the SpMV passes use rows(smem, load, value, body) instead.
// body(i, valid, entries, own) is called by every thread of the block for
// each row it owns (valid = false for slots past the last row); inside it,
// entries(consume) calls consume(j, a_ij, x_j) for the row's entries in
// stored order with x_j = value(load(j)), and own() returns x_i.  entries
// must be called once per body call, by every thread (the CSR operator
// synchronises the block inside it).  The CSR operators walk 1-D tiles; the
// stencil operator marches 2-D tiles along z with the vector staged in LDS.
#pragma once

#include "common.hpp"

namespace its {

constexpr int kGather = 8;

// An operator whose 1-D tile sweep (tiled_rows, tiled_own_rows) runs
// backwards (sched_place); only for the CSR operators, whose rows() is the
// tile sweep.  The direction is part of the type, so a forward kernel pays
// nothing for it.
template <class Op>
struct Backwards;

template <class Op>
__host__ __device__ constexpr bool rev_of(const Op &) {
  return false;
}
template <class Op>
__host__ __device__ constexpr bool rev_of(const Backwards<Op> &) {
  return true;
}

// rows() for the operators that walk 1-D tiles of kBlock rows.
template <class Op, class Load, class Value, class Body>
__device__ __forceinline__ void tiled_rows(const Op &A, typename Op::Smem &sm, Load &&load,
                                           Value &&value, Body &&body) {
  for_tiles(A.n, [&](int32_t r0, int32_t r1) {
    const int32_t i = r0 + int32_t(threadIdx.x);
    auto entries = [&](auto &&consume) {
      A.tile_entries(r0, r1, sm, load, [&](int32_t j, auto av, const auto &raw) {
        consume(j, av, value(raw));
      });
    };
    auto own = [&]() { return value(load(i)); };
    body(i, i < r1, entries, own);
  }, rev_of(A));
}

// The rows a thread owns in tiled_rows(), in the same order: body(i).  A
// pass that walks own_rows() after a rows() pass touches exactly the rows
// this thread handled there.
template <class Op, class Body>
__device__ __forceinline__ void tiled_own_rows(const Op &A, Body &&body) {
  for_rows(A.n, body, rev_of(A));
}

template <class Op>
struct Backwards : Op {
  template <class Load, class Value, class Body>
  __device__ __forceinline__ void rows(typename Op::Smem &sm, Load &&load, Value &&value,
                                       Body &&body) const {
    tiled_rows(*this, sm, load, value, body);
  }
  template <class Body>
  __device__ __forceinline__ void own_rows(Body &&body) const {
    tiled_own_rows(*this, body);
  }
};

__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ float widen(float v) { return v; }
__device__ __forceinline__ float widen(__half v) { return __half2float(v); }

}  // namespace its
