// Matrix operators.  Every operator applies row i as a fused multiply-add
// chain over the row's entries in ascending column order, starting from +0,
// with the vector entry x_j derived from what a fetch functor loads for
// column j -- so a kernel can apply A to a vector it forms on the fly
// (p = r + beta p, s = r - alpha v) without storing it first.  The SpMV of
// the paper (Sections 2.1-2.2) is the chain with x_j = x[j].
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
#pragma once

#include "common.hpp"

namespace its {

constexpr int kGather = 8;

__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ float widen(float v) { return v; }
__device__ __forceinline__ float widen(__half v) { return __half2float(v); }

}  // namespace its
