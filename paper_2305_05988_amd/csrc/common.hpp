// Device building blocks shared by every kernel of the library: error-free
// floating-point transformations, the deterministic two-level dot-product
// reduction, the XCD-aware tile schedule and the device-resident solver
// state.  gfx950 (CDNA4): 64-wide wavefronts, 256 CUs in 8 XCDs.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace its {

constexpr int kBlock = 256;             // threads per block: 4 wave64
constexpr int kWaves = kBlock / 64;
constexpr int kGroup = 256;             // blocks per first-level reduction group
constexpr int kMaxGrid = kGroup * kGroup;  // 65536 blocks: one 256-row tile each up to 16.7M rows
constexpr int kMaxDots = 2;             // dot products reduced per kernel
constexpr int kXcds = 8;                // MI355X: 8 XCDs, blocks dealt round-robin

// Solver status flags kept on the device.
enum : int32_t { kRunning = 0, kConverged = 1, kMaxIter = 2, kBreakdown = 3 };

// Device-resident scalars of one solve.  Kernels read them at entry and the
// finishing kernel of each reduction updates them; the host reads a snapshot
// only when it polls.
struct alignas(256) State {
  int32_t flag;       // kRunning / kConverged / kMaxIter / kBreakdown
  int32_t restart;    // BiCGStab: the next A p pass starts from a restart
  int64_t k;          // completed iterations
  int32_t restarts;   // BiCGStab restarts so far
  int32_t pad;
  uint32_t counter[8];// flags and counters of the setup checks (counter[7]: rows without a diagonal)
  double rho;         // r.r of the current iterate (CG); beta = r.r (BiCGStab)
  double alpha;       // step length
  double beta;        // CG: direction coefficient; BiCGStab: p coefficient
  double omega;       // BiCGStab stabilising step
  double alpha_n;     // BiCGStab r.r'
  double alpha_d;     // BiCGStab (A p).r'
  double ts, tt;      // BiCGStab (A s).s and (A s).(A s)
  double gamma;       // CG-NB x-update coefficient
  double alpha_x;     // CG: step of the x update deferred from an even iteration
  double thr2;        // stopping threshold on the squared residual norm
  int64_t max_iter;   // iteration cap
  double dot[4];      // scratch results (dot products, residual norms)
};

// ---------------------------------------------------------------- floating point
// Written-out roundings: the library is compiled with -ffp-contract=off, so
// a*b+c is two roundings and fma() is one, exactly as written.

struct DD {  // unevaluated sum hi + lo, |lo| <= ulp(hi)/2 when normalised
  double hi, lo;
};

__device__ __forceinline__ DD two_sum(double a, double b) {
  const double s = a + b;
  const double bp = s - a;
  const double e = (a - (s - bp)) + (b - bp);
  return {s, e};
}

__device__ __forceinline__ DD fast_two_sum(double a, double b) {  // |a| >= |b|
  const double s = a + b;
  return {s, b - (s - a)};
}

// Accurate double-double addition (error ~ 2^-104 relative to |a|+|b|).
__device__ __forceinline__ DD dd_add(DD a, DD b) {
  DD s = two_sum(a.hi, b.hi);
  const DD t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}

// Per-thread compensated dot accumulator (Ogita-Rump-Oishi Dot2): the
// product error comes from fma, the sum error from two_sum; both are summed
// into c.  A float*float product is exact in double, so its error term is 0.
struct Dot2 {
  double s = 0.0, c = 0.0;
  __device__ __forceinline__ void add(double x, double y) {
    const double p = x * y;
    const double e = fma(x, y, -p);
    const DD t = two_sum(s, p);
    s = t.hi;
    c += t.lo + e;
  }
  // (s, c) as an unevaluated pair: the reductions add such pairs with
  // dd_cascade / dd_add, which need no normalised input
  __device__ __forceinline__ DD get() const { return {s, c}; }
};

__device__ __forceinline__ double dd_round(DD v) { return v.hi + v.lo; }

__device__ __forceinline__ bool finite(double v) { return __builtin_isfinite(v); }

// Two-element vectors for interleaved pairs (one 16- or 8-byte access).
typedef double double2_t __attribute__((ext_vector_type(2)));
typedef float float2_t __attribute__((ext_vector_type(2)));
typedef float float4_t __attribute__((ext_vector_type(4)));
template <class T> struct Pair;
template <> struct Pair<double> { using type = double2_t; };
template <> struct Pair<float> { using type = float2_t; };

// Streaming (non-temporal) accesses for data used once per pass: the matrix
// arrays and the vectors a pass reads or writes only for its own rows.  They
// keep L2 for the vector entries that neighbouring rows gather, and leave
// little dirty data behind.
template <class T>
__device__ __forceinline__ T ld_nt(const T *p) {
  return __builtin_nontemporal_load(p);
}
__device__ __forceinline__ __half ld_nt(const __half *p) {
  const unsigned short b = __builtin_nontemporal_load(reinterpret_cast<const unsigned short *>(p));
  return __builtin_bit_cast(__half, b);
}
template <class T>
__device__ __forceinline__ void st_nt(T *p, T v) {
  __builtin_nontemporal_store(v, p);
}

// The pairs an update pass writes for the next SpMV pass to gather: with an
// operator that gathers them entry by entry (the CSR forms) the stores
// allocate, so the start of the next pass finds the lines the update pass
// wrote last still cached (256^3 CG +2.3 %, BiCGStab +4.5 %); the matrix-free
// brick marches, which stage each plane once in LDS, run faster when the
// update pass streams them past the caches (measured).
template <class Op> struct GathersPairs : std::true_type {};

template <bool Keep, class P>
__device__ __forceinline__ void st_pairs(P *p, P v) {
  if constexpr (Keep)
    *p = v;
  else
    st_nt(p, v);
}

__device__ __forceinline__ double fmaT(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return fmaf(a, b, c); }

// --------------------------------------------------------------- tile schedule
// Rows are processed in tiles of kBlock rows, one row per thread.  With at
// least 64 blocks (a multiple of 8) the tiles are cut into 8 contiguous
// chunks and chunk x is served by the blocks that the hardware places on XCD
// x (block ids congruent to x mod 8), so the neighbour rows a stencil-like
// matrix gathers (+-1, +-nx, +-nx*ny) stay in one XCD's L2.
struct Sched {
  int64_t begin, end, stride;
};

// The block's place in that schedule.  A pass that runs backwards (rev)
// gives block b the place mirrored among its XCD's blocks, so the blocks
// dispatched first take the ends of the chunks and the pass ends at their
// starts, where the next pass begins; its block partials are stored at the
// place, so the reduction, and every bit of the result, is the forward
// pass's.
__device__ __forceinline__ int sched_place(bool rev) {
  const int G = gridDim.x, b = blockIdx.x;
  if (!rev) return b;
  if (G < 64 || (G % kXcds) != 0) return G - 1 - b;
  return (G / kXcds - 1 - b / kXcds) * kXcds + b % kXcds;
}

__device__ __forceinline__ Sched my_tiles(int64_t ntiles, bool rev = false) {
  const int G = gridDim.x;
  const int b = sched_place(rev);
  if (G < 64 || (G % kXcds) != 0) return {b, ntiles, G};
  const int x = b % kXcds, slot = b / kXcds, per = G / kXcds;
  const int64_t lo = ntiles * x / kXcds, hi = ntiles * (x + 1) / kXcds;
  return {lo + slot, hi, per};
}

// Element-wise walk: body(i) for the thread's row of each of its tiles.
template <class Body>
__device__ __forceinline__ void for_rows(int32_t n, Body &&body, bool rev = false) {
  const int64_t ntiles = (int64_t(n) + kBlock - 1) / kBlock;
  const Sched s = my_tiles(ntiles, rev);
  for (int64_t t = s.begin; t < s.end; t += s.stride) {
    const int64_t i = t * kBlock + threadIdx.x;
    if (i < n) body(int32_t(i));
  }
}

// Tile walk: body(r0, r1) for each of the block's tiles, called by every
// thread of the block (the body may synchronise the block).
template <class Body>
__device__ __forceinline__ void for_tiles(int32_t n, Body &&body, bool rev = false) {
  const int64_t ntiles = (int64_t(n) + kBlock - 1) / kBlock;
  const Sched s = my_tiles(ntiles, rev);
  for (int64_t t = s.begin; t < s.end; t += s.stride) {
    const int32_t r0 = int32_t(t * kBlock);
    const int32_t r1 = int32_t(min(int64_t(n), t * kBlock + kBlock));
    body(r0, r1);
  }
}

// --------------------------------------------------------------- reductions

// Cascaded sum of unevaluated pairs (the Sum2 step of Ogita-Rump-Oishi):
// the high parts are added error-free, their error joins the low parts.
// The result is the sum of the operands' values up to an error of about
// 2^-106 times the sum of their magnitudes, the accuracy class of Dot2
// itself, so a reduction of Dot2 partials through it keeps Dot2's bound; it
// costs 8 additions instead of dd_add's 20.
__device__ __forceinline__ DD dd_cascade(DD a, DD b) {
  const DD s = two_sum(a.hi, b.hi);
  return {s.hi, (a.lo + b.lo) + s.lo};
}

__device__ __forceinline__ DD wave_reduce(DD v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    DD o;
    o.hi = __shfl_xor(v.hi, off);
    o.lo = __shfl_xor(v.lo, off);
    v = dd_cascade(v, o);
  }
  return v;
}

// Reduces ND per-thread values over the block; the result is valid in
// thread 0.  Fixed order: butterfly within each wave, then waves 0..3.
template <int ND>
__device__ __forceinline__ void block_reduce(DD (&v)[ND]) {
  __shared__ DD sm[ND][kWaves];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int d = 0; d < ND; ++d) v[d] = wave_reduce(v[d]);
  if (lane == 0) {
#pragma unroll
    for (int d = 0; d < ND; ++d) sm[d][w] = v[d];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      DD t = sm[d][0];
      for (int j = 1; j < kWaves; ++j) t = dd_cascade(t, sm[d][j]);
      v[d] = t;
    }
  }
  __syncthreads();
}

// Scratch of the grid-wide reductions: first-level partials (one per block
// of a streaming pass) and second-level partials (one per group of kGroup
// first-level partials).
struct Reduce {
  DD p1[kMaxDots][kMaxGrid];
  DD p2[kMaxDots][kGroup];
  uint32_t count;  // unused; kept for layout stability
};

// First level: the block's partial, stored by thread 0 with plain stores.
// No fence and no atomic: the finishing kernels, launched after this one on
// the same stream, see the stores at the kernel boundary.
template <int ND>
__device__ __forceinline__ void block_partial(DD (&v)[ND], Reduce *R, bool rev = false) {
  block_reduce<ND>(v);
  if (threadIdx.x == 0) {
    const int at = sched_place(rev);
#pragma unroll
    for (int d = 0; d < ND; ++d) R->p1[d][at] = v[d];
  }
}

// The partials of a pass with G blocks are finished by one kernel when
// G <= kFinishOne, else by two: k_finish_group (block b sums first-level
// partials kGroup*b .. kGroup*b+kGroup-1 into p2[b]) and k_finish_final over
// the group sums.  The order of the additions is fixed at both levels, so
// the total does not depend on scheduling, and no fence is needed: each
// level reads what the previous kernel stored.  (An in-kernel "last block"
// needs agent-scope fences, which on this GPU write back and invalidate L2
// and cost more than the extra launch.)
constexpr int kFinishOne = 16 * kBlock;

template <int ND>
__global__ void __launch_bounds__(kBlock) k_finish_group(Reduce *R, int G) {
  DD v[ND];
  const int j = blockIdx.x * kGroup + int(threadIdx.x);
#pragma unroll
  for (int d = 0; d < ND; ++d) v[d] = (j < G) ? R->p1[d][j] : DD{0.0, 0.0};
  block_reduce<ND>(v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int d = 0; d < ND; ++d) R->p2[d][blockIdx.x] = v[d];
  }
}

// One block reduces `count` partials src[d][0 .. count) (thread t adds
// partials t, t + kBlock, ... in that order), then thread 0 applies Fin (the
// pass's scalar update) to the totals.  Every thread of the block calls it.
template <int ND, class Fin>
__device__ __forceinline__ void finish_in_block(const DD *const (&src)[ND], int count, Fin fin) {
  DD v[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) v[d] = DD{0.0, 0.0};
  // eight partials per thread in flight at a time, added in the same order
  constexpr int kU = 8;
  for (int j0 = int(threadIdx.x); j0 < count; j0 += kU * kBlock) {
    DD t[kU][ND];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int j = j0 + u * kBlock;
#pragma unroll
      for (int d = 0; d < ND; ++d) t[u][d] = j < count ? src[d][j] : DD{0.0, 0.0};
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
#pragma unroll
      for (int d = 0; d < ND; ++d) v[d] = dd_add(v[d], t[u][d]);
  }
  block_reduce<ND>(v);
  if (threadIdx.x == 0) fin(v);
}

// Single block: reduce `count` partials (from p1 if `level` is 1, else p2)
// and apply Fin to the totals.
template <int ND, class Fin>
__global__ void __launch_bounds__(kBlock) k_finish_final(Reduce *R, int count, int level, Fin fin) {
  if (!fin.active()) return;
  const DD *src[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) src[d] = level == 1 ? R->p1[d] : R->p2[d];
  finish_in_block<ND>(src, count, fin);
}

// Blocks of the first finishing level (0 when one kernel finishes).
inline int finish_grid(int G) { return G <= kFinishOne ? 0 : (G + kGroup - 1) / kGroup; }

// ------------------------------------------------------- grid barrier
// For the persistent solver kernels: every block of a cooperative launch
// (all co-resident) arrives at a barrier and waits for the others, with no
// kernel boundary in between.
//
// On gfx950 each XCD has its own L2, and the L2s are not kept coherent with
// each other: a block's stores reach the other XCDs only after its L2 is
// written back (an agent-scope release fence), and a block sees them only
// after invalidating its own stale lines (an agent-scope acquire fence).  A
// write-back walks the whole L2, so the barrier does one per XCD rather than
// one per block: the blocks of an XCD count themselves in a per-XCD counter
// (each first waits for its own stores to reach the L2); the last of them
// (the XCD's leader) releases the L2 and adds 1 to the global counter; when
// the global count shows every XCD, the leader acquires and publishes the
// barrier's epoch to its XCD, and every other block of the XCD acquires once
// it sees that epoch.  The XCD of a block is read from the hardware
// (XCC_ID); grid_init counts the blocks of each XCD once per launch.
//
// Between arrive and wait a block may do work that no other block reads
// before the next barrier (split phase); it is covered by the next barrier.
// Waits are bounded: a wait that has polled spin_limit times, or that finds
// the give-up word set, sets the word and returns false, and the kernel then
// leaves; every other block's wait then ends too, so the grid drains and the
// host reports the failure.  `extra` adds arrivals no launch can supply (a
// barrier that cannot complete, to force that path from the host).
//
// The sync block (unsigned long long words, zeroed before the launch; the
// counters sit on separate 64-byte lines):
//   [0] arrivals of XCD leaders   [8 + 8x] arrivals on XCD x   [136 + 8x]
//   released epoch of XCD x       [264 + x] blocks on XCD x    [280]
//   give-up word
constexpr int kMaxXcc = 16;
constexpr int kSyncWords = 288;

struct GridSync {
  unsigned long long *w;
  uint32_t extra;
  int64_t spin_limit;
};

struct SyncState {  // per block (thread 0's registers)
  uint64_t passed = 0;    // barriers completed
  uint32_t xcc = 0;       // this block's XCD
  uint64_t nx = 0;        // blocks on this XCD
  uint64_t nxcd = 0;      // XCDs holding blocks
  bool leader = false;    // last arrival of its XCD at the current barrier
};

__device__ __forceinline__ unsigned long long sync_load(unsigned long long *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Polls *p until it reaches t; false if the wait gave up.
__device__ __forceinline__ bool sync_spin(const GridSync &g, unsigned long long *p, unsigned long long t) {
  for (int64_t spins = 0;; ++spins) {
    if (sync_load(p) >= t) return true;
    if (spins >= g.spin_limit || sync_load(g.w + 280) != 0ull) {
      __hip_atomic_store(g.w + 280, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// Counts the blocks of each XCD; called once by every block at kernel start.
// Done when the per-XCD counts add up to the grid.
__device__ __forceinline__ bool grid_init(const GridSync &g, SyncState &ss) {
  __shared__ int ok;
  if (threadIdx.x == 0) {
    // HW_REG_XCC_ID (hardware register 20), bits [3:0]
    ss.xcc = __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & uint32_t(kMaxXcc - 1);
    atomicAdd(g.w + 264 + ss.xcc, 1ull);
    int good = 1;
    for (int64_t spins = 0;; ++spins) {
      unsigned long long total = 0, xcds = 0;
      for (int x = 0; x < kMaxXcc; ++x) {
        const unsigned long long c = sync_load(g.w + 264 + x);
        total += c;
        xcds += c != 0ull;
      }
      if (total == gridDim.x) {
        ss.nx = sync_load(g.w + 264 + ss.xcc);
        ss.nxcd = xcds;
        break;
      }
      if (spins >= g.spin_limit || sync_load(g.w + 280) != 0ull) {
        __hip_atomic_store(g.w + 280, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        good = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    ok = good;
  }
  __syncthreads();
  return ok != 0;
}

__device__ __forceinline__ void grid_arrive(const GridSync &g, SyncState &ss) {
  __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have reached the L2
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long e = ss.passed + 1;
    const unsigned long long mine = atomicAdd(g.w + 8 + 8 * ss.xcc, 1ull) + 1;
    ss.leader = mine == e * ss.nx;
    if (ss.leader) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // write the XCD's L2 back
      atomicAdd(g.w, 1ull);
    }
  }
}

__device__ __forceinline__ bool grid_wait(const GridSync &g, SyncState &ss) {
  __shared__ int ok;
  if (threadIdx.x == 0) {
    const unsigned long long e = ss.passed + 1;
    bool good;
    if (ss.leader) {
      good = sync_spin(g, g.w, e * ss.nxcd + g.extra);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __hip_atomic_store(g.w + 136 + 8 * ss.xcc, e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      good = sync_spin(g, g.w + 136 + 8 * ss.xcc, e);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    ok = good ? 1 : 0;
  }
  __syncthreads();
  ++ss.passed;
  return ok != 0;
}

// A block's partial of a persistent kernel's reduction: slot blockIdx.x of
// half `buf` (0 or 1) of the first-level partials.  Consecutive reductions
// alternate halves, so a block still reading one reduction's partials never
// sees them overwritten by a faster block's next reduction (that block must
// first pass a barrier this block has not reached).
template <int ND>
__device__ __forceinline__ void block_partial_half(DD (&v)[ND], Reduce *R, int buf) {
  block_reduce<ND>(v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int d = 0; d < ND; ++d) R->p1[d][buf * int(gridDim.x) + int(blockIdx.x)] = v[d];
  }
}

// Every block reduces all blocks' partials of half `buf` in the same fixed
// order, so every block computes the same totals and scalars.
template <int ND, class Fin>
__device__ __forceinline__ void finish_half(Reduce *R, int buf, Fin fin) {
  const DD *src[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) src[d] = R->p1[d] + buf * int(gridDim.x);
  finish_in_block<ND>(src, int(gridDim.x), fin);
  __syncthreads();
}

// ---------------------------------------------------------------- launch size

// One block per tile, except that up to four tiles share a block where that
// keeps the grid within one finishing level (mid-size vectors, where the
// second finishing kernel is a noticeable part of an iteration).
inline int grid_for(int64_t n, int max_blocks = kMaxGrid) {
  int64_t tiles = (n + kBlock - 1) / kBlock;
  if (tiles < 1) tiles = 1;
  if (tiles > kFinishOne && tiles <= 4 * kFinishOne) tiles = kFinishOne;
  int g = int(tiles < max_blocks ? tiles : max_blocks);
  if (g >= 64) g -= g % kXcds;
  return g;
}


}  // namespace its
