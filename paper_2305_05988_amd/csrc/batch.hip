// C ABI of the batched solve (include/itsolve.h): many independent
// variable-coefficient diffusion systems with several right-hand sides,
// FP64 CG on each (system, right-hand side), advanced together by one HIP
// graph of m iterations that is replayed until every (system, rhs) stops.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "batch.hpp"
#include "host.hpp"

using namespace its;

#define BHIP(expr)                                                                        \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return its_fail(ITS_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct its_batch {
  int32_t nsys = 0, nrhs = 0;
  int64_t ncell = 0;
  std::vector<BatchSys> sys;
  BatchSys *d_sys = nullptr;
  double *coef = nullptr;
  // work items of the update passes (tiles per item) and bricks of the SpMV
  // pass (planes per brick); 0 until the autotuner chooses at the next solve
  int32_t chunk = 0;
  std::vector<BatchItem> items;
  BatchItem *d_items = nullptr;
  int32_t item_cap = 0;
  int32_t zb = 0;
  std::vector<BatchBrick> bricks;
  BatchBrick *d_bricks = nullptr;
  int32_t brick_cap = 0;
  double tune_ms = 0.0;
  // the solve's own stream (graphs cannot be captured on the legacy stream)
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  // graph of m iterations, cached for one set of arguments
  hipGraphExec_t gexec = nullptr;
  std::vector<uintptr_t> gkey;
  int32_t *h_count = nullptr;  // pinned: items still running
};

namespace {

constexpr int kTuneTiles[] = {4, 8, 16, 32, 64};
constexpr int kTunePlanes[] = {4, 8, 16, 32, 64};

int cells_per_tile(int R) { return kBlock / R; }

void brick_shape(int R, int &tx, int &ty) {
  switch (R) {
    case 1: tx = BrickShape<1>::TX; ty = BrickShape<1>::TY; break;
    case 2: tx = BrickShape<2>::TX; ty = BrickShape<2>::TY; break;
    case 4: tx = BrickShape<4>::TX; ty = BrickShape<4>::TY; break;
    default: tx = BrickShape<8>::TX; ty = BrickShape<8>::TY; break;
  }
}

int64_t count_bricks(const its_batch *B, int zb) {
  int tx, ty;
  brick_shape(B->nrhs, tx, ty);
  int64_t c = 0;
  for (const BatchSys &sy : B->sys)
    c += int64_t((sy.nx + tx - 1) / tx) * ((sy.ny + ty - 1) / ty) * ((sy.nz + zb - 1) / zb);
  return c;
}

// Bricks of each system: x tiles fastest, then y tiles, then z runs of zb
// planes, so neighbouring bricks of a plane are dealt side by side.
void build_bricks(its_batch *B, int zb) {
  int tx, ty;
  brick_shape(B->nrhs, tx, ty);
  B->bricks.clear();
  for (int32_t s = 0; s < B->nsys; ++s) {
    BatchSys &sy = B->sys[size_t(s)];
    sy.brick0 = int32_t(B->bricks.size());
    for (int32_t z0 = 0; z0 < sy.nz; z0 += zb)
      for (int32_t y0 = 0; y0 < sy.ny; y0 += ty)
        for (int32_t x0 = 0; x0 < sy.nx; x0 += tx) {
          BatchBrick br{};
          br.sys = s;
          br.x0 = x0;
          br.y0 = y0;
          br.z0 = z0;
          br.z1 = std::min(sy.nz, z0 + zb);
          B->bricks.push_back(br);
        }
    sy.brick1 = int32_t(B->bricks.size());
  }
}

void build_items(its_batch *B, int chunk) {
  B->items.clear();
  for (int32_t s = 0; s < B->nsys; ++s) {
    BatchSys &sy = B->sys[size_t(s)];
    sy.item0 = int32_t(B->items.size());
    for (int32_t t = 0; t < sy.tiles; t += chunk) {
      BatchItem it{};
      it.sys = s;
      it.t0 = t;
      it.t1 = std::min(sy.tiles, t + chunk);
      B->items.push_back(it);
    }
    sy.item1 = int32_t(B->items.size());
  }
}

its_status upload_schedule(its_batch *B, hipStream_t s) {
  BHIP(hipMemcpyAsync(B->d_items, B->items.data(), B->items.size() * sizeof(BatchItem),
                      hipMemcpyHostToDevice, s));
  if (!B->bricks.empty())
    BHIP(hipMemcpyAsync(B->d_bricks, B->bricks.data(), B->bricks.size() * sizeof(BatchBrick),
                        hipMemcpyHostToDevice, s));
  BHIP(hipMemcpyAsync(B->d_sys, B->sys.data(), B->sys.size() * sizeof(BatchSys), hipMemcpyHostToDevice, s));
  BHIP(hipStreamSynchronize(s));
  return ITS_OK;
}

int pass_grid(int nitems) {
  int g = std::min(nitems, kMaxGrid);
  if (g >= 64) g -= g % kXcds;
  return std::max(g, 1);
}

// Workspace: [BatchCg S R][sys_run S][sys_base 2S][nact 2][act cap][act1 cap1]
// [partials cap R 2 DD][brick partials cap1 R 2 DD][pairs][q]
struct BatchWs {
  size_t st, run, base, nact, act, act1, part, part1, pairs, q, total;
};

BatchWs batch_layout(const its_batch *B) {
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  BatchWs L{};
  const size_t S = size_t(B->nsys), R = size_t(B->nrhs);
  L.st = 0;
  L.run = up(S * R * sizeof(BatchCg));
  L.base = L.run + up(S * sizeof(int32_t));
  L.nact = L.base + up(2 * S * sizeof(int32_t));
  L.act = L.nact + 256;
  L.act1 = L.act + up(size_t(B->item_cap) * sizeof(BatchAct));
  L.part = L.act1 + up(size_t(B->brick_cap) * sizeof(BatchActB));
  L.part1 = L.part + up(size_t(B->item_cap) * R * 2 * sizeof(DD));
  L.pairs = L.part1 + up(size_t(B->brick_cap) * R * 2 * sizeof(DD));
  L.q = L.pairs + up(size_t(B->ncell) * R * 16);
  L.total = L.q + up(size_t(B->ncell) * R * 8);
  return L;
}

BatchView view_of(const its_batch *B, char *ws, const BatchWs &L) {
  BatchView V{};
  V.nsys = B->nsys;
  V.nrhs = B->nrhs;
  V.cells = cells_per_tile(B->nrhs);
  V.nitems = int32_t(B->items.size());
  V.ncell = B->ncell;
  V.sys = B->d_sys;
  V.items = B->d_items;
  V.coef = B->coef;
  V.st = reinterpret_cast<BatchCg *>(ws + L.st);
  V.sys_run = reinterpret_cast<int32_t *>(ws + L.run);
  V.sys_base = reinterpret_cast<int32_t *>(ws + L.base);
  V.nact = reinterpret_cast<int32_t *>(ws + L.nact);
  V.act = reinterpret_cast<BatchAct *>(ws + L.act);
  V.act1 = reinterpret_cast<BatchActB *>(ws + L.act1);
  V.bricks = B->d_bricks;
  V.part = reinterpret_cast<DD *>(ws + L.part);
  V.part1 = reinterpret_cast<DD *>(ws + L.part1);
  return V;
}

// The running systems' items and bricks, gathered for the two passes.
void launch_compact(hipStream_t s, const BatchView &V) {
  hipLaunchKernelGGL(k_batch_scan, dim3(1), dim3(kBlock), 0, s, V);
  hipLaunchKernelGGL(k_batch_compact, dim3(V.nsys), dim3(kBlock), 0, s, V);
}

// The two passes, instantiated per right-hand-side count.
void launch_pass1(int G, hipStream_t s, const BatchView &V, const double2_t *pairs, double *q) {
  switch (V.nrhs) {
    case 1: hipLaunchKernelGGL(k_batch_pass1<1>, dim3(G), dim3(kBlock), 0, s, V, pairs, q); break;
    case 2: hipLaunchKernelGGL(k_batch_pass1<2>, dim3(G), dim3(kBlock), 0, s, V, pairs, q); break;
    case 4: hipLaunchKernelGGL(k_batch_pass1<4>, dim3(G), dim3(kBlock), 0, s, V, pairs, q); break;
    default: hipLaunchKernelGGL(k_batch_pass1<8>, dim3(G), dim3(kBlock), 0, s, V, pairs, q); break;
  }
}

void launch_pass2(int G, hipStream_t s, const BatchView &V, double *x, double2_t *pairs, const double *q) {
  switch (V.nrhs) {
    case 1: hipLaunchKernelGGL(k_batch_pass2<1>, dim3(G), dim3(kBlock), 0, s, V, x, pairs, q); break;
    case 2: hipLaunchKernelGGL(k_batch_pass2<2>, dim3(G), dim3(kBlock), 0, s, V, x, pairs, q); break;
    case 4: hipLaunchKernelGGL(k_batch_pass2<4>, dim3(G), dim3(kBlock), 0, s, V, x, pairs, q); break;
    default: hipLaunchKernelGGL(k_batch_pass2<8>, dim3(G), dim3(kBlock), 0, s, V, x, pairs, q); break;
  }
}

__global__ void k_batch_fill_run(int32_t *run, int n) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) run[i] = 1;
}

// State for timing the passes: every (system, rhs) running at an even
// iteration past the first, alpha = beta = 0, so the update pass reads and
// writes the pairs and q but leaves x alone.
__global__ void k_batch_tune_state(BatchView V) {
  const int64_t m = int64_t(V.nsys) * V.nrhs;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < m; i += int64_t(gridDim.x) * kBlock) {
    BatchCg &c = V.st[i];
    c.k = 2;
    c.flag = kRunning;
    c.alpha = c.beta = c.alpha_x = 0.0;
  }
}

// Autotuner, run at the first solve for whichever of the two lengths is not
// fixed.  The two passes of an iteration depend on one length each (the SpMV
// pass on the bricks' planes, the update pass on the items' tiles), so the
// best pair is the pair of per-pass bests: each candidate is timed over three
// launches of its pass and the fastest kept.  The SpMV pass writes q and the
// brick partials only; the update pass, at the state above, writes the pairs
// and the item partials only; the prologue of the solve overwrites all four.
its_status autotune(its_batch *B, char *ws, const BatchWs &L, double *x) {
  hipStream_t s = B->stream;
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    if (a) (void)hipEventDestroy(a);
    return its_fail(ITS_E_HIP, "autotune events");
  }
  const auto t0 = std::chrono::steady_clock::now();
  its_status rs = ITS_OK;
  auto *pairs = reinterpret_cast<double2_t *>(ws + L.pairs);
  auto *q = reinterpret_cast<double *>(ws + L.q);
  // times three launches after one warm-up; negative on failure
  auto timed = [&](auto &&launch) -> float {
    launch();
    (void)hipEventRecord(a, s);
    for (int rep = 0; rep < 3; ++rep) launch();
    (void)hipEventRecord(b, s);
    if (hipEventSynchronize(b) != hipSuccess) return -1.f;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    return ms;
  };
  auto prepare = [&](const BatchView &V) {
    hipLaunchKernelGGL(k_batch_tune_state, dim3(std::min(1024, (B->nsys * B->nrhs + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, V);
    hipLaunchKernelGGL(k_batch_fill_run, dim3(std::max(1, (B->nsys + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       V.sys_run, B->nsys);
    launch_compact(s, V);
  };
  const bool tune_planes = B->zb == 0, tune_tiles = B->chunk == 0;
  if (tune_planes) {
    float best = 1e30f;
    int best_zb = kTunePlanes[0];
    for (int zb : kTunePlanes) {
      build_bricks(B, zb);
      if (int64_t(B->bricks.size()) > B->brick_cap) continue;
      if ((rs = upload_schedule(B, s)) != ITS_OK) break;
      const BatchView V = view_of(B, ws, L);
      const int G = pass_grid(int32_t(B->bricks.size()));
      prepare(V);
      const float ms = timed([&] { launch_pass1(G, s, V, pairs, q); });
      if (ms < 0.f) {
        rs = its_fail(ITS_E_HIP, "autotune timing");
        break;
      }
      if (ms < best) {
        best = ms;
        best_zb = zb;
      }
    }
    if (rs == ITS_OK) {
      B->zb = best_zb;
      build_bricks(B, best_zb);
    }
  }
  if (rs == ITS_OK && tune_tiles) {
    float best = 1e30f;
    int best_chunk = kTuneTiles[0];
    for (int chunk : kTuneTiles) {
      build_items(B, chunk);
      if ((rs = upload_schedule(B, s)) != ITS_OK) break;
      const BatchView V = view_of(B, ws, L);
      const int G = pass_grid(V.nitems);
      prepare(V);
      const float ms = timed([&] { launch_pass2(G, s, V, x, pairs, q); });
      if (ms < 0.f) {
        rs = its_fail(ITS_E_HIP, "autotune timing");
        break;
      }
      if (ms < best) {
        best = ms;
        best_chunk = chunk;
      }
    }
    if (rs == ITS_OK) {
      B->chunk = best_chunk;
      build_items(B, best_chunk);
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rs != ITS_OK) return rs;
  B->tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return upload_schedule(B, s);
}

void drop_graph(its_batch *B) {
  if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
  B->gexec = nullptr;
  B->gkey.clear();
}

}  // namespace

extern "C" {

its_status its_batch_create(int32_t nsys, const int32_t *dims, const double *k, int32_t nrhs,
                            void *stream, its_batch **out) {
  if (!out) return its_fail(ITS_E_INVALID, "out is null");
  *out = nullptr;
  if (nsys < 1 || !dims || !k) return its_fail(ITS_E_INVALID, "need at least one system, dims and k");
  if (nrhs != 1 && nrhs != 2 && nrhs != 4 && nrhs != 8)
    return its_fail(ITS_E_UNSUPPORTED, "nrhs must be 1, 2, 4 or 8");
  its_batch *B = new (std::nothrow) its_batch();
  if (!B) return its_fail(ITS_E_INVALID, "out of host memory");
  B->nsys = nsys;
  B->nrhs = nrhs;
  const int cpt = cells_per_tile(nrhs);
  int64_t off = 0, max_tiles_items = 0;
  for (int32_t s = 0; s < nsys; ++s) {
    const int32_t nx = dims[3 * s], ny = dims[3 * s + 1], nz = dims[3 * s + 2];
    if (nx < 1 || ny < 1 || nz < 1) {
      delete B;
      return its_fail(ITS_E_INVALID, "system " + std::to_string(s) + " has an empty grid");
    }
    if (int64_t(nx) * ny >= (int64_t(1) << 31)) {
      delete B;
      return its_fail(ITS_E_UNSUPPORTED, "system " + std::to_string(s) + " has 2^31 or more cells per plane");
    }
    BatchSys sy{};
    sy.off = off;
    sy.nx = nx;
    sy.ny = ny;
    sy.nz = nz;
    const int64_t n = int64_t(nx) * ny * nz;
    sy.tiles = int32_t((n + cpt - 1) / cpt);
    max_tiles_items += sy.tiles;
    off += n;
    B->sys.push_back(sy);
  }
  B->ncell = off;
  if (off * nrhs >= (int64_t(1) << 40)) {
    delete B;
    return its_fail(ITS_E_UNSUPPORTED, "batch too large");
  }
  const int64_t max_bricks = count_bricks(B, 1);
  if (max_tiles_items >= (int64_t(1) << 30) || max_bricks >= (int64_t(1) << 30)) {
    delete B;
    return its_fail(ITS_E_UNSUPPORTED, "batch too large");
  }
  B->item_cap = int32_t(max_tiles_items);  // items of one tile each at most
  B->brick_cap = int32_t(max_bricks);      // bricks of one plane each at most
  its_status rs = ITS_OK;
  do {
    if (hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&B->ev, hipEventDisableTiming) != hipSuccess) {
      rs = its_fail(ITS_E_HIP, "stream creation failed");
      break;
    }
    void *p = nullptr;
    if (hipHostMalloc(&p, sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
      rs = its_fail(ITS_E_HIP, "hipHostMalloc failed");
      break;
    }
    B->h_count = static_cast<int32_t *>(p);
    if (hipMalloc(&B->d_sys, sizeof(BatchSys) * size_t(nsys)) != hipSuccess ||
        hipMalloc(&B->d_items, sizeof(BatchItem) * size_t(B->item_cap)) != hipSuccess ||
        hipMalloc(&B->d_bricks, sizeof(BatchBrick) * size_t(B->brick_cap)) != hipSuccess ||
        hipMalloc(&B->coef, sizeof(double) * kCoefs * size_t(off)) != hipSuccess) {
      rs = its_fail(ITS_E_HIP, "device allocation failed");
      break;
    }
    build_items(B, kTuneTiles[0]);    // both replaced by the autotuner's choice
    build_bricks(B, kTunePlanes[0]);
    // the coefficients are formed on the caller's stream, after k is ready
    hipStream_t cs = reinterpret_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(B->d_sys, B->sys.data(), sizeof(BatchSys) * size_t(nsys), hipMemcpyHostToDevice, cs) != hipSuccess) {
      rs = its_fail(ITS_E_HIP, "upload failed");
      break;
    }
    BatchView V{};
    V.nsys = nsys;
    V.nrhs = nrhs;
    V.ncell = off;
    V.sys = B->d_sys;
    hipLaunchKernelGGL(k_batch_coef, dim3(std::min(nsys, 65536)), dim3(kBlock), 0, cs, V, k, B->coef);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(cs) != hipSuccess) {
      rs = its_fail(ITS_E_HIP, "coefficient kernel failed");
      break;
    }
  } while (0);
  if (rs != ITS_OK) {
    its_batch_destroy(B);
    return rs;
  }
  *out = B;
  return ITS_OK;
}

its_status its_batch_destroy(its_batch *B) {
  if (!B) return ITS_OK;
  drop_graph(B);
  if (B->d_sys) (void)hipFree(B->d_sys);
  if (B->d_items) (void)hipFree(B->d_items);
  if (B->d_bricks) (void)hipFree(B->d_bricks);
  if (B->coef) (void)hipFree(B->coef);
  if (B->h_count) (void)hipHostFree(B->h_count);
  if (B->ev) (void)hipEventDestroy(B->ev);
  if (B->stream) (void)hipStreamDestroy(B->stream);
  delete B;
  return ITS_OK;
}

int64_t its_batch_cells(const its_batch *B) { return B ? B->ncell : -1; }

size_t its_batch_workspace_size(const its_batch *B) { return B ? batch_layout(B).total : 0; }

its_status its_batch_set_schedule(its_batch *B, int32_t tiles_per_item, int32_t planes_per_brick) {
  if (!B) return its_fail(ITS_E_INVALID, "null batch");
  if (tiles_per_item < 0 || planes_per_brick < 0)
    return its_fail(ITS_E_INVALID, "tiles_per_item and planes_per_brick must be >= 0");
  drop_graph(B);
  B->chunk = tiles_per_item;
  B->zb = planes_per_brick;
  B->tune_ms = 0.0;
  if (tiles_per_item > 0) build_items(B, tiles_per_item);
  if (planes_per_brick > 0) build_bricks(B, planes_per_brick);
  // the device copy of the systems carries both ranges; autotuned lists are
  // uploaded by the tuner
  return upload_schedule(B, B->stream);
}

its_status its_batch_solve(its_batch *B, const its_options *o, const double *b, double *x,
                           void *workspace, size_t ws_bytes, void *stream, its_batch_result *res,
                           int64_t *iters, int32_t *status) {
  if (!B || !o || !b || !x || !res) return its_fail(ITS_E_INVALID, "null argument");
  if (o->method != ITS_CG || o->inner_dtype != ITS_F64 || o->transpose != 0)
    return its_fail(ITS_E_UNSUPPORTED, "the batched solve runs FP64 CG");
  if (!(o->rtol >= 0.0) || !std::isfinite(o->rtol) || o->max_iter < 0 || o->check_every < 0)
    return its_fail(ITS_E_INVALID, "bad options");
  if (b == x) return its_fail(ITS_E_INVALID, "b and x alias");
  const BatchWs L = batch_layout(B);
  if (!workspace || ws_bytes < L.total) return its_fail(ITS_E_WORKSPACE, "workspace missing or too small");
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return its_fail(ITS_E_WORKSPACE, "workspace must be 256-byte aligned");
  std::memset(res, 0, sizeof(*res));
  char *ws = static_cast<char *>(workspace);
  hipStream_t cs = reinterpret_cast<hipStream_t>(stream), s = B->stream;
  const auto t_start = std::chrono::steady_clock::now();
  // order the solve after the caller's work
  BHIP(hipEventRecord(B->ev, cs));
  BHIP(hipStreamWaitEvent(s, B->ev, 0));
  if (B->zb == 0 || B->chunk == 0) {
    its_status rs = autotune(B, ws, L, x);
    if (rs != ITS_OK) return rs;
  }
  BatchView V = view_of(B, ws, L);
  const int G = pass_grid(V.nitems), G1 = pass_grid(int32_t(B->bricks.size()));
  auto *pairs = reinterpret_cast<double2_t *>(ws + L.pairs);
  auto *q = reinterpret_cast<double *>(ws + L.q);
  const int S = B->nsys, R = B->nrhs;
  // prologue: r = b - A x0, r.r, b.b; thresholds on the host, as the
  // single-system solve computes them
  hipLaunchKernelGGL(k_batch_residual, dim3(G), dim3(kBlock), 0, s, V, b, (const double *)x, pairs);
  hipLaunchKernelGGL(k_batch_sums, dim3(S), dim3(kBlock), 0, s, V);
  BHIP(hipGetLastError());
  std::vector<BatchCg> hst(size_t(S) * R);
  BHIP(hipMemcpyAsync(hst.data(), V.st, hst.size() * sizeof(BatchCg), hipMemcpyDeviceToHost, s));
  BHIP(hipStreamSynchronize(s));
  for (auto &c : hst) {
    if (!std::isfinite(c.bb)) return its_fail(ITS_E_INVALID, "b contains NaN or Inf");
    const double t = o->rtol * std::sqrt(c.bb);
    c.thr2 = t * t;
  }
  BHIP(hipMemcpyAsync(V.st, hst.data(), hst.size() * sizeof(BatchCg), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_batch_begin, dim3(S), dim3(kBlock), 0, s, V, (int64_t)o->max_iter);
  hipLaunchKernelGGL(k_batch_zero, dim3(G), dim3(kBlock), 0, s, V, x);
  launch_compact(s, V);
  BHIP(hipGetLastError());
  BHIP(hipMemcpyAsync(B->h_count, V.nact, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  BHIP(hipStreamSynchronize(s));
  // m = 64 iterations per replay: about ten host polls per solve (the
  // replays cost the same with 16)
  const int m = o->check_every > 0 ? o->check_every : 64;
  int64_t replays = 0;
  if (*B->h_count > 0) {
    // one graph: m iterations (the four CG kernels, then the gathering of
    // the running systems' items, whose count the host polls)
    const std::vector<uintptr_t> key = {reinterpret_cast<uintptr_t>(b), reinterpret_cast<uintptr_t>(x),
                                        reinterpret_cast<uintptr_t>(ws), uintptr_t(m),
                                        uintptr_t(o->max_iter), uintptr_t(B->chunk),
                                        uintptr_t(B->zb)};
    if (!B->gexec || B->gkey != key) {
      drop_graph(B);
      hipGraph_t g = nullptr;
      BHIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      for (int it = 0; it < m; ++it) {
        launch_pass1(G1, s, V, pairs, q);
        hipLaunchKernelGGL(k_batch_fin1, dim3(S), dim3(kBlock), 0, s, V);
        launch_pass2(G, s, V, x, pairs, q);
        hipLaunchKernelGGL(k_batch_fin2, dim3(S), dim3(kBlock), 0, s, V, (int64_t)o->max_iter);
        launch_compact(s, V);
      }
      hipError_t ce = hipStreamEndCapture(s, &g);
      if (ce != hipSuccess) return its_fail(ITS_E_HIP, std::string("graph capture: ") + hipGetErrorString(ce));
      ce = hipGraphInstantiate(&B->gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ce != hipSuccess) {
        B->gexec = nullptr;
        return its_fail(ITS_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(ce));
      }
      B->gkey = key;
    }
    // every (system, rhs) stops within max_iter iterations
    const int64_t max_replays = o->max_iter / m + 2;
    for (;;) {
      BHIP(hipGraphLaunch(B->gexec, s));
      ++replays;
      BHIP(hipMemcpyAsync(B->h_count, V.nact, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      BHIP(hipStreamSynchronize(s));
      if (*B->h_count == 0) break;
      if (replays > max_replays) return its_fail(ITS_E_HIP, "batched solve still running after max_iter");
    }
  }
  hipLaunchKernelGGL(k_batch_flush_x, dim3(S, kFlushParts), dim3(kBlock), 0, s, V, x, (const double2_t *)pairs);
  BHIP(hipGetLastError());
  BHIP(hipMemcpyAsync(hst.data(), V.st, hst.size() * sizeof(BatchCg), hipMemcpyDeviceToHost, s));
  BHIP(hipStreamSynchronize(s));
  int32_t worst = ITS_OK;
  int64_t kmax = 0;
  for (size_t i = 0; i < hst.size(); ++i) {
    const int32_t st = hst[i].flag == kConverged ? ITS_OK : (hst[i].flag == kMaxIter ? ITS_NOT_CONVERGED : ITS_BREAKDOWN);
    if (iters) iters[i] = hst[i].k;
    if (status) status[i] = st;
    if (st == ITS_BREAKDOWN || (st == ITS_NOT_CONVERGED && worst == ITS_OK)) worst = st;
    kmax = std::max<int64_t>(kmax, hst[i].k);
  }
  res->status = worst;
  res->tiles_per_item = B->chunk;
  res->planes_per_brick = B->zb;
  res->graph_iters = m;
  res->max_iters = kmax;
  res->replays = replays;
  res->tune_ms = B->tune_ms;
  res->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  return static_cast<its_status>(worst);
}

}  // extern "C"
