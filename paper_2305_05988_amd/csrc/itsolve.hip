// The C ABI of include/itsolve.h: argument validation, matrix handles,
// workspace layout and the host drivers of each method.  A driver launches
// the fused passes of m iterations back to back (m = check_every) and then
// reads the device State once; scalars never leave the device in between.
#include "../../include/itsolve.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <limits>
#include <mutex>
#include <type_traits>
#include <utility>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <string>
#include <vector>

#include "host.hpp"
#include "kernels.hpp"

using namespace its;

enum MatKind { kCsr = 0, kSten7 = 1, kSten27 = 2, kVar7 = 3 };

struct its_matrix {
  int kind = kCsr;
  int64_t n = 0, nnz = 0;
  const int32_t *rp = nullptr, *col = nullptr;
  const double *val = nullptr;
  const float *val32 = nullptr;
  const __half *val16 = nullptr;
  int32_t nx = 0, ny = 0, nz = 0;
  double coef[27] = {};
  const double *kcoef = nullptr;  // variable-coefficient diffusion: per-cell k (borrowed)
  // Gauss-Seidel colouring (CSR): rows grouped by colour, owned
  int32_t ncolors = 0;
  int32_t *color_rows = nullptr;
  std::vector<int32_t> color_off;
  int diag_state = 0;  // CSR: 0 unchecked, 1 every row has a nonzero diagonal, -1 not
  State *host_state = nullptr;  // pinned snapshot buffer for polling (two States and
                                // one more block for words read back after a
                                // persistent kernel)
  // Packed copy (its_csr_pack), owned: sliced ELLPACK of col/val and of the
  // low-precision values that were set when it was packed.
  int64_t *sp = nullptr;
  int32_t *scol = nullptr;  // null when every slice is an offset slice
  double *sval = nullptr;
  float *sval32 = nullptr;
  __half *sval16 = nullptr;
  int32_t *soff = nullptr;    // offset-slice descriptors
  uint64_t *smask = nullptr;
  int64_t sell_entries = 0;
  int64_t sell_col_slots = 0;  // slots of the slices that store columns
  int32_t sell_wmax = 0;       // widest slice
  double pack_fill = 0.0;  // max_fill of the last its_csr_pack (0: not packed)
  // Gauss-Seidel: each colour's rows packed the same way, in colour order
  struct ColorPack {
    int64_t *sp = nullptr;
    int32_t *col = nullptr;
    double *val = nullptr;
    int32_t *soff = nullptr;
    uint64_t *smask = nullptr;
  };
  std::vector<ColorPack> cpack;
  // A^T (its_csr_transpose): a CSR handle that owns its arrays (own_*)
  its_matrix *tr = nullptr;
  int32_t *own_rp = nullptr, *own_col = nullptr;
  double *own_val = nullptr;
  // the iteration loop captured as a HIP graph, cached for one argument set
  struct GraphCache {
    hipStream_t s = nullptr;  // own stream: the caller's may be the legacy stream
    hipEvent_t ev = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<uint64_t> key;
  } graph;
};

static void drop_graph(its_matrix *A) {
  if (A->graph.exec) (void)hipGraphExecDestroy(A->graph.exec);
  A->graph.exec = nullptr;
  A->graph.key.clear();
}

static void free_color_packs(its_matrix *A) {
  for (auto &c : A->cpack) {
    if (c.sp) (void)hipFree(c.sp);
    if (c.col) (void)hipFree(c.col);
    if (c.val) (void)hipFree(c.val);
    if (c.soff) (void)hipFree(c.soff);
    if (c.smask) (void)hipFree(c.smask);
  }
  A->cpack.clear();
}

static void drop_graph(its_matrix *A);
static void free_packed(its_matrix *A) {
  drop_graph(A);
  if (A->sp) (void)hipFree(A->sp);
  if (A->scol) (void)hipFree(A->scol);
  if (A->sval) (void)hipFree(A->sval);
  if (A->sval32) (void)hipFree(A->sval32);
  if (A->sval16) (void)hipFree(A->sval16);
  if (A->soff) (void)hipFree(A->soff);
  if (A->smask) (void)hipFree(A->smask);
  A->sp = nullptr;
  A->scol = nullptr;
  A->sval = nullptr;
  A->sval32 = nullptr;
  A->sval16 = nullptr;
  A->soff = nullptr;
  A->smask = nullptr;
  A->sell_entries = 0;
  A->sell_col_slots = 0;
  A->sell_wmax = 0;
  A->pack_fill = 0.0;
  free_color_packs(A);
}

// ------------------------------------------------------------------ errors

static thread_local std::string g_err;

its_status its_fail(its_status st, const std::string &msg) {
  g_err = msg;
  return st;
}
static its_status fail(its_status st, const std::string &msg) { return its_fail(st, msg); }

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(ITS_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));          \
  } while (0)

static hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

// ------------------------------------------------------------- profiling

namespace {

constexpr int kClassFinish = 6;  // profile class of the finishing reductions
constexpr int kClassOther = 7;   // setup and bookkeeping kernels

struct Prof {
  int every = 0;  // 0: off; k: time every k-th launch of each class
  its_result *res = nullptr;
  std::vector<hipEvent_t> ev;
  std::vector<int> cls;
  int64_t seen[ITS_MAX_KERNEL_CLASSES] = {};
  size_t used = 0;
  bool open = false;
  ~Prof() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
  void begin(int c, hipStream_t s) {
    open = false;
    if (every <= 0 || (seen[c]++ % every) != 0) return;
    while (ev.size() < used + 2) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) {
        every = 0;
        return;
      }
      ev.push_back(e);
    }
    (void)hipEventRecord(ev[used], s);
    cls.push_back(c);
    open = true;
  }
  void end(hipStream_t s) {
    if (!open) return;
    (void)hipEventRecord(ev[used + 1], s);
    used += 2;
    open = false;
  }
  void flush() {  // after a stream synchronisation
    for (size_t p = 0; p < cls.size(); ++p) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[2 * p], ev[2 * p + 1]) == hipSuccess) {
        res->kernel_ms[cls[p]] += ms;
        res->kernel_launches[cls[p]] += 1;
      }
    }
    cls.clear();
    used = 0;
  }
};

struct Run {
  hipStream_t s;
  Prof prof;
  its_matrix::GraphCache *gc = nullptr;  // null: launch each iteration eagerly
  std::vector<uint64_t> key;             // what the captured launches depend on
  template <class K, class... Args>
  hipError_t launch(int cls, K kernel, int grid, Args... args) {
    prof.begin(cls, s);
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), 0, s, args...);
    prof.end(s);
    return hipGetLastError();
  }
  // The finishing kernel(s) of a reducing pass that ran with G blocks.
  template <int ND, class Fin>
  hipError_t finish(Reduce *R, int G, Fin fin) {
    const int nb = finish_grid(G);
    if (nb == 0) return launch(kClassFinish, k_finish_final<ND, Fin>, 1, R, G, 1, fin);
    hipError_t e = launch(kClassFinish, k_finish_group<ND>, nb, R, G);
    if (e != hipSuccess) return e;
    return launch(kClassFinish, k_finish_final<ND, Fin>, 1, R, nb, 2, fin);
  }
};

#define FINISH(run, nd, R, G, fin)                                                              \
  do {                                                                                        \
    hipError_t e_ = (run).template finish<nd>(R, G, fin);                                     \
    if (e_ != hipSuccess) return fail(ITS_E_HIP, std::string("launch: ") + hipGetErrorString(e_)); \
  } while (0)

#define LAUNCH(run, cls, kernel, grid, ...)                                                   \
  do {                                                                                        \
    hipError_t e_ = (run).launch(cls, kernel, grid, __VA_ARGS__);                             \
    if (e_ != hipSuccess) return fail(ITS_E_HIP, std::string("launch: ") + hipGetErrorString(e_)); \
  } while (0)

// ------------------------------------------------------------ workspace
// [State main][State inner][grid-barrier words][Reduce scratch][vectors...],
// every section 256-byte aligned.
constexpr size_t kAlign = 256;
inline size_t up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

constexpr int kGuardPairs = 32;  // 256 bytes of FP32 pairs

struct Layout {
  size_t state = 0, state2 = 0, sync = 0, reduce = 0, total = 0;
  size_t off[8] = {};  // offsets of the method's vector regions
  int nreg = 0;
};

// Vector regions per method (bytes per row):
//   Jacobi   : x ping-pong buffer (8)
//   SGS      : the saved black rows of the iterate under test (8; CSR, two colours)
//   CG       : {r, p} interleaved pairs (16), q (8)
//   IR-CG    : r (8), {r, p} FP32 pairs (8, + 256 bytes of guard pairs at each end), q (4), d (4)
//   BiCGStab : {r, u} pairs (16), r' (8), p (8), {r, v} pairs (16), t (8)
//   CG-NB    : {r, Ap} interleaved pairs (16), p (8), w = A r (8); persistent:
//              a second pair buffer (16)
Layout layout_for(int64_t n, int method, int inner_dtype, int persistent = 0) {
  Layout L;
  L.state = 0;
  L.state2 = up(sizeof(State));
  L.sync = L.state2 + up(sizeof(State));
  L.reduce = L.sync + up(sizeof(unsigned long long) * kSyncWords);
  size_t at = L.reduce + up(sizeof(Reduce));
  int per[8] = {};
  switch (method) {
    case ITS_JACOBI: L.nreg = 1; per[0] = 8; break;
    case ITS_SGS: L.nreg = 1; per[0] = 8; break;
    case ITS_CG:
      if (inner_dtype == ITS_F64) {
        L.nreg = 2; per[0] = 16; per[1] = 8;
      } else {
        L.nreg = 4; per[0] = 8; per[1] = 8; per[2] = 4; per[3] = 4;
      }
      break;
    case ITS_BICGSTAB:
      L.nreg = 5; per[0] = 16; per[1] = 8; per[2] = 8; per[3] = 16; per[4] = 8;
      break;
    case ITS_CG_NB:
      // persistent: a second {r, Ap} pair buffer (iterations alternate)
      L.nreg = persistent ? 4 : 3; per[0] = 16; per[1] = 8; per[2] = 8; per[3] = 16;
      break;
    default: break;
  }
  // the refinement's FP32 pairs carry two guard pairs at each end
  size_t pad[8] = {};
  if (method == ITS_CG && inner_dtype != ITS_F64) pad[1] = 2 * kGuardPairs * sizeof(float2_t);
  for (int i = 0; i < L.nreg; ++i) {
    L.off[i] = at;
    at += up(size_t(n) * size_t(per[i]) + pad[i]);
  }
  L.total = at;
  return L;
}

struct WS {
  State *st, *st2;
  Reduce *R;
  unsigned long long *sync;
  char *base;
  Layout L;
  template <class T>
  T *reg(int i) const { return reinterpret_cast<T *>(base + L.off[i]); }
  double *v64(int i) const { return reg<double>(i); }
};

WS carve(void *ws, const Layout &L, int64_t) {
  char *b = static_cast<char *>(ws);
  WS w;
  w.st = reinterpret_cast<State *>(b + L.state);
  w.st2 = reinterpret_cast<State *>(b + L.state2);
  w.R = reinterpret_cast<Reduce *>(b + L.reduce);
  w.sync = reinterpret_cast<unsigned long long *>(b + L.sync);
  w.base = b;
  w.L = L;
  return w;
}

// ------------------------------------------------------------ operators

// Blocks of the FP64 CG update pass and BiCGStab's pass C (each walks several
// tiles backwards or forwards): 1024 measured best at 256^3 (update pass
// 120.8 us against 123.6 us with 4096 blocks, 122.1 with 768, 143.7 with
// 512), and for BiCGStab on 192^3; the FP32 inner update pass keeps 4096.
constexpr int kUpdateGrid = 1024;

// A CSR operator's launch that sweeps its tiles backwards (Backwards); the
// matrix-free operators are launched as they are.
#define LAUNCH_OP(run, cls, K, rev, grid, op, ...)                                              \
  do {                                                                                        \
    using Op_ = decltype(op);                                                                 \
    if constexpr (GathersPairs<Op_>::value) {                                                 \
      if (rev) {                                                                              \
        LAUNCH(run, cls, K<Backwards<Op_>>, grid, Backwards<Op_>{op}, __VA_ARGS__);           \
        break;                                                                                \
      }                                                                                       \
    }                                                                                         \
    LAUNCH(run, cls, K<Op_>, grid, op, __VA_ARGS__);                                          \
  } while (0)

template <class F>
its_status with_op64(const its_matrix *A, F &&f) {
  switch (A->kind) {
    case kCsr:
      if (A->sp && !A->scol)
        return f(SellOp<double, double, true>{A->sp, A->scol, A->sval, int32_t(A->n), A->soff, A->smask, nullptr});
      if (A->sp) return f(SellOp<double, double>{A->sp, A->scol, A->sval, int32_t(A->n), A->soff, A->smask, nullptr});
      return f(CsrOp<double, double>{A->rp, A->col, A->val, int32_t(A->n)});
    case kSten7: {
      StencilOp<7, double> op{A->nx, A->ny, A->nz, int32_t(A->n), {}};
      for (int o = 0; o < 7; ++o) op.c[o] = A->coef[o];
      op.plan();
      return f(op);
    }
    case kVar7: {
      VarCoefOp op{A->nx, A->ny, A->nz, int32_t(A->n), A->kcoef};
      op.plan();
      return f(op);
    }
    default: {
      StencilOp<27, double> op{A->nx, A->ny, A->nz, int32_t(A->n), {}};
      for (int o = 0; o < 27; ++o) op.c[o] = A->coef[o];
      op.plan();
      return f(op);
    }
  }
}

template <class F>
its_status with_op32(const its_matrix *A, int dtype, F &&f) {
  switch (A->kind) {
    case kVar7: return fail(ITS_E_UNSUPPORTED, "mixed precision is not available for variable coefficients");
    case kCsr:
      if (dtype == ITS_F32) {
        if (A->sp && !A->scol)
          return f(SellOp<float, float, true>{A->sp, A->scol, A->sval32, int32_t(A->n), A->soff, A->smask, nullptr});
        if (A->sp) return f(SellOp<float, float>{A->sp, A->scol, A->sval32, int32_t(A->n), A->soff, A->smask, nullptr});
        return f(CsrOp<float, float>{A->rp, A->col, A->val32, int32_t(A->n)});
      }
      if (A->sp && !A->scol)
        return f(SellOp<__half, float, true>{A->sp, A->scol, A->sval16, int32_t(A->n), A->soff, A->smask, nullptr});
      if (A->sp) return f(SellOp<__half, float>{A->sp, A->scol, A->sval16, int32_t(A->n), A->soff, A->smask, nullptr});
      return f(CsrOp<__half, float>{A->rp, A->col, A->val16, int32_t(A->n)});
    case kSten7: {
      StencilOp<7, float> op{A->nx, A->ny, A->nz, int32_t(A->n), {}};
      for (int o = 0; o < 7; ++o)
        op.c[o] = dtype == ITS_F32 ? float(A->coef[o]) : float(static_cast<_Float16>(A->coef[o]));
      op.plan();
      return f(op);
    }
    default: {
      StencilOp<27, float> op{A->nx, A->ny, A->nz, int32_t(A->n), {}};
      for (int o = 0; o < 27; ++o)
        op.c[o] = dtype == ITS_F32 ? float(A->coef[o]) : float(static_cast<_Float16>(A->coef[o]));
      op.plan();
      return f(op);
    }
  }
}

// ------------------------------------------------------------- polling

its_status poll(Run &run, const State *dev, State *host) {
  HIP_TRY(hipMemcpyAsync(host, dev, sizeof(State), hipMemcpyDeviceToHost, run.s));
  HIP_TRY(hipStreamSynchronize(run.s));
  run.prof.flush();
  return ITS_OK;
}

its_status flag_to_status(int32_t f) {
  switch (f) {
    case kConverged: return ITS_OK;
    case kMaxIter: return ITS_NOT_CONVERGED;
    default: return ITS_BREAKDOWN;
  }
}

int batch_size(const its_options *o, int64_t n) {
  if (o->check_every > 0) return o->check_every;
  return n >= (int64_t(1) << 20) ? 8 : 32;
}

// Runs iterations j = j0, j0+1, ... until the device flag leaves kRunning or
// max_iter iterations were launched; `step(j)` launches iteration j.
// Graph form of the loop: iterations 0..m-1 (or 1..m with the first run
// eagerly, for a step whose first iteration differs) are captured once on
// the handle's stream and replayed, with one poll of the State per replay.
// m is even so that steps alternating buffers by the parity of j line up.
// The limits live in the State, so the same graph serves every right-hand
// side; the key holds every value the captured launches bake in.
template <class Step>
its_status iterate_graph(Run &run, const State *dev, State *host, int64_t max_iter, int m,
                         bool eager_first, Step &&step) {
  its_matrix::GraphCache &G = *run.gc;
  if (m & 1) ++m;
  if (!G.s) {
    HIP_TRY(hipStreamCreateWithFlags(&G.s, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&G.ev, hipEventDisableTiming));
  }
  int64_t j = 0;
  if (eager_first) {
    its_status st = step(0);
    if (st != ITS_OK) return st;
    j = 1;
  }
  std::vector<uint64_t> key = run.key;
  key.push_back(uint64_t(m));
  key.push_back(uint64_t(eager_first));
  // order the graph after the work already on the caller's stream
  HIP_TRY(hipEventRecord(G.ev, run.s));
  HIP_TRY(hipStreamWaitEvent(G.s, G.ev, 0));
  if (!G.exec || G.key != key) {
    if (G.exec) (void)hipGraphExecDestroy(G.exec);
    G.exec = nullptr;
    G.key.clear();
    const hipStream_t saved = run.s;
    run.s = G.s;
    HIP_TRY(hipStreamBeginCapture(G.s, hipStreamCaptureModeThreadLocal));
    its_status st = ITS_OK;
    for (int t = 0; t < m && st == ITS_OK; ++t) st = step(j + t);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(G.s, &g);
    run.s = saved;
    if (st != ITS_OK) {
      if (e == hipSuccess && g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return fail(ITS_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&G.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      G.exec = nullptr;
      return fail(ITS_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    G.key = key;
  }
  for (;;) {
    HIP_TRY(hipGraphLaunch(G.exec, G.s));
    j += m;
    HIP_TRY(hipMemcpyAsync(host, dev, sizeof(State), hipMemcpyDeviceToHost, G.s));
    HIP_TRY(hipStreamSynchronize(G.s));
    if (host->flag != kRunning) return ITS_OK;
    if (j >= max_iter + m) return fail(ITS_E_HIP, "device state still running after max_iter");
  }
}

template <class Step>
its_status iterate(Run &run, const State *dev, State *host, int64_t max_iter, int m, Step &&step,
                   bool eager_first = false) {
  if (run.gc && run.prof.every == 0) return iterate_graph(run, dev, host, max_iter, m, eager_first, step);
  int64_t j = 0;
  for (;;) {
    const int64_t todo = std::min<int64_t>(m, max_iter - j);
    for (int64_t t = 0; t < todo; ++t, ++j) {
      its_status st = step(j);
      if (st != ITS_OK) return st;
    }
    its_status st = poll(run, dev, host);
    if (st != ITS_OK) return st;
    if (host->flag != kRunning) return ITS_OK;
    if (j >= max_iter) return fail(ITS_E_HIP, "device state still running after max_iter");
  }
}

// Steps of a loop whose step j tests iterate j: one more than the tests.
int64_t steps_for(int64_t max_iter) {
  return max_iter < std::numeric_limits<int64_t>::max() ? max_iter + 1 : max_iter;
}

// Common prologue: zero the States, b.b, r0 = b - A x0 (stored in r if
// non-null) and r0.r0.  Returns bb and rr0 through `host`.
its_status prologue(Run &run, const its_matrix *A, const WS &w, const double *b, const double *x,
                    double *r, int rstride, State *host, double &bb, double &rr) {
  const int32_t n = int32_t(A->n);
  const int G = grid_for(n);
  LAUNCH(run, kClassOther, k_reset, 1, w.st, 2, w.R);
  LAUNCH(run, kClassOther, k_dot, G, n, b, b, w.R);
  FINISH(run, 1, w.R, G, (FinDot{w.st, 0}));
  its_status s = with_op64(A, [&](auto op) -> its_status {
    const int GA = op.grid();
    LAUNCH(run, kClassOther, k_residual<decltype(op)>, GA, op, b, x, r, rstride, w.R);
    FINISH(run, 1, w.R, GA, (FinDot{w.st, 1}));
    return ITS_OK;
  });
  if (s != ITS_OK) return s;
  s = poll(run, w.st, host);
  if (s != ITS_OK) return s;
  bb = host->dot[0];
  rr = host->dot[1];
  return ITS_OK;
}

double threshold2(double rtol, double bb) {
  const double t = rtol * std::sqrt(bb);
  return t * t;
}

its_status true_residual(Run &run, const its_matrix *A, const WS &w, const double *b,
                         const double *x, State *host, double bb, its_result *res) {
  its_status s = with_op64(A, [&](auto op) -> its_status {
    const int GA = op.grid();
    LAUNCH(run, kClassOther, k_residual<decltype(op)>, GA, op, b, x, (double *)nullptr, 1, w.R);
    FINISH(run, 1, w.R, GA, (FinDot{w.st2, 2}));
    return ITS_OK;
  });
  if (s != ITS_OK) return s;
  s = poll(run, w.st2, host);
  if (s != ITS_OK) return s;
  res->true_rel_res = std::sqrt(host->dot[2]) / std::sqrt(bb);
  return ITS_OK;
}

// ------------------------------------------------------ persistent loops
// One cooperative launch of a persistent solver kernel (kernels_persist.hpp)
// with as many blocks as are co-resident, capped by the work units of the
// operator (tiles or bricks) and by kPersistBlocks (fewer participants make
// a cheaper barrier; the environment variable ITS_PERSISTENT_BLOCKS
// overrides the cap).  The barrier words live in the workspace and are
// zeroed before the launch.

constexpr int kPersistBlocks = 256;

int64_t env_int(const char *name, int64_t dflt) {
  const char *v = std::getenv(name);
  if (!v || !*v) return dflt;
  char *end = nullptr;
  const long long r = std::strtoll(v, &end, 10);
  return (end && *end == '\0') ? int64_t(r) : dflt;
}

template <class K, class... Args>
its_status persist_launch(Run &run, State *h, K kernel, int units, const WS &w, Args... args) {
  int dev = 0, cus = 0, per = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kBlock, 0));
  int64_t G = std::min<int64_t>(int64_t(per) * cus, env_int("ITS_PERSISTENT_BLOCKS", kPersistBlocks));
  G = std::min<int64_t>(G, std::max(units, 1));
  if (G >= 64) G -= G % kXcds;
  if (G < 1) return fail(ITS_E_UNSUPPORTED, "the persistent kernel does not fit on this device");
  GridSync gs;
  gs.w = w.sync;
  gs.extra = uint32_t(std::max<int64_t>(0, env_int("ITS_BARRIER_TEST_EXTRA", 0)));
  gs.spin_limit = std::max<int64_t>(0, env_int("ITS_BARRIER_SPIN_LIMIT", int64_t(1) << 24));
  LAUNCH(run, kClassOther, k_zero_words, 1, w.sync, kSyncWords);
  void *argv[] = {static_cast<void *>(&args)..., static_cast<void *>(&gs)};
  run.prof.begin(0, run.s);
  HIP_TRY(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(kernel), dim3(unsigned(G)),
                                     dim3(kBlock), argv, 0, run.s));
  run.prof.end(run.s);
  // the solver's State and the give-up word
  unsigned long long *gave_up = reinterpret_cast<unsigned long long *>(h + 2);
  HIP_TRY(hipMemcpyAsync(h, w.st, sizeof(State), hipMemcpyDeviceToHost, run.s));
  HIP_TRY(hipMemcpyAsync(gave_up, w.sync + 280, sizeof(unsigned long long), hipMemcpyDeviceToHost, run.s));
  HIP_TRY(hipStreamSynchronize(run.s));
  run.prof.flush();
  if (*gave_up != 0)
    return fail(ITS_E_HIP, "persistent kernel: a grid barrier wait gave up after " +
                               std::to_string(gs.spin_limit) + " polls; x is undefined");
  return ITS_OK;
}

// ------------------------------------------------------------------- CG

its_status solve_cg(Run &run, const its_matrix *A, const its_options *o, const double *b, double *x,
                    const WS &w, its_result *res) {
  State *h = A->host_state;
  const int32_t n = int32_t(A->n);
  const int G = grid_for(n);
  // the update pass: two rows per thread, at most kUpdateGrid blocks
  const int G2 = grid_for((int64_t(n) + 1) / 2, kUpdateGrid);
  double2_t *rp = w.reg<double2_t>(0);  // {r, p} pairs
  double *q = w.v64(1);
  double bb, rr;
  its_status s = prologue(run, A, w, b, x, reinterpret_cast<double *>(rp), 2, h, bb, rr);
  if (s != ITS_OK) return s;
  if (!std::isfinite(bb)) return fail(ITS_E_INVALID, "b contains NaN or Inf");
  if (bb == 0.0) {
    LAUNCH(run, kClassOther, k_fill, G, n, x, 0.0);
    HIP_TRY(hipStreamSynchronize(run.s));
    res->status = ITS_OK;
    return ITS_OK;
  }
  const double thr2 = threshold2(o->rtol, bb);
  int32_t flag = kRunning;
  if (rr <= thr2) flag = kConverged;
  else if (!std::isfinite(rr)) flag = kBreakdown;
  else if (o->max_iter <= 0) flag = kMaxIter;
  LAUNCH(run, kClassOther, k_begin, 1, w.st, flag, rr, thr2, (int64_t)o->max_iter);
  if (flag == kRunning && o->persistent) {
    s = with_op64(A, [&](auto op) -> its_status {
      return persist_launch(run, h, k_cg_persist<decltype(op)>, op.grid(), w, op, x, rp, q, b, w.st, w.R);
    });
    if (s != ITS_OK) return s;
    res->status = flag_to_status(h->flag);
    res->iters = h->k;
    res->rel_res = std::sqrt(h->rho) / std::sqrt(bb);
    res->true_rel_res = std::sqrt(h->dot[2]) / std::sqrt(bb);
    return ITS_OK;
  }
  if (flag == kRunning) {
    s = with_op64(A, [&](auto op) -> its_status {
      const int GA = op.grid();
      return iterate(run, w.st, h, o->max_iter, batch_size(o, n), [&](int64_t) -> its_status {
        LAUNCH(run, 0, (k_cg_pass1<decltype(op), double>), GA, op, (const double2_t *)rp, q, (const State *)w.st, w.R);
        // p.q: with two reduction levels the update pass sums the group sums
        // (at most kGroup) itself instead of a finishing kernel.  It never
        // reads first-level partials: its own blocks overwrite those with
        // their r.r partials while others may still be starting.
        const DD *pq = nullptr;
        int32_t pqn = 0;
        if (GA > kFinishOne) {
          const int nb = finish_grid(GA);
          LAUNCH(run, kClassFinish, k_finish_group<1>, nb, w.R, GA);
          pq = reinterpret_cast<const DD *>(reinterpret_cast<const char *>(w.R) + offsetof(Reduce, p2));
          pqn = nb;
        } else {
          FINISH(run, 1, w.R, GA, (FinCg1{w.st}));
        }
        LAUNCH(run, 1, (k_cg_pass2<double, GathersPairs<decltype(op)>::value>), G2, n, x, rp, (const double *)q, w.st, w.R, pq, pqn);
        FINISH(run, 1, w.R, G2, (FinCg2{w.st}));
        return ITS_OK;
      });
    });
    if (s != ITS_OK) return s;
    LAUNCH(run, kClassOther, k_cg_flush_x, G, n, x, (const double2_t *)rp, (const State *)w.st);
  } else {
    s = poll(run, w.st, h);
    if (s != ITS_OK) return s;
  }
  res->status = flag_to_status(h->flag);
  res->iters = h->k;
  res->rel_res = std::sqrt(h->rho) / std::sqrt(bb);
  return true_residual(run, A, w, b, x, h, bb, res);
}

// ---------------------------------------------------------------- CG-NB

its_status solve_cgnb(Run &run, const its_matrix *A, const its_options *o, const double *b,
                      double *x, const WS &w, its_result *res) {
  State *h = A->host_state;
  const int32_t n = int32_t(A->n);
  const int G = grid_for(n);
  double2_t *ra = w.reg<double2_t>(0);  // {r, Ap} pairs
  double *p = w.v64(1), *wv = w.v64(2);
  double bb, rr;
  its_status s = prologue(run, A, w, b, x, reinterpret_cast<double *>(ra), 2, h, bb, rr);
  if (s != ITS_OK) return s;
  if (!std::isfinite(bb)) return fail(ITS_E_INVALID, "b contains NaN or Inf");
  if (bb == 0.0) {
    LAUNCH(run, kClassOther, k_fill, G, n, x, 0.0);
    HIP_TRY(hipStreamSynchronize(run.s));
    res->status = ITS_OK;
    return ITS_OK;
  }
  const double thr2 = threshold2(o->rtol, bb);
  int32_t flag = kRunning;
  if (rr <= thr2) flag = kConverged;
  else if (!std::isfinite(rr)) flag = kBreakdown;
  else if (o->max_iter <= 0) flag = kMaxIter;
  LAUNCH(run, kClassOther, k_begin, 1, w.st, flag, rr, thr2, (int64_t)o->max_iter);
  if (flag == kRunning) {
    s = with_op64(A, [&](auto op) -> its_status {
      const int GA = op.grid();
      LAUNCH(run, kClassOther, k_cgnb_init<decltype(op)>, GA, op, ra, p, w.R);
      FINISH(run, 1, w.R, GA, (FinCgnbInit{w.st}));
      if (o->persistent)
        return persist_launch(run, h, k_cgnb_persist<decltype(op)>, GA, w, op, x, ra, w.reg<double2_t>(3), p, wv, b,
                              w.st, w.R);
      return iterate(run, w.st, h, o->max_iter, batch_size(o, n), [&](int64_t) -> its_status {
        LAUNCH(run, 0, k_cgnb_x<decltype(op)>, GA, op, (const double2_t *)ra, wv, (const State *)w.st, w.R);
        FINISH(run, 1, w.R, GA, (FinCgnbX{w.st}));
        LAUNCH(run, 1, k_cgnb_y<GathersPairs<decltype(op)>::value>, G, n, x, ra, p, (const double *)wv, (const State *)w.st, w.R);
        FINISH(run, 1, w.R, G, (FinCgnbY{w.st}));
        return ITS_OK;
      });
    });
    if (s != ITS_OK) return s;
  } else {
    s = poll(run, w.st, h);
    if (s != ITS_OK) return s;
  }
  res->status = flag_to_status(h->flag);
  res->iters = h->k;
  res->rel_res = std::sqrt(h->rho) / std::sqrt(bb);
  if (flag == kRunning && o->persistent) {  // the kernel formed the true residual
    res->true_rel_res = std::sqrt(h->dot[2]) / std::sqrt(bb);
    return ITS_OK;
  }
  return true_residual(run, A, w, b, x, h, bb, res);
}

// ------------------------------------------- mixed-precision refinement CG

its_status solve_ir(Run &run, const its_matrix *A, const its_options *o, const double *b, double *x,
                    const WS &w, its_result *res) {
  State *h = A->host_state;
  const int32_t n = int32_t(A->n);
  const int G = grid_for(n), G2 = grid_for(n >> 1, kFinishOne);  // G2: row pairs of the FP32 pass 2
  const int dt = o->inner_dtype;
  if (A->kind == kCsr && ((dt == ITS_F32 && !A->val32) || (dt == ITS_F16 && !A->val16)))
    return fail(ITS_E_INVALID, "mixed precision needs its_csr_set_lowp values of that dtype");
  double *r = w.v64(0);
  // inner {r, p} pairs, with guard pairs before index 0 and after index
  // n - 1 (the two-rows-per-lane pass reads a pair past either end); 256
  // bytes of them in front keep the pairs' alignment
  float2_t *rhp = w.reg<float2_t>(1) + kGuardPairs;
  float *q = w.reg<float>(2), *d = w.reg<float>(3);
  double bb, rr;
  its_status s = prologue(run, A, w, b, x, r, 1, h, bb, rr);
  if (s != ITS_OK) return s;
  if (!std::isfinite(bb)) return fail(ITS_E_INVALID, "b contains NaN or Inf");
  if (bb == 0.0) {
    LAUNCH(run, kClassOther, k_fill, G, n, x, 0.0);
    HIP_TRY(hipStreamSynchronize(run.s));
    res->status = ITS_OK;
    return ITS_OK;
  }
  const double thr2 = threshold2(o->rtol, bb);
  int64_t inner_total = 0;
  int64_t outer = 0;
  for (;; ++outer) {
    if (outer > 0) {  // r = b - A x of the refined iterate
      s = with_op64(A, [&](auto op) -> its_status {
        const int GA = op.grid();
        LAUNCH(run, 2, k_residual<decltype(op)>, GA, op, b, (const double *)x, r, 1, w.R);
        FINISH(run, 1, w.R, GA, (FinDot{w.st, 1}));
        return ITS_OK;
      });
      if (s != ITS_OK) return s;
      s = poll(run, w.st, h);
      if (s != ITS_OK) return s;
      rr = h->dot[1];
    }
    if (rr <= thr2) { res->status = ITS_OK; break; }
    if (!std::isfinite(rr)) { res->status = ITS_BREAKDOWN; break; }
    if (outer == o->max_outer || inner_total >= o->max_iter) { res->status = ITS_NOT_CONVERGED; break; }
    const double rn = std::sqrt(rr);
    LAUNCH(run, 3, k_ir_scale, G, n, (const double *)r, reinterpret_cast<float *>(rhp), d, w.R, rn);
    FINISH(run, 1, w.R, G, (FinDot{w.st2, 1}));
    s = poll(run, w.st2, h);
    if (s != ITS_OK) return s;
    const double rho_i = h->dot[1];
    const double ithr2 = threshold2(o->inner_rtol, rho_i);
    const int64_t budget = o->max_iter - inner_total;
    if (!(rho_i <= ithr2)) {
      LAUNCH(run, kClassOther, k_begin, 1, w.st2, (int32_t)kRunning, rho_i, ithr2, budget);
      s = with_op32(A, dt, [&](auto op) -> its_status {
        // two rows per lane where it pays (measured): FP16 values, or
        // slices wider than one group of seven entries
        bool pairs = false;
        if constexpr (PairWalk<decltype(op)>::value)
          pairs = sizeof(typename decltype(op)::value_type) == 2 || A->sell_wmax > 7;
        int GA = op.grid();
        if constexpr (PairWalk<decltype(op)>::value)
          if (pairs) GA = op.grid_pairs(A->sell_wmax > 7);
        return iterate(run, w.st2, h, budget, batch_size(o, n), [&](int64_t) -> its_status {
          if constexpr (PairWalk<decltype(op)>::value)
            if (pairs) {
              LAUNCH(run, 0, (k_cg_pass1_pairs<decltype(op)>), GA, op, (const float2_t *)rhp, q, (const State *)w.st2, w.R);
              FINISH(run, 1, w.R, GA, (FinCg1{w.st2}));
              LAUNCH(run, 1, k_cg_pass2_f32x2<GathersPairs<decltype(op)>::value>, G2, n, d, rhp, (const float *)q, (const State *)w.st2, w.R);
              FINISH(run, 1, w.R, G2, (FinCg2{w.st2}));
              return ITS_OK;
            }
          LAUNCH(run, 0, (k_cg_pass1<decltype(op), float>), GA, op, (const float2_t *)rhp, q, (const State *)w.st2, w.R);
          FINISH(run, 1, w.R, GA, (FinCg1{w.st2}));
          LAUNCH(run, 1, k_cg_pass2_f32x2<GathersPairs<decltype(op)>::value>, G2, n, d, rhp, (const float *)q, (const State *)w.st2, w.R);
          FINISH(run, 1, w.R, G2, (FinCg2{w.st2}));
          return ITS_OK;
        });
      });
      if (s != ITS_OK) return s;
      LAUNCH(run, kClassOther, k_cg_flush_x32, G, n, d, (const float2_t *)rhp, (const State *)w.st2);
      inner_total += h->k;
      if (h->flag == kBreakdown) { res->status = ITS_BREAKDOWN; break; }
    }
    LAUNCH(run, 3, k_ir_update, G, n, x, (const float *)d, rn);
  }
  res->iters = outer;
  res->inner_iters = inner_total;
  res->rel_res = std::sqrt(rr) / std::sqrt(bb);
  res->true_rel_res = res->rel_res;
  HIP_TRY(hipStreamSynchronize(run.s));
  run.prof.flush();
  return ITS_OK;
}

// ------------------------------------------------------------- BiCGStab

its_status solve_bicgstab(Run &run, const its_matrix *A, const its_options *o, const double *b,
                          double *x, const WS &w, its_result *res) {
  State *h = A->host_state;
  const int32_t n = int32_t(A->n);
  const int G = grid_for(n);
  const int GC = grid_for((int64_t(n) + 1) / 2, kUpdateGrid);  // pass C: two rows per thread
  double2_t *ru = w.reg<double2_t>(0), *rv = w.reg<double2_t>(3);
  double *rs = w.v64(1), *p = w.v64(2), *t = w.v64(4);
  double bb, rr;
  its_status s = prologue(run, A, w, b, x, reinterpret_cast<double *>(ru), 2, h, bb, rr);
  if (s != ITS_OK) return s;
  if (!std::isfinite(bb)) return fail(ITS_E_INVALID, "b contains NaN or Inf");
  if (bb == 0.0) {
    LAUNCH(run, kClassOther, k_fill, G, n, x, 0.0);
    HIP_TRY(hipStreamSynchronize(run.s));
    res->status = ITS_OK;
    return ITS_OK;
  }
  const double thr2 = threshold2(o->rtol, bb);
  int32_t flag = kRunning;
  if (rr <= thr2) flag = kConverged;
  else if (!std::isfinite(rr)) flag = kBreakdown;
  else if (o->max_iter <= 0) flag = kMaxIter;
  LAUNCH(run, kClassOther, k_begin, 1, w.st, flag, rr, thr2, (int64_t)o->max_iter);
  if (flag == kRunning) {
    LAUNCH(run, kClassOther, k_bicg_init, G, n, (const double2_t *)ru, rs, w.R, std::sqrt(rr));
    FINISH(run, 1, w.R, G, (FinBicgInit{w.st}));
    const double rt2 = o->restart_tol * o->restart_tol;
    const int32_t paper = o->restart_mode == ITS_RESTART_PAPER;
    s = with_op64(A, [&](auto op) -> its_status {
      const int GA = op.grid();
      if (o->persistent) {
        // BiCGStab-B1's split-phase schedule (ITS_BICGSTAB_SPLIT=0: the same
        // updates after the waits, classical BiCGStab's blocking points)
        if (env_int("ITS_BICGSTAB_SPLIT", 1) != 0)
          return persist_launch(run, h, k_bicg_persist<decltype(op), true>, GA, w, op, x, ru, rs, p, rv, t, b,
                                w.st, w.R, rt2, paper);
        return persist_launch(run, h, k_bicg_persist<decltype(op), false>, GA, w, op, x, ru, rs, p, rv, t, b,
                              w.st, w.R, rt2, paper);
      }
      return iterate(run, w.st, h, o->max_iter, batch_size(o, n), [&](int64_t) -> its_status {
        LAUNCH(run, 0, k_bicg_a<decltype(op)>, GA, op, (const double2_t *)ru, rs, p, rv, (const State *)w.st, w.R);
        FINISH(run, 1, w.R, GA, (FinBicgA{w.st}));
        // backwards: it starts on the {r, v} pairs pass A wrote last
        LAUNCH_OP(run, 1, k_bicg_b, true, GA, op, (const double2_t *)rv, t, (const State *)w.st, w.R);
        FINISH(run, 2, w.R, GA, (FinBicgB{w.st}));
        LAUNCH(run, 2, k_bicg_c<GathersPairs<decltype(op)>::value>, GC, n, x, ru, (const double *)rs, (const double *)p, (const double2_t *)rv, (const double *)t, (const State *)w.st, w.R);
        FINISH(run, 2, w.R, GC, (FinBicgC{w.st, rt2, paper}));
        return ITS_OK;
      });
    });
    if (s != ITS_OK) return s;
  } else {
    s = poll(run, w.st, h);
    if (s != ITS_OK) return s;
  }
  res->status = flag_to_status(h->flag);
  res->iters = h->k;
  res->restarts = h->restarts;
  res->rel_res = std::sqrt(h->rho) / std::sqrt(bb);
  if (flag == kRunning && o->persistent) {  // the kernel formed the true residual
    res->true_rel_res = std::sqrt(h->dot[2]) / std::sqrt(bb);
    return ITS_OK;
  }
  return true_residual(run, A, w, b, x, h, bb, res);
}

// --------------------------------------------------------------- Jacobi

its_status check_diag(Run &run, its_matrix *A, const WS &w);

its_status solve_jacobi(Run &run, its_matrix *A, const its_options *o, const double *b, double *x,
                        const WS &w, its_result *res) {
  State *h = A->host_state;
  const int32_t n = int32_t(A->n);
  const int G = grid_for(n);
  double *X[2] = {x, w.v64(0)};
  double bb, rr;
  its_status s = prologue(run, A, w, b, x, nullptr, 1, h, bb, rr);
  if (s != ITS_OK) return s;
  if (!std::isfinite(bb)) return fail(ITS_E_INVALID, "b contains NaN or Inf");
  if (bb == 0.0) {
    LAUNCH(run, kClassOther, k_fill, G, n, x, 0.0);
    HIP_TRY(hipStreamSynchronize(run.s));
    res->status = ITS_OK;
    return ITS_OK;
  }
  const double thr2 = threshold2(o->rtol, bb);
  LAUNCH(run, kClassOther, k_begin, 1, w.st, (int32_t)kRunning, 0.0, thr2, (int64_t)o->max_iter);
  // sweep j tests x_j and forms x_{j+1}: max_iter + 1 launches at most
  s = with_op64(A, [&](auto op) -> its_status {
    const int GA = op.grid();
    return iterate(run, w.st, h, steps_for(o->max_iter), batch_size(o, n), [&](int64_t j) -> its_status {
      const int a = int(j & 1);
      // odd sweeps run backwards: each starts on the x values the previous one wrote last
      LAUNCH_OP(run, 0, k_jacobi, a == 1, GA, op, b, (const double *)X[a], X[a ^ 1], (const State *)w.st, w.R);
      FINISH(run, 1, w.R, GA, (FinJacobi{w.st}));
      return ITS_OK;
    });
  });
  if (s != ITS_OK) return s;
  if (h->k & 1) HIP_TRY(hipMemcpyAsync(x, X[1], size_t(n) * 8, hipMemcpyDeviceToDevice, run.s));
  HIP_TRY(hipStreamSynchronize(run.s));
  res->status = flag_to_status(h->flag);
  res->iters = h->k;
  res->rel_res = std::sqrt(h->rho) / std::sqrt(bb);
  res->true_rel_res = res->rel_res;
  return ITS_OK;
}

// ----------------------------------------------------- symmetric Gauss-Seidel

its_status solve_sgs(Run &run, its_matrix *A, const its_options *o, const double *b, double *x,
                     const WS &w, its_result *res) {
  State *h = A->host_state;
  const int32_t n = int32_t(A->n);
  const int G = grid_for(n);
  if (A->kind == kVar7) return fail(ITS_E_UNSUPPORTED, "Gauss-Seidel is not available for variable coefficients");
  const int nc = A->kind == kCsr ? A->ncolors : (A->kind == kSten7 ? 2 : 8);
  double bb, rr;
  its_status s = prologue(run, A, w, b, x, nullptr, 1, h, bb, rr);
  if (s != ITS_OK) return s;
  if (!std::isfinite(bb)) return fail(ITS_E_INVALID, "b contains NaN or Inf");
  if (bb == 0.0) {
    LAUNCH(run, kClassOther, k_fill, G, n, x, 0.0);
    HIP_TRY(hipStreamSynchronize(run.s));
    res->status = ITS_OK;
    return ITS_OK;
  }
  const double thr2 = threshold2(o->rtol, bb);
  int32_t flag = kRunning;
  if (rr <= thr2) flag = kConverged;
  else if (!std::isfinite(rr)) flag = kBreakdown;
  else if (o->max_iter <= 0) flag = kMaxIter;
  LAUNCH(run, kClassOther, k_begin, 1, w.st, flag, rr, thr2, (int64_t)o->max_iter);
  // Colour order of iteration j: forward 0..nc-1 then backward nc-1..0.  The
  // backward sweep's first colour repeats the forward sweep's last one on
  // unchanged inputs, and the next forward sweep's colour 0 repeats this
  // backward sweep's last one; both repeats reproduce identical bits and
  // are skipped.
  double *xs = w.v64(0);  // CSR, two colours: the black rows of the iterate under test
  int32_t count[2] = {0, 0};
  if (A->kind == kCsr)
    for (int c = 0; c < 2 && c < nc; ++c) count[c] = A->color_off[c + 1] - A->color_off[c];
  // with two colours both half-sweeps' residual partials line up on one grid
  const int G2 = grid_for(std::max(count[0], count[1]));
  auto sweep = [&](int c, auto mode_tag) -> its_status {
    constexpr int M = decltype(mode_tag)::value;
    if (A->kind == kCsr) {
      const int32_t beg = A->color_off[c], cnt = A->color_off[c + 1] - beg;
      const int Gc = M == kGsPlain ? grid_for(cnt) : G2;
      if (cnt == 0 && M == kGsPlain) return ITS_OK;
      if (!A->cpack.empty()) {
        const auto &cp = A->cpack[size_t(c)];
        const int32_t *rows = A->color_rows + beg;
        if (!cp.col) {  // every slice an offset slice
          // with two colours the red half-sweeps run backwards: each starts on the rows
          // the black one before it wrote last
          const SellOp<double, double, true> op{cp.sp, cp.col, cp.val, cnt, cp.soff, cp.smask, rows};
          if (nc == 2 && c == 0)
            LAUNCH(run, 0, (k_gs_rows_packed<M, Backwards<SellOp<double, double, true>>>), Gc, Backwards<SellOp<double, double, true>>{op}, rows, b, x, xs, (const State *)w.st, w.R);
          else
            LAUNCH(run, 0, (k_gs_rows_packed<M, SellOp<double, double, true>>), Gc, op, rows, b, x, xs, (const State *)w.st, w.R);
        } else {
          LAUNCH(run, 0, (k_gs_rows_packed<M, SellOp<double, double>>), Gc, SellOp<double, double>{cp.sp, cp.col, cp.val, cnt, cp.soff, cp.smask, rows}, rows, b, x, xs, (const State *)w.st, w.R);
        }
        return ITS_OK;
      }
      LAUNCH(run, 0, k_gs_rows_csr<M>, Gc, CsrOp<double, double>{A->rp, A->col, A->val, n}, (const int32_t *)(A->color_rows + beg), cnt, b, x, xs, (const State *)w.st, w.R);
    } else if (A->kind == kSten7) {
      StencilOp<7, double> op{A->nx, A->ny, A->nz, n, {}};
      for (int q = 0; q < 7; ++q) op.c[q] = A->coef[q];
      LAUNCH(run, 0, k_gs_stencil<7>, grid_for(gs_colour_cells<7>(A->nx, A->ny, A->nz)), op, (int32_t)c, b, x, (const State *)w.st);
    } else {
      StencilOp<27, double> op{A->nx, A->ny, A->nz, n, {}};
      for (int q = 0; q < 27; ++q) op.c[q] = A->coef[q];
      LAUNCH(run, 0, k_gs_stencil<27>, grid_for(gs_colour_cells<27>(A->nx, A->ny, A->nz)), op, (int32_t)c, b, x, (const State *)w.st);
    }
    return ITS_OK;
  };
  using Plain = std::integral_constant<int, kGsPlain>;
  using Final = std::integral_constant<int, kGsFinal>;
  using Lagged = std::integral_constant<int, kGsLagged>;
  if (flag == kRunning && nc == 2 && A->kind == kCsr) {
    // Iteration 1 sweeps red, black, red; iteration j > 1 black, red.  The
    // test of iterate j rides on the sweeps: its red residual on iteration
    // j's last (red) sweep, its black residual on iteration j + 1's black
    // sweep, after which the test runs; so step j (0-based) finishes
    // iterate j's test before making iterate j + 1, and max_iter + 1 steps
    // cover max_iter tests.
    s = iterate(run, w.st, h, steps_for(o->max_iter), batch_size(o, n), [&](int64_t j) -> its_status {
      its_status e;
      if (j == 0) {
        if ((e = sweep(0, Plain{})) != ITS_OK) return e;
        if ((e = sweep(1, Plain{})) != ITS_OK) return e;
      } else {
        if ((e = sweep(1, Lagged{})) != ITS_OK) return e;
        FINISH(run, 2, w.R, G2, (FinGs2{w.st}));
      }
      return sweep(0, Final{});
    }, /*eager_first=*/true);
    if (s != ITS_OK) return s;
    // the stopping test ran after a black sweep: put the tested black rows back
    LAUNCH(run, kClassOther, k_gs_restore_rows, grid_for(count[1]), (const int32_t *)(A->color_rows + A->color_off[1]), count[1], (const double *)xs, x);
    HIP_TRY(hipStreamSynchronize(run.s));
  } else if (flag == kRunning) {
    s = with_op64(A, [&](auto op) -> its_status {
      const int GA = op.grid();
      return iterate(run, w.st, h, o->max_iter, batch_size(o, n), [&](int64_t j) -> its_status {
        for (int c = (j == 0 ? 0 : 1); c < nc; ++c) {
          its_status e = sweep(c, Plain{});
          if (e != ITS_OK) return e;
        }
        for (int c = nc - 2; c >= 0; --c) {
          its_status e = sweep(c, Plain{});
          if (e != ITS_OK) return e;
        }
        LAUNCH(run, 1, k_gs_check<decltype(op)>, GA, op, b, (const double *)x, (const State *)w.st, w.R);
        FINISH(run, 1, w.R, GA, (FinGs{w.st}));
        return ITS_OK;
      }, /*eager_first=*/true);
    });
    if (s != ITS_OK) return s;
  } else {
    s = poll(run, w.st, h);
    if (s != ITS_OK) return s;
  }
  res->status = flag_to_status(h->flag);
  res->iters = h->k;
  res->rel_res = std::sqrt(h->rho) / std::sqrt(bb);
  res->true_rel_res = res->rel_res;
  return ITS_OK;
}

its_status check_diag(Run &run, its_matrix *A, const WS &w) {
  if (A->kind == kVar7) {  // diagonal = sum of positive face coefficients
    A->diag_state = 1;
    return ITS_OK;
  }
  if (A->kind != kCsr) {
    A->diag_state = A->coef[A->kind == kSten7 ? 3 : 13] != 0.0 ? 1 : -1;
    return ITS_OK;
  }
  if (A->diag_state != 0) return ITS_OK;
  uint32_t *bad = &w.st2->counter[7];
  LAUNCH(run, kClassOther, k_reset, 1, w.st2, 1, w.R);
  LAUNCH(run, kClassOther, k_csr_check, grid_for(A->n), int32_t(A->n), int32_t(A->nnz), A->rp, A->col, A->val, (int32_t)1, bad);
  its_status s = poll(run, w.st2, A->host_state);
  if (s != ITS_OK) return s;
  A->diag_state = A->host_state->counter[7] == 0 ? 1 : -1;
  return ITS_OK;
}

bool options_ok(const its_options *o, std::string &why) {
  if (o->method < ITS_JACOBI || o->method > ITS_CG_NB) { why = "unknown method"; return false; }
  if (!(o->rtol >= 0.0) || !std::isfinite(o->rtol)) { why = "rtol must be finite and >= 0"; return false; }
  if (o->max_iter < 0) { why = "max_iter must be >= 0"; return false; }
  if (!(o->restart_tol >= 0.0) || !std::isfinite(o->restart_tol)) { why = "restart_tol must be finite and >= 0"; return false; }
  if (o->restart_mode != ITS_RESTART_COSINE && o->restart_mode != ITS_RESTART_PAPER) { why = "unknown restart_mode"; return false; }
  if (o->check_every < 0) { why = "check_every must be >= 0"; return false; }
  if (o->inner_dtype < ITS_F64 || o->inner_dtype > ITS_F16) { why = "unknown inner_dtype"; return false; }
  if (o->inner_dtype != ITS_F64 && o->method != ITS_CG) { why = "mixed precision is for CG only"; return false; }
  if (!(o->inner_rtol >= 0.0) || !std::isfinite(o->inner_rtol)) { why = "inner_rtol must be finite and >= 0"; return false; }
  if (o->max_outer < 0) { why = "max_outer must be >= 0"; return false; }
  if (o->profile < 0) { why = "profile must be >= 0"; return false; }
  if (o->transpose != 0 && o->transpose != 1) { why = "transpose must be 0 or 1"; return false; }
  if (o->graph != 0 && o->graph != 1) { why = "graph must be 0 or 1"; return false; }
  if (o->persistent != 0 && o->persistent != 1) { why = "persistent must be 0 or 1"; return false; }
  return true;
}

}  // namespace

// ====================================================================== ABI

extern "C" {

void its_default_options(its_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->method = ITS_CG;
  o->restart_mode = ITS_RESTART_COSINE;
  o->rtol = 1e-8;
  o->max_iter = 10000;
  o->restart_tol = 1e-5;
  o->check_every = 0;
  o->inner_dtype = ITS_F64;
  o->inner_rtol = 1e-4;
  o->max_outer = 30;
  o->profile = 0;
  o->transpose = 0;
  o->graph = 0;
}

const char *its_status_string(int32_t st) {
  switch (st) {
    case ITS_OK: return "ITS_OK";
    case ITS_NOT_CONVERGED: return "ITS_NOT_CONVERGED";
    case ITS_BREAKDOWN: return "ITS_BREAKDOWN";
    case ITS_E_INVALID: return "ITS_E_INVALID";
    case ITS_E_HIP: return "ITS_E_HIP";
    case ITS_E_WORKSPACE: return "ITS_E_WORKSPACE";
    case ITS_E_UNSUPPORTED: return "ITS_E_UNSUPPORTED";
    default: return "unknown status";
  }
}

const char *its_last_error(void) { return g_err.c_str(); }

static its_status new_matrix(its_matrix **out) {
  its_matrix *A = new (std::nothrow) its_matrix();
  if (!A) return fail(ITS_E_INVALID, "out of host memory");
  void *p = nullptr;
  if (hipHostMalloc(&p, 3 * sizeof(State), hipHostMallocDefault) != hipSuccess) {
    delete A;
    return fail(ITS_E_HIP, "hipHostMalloc of the state snapshot failed");
  }
  A->host_state = static_cast<State *>(p);
  std::memset(A->host_state, 0, 3 * sizeof(State));
  *out = A;
  return ITS_OK;
}

its_status its_csr_create(int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col,
                          const double *val, its_matrix **out) {
  if (!out) return fail(ITS_E_INVALID, "out is null");
  *out = nullptr;
  if (n < 0 || nnz < 0) return fail(ITS_E_INVALID, "negative size");
  if (n >= (int64_t(1) << 31) - 1 || nnz >= (int64_t(1) << 31))
    return fail(ITS_E_UNSUPPORTED, "n and nnz must be below 2^31");
  if (!row_ptr || (nnz > 0 && (!col || !val))) return fail(ITS_E_INVALID, "null CSR array");
  if ((reinterpret_cast<uintptr_t>(col) | reinterpret_cast<uintptr_t>(val)) % 16)
    return fail(ITS_E_INVALID, "col and val must be 16-byte aligned");
  its_matrix *A;
  its_status s = new_matrix(&A);
  if (s != ITS_OK) return s;
  A->kind = kCsr;
  A->n = n;
  A->nnz = nnz;
  A->rp = row_ptr;
  A->col = col;
  A->val = val;
  *out = A;
  return ITS_OK;
}

its_status its_csr_create64(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                            const double *val, void *stream, its_matrix **out) {
  if (!out) return fail(ITS_E_INVALID, "out is null");
  *out = nullptr;
  if (n < 0 || nnz < 0) return fail(ITS_E_INVALID, "negative size");
  if (n >= (int64_t(1) << 31) - 1 || nnz >= (int64_t(1) << 31))
    return fail(ITS_E_UNSUPPORTED, "n and nnz must be below 2^31 to narrow the row pointers");
  if (!row_ptr || (nnz > 0 && (!col || !val))) return fail(ITS_E_INVALID, "null CSR array");
  if ((reinterpret_cast<uintptr_t>(col) | reinterpret_cast<uintptr_t>(val)) % 16)
    return fail(ITS_E_INVALID, "col and val must be 16-byte aligned");
  int32_t *rp32 = nullptr;
  uint32_t *bad = nullptr;
  HIP_TRY(hipMalloc(&rp32, sizeof(int32_t) * size_t(n + 1)));
  if (hipMalloc(&bad, sizeof(uint32_t)) != hipSuccess) {
    (void)hipFree(rp32);
    return fail(ITS_E_HIP, "device allocation failed");
  }
  hipStream_t s = S(stream);
  uint32_t hbad = 0;
  hipError_t e = hipMemsetAsync(bad, 0, sizeof(uint32_t), s);
  if (e == hipSuccess) {
    const int grid = int(std::min<int64_t>((n + 1 + kBlock - 1) / kBlock, 65536));
    hipLaunchKernelGGL(k_narrow_rp, dim3(grid), dim3(kBlock), 0, s, n + 1, nnz, row_ptr, rp32, bad);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(bad);
  if (e != hipSuccess || hbad) {
    (void)hipFree(rp32);
    if (e != hipSuccess) return fail(ITS_E_HIP, std::string("narrowing row pointers: ") + hipGetErrorString(e));
    return fail(ITS_E_INVALID, std::to_string(hbad) + " row pointers outside [0, nnz]");
  }
  its_status st = its_csr_create(n, nnz, rp32, col, val, out);
  if (st != ITS_OK) {
    (void)hipFree(rp32);
    return st;
  }
  (*out)->own_rp = rp32;  // freed by its_matrix_destroy
  return ITS_OK;
}

its_status its_stencil_create(int32_t nx, int32_t ny, int32_t nz, int32_t npts, const double *coef,
                              its_matrix **out) {
  if (!out) return fail(ITS_E_INVALID, "out is null");
  *out = nullptr;
  if (nx < 0 || ny < 0 || nz < 0) return fail(ITS_E_INVALID, "negative grid size");
  if (npts != 7 && npts != 27) return fail(ITS_E_INVALID, "npts must be 7 or 27");
  if (!coef) return fail(ITS_E_INVALID, "coef is null");
  const int64_t n = int64_t(nx) * ny * nz;
  if (n >= (int64_t(1) << 31) - 1) return fail(ITS_E_UNSUPPORTED, "grid must have < 2^31 nodes");
  for (int o = 0; o < npts; ++o)
    if (!std::isfinite(coef[o])) return fail(ITS_E_INVALID, "non-finite coefficient");
  its_matrix *A;
  its_status s = new_matrix(&A);
  if (s != ITS_OK) return s;
  A->kind = npts == 7 ? kSten7 : kSten27;
  A->n = n;
  A->nx = nx;
  A->ny = ny;
  A->nz = nz;
  for (int o = 0; o < npts; ++o) A->coef[o] = coef[o];
  *out = A;
  return ITS_OK;
}

its_status its_matrix_destroy(its_matrix *A) {
  if (!A) return ITS_OK;
  if (A->tr) its_matrix_destroy(A->tr);
  if (A->own_rp) (void)hipFree(A->own_rp);
  if (A->own_col) (void)hipFree(A->own_col);
  if (A->own_val) (void)hipFree(A->own_val);
  if (A->color_rows) (void)hipFree(A->color_rows);
  if (A->host_state) (void)hipHostFree(A->host_state);
  free_packed(A);
  drop_graph(A);
  if (A->graph.ev) (void)hipEventDestroy(A->graph.ev);
  if (A->graph.s) (void)hipStreamDestroy(A->graph.s);
  delete A;
  return ITS_OK;
}

int64_t its_matrix_rows(const its_matrix *A) { return A ? A->n : -1; }

its_status its_stencil_plan(const its_matrix *A, int32_t *plan) {
  if (!A || !plan) return fail(ITS_E_INVALID, "null argument");
  if (A->kind == kCsr) return fail(ITS_E_INVALID, "not a matrix-free operator");
  return with_op64(A, [&](auto op) -> its_status {
    if constexpr (std::is_same_v<decltype(op), VarCoefOp> ||
                  std::is_same_v<decltype(op), StencilOp<7, double>> ||
                  std::is_same_v<decltype(op), StencilOp<27, double>>) {
      plan[0] = op.nbx;
      plan[1] = op.nby;
      plan[2] = op.nbz;
      plan[3] = op.zb;
      return ITS_OK;
    } else {
      return fail(ITS_E_INVALID, "not a matrix-free operator");
    }
  });
}

its_status its_varcoef_create(int32_t nx, int32_t ny, int32_t nz, const double *k,
                              its_matrix **out) {
  if (!out) return fail(ITS_E_INVALID, "out is null");
  *out = nullptr;
  if (nx < 0 || ny < 0 || nz < 0) return fail(ITS_E_INVALID, "negative grid size");
  const int64_t n = int64_t(nx) * ny * nz;
  if (n >= (int64_t(1) << 31) - 1) return fail(ITS_E_UNSUPPORTED, "grid must have < 2^31 nodes");
  if (n > 0 && !k) return fail(ITS_E_INVALID, "k is null");
  its_matrix *A;
  its_status s = new_matrix(&A);
  if (s != ITS_OK) return s;
  A->kind = kVar7;
  A->n = n;
  A->nx = nx;
  A->ny = ny;
  A->nz = nz;
  A->kcoef = k;
  *out = A;
  return ITS_OK;
}

its_status its_varcoef_grad(const its_matrix *A, const double *x, const double *lam, double *dk,
                            void *stream) {
  if (!A || A->kind != kVar7) return fail(ITS_E_INVALID, "not a variable-coefficient operator");
  if (A->n == 0) return ITS_OK;
  if (!x || !lam || !dk) return fail(ITS_E_INVALID, "null vector");
  if (dk == x || dk == lam || dk == A->kcoef) return fail(ITS_E_INVALID, "dk aliases an input");
  VarCoefOp op{A->nx, A->ny, A->nz, int32_t(A->n), A->kcoef};
  hipLaunchKernelGGL(k_varcoef_grad, dim3(grid_for(A->n)), dim3(kBlock), 0, S(stream), op, x, lam, dk);
  HIP_TRY(hipGetLastError());
  return ITS_OK;
}

its_status its_csr_validate(its_matrix *A, int32_t need_diag, void *stream) {
  if (!A || A->kind != kCsr) return fail(ITS_E_INVALID, "not a CSR matrix");
  if (A->n == 0) return ITS_OK;
  uint32_t *bad = nullptr;
  HIP_TRY(hipMalloc(&bad, sizeof(uint32_t)));
  hipStream_t s = S(stream);
  its_status rs = ITS_OK;
  uint32_t hbad = 0;
  do {
    if (hipMemsetAsync(bad, 0, sizeof(uint32_t), s) != hipSuccess) { rs = fail(ITS_E_HIP, "memset"); break; }
    hipLaunchKernelGGL(k_csr_check, dim3(grid_for(A->n)), dim3(kBlock), 0, s, int32_t(A->n),
                       int32_t(A->nnz), A->rp, A->col, A->val, need_diag, bad);
    if (hipGetLastError() != hipSuccess) { rs = fail(ITS_E_HIP, "launch k_csr_check"); break; }
    if (hipMemcpyAsync(&hbad, bad, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) { rs = fail(ITS_E_HIP, "readback"); break; }
  } while (0);
  (void)hipFree(bad);
  if (rs != ITS_OK) return rs;
  if (need_diag) A->diag_state = hbad == 0 ? 1 : -1;
  if (hbad) return fail(ITS_E_INVALID, std::to_string(hbad) + " invalid CSR rows");
  return ITS_OK;
}

its_status its_csr_transpose(its_matrix *A, void *stream) {
  if (!A || A->kind != kCsr) return fail(ITS_E_INVALID, "not a CSR matrix");
  its_status rs = its_csr_validate(A, 0, stream);  // columns in range and ascending
  if (rs != ITS_OK) return rs;
  drop_graph(A);
  if (A->tr) {
    its_matrix_destroy(A->tr);
    A->tr = nullptr;
  }
  its_matrix *T;
  if ((rs = new_matrix(&T)) != ITS_OK) return rs;
  T->kind = kCsr;
  T->n = A->n;
  T->nnz = A->nnz;
  const int32_t n = int32_t(A->n);
  hipStream_t s = S(stream);
  int32_t *cnt = nullptr;
  do {
    if (hipMalloc(&T->own_rp, sizeof(int32_t) * size_t(n + 1)) != hipSuccess ||
        hipMalloc(&T->own_col, sizeof(int32_t) * size_t(std::max<int64_t>(A->nnz, 1))) != hipSuccess ||
        hipMalloc(&T->own_val, sizeof(double) * size_t(std::max<int64_t>(A->nnz, 1))) != hipSuccess ||
        hipMalloc(&cnt, sizeof(int32_t) * size_t(std::max(n, 1))) != hipSuccess) {
      rs = fail(ITS_E_HIP, "device allocation failed");
      break;
    }
    std::vector<int32_t> h(size_t(n) + 1, 0);
    if (n > 0) {
      if (hipMemsetAsync(cnt, 0, sizeof(int32_t) * size_t(n), s) != hipSuccess) {
        rs = fail(ITS_E_HIP, "memset");
        break;
      }
      hipLaunchKernelGGL(k_tr_count, dim3(grid_for(n)), dim3(kBlock), 0, s, n, A->rp, A->col, cnt);
      if (hipGetLastError() != hipSuccess ||
          hipMemcpyAsync(h.data() + 1, cnt, sizeof(int32_t) * size_t(n), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        rs = fail(ITS_E_HIP, "column counts");
        break;
      }
    }
    for (int32_t j = 0; j < n; ++j) h[size_t(j) + 1] += h[size_t(j)];  // row pointers of A^T
    if (hipMemcpyAsync(T->own_rp, h.data(), sizeof(int32_t) * size_t(n + 1), hipMemcpyHostToDevice, s) != hipSuccess) {
      rs = fail(ITS_E_HIP, "upload");
      break;
    }
    if (n > 0) {
      // cursors start at the row starts of A^T
      if (hipMemcpyAsync(cnt, h.data(), sizeof(int32_t) * size_t(n), hipMemcpyHostToDevice, s) != hipSuccess) {
        rs = fail(ITS_E_HIP, "upload");
        break;
      }
      hipLaunchKernelGGL(k_tr_scatter, dim3(grid_for(n)), dim3(kBlock), 0, s, n, A->rp, A->col, A->val, cnt,
                         T->own_col, T->own_val);
      hipLaunchKernelGGL(k_tr_sort, dim3(grid_for(n)), dim3(kBlock), 0, s, n, (const int32_t *)T->own_rp,
                         T->own_col, T->own_val);
      if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
        rs = fail(ITS_E_HIP, "transpose kernels");
        break;
      }
    }
  } while (0);
  if (cnt) (void)hipFree(cnt);
  if (rs != ITS_OK) {
    its_matrix_destroy(T);
    return rs;
  }
  T->rp = T->own_rp;
  T->col = T->own_col;
  T->val = T->own_val;
  // packed like A where A^T's rows fit the same max_fill (else CSR form)
  if (A->pack_fill > 0.0) (void)its_csr_pack(T, A->pack_fill, stream);
  A->tr = T;
  return ITS_OK;
}

its_status its_csr_value_grad(const its_matrix *A, const double *x, const double *lam, double *dval,
                              void *stream) {
  if (!A || A->kind != kCsr) return fail(ITS_E_INVALID, "not a CSR matrix");
  if (A->n == 0 || A->nnz == 0) return ITS_OK;
  if (!x || !lam || !dval) return fail(ITS_E_INVALID, "null vector");
  if (dval == A->val) return fail(ITS_E_INVALID, "dval aliases the matrix values");
  hipLaunchKernelGGL(k_csr_value_grad, dim3(grid_for(A->n)), dim3(kBlock), 0, S(stream), int32_t(A->n),
                     A->rp, A->col, x, lam, dval);
  HIP_TRY(hipGetLastError());
  return ITS_OK;
}

its_status its_csr_set_lowp(its_matrix *A, const void *val_lo, int32_t dtype) {
  if (!A || A->kind != kCsr) return fail(ITS_E_INVALID, "not a CSR matrix");
  drop_graph(A);
  if (A->sp) return fail(ITS_E_INVALID, "set low-precision values before its_csr_pack");
  if (!val_lo && A->nnz > 0) return fail(ITS_E_INVALID, "null values");
  if (reinterpret_cast<uintptr_t>(val_lo) % 16)
    return fail(ITS_E_INVALID, "low-precision values must be 16-byte aligned");
  if (dtype == ITS_F32) A->val32 = static_cast<const float *>(val_lo);
  else if (dtype == ITS_F16) A->val16 = static_cast<const __half *>(val_lo);
  else return fail(ITS_E_INVALID, "dtype must be ITS_F32 or ITS_F16");
  return ITS_OK;
}

namespace {
struct DevTmp {  // device allocation freed on scope exit
  void *p = nullptr;
  ~DevTmp() {
    if (p) (void)hipFree(p);
  }
};
}  // namespace

// Packs rows rows[0 .. count) (all rows in order when rows is null) of a CSR
// matrix into the sliced layout; lowp also packs the low-precision values.
// On success the new arrays are returned in out (owned by the caller).
struct PackOut {
  int64_t *sp = nullptr;
  int32_t *col = nullptr;
  double *val = nullptr;
  float *val32 = nullptr;
  __half *val16 = nullptr;
  int32_t *soff = nullptr;
  uint64_t *smask = nullptr;
  int64_t slots = 0;
  int32_t wmax = 0;
  int64_t col_slots = 0;
  void release() {
    if (sp) (void)hipFree(sp);
    if (col) (void)hipFree(col);
    if (val) (void)hipFree(val);
    if (val32) (void)hipFree(val32);
    if (val16) (void)hipFree(val16);
    if (soff) (void)hipFree(soff);
    if (smask) (void)hipFree(smask);
    *this = PackOut();
  }
};

static its_status pack_rows(const its_matrix *A, const int32_t *rows, int64_t count, double max_fill,
                            bool lowp, hipStream_t s, PackOut &out) {
  const int64_t ns = (count + kSlice - 1) / kSlice;
  if (count == 0) return ITS_OK;
  DevTmp width, bad;
  HIP_TRY(hipMalloc(&width.p, size_t(ns) * sizeof(int32_t)));
  HIP_TRY(hipMalloc(&bad.p, sizeof(uint32_t)));
  HIP_TRY(hipMemsetAsync(bad.p, 0, sizeof(uint32_t), s));
  const int gw = int(std::min<int64_t>((ns + kBlock - 1) / kBlock, 65536));
  hipLaunchKernelGGL(k_sell_width, dim3(gw), dim3(kBlock), 0, s, int32_t(count), int32_t(A->nnz), A->rp,
                     rows, static_cast<int32_t *>(width.p), static_cast<uint32_t *>(bad.p));
  HIP_TRY(hipGetLastError());
  std::vector<int32_t> hw(static_cast<size_t>(ns));
  uint32_t hbad = 0;
  HIP_TRY(hipMemcpyAsync(hw.data(), width.p, size_t(ns) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&hbad, bad.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (hbad) return fail(ITS_E_INVALID, std::to_string(hbad) + " rows with invalid row pointers");
  std::vector<int64_t> hsp(static_cast<size_t>(ns) + 1, 0);
  for (int64_t q = 0; q < ns; ++q) hsp[size_t(q) + 1] = hsp[size_t(q)] + int64_t(kSlice) * hw[size_t(q)];
  const int64_t total = hsp[size_t(ns)];
  // slots of the real rows (the positions past count in the last slice do
  // not count) against the entries of those rows
  int64_t row_slots = 0;
  for (int64_t q = 0; q < ns; ++q) row_slots += std::min<int64_t>(kSlice, count - q * kSlice) * hw[size_t(q)];
  int64_t entries = A->nnz;
  if (rows) {
    entries = 0;  // the rows' own entries: the widths bound them from above
    std::vector<int32_t> hr(static_cast<size_t>(count));
    std::vector<int32_t> hrp(static_cast<size_t>(A->n) + 1);
    HIP_TRY(hipMemcpyAsync(hr.data(), rows, size_t(count) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hrp.data(), A->rp, size_t(A->n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int32_t i : hr) entries += hrp[size_t(i) + 1] - hrp[size_t(i)];
  }
  if (double(row_slots) > max_fill * double(entries) + kSlice)
    return fail(ITS_E_UNSUPPORTED, "row lengths vary too much: the packed rows would hold " +
                                       std::to_string(row_slots) + " slots for " +
                                       std::to_string(entries) + " entries");
  PackOut P;
  hipError_t e = hipMalloc(&P.sp, size_t(ns + 1) * sizeof(int64_t));
  const int64_t cols = total / kSlice;  // entry positions over all slices
  if (e == hipSuccess && total > 0) e = hipMalloc(&P.soff, size_t(cols) * sizeof(int32_t));
  if (e == hipSuccess && total > 0) e = hipMalloc(&P.smask, size_t(cols) * sizeof(uint64_t));
  if (e == hipSuccess && total > 0) e = hipMalloc(&P.val, size_t(total) * sizeof(double));
  if (e == hipSuccess && total > 0 && lowp && A->val32) e = hipMalloc(&P.val32, size_t(total) * sizeof(float));
  if (e == hipSuccess && total > 0 && lowp && A->val16) e = hipMalloc(&P.val16, size_t(total) * sizeof(__half));
  if (e == hipSuccess)
    e = hipMemcpyAsync(P.sp, hsp.data(), size_t(ns + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s);
  const int32_t ci = int32_t(count);
  if (e == hipSuccess && total > 0) {
    // offset slices, then columns for the slices that keep them
    DevTmp nslots;
    unsigned long long hslots = 0;
    e = hipMalloc(&nslots.p, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemsetAsync(nslots.p, 0, sizeof(unsigned long long), s);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_sell_offsets, dim3(gw), dim3(kBlock), 0, s, ci, A->rp, rows, A->col, P.sp,
                         P.soff, P.smask, static_cast<unsigned long long *>(nslots.p));
      e = hipGetLastError();
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(&hslots, nslots.p, sizeof(hslots), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    P.col_slots = int64_t(hslots);
    // columns are addressed by slot, so any explicit slice needs the full array
    if (e == hipSuccess && P.col_slots > 0) e = hipMalloc(&P.col, size_t(total) * sizeof(int32_t));
  }
  if (e == hipSuccess && total > 0) {
    const int gs = int(std::min<int64_t>((ns * kSlice + kBlock - 1) / kBlock, 65536));
    hipLaunchKernelGGL(k_sell_scatter<double>, dim3(gs), dim3(kBlock), 0, s, ci, A->rp, rows, A->col,
                       A->val, (const int64_t *)P.sp, (const int32_t *)P.soff, P.col, P.val);
    if (P.val32)
      hipLaunchKernelGGL(k_sell_scatter<float>, dim3(gs), dim3(kBlock), 0, s, ci, A->rp, rows, A->col,
                         A->val32, (const int64_t *)P.sp, (const int32_t *)P.soff, (int32_t *)nullptr,
                         P.val32);
    if (P.val16)
      hipLaunchKernelGGL(k_sell_scatter<__half>, dim3(gs), dim3(kBlock), 0, s, ci, A->rp, rows, A->col,
                         A->val16, (const int64_t *)P.sp, (const int32_t *)P.soff, (int32_t *)nullptr,
                         P.val16);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    P.release();
    return fail(ITS_E_HIP, std::string("packing: ") + hipGetErrorString(e));
  }
  P.slots = total;
  for (int32_t w : hw) P.wmax = std::max(P.wmax, w);
  out = P;
  return ITS_OK;
}

// Packs each colour's rows for the Gauss-Seidel half-sweeps; a colour that
// would exceed the fill bound leaves every colour on the CSR arrays.
static its_status pack_colors(its_matrix *A, hipStream_t s) {
  drop_graph(A);
  free_color_packs(A);
  if (A->ncolors == 0 || A->pack_fill == 0.0) return ITS_OK;
  std::vector<its_matrix::ColorPack> packs;
  for (int32_t c = 0; c < A->ncolors; ++c) {
    const int32_t beg = A->color_off[size_t(c)], cnt = A->color_off[size_t(c) + 1] - beg;
    PackOut P;
    its_status st = pack_rows(A, A->color_rows + beg, cnt, A->pack_fill, false, s, P);
    if (st != ITS_OK) {
      for (auto &q : packs) {
        if (q.sp) (void)hipFree(q.sp);
        if (q.col) (void)hipFree(q.col);
        if (q.val) (void)hipFree(q.val);
        if (q.soff) (void)hipFree(q.soff);
        if (q.smask) (void)hipFree(q.smask);
      }
      if (st == ITS_E_UNSUPPORTED) {
        g_err.clear();
        return ITS_OK;
      }
      return st;
    }
    its_matrix::ColorPack cp;
    cp.sp = P.sp;
    cp.col = P.col;
    cp.val = P.val;
    cp.soff = P.soff;
    cp.smask = P.smask;
    packs.push_back(cp);
  }
  A->cpack = packs;
  return ITS_OK;
}

its_status its_csr_pack(its_matrix *A, double max_fill, void *stream) {
  if (!A || A->kind != kCsr) return fail(ITS_E_INVALID, "not a CSR matrix");
  if (!(max_fill >= 1.0) || !std::isfinite(max_fill))
    return fail(ITS_E_INVALID, "max_fill must be finite and >= 1");
  free_packed(A);
  if (A->n == 0) return ITS_OK;
  hipStream_t s = S(stream);
  PackOut P;
  its_status st = pack_rows(A, nullptr, A->n, max_fill, true, s, P);
  if (st != ITS_OK) return st;
  A->sp = P.sp;
  A->scol = P.col;
  A->sval = P.val;
  A->sval32 = P.val32;
  A->sval16 = P.val16;
  A->soff = P.soff;
  A->smask = P.smask;
  A->sell_entries = P.slots;
  A->sell_col_slots = P.col_slots;
  A->sell_wmax = P.wmax;
  A->pack_fill = max_fill;
  // A^T alike where its rows fit max_fill (else it stays in CSR form)
  if (A->tr) (void)its_csr_pack(A->tr, max_fill, stream);
  return pack_colors(A, s);
}

int64_t its_csr_packed_slots(const its_matrix *A) { return A && A->sp ? A->sell_entries : 0; }

int64_t its_csr_packed_column_slots(const its_matrix *A) {
  return A && A->sp ? A->sell_col_slots : 0;
}

its_status its_csr_set_colors(its_matrix *A, const uint8_t *color, int32_t ncolors, void *stream) {
  if (!A || A->kind != kCsr) return fail(ITS_E_INVALID, "not a CSR matrix");
  if (ncolors < 1 || ncolors > 255) return fail(ITS_E_INVALID, "ncolors must be in 1..255");
  if (!color && A->n > 0) return fail(ITS_E_INVALID, "color is null");
  hipStream_t s = S(stream);
  const int64_t n = A->n;
  std::vector<uint8_t> hc(static_cast<size_t>(n));
  if (n > 0) {
    uint32_t *bad = nullptr;
    HIP_TRY(hipMalloc(&bad, sizeof(uint32_t)));
    uint32_t hbad = 0;
    hipError_t e = hipMemsetAsync(bad, 0, sizeof(uint32_t), s);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_color_check, dim3(grid_for(n)), dim3(kBlock), 0, s, int32_t(n), A->rp,
                         A->col, color, ncolors, bad);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hc.data(), color, size_t(n), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(bad);
    if (e != hipSuccess) return fail(ITS_E_HIP, std::string("colour check: ") + hipGetErrorString(e));
    if (hbad) return fail(ITS_E_INVALID, std::to_string(hbad) + " rows violate the colouring");
  }
  // group rows by colour (counting sort, ascending rows within a colour)
  std::vector<int32_t> off(static_cast<size_t>(ncolors) + 1, 0);
  std::vector<int32_t> rows(static_cast<size_t>(n));
  for (int64_t i = 0; i < n; ++i) off[hc[size_t(i)] + 1]++;
  for (int c = 0; c < ncolors; ++c) off[c + 1] += off[c];
  std::vector<int32_t> pos(off.begin(), off.end() - 1);
  for (int64_t i = 0; i < n; ++i) rows[size_t(pos[hc[size_t(i)]]++)] = int32_t(i);
  int32_t *d = nullptr;
  if (n > 0) {
    HIP_TRY(hipMalloc(&d, size_t(n) * sizeof(int32_t)));
    if (hipMemcpy(d, rows.data(), size_t(n) * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(d);
      return fail(ITS_E_HIP, "upload of colour rows failed");
    }
  }
  if (A->color_rows) (void)hipFree(A->color_rows);
  A->color_rows = d;
  A->color_off = off;
  A->ncolors = ncolors;
  return pack_colors(A, s);
}

its_status its_spmv(const its_matrix *A, const double *x, double *y, void *stream) {
  if (!A) return fail(ITS_E_INVALID, "A is null");
  if (A->n == 0) return ITS_OK;
  if (!x || !y) return fail(ITS_E_INVALID, "null vector");
  if (x == y) return fail(ITS_E_INVALID, "x and y alias");
  hipStream_t s = S(stream);
  its_status st = with_op64(A, [&](auto op) -> its_status {
    const int grid = op.grid();
    hipLaunchKernelGGL(k_spmv<decltype(op)>, dim3(grid), dim3(kBlock), 0, s, op, x, y);
    return ITS_OK;
  });
  if (st != ITS_OK) return st;
  HIP_TRY(hipGetLastError());
  return ITS_OK;
}

size_t its_dot_workspace_size(int64_t) { return up(sizeof(State)) + up(sizeof(Reduce)); }

its_status its_dot(int64_t n, const double *x, const double *y, double *result, void *workspace,
                   size_t ws_bytes, void *stream) {
  if (!result) return fail(ITS_E_INVALID, "result is null");
  if (n < 0) return fail(ITS_E_INVALID, "negative n");
  if (n >= (int64_t(1) << 31) - 1) return fail(ITS_E_UNSUPPORTED, "n must be below 2^31");
  if (n > 0 && (!x || !y)) return fail(ITS_E_INVALID, "null vector");
  if (!workspace || ws_bytes < its_dot_workspace_size(n))
    return fail(ITS_E_WORKSPACE, "workspace missing or too small");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
    return fail(ITS_E_WORKSPACE, "workspace must be 256-byte aligned");
  State *st = static_cast<State *>(workspace);
  Reduce *R = reinterpret_cast<Reduce *>(static_cast<char *>(workspace) + up(sizeof(State)));
  hipStream_t s = S(stream);
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(kBlock), 0, s, st, 1, R);
  const int G = grid_for(n);
  hipLaunchKernelGGL(k_dot, dim3(G), dim3(kBlock), 0, s, int32_t(n), x, y, R);
  const int nb = finish_grid(G);
  if (nb == 0) {
    hipLaunchKernelGGL((k_finish_final<1, FinDot>), dim3(1), dim3(kBlock), 0, s, R, G, 1, FinDot{st, 0});
  } else {
    hipLaunchKernelGGL(k_finish_group<1>, dim3(nb), dim3(kBlock), 0, s, R, G);
    hipLaunchKernelGGL((k_finish_final<1, FinDot>), dim3(1), dim3(kBlock), 0, s, R, nb, 2, FinDot{st, 0});
  }
  HIP_TRY(hipGetLastError());
  double v = 0.0;
  HIP_TRY(hipMemcpyAsync(&v, &st->dot[0], sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *result = v;
  return ITS_OK;
}

its_status its_workspace_size(const its_matrix *A, const its_options *o, size_t *bytes) {
  if (!A || !o || !bytes) return fail(ITS_E_INVALID, "null argument");
  std::string why;
  if (!options_ok(o, why)) return fail(ITS_E_INVALID, why);
  *bytes = layout_for(A->n, o->method, o->inner_dtype, o->persistent).total;
  return ITS_OK;
}

}  // extern "C"

// ------------------------------------------------------------ static scratch
// The workspace of its_solve_noalloc: one array per device in the code
// object's device memory, for callers that cannot allocate.  Its device
// address is looked up once per device (hipGetSymbolAddress, with that device
// current) and only that address is used by the host; the array's name here
// is a host-side stand-in.
namespace {
constexpr size_t kScratchBytes = ITS_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
__device__ __align__(256) char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

its_status scratch_for_current_device(void **out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(ITS_E_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(ITS_E_HIP, "hipGetSymbolAddress returned a null scratch address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return ITS_OK;
}
}  // namespace

// The body of its_solve and its_solve_noalloc.  cache_graph: the iteration
// loop may run as the handle's cached HIP graph (its_options.graph).
static its_status solve_impl(const its_matrix *Ac, const its_options *o, const double *b, double *x,
                             void *workspace, size_t ws_bytes, void *stream, its_result *res,
                             bool cache_graph);

extern "C" {

its_status its_solve(const its_matrix *Ac, const its_options *o, const double *b, double *x,
                     void *workspace, size_t ws_bytes, void *stream, its_result *res) {
  return solve_impl(Ac, o, b, x, workspace, ws_bytes, stream, res, true);
}

its_status its_solve_noalloc(const its_matrix *A, const its_options *o, const double *b, double *x,
                             void *stream, its_result *res) {
  if (!A || !o || !res) return fail(ITS_E_INVALID, "null argument");
  std::string why;
  if (!options_ok(o, why)) return fail(ITS_E_INVALID, why);
  if (o->graph != 0) return fail(ITS_E_UNSUPPORTED, "its_solve_noalloc does not capture graphs (graph must be 0)");
  if (o->profile != 0) return fail(ITS_E_UNSUPPORTED, "its_solve_noalloc does not profile (profile must be 0)");
  const size_t need = layout_for(A->n, o->method, o->inner_dtype, o->persistent).total;
  if (need > kScratchBytes)
    return fail(ITS_E_WORKSPACE, "its_solve_noalloc: this solve needs " + std::to_string(need) +
                                     " bytes of scratch; the static buffer holds " +
                                     std::to_string(kScratchBytes) + " (use its_solve with a workspace)");
  void *ws = nullptr;
  its_status st = scratch_for_current_device(&ws);
  if (st != ITS_OK) return st;
  return solve_impl(A, o, b, x, ws, kScratchBytes, stream, res, false);
}

}  // extern "C"

static its_status solve_impl(const its_matrix *Ac, const its_options *o, const double *b, double *x,
                             void *workspace, size_t ws_bytes, void *stream, its_result *res,
                             bool cache_graph) {
  its_matrix *A = const_cast<its_matrix *>(Ac);  // only cached validation state changes
  if (!A || !o || !res) return fail(ITS_E_INVALID, "null argument");
  // A^T: a constant stencil with its offsets reflected (entry (i, i+d) of A^T
  // is A's entry for offset -d, with the same grid truncation); the
  // variable-coefficient operator is symmetric.
  its_matrix At;
  if (o->transpose == 1 && A->kind == kCsr) {
    // A^T of a CSR matrix: the handle built by its_csr_transpose
    if (!A->tr) return fail(ITS_E_INVALID, "transposed CSR solves need its_csr_transpose first");
    if (o->method == ITS_SGS)
      return fail(ITS_E_UNSUPPORTED, "Gauss-Seidel with the transpose needs a stencil operator");
    if (o->inner_dtype != ITS_F64)
      return fail(ITS_E_UNSUPPORTED, "mixed precision with the transpose needs a stencil operator");
    A = A->tr;
  } else if (o->transpose == 1 && A->kind != kVar7) {
    At.kind = A->kind;
    At.n = A->n;
    At.nx = A->nx;
    At.ny = A->ny;
    At.nz = A->nz;
    const int np = A->kind == kSten7 ? 7 : 27;
    for (int q = 0; q < np; ++q) At.coef[q] = A->coef[np - 1 - q];
    At.diag_state = A->diag_state;
    At.host_state = A->host_state;
    A = &At;
  }
  std::string why;
  if (!options_ok(o, why)) return fail(ITS_E_INVALID, why);
  if (A->n > 0 && (!b || !x)) return fail(ITS_E_INVALID, "null vector");
  if (A->n > 0 && b == x) return fail(ITS_E_INVALID, "b and x alias");
  const Layout L = layout_for(A->n, o->method, o->inner_dtype, o->persistent);
  if (!workspace || ws_bytes < L.total) return fail(ITS_E_WORKSPACE, "workspace missing or too small");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
    return fail(ITS_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (o->persistent && !((o->method == ITS_CG && o->inner_dtype == ITS_F64) || o->method == ITS_CG_NB ||
                         o->method == ITS_BICGSTAB))
    return fail(ITS_E_UNSUPPORTED, "persistent is for FP64 CG, CG-NB and BiCGStab");
  if ((o->method == ITS_SGS) && A->kind == kCsr && A->ncolors == 0)
    return fail(ITS_E_INVALID, "Gauss-Seidel on CSR needs its_csr_set_colors");
  std::memset(res, 0, sizeof(*res));
  if (A->n == 0) {
    res->status = ITS_OK;
    return ITS_OK;
  }
  Run run;
  run.s = S(stream);
  run.prof.every = o->profile;
  run.prof.res = res;
  // the iteration loops run as a cached HIP graph (eagerly when profiling);
  // the key lists what the captured launches depend on
  its_matrix *owner = const_cast<its_matrix *>(Ac);
  run.gc = (o->graph == 1 && cache_graph) ? &owner->graph : nullptr;
  if (run.gc) {
    uint64_t rt;
    std::memcpy(&rt, &o->restart_tol, sizeof(rt));
    run.key = {uint64_t(o->method), uint64_t(o->inner_dtype), uint64_t(o->restart_mode), rt,
               uint64_t(o->transpose), uint64_t(reinterpret_cast<uintptr_t>(Ac)),
               uint64_t(reinterpret_cast<uintptr_t>(A->sp)), uint64_t(A->cpack.size()),
               uint64_t(reinterpret_cast<uintptr_t>(A->color_rows)), uint64_t(A->kind),
               uint64_t(reinterpret_cast<uintptr_t>(b)), uint64_t(reinterpret_cast<uintptr_t>(x)),
               uint64_t(reinterpret_cast<uintptr_t>(workspace)), uint64_t(A->n),
               uint64_t(reinterpret_cast<uintptr_t>(A->val32)),
               uint64_t(reinterpret_cast<uintptr_t>(A->val16))};
    for (int q = 0; q < 27; ++q) {
      uint64_t c;
      std::memcpy(&c, &A->coef[q], sizeof(c));
      run.key.push_back(c);
    }
  }
  const WS w = carve(workspace, L, A->n);
  if (o->method == ITS_JACOBI || o->method == ITS_SGS) {
    its_status s = check_diag(run, A, w);
    if (s != ITS_OK) return s;
    if (A->diag_state < 0) return fail(ITS_E_INVALID, "a row lacks a nonzero diagonal entry");
  }
  its_status s;
  switch (o->method) {
    case ITS_CG:
      s = o->inner_dtype == ITS_F64 ? solve_cg(run, A, o, b, x, w, res) : solve_ir(run, A, o, b, x, w, res);
      break;
    case ITS_BICGSTAB: s = solve_bicgstab(run, A, o, b, x, w, res); break;
    case ITS_CG_NB: s = solve_cgnb(run, A, o, b, x, w, res); break;
    case ITS_JACOBI: s = solve_jacobi(run, A, o, b, x, w, res); break;
    default: s = solve_sgs(run, A, o, b, x, w, res); break;
  }
  if (s != ITS_OK) return s;
  return static_cast<its_status>(res->status);
}

extern "C" {

its_status its_cast_values(const double *src, void *dst, int32_t dtype, int64_t count, void *stream) {
  if (count < 0) return fail(ITS_E_INVALID, "negative count");
  if (count == 0) return ITS_OK;
  if (!src || !dst) return fail(ITS_E_INVALID, "null pointer");
  const int grid = int(std::min<int64_t>((count + kBlock - 1) / kBlock, 65536));
  hipStream_t s = S(stream);
  if (dtype == ITS_F32)
    hipLaunchKernelGGL(k_cast_f32, dim3(grid), dim3(kBlock), 0, s, count, src, static_cast<float *>(dst));
  else if (dtype == ITS_F16)
    hipLaunchKernelGGL(k_cast_f16, dim3(grid), dim3(kBlock), 0, s, count, src, static_cast<_Float16 *>(dst));
  else
    return fail(ITS_E_INVALID, "dtype must be ITS_F32 or ITS_F16");
  HIP_TRY(hipGetLastError());
  return ITS_OK;
}

its_status its_stream_copy(const double *src, double *dst, int64_t n, void *stream) {
  if (n < 0) return fail(ITS_E_INVALID, "negative n");
  if (n == 0) return ITS_OK;
  if (!src || !dst) return fail(ITS_E_INVALID, "null pointer");
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16)
    return fail(ITS_E_INVALID, "copy buffers must be 16-byte aligned");
  const int grid = int(std::min<int64_t>((n / 2 + kBlock - 1) / kBlock + 1, int64_t(1) << 20));
  hipLaunchKernelGGL(k_copy, dim3(grid), dim3(kBlock), 0, S(stream), n, src, dst);
  HIP_TRY(hipGetLastError());
  return ITS_OK;
}

}  // extern "C"
