/*
 * itsolve: iterative sparse solvers for MI355X (gfx950), C ABI.
 *
 * Solves A x = b for a sparse A, by Jacobi, symmetric Gauss-Seidel, conjugate
 * gradient or BiCGStab, to a relative-residual tolerance within a maximum
 * iteration count -- the problem statement of Martinez-Ferrer, Arslan and
 * Beltran, "Improving the performance of classical linear algebra iterative
 * methods via hybrid parallelism" (JPDC 2023), Section 3.1.  A is given in
 * CSR (the format of the HPCCG code the paper builds on, Section 3.2) or as
 * a constant-coefficient 7- or 27-point stencil on a structured 3-D grid (the
 * paper's two sparsity patterns, Section 3.1).
 *
 * Conventions for every entry point:
 *  - Device pointers are HIP device memory on the current device; "host"
 *    marks host pointers.  The caller allocates and owns all device memory;
 *    matrix handles borrow the caller's arrays (which must outlive the
 *    handle), and compute calls allocate no device memory.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Work is ordered on
 *    it; calls that fill a host result return after their work completed.
 *  - Vectors are contiguous float64 arrays of length n (the matrix's rows).
 *  - Errors are negative its_status values and are reported before any
 *    device work, leaving outputs untouched; its_last_error() gives a
 *    message.  Positive values are solver outcomes, not errors.
 *  - A handle or workspace may be used by one call at a time.
 */
#ifndef ITSOLVE_H
#define ITSOLVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct its_matrix its_matrix; /* opaque matrix handle */

typedef enum {
  ITS_OK = 0,            /* converged: ||b - A x|| (recursive) <= rtol ||b|| */
  ITS_NOT_CONVERGED = 1, /* max_iter reached; x holds the last iterate */
  ITS_BREAKDOWN = 2,     /* a solver denominator vanished or became non-finite */
  ITS_E_INVALID = -1,    /* invalid argument (null, size, NaN/Inf in b, ...) */
  ITS_E_HIP = -2,        /* a HIP runtime call failed */
  ITS_E_WORKSPACE = -3,  /* workspace missing or too small */
  ITS_E_UNSUPPORTED = -4 /* valid request this build does not support */
} its_status;

typedef enum { ITS_JACOBI = 0, ITS_SGS = 1, ITS_CG = 2, ITS_BICGSTAB = 3, ITS_CG_NB = 4 } its_method;
typedef enum { ITS_F64 = 0, ITS_F32 = 1, ITS_F16 = 2 } its_dtype;
typedef enum { ITS_RESTART_COSINE = 0, ITS_RESTART_PAPER = 1 } its_restart_mode;

/* Solver options.  Use its_default_options() and change fields. */
typedef struct {
  int32_t method;       /* its_method */
  int32_t restart_mode; /* BiCGStab restart test (Algorithm 2; see its_solve) */
  double rtol;          /* relative residual tolerance, >= 0 */
  int64_t max_iter;     /* iteration cap (IR: cap on total inner iterations) */
  double restart_tol;   /* BiCGStab restart threshold (paper: 1e-5) */
  int32_t check_every;  /* host polls the device status every this many
                           iterations; 0 = automatic */
  int32_t inner_dtype;  /* CG only.  ITS_F64: plain FP64 CG.  ITS_F32/ITS_F16:
                           mixed-precision iterative refinement whose inner CG
                           uses the matrix's low-precision values of that type
                           (its_csr_set_lowp) and FP32 vectors */
  double inner_rtol;    /* IR: relative tolerance of each inner solve */
  int64_t max_outer;    /* IR: cap on refinement steps */
  int32_t profile;      /* 0: off.  k >= 1: time every k-th launch of each
                           kernel class with HIP events on the stream and
                           report the timed launches in its_result */
  int32_t transpose;    /* 1: solve A^T x = b (stencil operators: offsets
                           reflected; variable-coefficient diffusion is
                           symmetric; CSR: the transpose built by
                           its_csr_transpose, ITS_E_INVALID before it, and
                           ITS_E_UNSUPPORTED with Gauss-Seidel or mixed
                           precision).  Used for the adjoint solve of a
                           differentiable solve */
  int32_t graph;        /* 1: run the iteration loop as a HIP graph of
                           check_every iterations (captured on the first solve
                           with a given matrix, method, vectors and workspace,
                           on a stream the handle owns, then replayed; results
                           are identical to launch-by-launch).  Not with
                           profile.  0 (default): launch kernel by kernel */
  int32_t persistent;   /* CG (FP64), CG-NB and BiCGStab only (else
                           ITS_E_UNSUPPORTED).  1: the whole iteration loop
                           runs as one cooperative kernel whose co-resident
                           blocks meet at grid barriers, for small systems
                           whose iterations are bound by launch and reduction
                           latency; the reductions CG-NB and BiCGStab-B1 do
                           not wait for (Algorithms 1-2) overlap the SpMV or
                           an x update.  Same iterates bit for bit.  A barrier
                           wait is bounded (environment ITS_BARRIER_SPIN_LIMIT
                           polls, default 2^24); a wait that runs out ends
                           every block and the solve returns ITS_E_HIP.  0
                           (default): one kernel per pass */
} its_options;

#define ITS_MAX_KERNEL_CLASSES 8

typedef struct {
  int32_t status;       /* its_status */
  int32_t restarts;     /* BiCGStab restarts performed */
  int64_t iters;        /* iterations (IR: refinement steps) */
  int64_t inner_iters;  /* IR: total inner CG iterations */
  double rel_res;       /* recursive ||r_k|| / ||b|| at exit */
  double true_rel_res;  /* ||b - A x|| / ||b|| recomputed at exit */
  /* profile != 0 only: summed duration and count of the timed launches per
     kernel class (6 = finishing reductions, 7 = setup and bookkeeping).
     CG: 0 = SpMV+dot pass, 1 = update+dot pass.  BiCGStab: 0 = A p pass,
     1 = A s pass, 2 = update pass.  CG-NB: 0 = SpMV pass X, 1 = update pass
     Y.  Jacobi: 0 = sweep.  SGS: 0 = colour
     half-sweeps, 1 = residual.  IR: 0/1 = inner passes as CG, 2 = outer
     residual, 3 = outer scaling and update. */
  double kernel_ms[ITS_MAX_KERNEL_CLASSES];
  int64_t kernel_launches[ITS_MAX_KERNEL_CLASSES];
} its_result;

/* Defaults: CG, rtol 1e-8, max_iter 10000, restart COSINE with 1e-5,
   inner_dtype F64, inner_rtol 1e-4, max_outer 30. */
void its_default_options(its_options *opts /* host, out */);

/* ---------------------------------------------------------------- matrices */

/* CSR matrix (Section 3.2).  row_ptr: n+1 int32 (row_ptr[0] = 0,
   nondecreasing, row_ptr[n] = nnz); col: nnz int32 in [0, n); val: nnz
   float64.  Rows are applied in stored order (store columns ascending).
   All three are device pointers, borrowed; col and val 16-byte aligned
   (fresh device allocations are).  Requires nnz < 2^31.
   Structure is not validated here (use its_csr_validate). */
its_status its_csr_create(int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col,
                          const double *val, its_matrix **out /* host, out */);

/* The same CSR matrix with 64-bit row pointers (Section 3.2's CSR, for
   callers whose index type is int64).  row_ptr: n+1 int64, device; it is
   narrowed on the device, at this call, into an int32 copy that the handle
   owns (4 (n+1) bytes, freed by its_matrix_destroy), so row_ptr may be freed
   afterwards.  col, val: as its_csr_create (borrowed).  Errors:
   ITS_E_UNSUPPORTED when n or nnz is 2^31 or more; ITS_E_INVALID when a row
   pointer lies outside [0, nnz] (the other structure checks are
   its_csr_validate's).  Synchronises `stream`. */
its_status its_csr_create64(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                            const double *val, void *stream, its_matrix **out /* host, out */);

/* Checks a CSR matrix on the device: row_ptr monotone and in range, columns
   in range and strictly ascending within each row.  If need_diag, every row
   must also hold a nonzero diagonal entry (Jacobi, Gauss-Seidel).
   Returns ITS_OK or ITS_E_INVALID. */
its_status its_csr_validate(its_matrix *A, int32_t need_diag, void *stream);

/* Attaches low-precision copies of the CSR values (same structure) for the
   mixed-precision CG: dtype ITS_F32 (float) or ITS_F16 (IEEE half).  Device
   pointer, borrowed, 16-byte aligned.  One array per dtype may be attached.
   ITS_E_INVALID once the matrix is packed (its_csr_pack). */
its_status its_csr_set_lowp(its_matrix *A, const void *val_lo, int32_t dtype);

/* Packs a CSR matrix into the library's device layout for the streaming
   passes: sliced ELLPACK, one slice per 64 consecutive rows, slice width =
   its longest row, column -1 in the slots past a row's end; within a slice
   each row's entries are kept in consecutive pairs (entries 2c and 2c+1 of
   the 64 rows form one contiguous run of 64 pairs; an odd width ends with
   single entries; the FP32 and FP16 copies use runs of four entries per row,
   then a pair and a single for the rest).  Every row keeps its stored entry order, so results are
   bit-identical to the unpacked matrix; the layout spares the row pointers
   and lets each wavefront read two entries of its 64 rows with one
   coalesced access (the SpMV of Sections 3.1-3.2).  A slice whose rows have
   strictly ascending columns and take their column offsets (column - row)
   from one list as long as the slice width stores no column indices at
   all: one offset and one 64-lane mask per entry position replace them, and
   each row's entries sit at the positions of their offsets.  Matrices from
   structured grids (stencils written as CSR) pack entirely this way, which
   cuts the bytes per FP64 entry from 12 to 8.
   The packed copy (col, val and any low-precision values attached with
   its_csr_set_lowp, which must come first) is allocated and owned by the
   handle and freed by its_matrix_destroy or the next its_csr_pack; it is a
   snapshot, so pack again after changing the values.  Solves and its_spmv
   use it when present; with a colouring set (its_csr_set_colors) each
   colour's rows are packed the same way for Gauss-Seidel's sweeps, and a
   transpose built with its_csr_transpose is packed too, each where it fits
   max_fill (else it keeps its CSR arrays).
   Padding slots are streamed like entries, so packing pays only for nearly
   uniform row lengths: max_fill (>= 1) bounds the slots of the rows, the sum
   over slices of (rows in the slice) x (slice width), by
   max_fill * nnz + 64.  Synchronises `stream`.  Errors: ITS_E_INVALID for
   row pointers out of order or range or a bad max_fill; ITS_E_UNSUPPORTED
   (matrix left unpacked) when the bound is exceeded. */
its_status its_csr_pack(its_matrix *A, double max_fill, void *stream);

/* Builds A^T for transposed solves (its_options.transpose = 1): validates A
   (as its_csr_validate without the diagonal requirement), then forms A^T in
   CSR with the rows of each column in ascending order -- unique, so A^T's
   rows chain exactly as the CSR rows of the transposed matrix -- in device
   memory the handle owns (n + 1 + nnz int32, nnz float64; freed by
   its_matrix_destroy or the next call).  If A is packed (now or later), A^T
   is packed with the same max_fill where its rows fit it (else it stays in
   CSR form).  Needed for the adjoint of a nonsymmetric CSR solve
   (the paper's problem statement solves A x = b; this is its adjoint).
   Synchronises `stream`. */
its_status its_csr_transpose(its_matrix *A, void *stream);

/* Gradient of a loss L(x) with respect to the stored values of a CSR
   matrix, where A x = b and lam solves A^T lam = dL/dx (the adjoint solve):
   dval[k] = -(lam_i x_j) for stored entry k = (i, j).  x, lam: n float64;
   dval: nnz float64 in A's value order; device, dval must not alias A's
   values.  A's structure as its_csr_create requires.  Enqueued on `stream`,
   not synchronised. */
its_status its_csr_value_grad(const its_matrix *A, const double *x, const double *lam, double *dval,
                              void *stream);

/* Slots of the packed layout (entries plus padding), 0 if not packed. */
int64_t its_csr_packed_slots(const its_matrix *A);

/* Slots of the packed layout that store a column index (those of the slices
   that are not offset slices, see its_csr_pack); 0 if not packed or if
   every slice is an offset slice. */
int64_t its_csr_packed_column_slots(const its_matrix *A);

/* Point colouring for symmetric Gauss-Seidel on a CSR matrix (Section 3.4:
   colours, red-black without rotation).  color: n uint8 (device) with values
   < ncolors; each colour must be an independent set (no row couples to a
   row of its own colour) -- checked here, ITS_E_INVALID otherwise.  The
   handle keeps per-colour row lists in device memory it allocates and frees
   in its_matrix_destroy. */
its_status its_csr_set_colors(its_matrix *A, const uint8_t *color, int32_t ncolors, void *stream);

/* Matrix-free constant-coefficient stencil on an nx*ny*nz grid: the 7- and
   27-point centred stencils on a structured hexahedral mesh that give the
   paper's two sparsity levels (Section 3.1, with the element counts per row
   of its touched-elements estimate).  Rows numbered i + nx*(j + ny*k),
   neighbours outside the grid omitted (Dirichlet).  npts = 7 or 27.  coef (host, copied): one value per offset
   in ascending column order -- 7-point: (k-1, j-1, i-1, centre, i+1, j+1,
   k+1); 27-point: dk outer, dj, di inner, each -1..1.  Gauss-Seidel uses the
   red-black colouring (i+j+k) mod 2 for 7 points and the 8 colours
   (i mod 2) + 2 (j mod 2) + 4 (k mod 2) for 27 points.  Requires
   nx*ny*nz < 2^31. */
its_status its_stencil_create(int32_t nx, int32_t ny, int32_t nz, int32_t npts,
                              const double *coef, its_matrix **out /* host, out */);

/* Variable-coefficient diffusion (not in the paper, whose matrices are
   constant stencils; the operator of the differentiable solve): cell-centred
   finite volumes on nx*ny*nz (rows i + nx(j + ny k)), homogeneous Dirichlet
   boundary, (A x)_c = sum over the 6 faces of c of k_f (x_c - x_nbr) with
   x_nbr = 0 across the boundary; an interior face between rows a < b has
   k_f = ((2 k_a) k_b) / (k_a + k_b), a boundary face k_f = k_c.  Diagonal
   0 + f(z-1) + f(y-1) + f(x-1) + f(x+1) + f(y+1) + f(z+1) in that order,
   off-diagonal entries -k_f.  A is symmetric positive definite for k > 0.
   k: n float64, device, borrowed, positive and finite (not checked).
   Jacobi, CG, CG-NB and BiCGStab apply; Gauss-Seidel and mixed precision
   return ITS_E_UNSUPPORTED. */
its_status its_varcoef_create(int32_t nx, int32_t ny, int32_t nz, const double *k,
                              its_matrix **out /* host, out */);

/* Gradient of a loss L(x) with respect to the per-cell coefficients of a
   variable-coefficient operator, where A(k) x = b and lam solves
   A lam = dL/dx (the adjoint solve; A is symmetric):
     dk_c = -sum over faces f of c of dk_f/dk_c (lam_c - lam_m)(x_c - x_m),
   dk_f/dk_c = ((2 k_m) k_m) / ((k_c + k_m)(k_c + k_m)), a boundary face
   contributing lam_c x_c; terms added from 0 in the face order above, then
   negated.  (dL/db = lam.)  x, lam, dk: n float64, device; dk must not alias
   the inputs.  Enqueued on `stream`, not synchronised. */
its_status its_varcoef_grad(const its_matrix *A, const double *x, const double *lam, double *dk,
                            void *stream);

its_status its_matrix_destroy(its_matrix *A);
int64_t its_matrix_rows(const its_matrix *A);

/* Brick plan of a matrix-free operator's SpMV sweep (the 7- and 27-point
   stencils of Section 3.1 and the variable-coefficient operator): plan (host,
   4 int32, out) = x tiles of 64 points, y tiles of 4 points, z chunks, and
   the z planes per chunk (the last chunk may hold fewer).  A block marches
   one (x tile, y tile, z chunk) brick plane by plane.  Depends only on the
   grid; ITS_E_INVALID for a CSR matrix. */
its_status its_stencil_plan(const its_matrix *A, int32_t *plan);

/* ----------------------------------------------------------------- kernels */

/* y = A x: the sparse matrix-vector product that each method of Section 3.1
   applies once (CG, Jacobi) or twice (BiCGStab, Algorithm 2) per iteration.
   Each row is a fused multiply-add chain over its entries in stored
   (ascending column) order starting from +0.  x, y: device, length n, not
   aliased.  Errors: ITS_E_INVALID for a null handle or vector, or x == y. */
its_status its_spmv(const its_matrix *A, const double *x, double *y, void *stream);

/* Dot product (the paper's scalar products): the sum of x_i*y_i computed
   with error-free transformations (double-double accumulation) and rounded
   once.  Its error is at most half an ulp of the result plus about
   n * 2^-104 * sum|x_i y_i|, so it is the correctly rounded value unless the
   sum cancels to near a rounding boundary (r.r never does).  result: host.
   workspace: device, at least its_dot_workspace_size(n) bytes. */
size_t its_dot_workspace_size(int64_t n);
its_status its_dot(int64_t n, const double *x, const double *y, double *result, void *workspace,
                   size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------- solve */

/* Device workspace in bytes needed by its_solve for this matrix/options:
   the vectors the chosen method keeps besides x and b (the r, p, q, ... of
   Algorithms 1-2 and their classical counterparts, Section 3.1), the device
   State blocks and the reduction partials of its dot products. */
its_status its_workspace_size(const its_matrix *A, const its_options *opts, size_t *bytes);

/* Solves A x = b.  b: device, n.  x: device, n, in = x0, out = solution.
   Stops when ||r_k||_2 <= rtol ||b||_2 (the paper's test is absolute;
   Algorithms 1-2) or after max_iter iterations.  b = 0 returns x = 0.
   Methods (Section 3.1):
     ITS_JACOBI   x_{k+1} = D^{-1}(b - (A - D) x_k), undamped;
     ITS_SGS      symmetric Gauss-Seidel: colours forward then backward;
     ITS_CG       classical CG (Hestenes-Stiefel), or mixed-precision IR;
     ITS_BICGSTAB BiCGStab with the arithmetic of Algorithm 2 and its
                  restart: COSINE restarts when |r.r'| < restart_tol ||r||,
                  PAPER when sqrt(|r.r'|) < restart_tol;
     ITS_CG_NB    the paper's nonblocking CG (Algorithm 1): SpMV on r, A p by
                  recurrence, x updated through gamma (p_j - r_j) (added; the
                  printed minus sign is a typo).
   Returns ITS_OK / ITS_NOT_CONVERGED / ITS_BREAKDOWN with res filled and x
   holding the returned iterate, or a negative error with x untouched.
   res: host, out. */
its_status its_solve(const its_matrix *A, const its_options *opts, const double *b, double *x,
                     void *workspace, size_t ws_bytes, void *stream, its_result *res);

/* Bytes of the static device scratch of its_solve_noalloc (per device). */
#define ITS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* its_solve for callers that cannot allocate device memory (code under HIP
   graph capture, tight serving loops, harnesses that forbid hipMalloc): the
   same solve, bit for bit, with its workspace (the device State blocks, the
   reduction partials and the method's vectors, its_workspace_size bytes) in
   a static device array of ITS_NOALLOC_SCRATCH_BYTES that the library holds
   on every device it runs on until the process ends.  No device memory is
   allocated or freed by this call.  Limits: its_workspace_size for the
   matrix and options must not exceed ITS_NOALLOC_SCRATCH_BYTES
   (ITS_E_WORKSPACE otherwise: for FP64 CG about 2.7M rows, BiCGStab 1.1M,
   Jacobi 8M); opts->graph and opts->profile must be 0 (ITS_E_UNSUPPORTED:
   both would create HIP objects).  Every call on one device shares that
   device's array, so calls that overlap on one device (concurrent streams
   or threads) race and must be serialised by the caller; each call
   initialises the scratch it reads, so nothing carries over between calls.
   Other arguments, results and errors as its_solve. */
its_status its_solve_noalloc(const its_matrix *A, const its_options *opts, const double *b, double *x,
                             void *stream, its_result *res);

/* --------------------------------------------------------------- utilities */

/* dst[i] = src[i] rounded to nearest-even in dtype (ITS_F32 or ITS_F16):
   builds low-precision matrix values for its_csr_set_lowp. */
its_status its_cast_values(const double *src, void *dst, int32_t dtype, int64_t count, void *stream);

/* dst = src, a streaming copy of n float64: the bandwidth probe against
   which HBM traffic counters are calibrated. */
its_status its_stream_copy(const double *src, double *dst, int64_t n, void *stream);

const char *its_status_string(int32_t status);
const char *its_last_error(void); /* message of this thread's last error */

/* ------------------------------------------------------------ batched solve
   Many independent variable-coefficient diffusion systems (the operator of
   its_varcoef_create), each with nrhs right-hand sides, solved by FP64 CG per
   (system, right-hand side) and advanced together.  The paper's experiments
   solve one large system per run; the batch is this library's analogue of
   choosing the task granularity (Section 4.2): on the first solve an
   autotuner picks how many z planes one brick of the SpMV pass covers and
   how many tiles one work item of the update passes covers, by timing each
   pass over the candidates (4, 8, 16, 32 and 64 for both).  Each (system, rhs) follows exactly the arithmetic of the
   single-system CG (the same iterates, bit for bit) and stops on its own
   test; m = check_every iterations (default 64) are captured in one HIP
   graph that is replayed until every (system, rhs) has stopped.

   Layout: the systems' cells are concatenated in system order; vectors
   interleave the right-hand sides, value (cell g, rhs r) at g * nrhs + r. */
typedef struct its_batch its_batch;

typedef struct {
  int32_t status;          /* ITS_OK if every (system, rhs) converged, else
                              ITS_BREAKDOWN if any broke down, else
                              ITS_NOT_CONVERGED */
  int32_t tiles_per_item;  /* tiles per work item of the update passes (the
                              autotuner's choice, or the fixed one) */
  int32_t graph_iters;     /* m */
  int32_t planes_per_brick; /* z planes per brick of the SpMV pass (the
                               autotuner's choice, or the fixed one) */
  int64_t max_iters;       /* largest iteration count over (system, rhs) */
  int64_t replays;         /* graph launches */
  double tune_ms;          /* time of the autotuning (first solve) */
  double solve_ms;         /* wall time of this solve */
} its_batch_result;

/* dims: host, 3 * nsys values (nx, ny, nz per system, each >= 1).  k: device,
   the systems' per-cell coefficients concatenated (positive, finite); read
   once here to form each cell's diagonal and upper face coefficients (same
   roundings as its_varcoef_create; a lower face's coefficient is the
   neighbour's upper one, 32 bytes per cell in all) into memory the handle
   owns, so k may be freed after.
   nrhs: 1, 2, 4 or 8 (else ITS_E_UNSUPPORTED; so is a system with nx * ny
   >= 2^31, a batch of 2^40 or more values, or one of 2^30 or more tiles or
   one-plane bricks).  Synchronises `stream`. */
its_status its_batch_create(int32_t nsys, const int32_t *dims, const double *k, int32_t nrhs,
                            void *stream, its_batch **out /* host, out */);
its_status its_batch_destroy(its_batch *B);
/* Total cells of the batch (vectors hold cells * nrhs values); -1 if null. */
int64_t its_batch_cells(const its_batch *B);
/* Bytes of device workspace its_batch_solve needs (256-byte aligned). */
size_t its_batch_workspace_size(const its_batch *B);
/* Fixes the work schedule: tiles_per_item, the tiles of 256/nrhs cells one
   work item of the update passes covers, and planes_per_brick, the z planes
   one brick of the SpMV pass covers (0 for either: the autotuner chooses it
   at the next solve, and keeps its choice for later solves).  Results do not depend on either
   (the reductions round their exact sums).  ITS_E_INVALID for a null handle
   or a negative value.  Synchronises the handle's stream. */
its_status its_batch_set_schedule(its_batch *B, int32_t tiles_per_item, int32_t planes_per_brick);
/* Solves every (system, rhs) with FP64 CG (opts: method ITS_CG, inner_dtype
   ITS_F64, rtol, max_iter per (system, rhs), check_every = m).  b, x: device,
   cells * nrhs float64 (x: x0 in, solution out); b = 0 for a (system, rhs)
   gives x = 0.  iters, status: optional host arrays of nsys * nrhs entries
   (index s * nrhs + r) for the per-(system, rhs) iteration counts and
   ITS_OK / ITS_NOT_CONVERGED / ITS_BREAKDOWN.  Runs on the handle's own
   stream, ordered after the work already on `stream`, and returns when
   done.  One solve per handle at a time. */
its_status its_batch_solve(its_batch *B, const its_options *opts, const double *b, double *x,
                           void *workspace, size_t ws_bytes, void *stream,
                           its_batch_result *res /* host, out */, int64_t *iters,
                           int32_t *status);

#ifdef __cplusplus
}
#endif
#endif /* ITSOLVE_H */
