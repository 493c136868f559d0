/*
 * Reference oracle for the iterative-solver hot path (TEST INFRASTRUCTURE).
 *
 * A plain, single-threaded, obviously-correct CPU implementation of what the
 * GPU path computes, written from the paper (Martinez-Ferrer, Arslan, Beltran,
 * "Improving the performance of classical linear algebra iterative methods via
 * hybrid parallelism", JPDC 2023).  It exists only to check the GPU library:
 * tests, the smoke check and the benchmark's CPU-baseline leg may call it;
 * the product path never does.  It shares no source with the GPU library.
 *
 * Conventions shared by every function (readings of points the paper leaves
 * open are listed with each function in oracle.c):
 *   - CSR with int64 row pointers, int32 column indices, values in the row's
 *     stored order (the generators store columns ascending);
 *   - every multiply-add that the GPU fuses is written as fma();
 *   - dot products are the exact sum rounded once to double;
 *   - a solve stops when ||r_k||_2 <= rtol*||b||_2, evaluated as
 *     r.r <= (rtol*sqrt(b.b))^2, or when k reaches max_iter.
 *
 * Functions return one of the status codes below; `x` is in/out (x0 in,
 * last iterate out).  Parity unpinned: none (every function has a pin in
 * tests/test_oracle_*.py).
 */
#ifndef ORC_ORACLE_H
#define ORC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_NOT_CONVERGED = 1, ORC_BREAKDOWN = 2, ORC_E_INVALID = -1 };
enum { ORC_RESTART_COSINE = 0, ORC_RESTART_PAPER = 1 };

typedef struct {
  int32_t status;
  int32_t restarts;
  int64_t iters;        /* outer iterations (IR) or iterations */
  int64_t inner_iters;  /* IR only: total inner CG iterations */
  double rel_res;       /* recursive ||r_k|| / ||b|| at exit */
  double true_rel_res;  /* ||b - A x|| / ||b|| recomputed at exit */
} orc_result;

double orc_dot(int64_t n, const double *x, const double *y);
double orc_dot_f32(int64_t n, const float *x, const float *y);

void orc_spmv(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
              const double *x, double *y);
void orc_spmv_f32(int64_t n, const int64_t *rp, const int32_t *col, const float *val,
                  const float *x, float *y);

int orc_jacobi(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
               const double *b, double *x, double rtol, int64_t max_iter, orc_result *res);
int orc_sgs(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
            const uint8_t *color, int32_t ncolors, const double *b, double *x, double rtol,
            int64_t max_iter, orc_result *res);
int orc_cg(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
           const double *b, double *x, double rtol, int64_t max_iter, orc_result *res);
int orc_cgnb(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
             const double *b, double *x, double rtol, int64_t max_iter, orc_result *res);
int orc_bicgstab(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
                 const double *b, double *x, double rtol, int64_t max_iter,
                 double restart_tol, int32_t restart_mode, orc_result *res);
int orc_ir_cg(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
              const float *val_lo, const double *b, double *x, double rtol,
              int64_t max_iter, double inner_rtol, int64_t max_outer, orc_result *res);

int orc_lu_solve(int64_t n, double *a, double *b);

/* variable-coefficient diffusion: CSR assembly (returns nnz; arrays sized for
   the 7-point structure) and the adjoint gradient with respect to k */
int64_t orc_varcoef_csr(int32_t nx, int32_t ny, int32_t nz, const double *k, int64_t *rp,
                        int32_t *col, double *val);
void orc_varcoef_grad(int32_t nx, int32_t ny, int32_t nz, const double *k, const double *x,
                      const double *lam, double *dk);

#ifdef __cplusplus
}
#endif
#endif
