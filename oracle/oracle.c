/*
 * Reference oracle (TEST INFRASTRUCTURE ONLY; see oracle.h).
 *
 * Plain single-threaded C99, compiled with -O2 -ffp-contract=off and no
 * fast-math, so every rounding below is the one written.  Each function cites
 * the passage of the paper it follows.  Readings of points the paper leaves
 * open or prints inconsistently are marked "Reading:".
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Exact accumulation.                                                       */
/*                                                                           */
/* The paper's scalar products (its third class of operations, Section 1;   */
/* alpha_n, alpha_d, beta, omega in Algorithms 1-2) are sums of products.  The */
/* oracle returns the exact value of that sum rounded once to double, so the */
/* result does not depend on summation order (the paper shows order-induced */
/* rounding changes BiCGStab's convergence, Section 3.3).                     */
/*                                                                           */
/* Method: Shewchuk's non-overlapping expansions (Discrete Comput. Geom.     */
/* 18, 1997): each new term is merged into a list of non-overlapping        */
/* partials by error-free two-sums; the partials are finally added from the  */
/* largest with the correction for a result lying exactly half-way between  */
/* two doubles.  A product x*y is split exactly into p + e with e computed by */
/* fma (the product error is representable unless it underflows).           */
/* ------------------------------------------------------------------------ */

#define ORC_ACC_CAP 160

typedef struct {
  double part[ORC_ACC_CAP];
  int len;
  double special; /* sum of non-finite terms (0 if none) */
} orc_acc;

static void acc_init(orc_acc *a) {
  a->len = 0;
  a->special = 0.0;
}

static void acc_add(orc_acc *a, double x) {
  int i, j = 0;
  if (!isfinite(x)) {
    a->special += x;
    return;
  }
  for (i = 0; i < a->len; i++) {
    double y = a->part[i];
    double hi, lo;
    if (fabs(x) < fabs(y)) {
      double t = x;
      x = y;
      y = t;
    }
    hi = x + y;
    if (!isfinite(hi)) { /* the running sum overflowed: result is +-inf */
      a->special += hi;
      a->len = 0;
      return;
    }
    lo = y - (hi - x);
    if (lo != 0.0) a->part[j++] = lo;
    x = hi;
  }
  if (j >= ORC_ACC_CAP) abort(); /* cannot happen for finite doubles */
  a->part[j++] = x;
  a->len = j;
}

static double acc_round(const orc_acc *a) {
  int n = a->len;
  double hi, lo = 0.0;
  if (a->special != 0.0 || a->special != a->special) return a->special;
  if (n == 0) return 0.0;
  hi = a->part[--n];
  while (n > 0) {
    double x = hi, y = a->part[--n];
    hi = x + y;
    lo = y - (hi - x);
    if (lo != 0.0) break;
  }
  /* hi is the round-to-nearest of hi+lo; if lo is exactly half an ulp the
     remaining partials decide the direction of the tie.  This final step
     (sum the partials from the top, stop at the first inexact addition, then
     correct a half-way case by the sign of the next partial) is the one of
     CPython's math.fsum (Hettinger's msum recipe built on Shewchuk's
     expansions). */
  if (n > 0 && ((lo < 0.0 && a->part[n - 1] < 0.0) || (lo > 0.0 && a->part[n - 1] > 0.0))) {
    double y = lo * 2.0;
    double x = hi + y;
    if (y == x - hi) hi = x;
  }
  return hi;
}

double orc_dot(int64_t n, const double *x, const double *y) {
  orc_acc a;
  int64_t i;
  acc_init(&a);
  for (i = 0; i < n; i++) {
    double p = x[i] * y[i];
    if (!isfinite(p)) {
      acc_add(&a, p);
      continue;
    }
    acc_add(&a, p);
    acc_add(&a, fma(x[i], y[i], -p));
  }
  return acc_round(&a);
}

/* float*float is exact in double (24+24 <= 53 significand bits). */
double orc_dot_f32(int64_t n, const float *x, const float *y) {
  orc_acc a;
  int64_t i;
  acc_init(&a);
  for (i = 0; i < n; i++) acc_add(&a, (double)x[i] * (double)y[i]);
  return acc_round(&a);
}

/* ------------------------------------------------------------------------ */
/* Sparse matrix-vector product on CSR (Section 3.2: HPCCG's CSR format;     */
/* SpMV is the dominant kernel, Section 4.2).                                 */
/* Reading: each row is a fused multiply-add chain over the stored entries,  */
/* in stored (ascending column) order, starting from +0.                     */
/* ------------------------------------------------------------------------ */

void orc_spmv(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
              const double *x, double *y) {
  int64_t i, k;
  for (i = 0; i < n; i++) {
    double acc = 0.0;
    for (k = rp[i]; k < rp[i + 1]; k++) acc = fma(val[k], x[col[k]], acc);
    y[i] = acc;
  }
}

void orc_spmv_f32(int64_t n, const int64_t *rp, const int32_t *col, const float *val,
                  const float *x, float *y) {
  int64_t i, k;
  for (i = 0; i < n; i++) {
    float acc = 0.0f;
    for (k = rp[i]; k < rp[i + 1]; k++) acc = fmaf(val[k], x[col[k]], acc);
    y[i] = acc;
  }
}

/* r = b - A x, each entry b_i minus the row's chain. */
static void residual(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
                     const double *b, const double *x, double *r) {
  int64_t i;
  orc_spmv(n, rp, col, val, x, r);
  for (i = 0; i < n; i++) r[i] = b[i] - r[i];
}

static double true_rel_res(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
                           const double *b, const double *x, double bb) {
  double *r = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double rr;
  residual(n, rp, col, val, b, x, r);
  rr = orc_dot(n, r, r);
  free(r);
  return sqrt(rr) / sqrt(bb);
}

/* Common start of every solver.  Reading of the stopping rule: the paper
   stops on the absolute test sqrt(alpha_n) < eps (Algorithms 1-2, Section
   4.1); here the test is relative, ||r|| <= rtol*||b||, evaluated without a
   square root as r.r <= thr2 with thr2 = (rtol*sqrt(b.b))^2.
   Returns 1 if the solve is already finished (invalid b, or b = 0, whose
   solution is x = 0). */
static int solve_prologue(int64_t n, const double *b, double *x, double rtol, double *bb,
                          double *thr2, orc_result *res) {
  double t;
  int64_t i;
  memset(res, 0, sizeof(*res));
  *bb = orc_dot(n, b, b);
  if (!isfinite(*bb) || !(rtol >= 0.0)) {
    res->status = ORC_E_INVALID;
    return 1;
  }
  if (*bb == 0.0) {
    for (i = 0; i < n; i++) x[i] = 0.0;
    res->status = ORC_OK;
    return 1;
  }
  t = rtol * sqrt(*bb);
  *thr2 = t * t;
  return 0;
}

/* Diagonal position of each row; 0 if every row has a nonzero diagonal. */
static int find_diag(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
                     int64_t *dpos) {
  int64_t i, k;
  for (i = 0; i < n; i++) {
    dpos[i] = -1;
    for (k = rp[i]; k < rp[i + 1]; k++)
      if (col[k] == i) dpos[i] = k;
    if (dpos[i] < 0 || val[dpos[i]] == 0.0) return -1;
  }
  return 0;
}

/* Relaxation update of row i (Section 3.1, Jacobi and Gauss-Seidel):
   x_i <- (b_i - sum_{j != i} a_ij x_j) / a_ii.  Reading: the off-diagonal
   sum is the row's fma chain with the diagonal entry skipped, followed by one
   subtraction and one IEEE division. */
static double relax_row(const int64_t *rp, const int32_t *col, const double *val,
                        const double *b, const double *x, int64_t i, int64_t dpos) {
  double s = 0.0;
  int64_t k;
  for (k = rp[i]; k < rp[i + 1]; k++)
    if (k != dpos) s = fma(val[k], x[col[k]], s);
  return (b[i] - s) / val[dpos];
}

/* ------------------------------------------------------------------------ */
/* Jacobi (Section 3.1): x_{k+1} = D^{-1} (b - (A - D) x_k), undamped        */
/* (Reading: the paper names no damping factor).  The residual of x_k is      */
/* evaluated before each sweep; the result is the first x_k that passes.      */
/* ------------------------------------------------------------------------ */
int orc_jacobi(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
               const double *b, double *x, double rtol, int64_t max_iter, orc_result *res) {
  double bb, thr2 = 0.0, rr = 0.0;
  int64_t i, k;
  int64_t *dpos;
  double *xa, *xb, *r;
  if (solve_prologue(n, b, x, rtol, &bb, &thr2, res)) return res->status;
  dpos = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  if (find_diag(n, rp, col, val, dpos)) {
    free(dpos);
    res->status = ORC_E_INVALID;
    return res->status;
  }
  xa = (double *)malloc(sizeof(double) * (size_t)n);
  xb = (double *)malloc(sizeof(double) * (size_t)n);
  r = (double *)malloc(sizeof(double) * (size_t)n);
  memcpy(xa, x, sizeof(double) * (size_t)n);
  for (k = 0;; k++) {
    double *t;
    residual(n, rp, col, val, b, xa, r);
    rr = orc_dot(n, r, r);
    if (rr <= thr2) {
      res->status = ORC_OK;
      break;
    }
    if (!isfinite(rr)) {
      res->status = ORC_BREAKDOWN;
      break;
    }
    if (k == max_iter) {
      res->status = ORC_NOT_CONVERGED;
      break;
    }
    for (i = 0; i < n; i++) xb[i] = relax_row(rp, col, val, b, xa, i, dpos[i]);
    t = xa;
    xa = xb;
    xb = t;
  }
  memcpy(x, xa, sizeof(double) * (size_t)n);
  res->iters = k;
  res->rel_res = sqrt(rr) / sqrt(bb);
  res->true_rel_res = res->rel_res;
  free(dpos);
  free(xa);
  free(xb);
  free(r);
  return res->status;
}

/* ------------------------------------------------------------------------ */
/* Symmetric Gauss-Seidel with a point colouring (Section 3.1: one forward    */
/* sweep then one backward sweep per iteration; Section 3.4: colours, with   */
/* red-black and no rotation as the configuration used).                      */
/* Reading: colours are point colours given by the caller and must be        */
/* independent sets (no row couples to a row of its own colour).  The forward */
/* sweep visits colours 0..nc-1, the backward sweep nc-1..0; within a colour  */
/* rows are updated in ascending order, in place.  Red-black is nc = 2 with   */
/* colour (i+j+k) mod 2, giving the colour order R, B, B, R.                  */
/* ------------------------------------------------------------------------ */
int orc_sgs(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
            const uint8_t *color, int32_t ncolors, const double *b, double *x, double rtol,
            int64_t max_iter, orc_result *res) {
  double bb, thr2 = 0.0, rr = 0.0;
  int64_t i, k, kk;
  int32_t c;
  int64_t *dpos;
  double *r;
  if (solve_prologue(n, b, x, rtol, &bb, &thr2, res)) return res->status;
  if (ncolors < 1 || ncolors > 255) {
    res->status = ORC_E_INVALID;
    return res->status;
  }
  for (i = 0; i < n; i++) {
    if (color[i] >= ncolors) {
      res->status = ORC_E_INVALID;
      return res->status;
    }
    for (kk = rp[i]; kk < rp[i + 1]; kk++)
      if (col[kk] != i && color[col[kk]] == color[i]) {
        res->status = ORC_E_INVALID;
        return res->status;
      }
  }
  dpos = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  if (find_diag(n, rp, col, val, dpos)) {
    free(dpos);
    res->status = ORC_E_INVALID;
    return res->status;
  }
  r = (double *)malloc(sizeof(double) * (size_t)n);
  for (k = 0;; k++) {
    residual(n, rp, col, val, b, x, r);
    rr = orc_dot(n, r, r);
    if (rr <= thr2) {
      res->status = ORC_OK;
      break;
    }
    if (!isfinite(rr)) {
      res->status = ORC_BREAKDOWN;
      break;
    }
    if (k == max_iter) {
      res->status = ORC_NOT_CONVERGED;
      break;
    }
    for (c = 0; c < ncolors; c++) /* forward sweep */
      for (i = 0; i < n; i++)
        if (color[i] == c) x[i] = relax_row(rp, col, val, b, x, i, dpos[i]);
    for (c = ncolors - 1; c >= 0; c--) /* backward sweep */
      for (i = 0; i < n; i++)
        if (color[i] == c) x[i] = relax_row(rp, col, val, b, x, i, dpos[i]);
  }
  res->iters = k;
  res->rel_res = sqrt(rr) / sqrt(bb);
  res->true_rel_res = res->rel_res;
  free(dpos);
  free(r);
  return res->status;
}

/* ------------------------------------------------------------------------ */
/* Conjugate gradient, classical Hestenes-Stiefel form (the CG that HPCCG    */
/* applies, Section 3.2; the paper's notation alpha_n = r.r and              */
/* alpha_d = (A p).p, Algorithm 1):                                           */
/*   r0 = b - A x0, p0 = r0                                                   */
/*   alpha = alpha_n / alpha_d, x += alpha p, r -= alpha A p,                 */
/*   beta = (r.r)_new / (r.r)_old, p = r + beta p.                             */
/* Reading: the returned x is the iterate whose recursive residual passed    */
/* the test (Algorithms 1-2 return one further update, an artefact of their */
/* task pipelining).  alpha_d == 0 or non-finite is a breakdown.              */
/* ------------------------------------------------------------------------ */
int orc_cg(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
           const double *b, double *x, double rtol, int64_t max_iter, orc_result *res) {
  double bb, thr2 = 0.0, rho, beta = 0.0;
  int64_t i, k;
  double *r, *p, *q;
  if (solve_prologue(n, b, x, rtol, &bb, &thr2, res)) return res->status;
  r = (double *)malloc(sizeof(double) * (size_t)n);
  p = (double *)malloc(sizeof(double) * (size_t)n);
  q = (double *)malloc(sizeof(double) * (size_t)n);
  residual(n, rp, col, val, b, x, r);
  rho = orc_dot(n, r, r);
  for (k = 0;; k++) {
    double pq, alpha, rho_new;
    if (rho <= thr2) {
      res->status = ORC_OK;
      break;
    }
    if (!isfinite(rho)) {
      res->status = ORC_BREAKDOWN;
      break;
    }
    if (k == max_iter) {
      res->status = ORC_NOT_CONVERGED;
      break;
    }
    if (k == 0)
      memcpy(p, r, sizeof(double) * (size_t)n);
    else
      for (i = 0; i < n; i++) p[i] = fma(beta, p[i], r[i]);
    orc_spmv(n, rp, col, val, p, q);
    pq = orc_dot(n, p, q);
    if (pq == 0.0 || !isfinite(pq)) {
      res->status = ORC_BREAKDOWN;
      break;
    }
    alpha = rho / pq;
    for (i = 0; i < n; i++) {
      x[i] = fma(alpha, p[i], x[i]);
      r[i] = fma(-alpha, q[i], r[i]);
    }
    rho_new = orc_dot(n, r, r);
    beta = rho_new / rho;
    rho = rho_new;
  }
  res->iters = k;
  res->rel_res = sqrt(rho) / sqrt(bb);
  res->true_rel_res = true_rel_res(n, rp, col, val, b, x, bb);
  free(r);
  free(p);
  free(q);
  return res->status;
}

/* ------------------------------------------------------------------------ */
/* CG-NB, the paper's nonblocking CG (Algorithm 1): the SpMV is applied to r  */
/* and A p is carried by the recurrence A p_j = A r_j + beta_j A p_{j-1}, so   */
/* the dot of r_j can overlap the SpMV (Section 3.1).                          */
/*   init: r0 = b - A x0, p0 = r0, (A p)0 = A r0, alpha_n = r0.r0,            */
/*         alpha_d = (A p)0.p0, alpha = alpha_n / alpha_d                      */
/*   j >= 1: r_j = r_{j-1} - alpha_{j-1} (A p)_{j-1}; alpha_n,j = r_j.r_j;     */
/*         beta = alpha_n,j / alpha_n,j-1; (A p)_j = A r_j + beta (A p)_{j-1}; */
/*         p_j = r_j + beta p_{j-1}; alpha_d,j = (A p)_j.p_j;                  */
/*         x_j = x_{j-1} + gamma (p_j - r_j),                                  */
/*         gamma = alpha_n,j-1^2 / (alpha_d,j-1 alpha_n,j)                      */
/* Readings:                                                                  */
/*  - sign: Algorithm 1 subtracts in the x update and in the final update;     */
/*    from p_j = r_j + beta_j p_{j-1} and x_j = x_{j-1} + alpha_{j-1} p_{j-1}  */
/*    the update is an addition (gamma (p_j - r_j) = alpha_{j-1} p_{j-1}).     */
/*  - the test is applied to r_j after x_j has been formed, and x_j (whose    */
/*    residual r_j is) is returned: no extra final update.                    */
/*  - the x update is the paper's three-term kernel z = a x + b y + c z with   */
/*    a = gamma, b = -gamma, c = 1: x = fma(gamma, p, fma(-gamma, r, x)).      */
/*  - alpha_d = 0 (or non-finite) is a breakdown with x unchanged.             */
/*  - if alpha_n,j = 0 exactly (exact convergence), gamma divides by zero;     */
/*    the update takes its exact value alpha_{j-1} p_{j-1}.                    */
/* ------------------------------------------------------------------------ */
int orc_cgnb(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
             const double *b, double *x, double rtol, int64_t max_iter, orc_result *res) {
  double bb, thr2 = 0.0, an, ad, alpha;
  int64_t i, k;
  double *r, *p, *ap, *w;
  if (solve_prologue(n, b, x, rtol, &bb, &thr2, res)) return res->status;
  r = (double *)malloc(sizeof(double) * (size_t)n);
  p = (double *)malloc(sizeof(double) * (size_t)n);
  ap = (double *)malloc(sizeof(double) * (size_t)n);
  w = (double *)malloc(sizeof(double) * (size_t)n);
  residual(n, rp, col, val, b, x, r);
  an = orc_dot(n, r, r);
  k = 0;
  if (an <= thr2) {
    res->status = ORC_OK;
  } else if (!isfinite(an)) {
    res->status = ORC_BREAKDOWN;
  } else if (max_iter <= 0) {
    res->status = ORC_NOT_CONVERGED;
  } else {
    memcpy(p, r, sizeof(double) * (size_t)n);
    orc_spmv(n, rp, col, val, r, ap);
    ad = orc_dot(n, ap, p);
    if (ad == 0.0 || !isfinite(ad)) {
      res->status = ORC_BREAKDOWN;
    } else {
      alpha = an / ad;
      for (k = 1;; k++) {
        double an_new, beta, gamma, ad_new;
        for (i = 0; i < n; i++) r[i] = fma(-alpha, ap[i], r[i]);
        an_new = orc_dot(n, r, r);
        beta = an_new / an;
        gamma = (an * an) / (ad * an_new);
        orc_spmv(n, rp, col, val, r, w);
        for (i = 0; i < n; i++) {
          const double p_old = p[i];
          ap[i] = fma(beta, ap[i], w[i]);
          p[i] = fma(beta, p[i], r[i]);
          if (an_new == 0.0) /* gamma = 1/0: take the exact limit alpha p_old */
            x[i] = fma(alpha, p_old, x[i]);
          else
            x[i] = fma(gamma, p[i], fma(-gamma, r[i], x[i]));
        }
        ad_new = orc_dot(n, ap, p);
        an = an_new;
        if (an <= thr2) {
          res->status = ORC_OK;
          break;
        }
        if (!isfinite(an)) {
          res->status = ORC_BREAKDOWN;
          break;
        }
        if (k == max_iter) {
          res->status = ORC_NOT_CONVERGED;
          break;
        }
        if (ad_new == 0.0 || !isfinite(ad_new)) {
          res->status = ORC_BREAKDOWN;
          break;
        }
        ad = ad_new;
        alpha = an / ad;
      }
    }
  }
  res->iters = k;
  res->rel_res = sqrt(an) / sqrt(bb);
  res->true_rel_res = true_rel_res(n, rp, col, val, b, x, bb);
  free(r);
  free(p);
  free(ap);
  free(w);
  return res->status;
}

/* ------------------------------------------------------------------------ */
/* BiCGStab with the operation list of Algorithm 2 (BiCGStab-B1), which is   */
/* arithmetically the classical method (Section 3.1), including its restart.  */
/*   init: r = b - A x, p = r, beta = r.r, r' = r/sqrt(beta), alpha_n = r.r'  */
/*   loop: v = A p, alpha_d = v.r', alpha = alpha_n/alpha_d, s = r - alpha v, */
/*         t = A s, omega = (t.s)/(t.t), x = (x + alpha p) + omega s,         */
/*         r = s - omega t, alpha_n' = r.r', beta = r.r, p' = p - omega v,     */
/*         restart ? (p = r, r' = r/sqrt(beta), alpha_n' = sqrt(beta))       */
/*                 : p = r + alpha_n'/(alpha_d omega) p'                      */
/* Readings:                                                                  */
/*  - alpha_j, used but not defined in Algorithm 2, is alpha_n/alpha_d.       */
/*  - the test uses beta = r.r at the top of each iteration (relative form). */
/*  - restart test: the paper compares sqrt(alpha_n) with 1e-5, but alpha_n  */
/*    can be negative and scales with ||r||.  COSINE mode (default) restarts  */
/*    when |r.r'| < restart_tol*||r|| (the cosine between r and the unit     */
/*    shadow r' is small), evaluated as alpha_n^2 < restart_tol^2 * beta;     */
/*    PAPER mode restarts when sqrt(|alpha_n|) < restart_tol, evaluated as    */
/*    |alpha_n| < restart_tol^2.                                              */
/*  - after a restart alpha_n = r.r'_new = sqrt(beta) exactly in exact        */
/*    arithmetic; that value is used (Algorithm 2 leaves it stale).           */
/*  - alpha_d == 0 (or non-finite) is a breakdown with x unchanged.  If       */
/*    t.t == 0 or omega == 0 the half step is kept (x += alpha p, r = s) and */
/*    the solve ends: converged if s passes the test, else a breakdown.       */
/* ------------------------------------------------------------------------ */
int orc_bicgstab(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
                 const double *b, double *x, double rtol, int64_t max_iter,
                 double restart_tol, int32_t restart_mode, orc_result *res) {
  double bb, thr2 = 0.0, beta, alpha_n, rnorm;
  int64_t i, k;
  double *r, *rs, *p, *v, *s, *t;
  if (solve_prologue(n, b, x, rtol, &bb, &thr2, res)) return res->status;
  if (!(restart_tol >= 0.0) || (restart_mode != ORC_RESTART_COSINE && restart_mode != ORC_RESTART_PAPER)) {
    res->status = ORC_E_INVALID;
    return res->status;
  }
  r = (double *)malloc(sizeof(double) * (size_t)n);
  rs = (double *)malloc(sizeof(double) * (size_t)n);
  p = (double *)malloc(sizeof(double) * (size_t)n);
  v = (double *)malloc(sizeof(double) * (size_t)n);
  s = (double *)malloc(sizeof(double) * (size_t)n);
  t = (double *)malloc(sizeof(double) * (size_t)n);
  residual(n, rp, col, val, b, x, r);
  beta = orc_dot(n, r, r);
  rnorm = sqrt(beta);
  for (i = 0; i < n; i++) {
    rs[i] = r[i] / rnorm;
    p[i] = r[i];
  }
  alpha_n = orc_dot(n, r, rs);
  for (k = 0;; k++) {
    double alpha_d, alpha, ts, tt, omega, an_new;
    int restart;
    if (beta <= thr2) {
      res->status = ORC_OK;
      break;
    }
    if (!isfinite(beta)) {
      res->status = ORC_BREAKDOWN;
      break;
    }
    if (k == max_iter) {
      res->status = ORC_NOT_CONVERGED;
      break;
    }
    orc_spmv(n, rp, col, val, p, v);
    alpha_d = orc_dot(n, v, rs);
    if (alpha_d == 0.0 || !isfinite(alpha_d)) {
      res->status = ORC_BREAKDOWN;
      break;
    }
    alpha = alpha_n / alpha_d;
    for (i = 0; i < n; i++) s[i] = fma(-alpha, v[i], r[i]);
    orc_spmv(n, rp, col, val, s, t);
    ts = orc_dot(n, t, s);
    tt = orc_dot(n, t, t);
    omega = (tt == 0.0) ? 0.0 : ts / tt;
    if (omega == 0.0) { /* keep the half step and stop */
      for (i = 0; i < n; i++) {
        x[i] = fma(alpha, p[i], x[i]);
        r[i] = s[i];
      }
      beta = orc_dot(n, r, r);
      k++;
      res->status = (beta <= thr2) ? ORC_OK : ORC_BREAKDOWN;
      break;
    }
    for (i = 0; i < n; i++) {
      x[i] = fma(omega, s[i], fma(alpha, p[i], x[i]));
      r[i] = fma(-omega, t[i], s[i]);
    }
    an_new = orc_dot(n, r, rs);
    beta = orc_dot(n, r, r);
    if (restart_mode == ORC_RESTART_COSINE)
      restart = an_new * an_new < (restart_tol * restart_tol) * beta;
    else
      restart = fabs(an_new) < restart_tol * restart_tol;
    if (restart && beta > 0.0 && isfinite(beta)) {
      rnorm = sqrt(beta);
      for (i = 0; i < n; i++) {
        p[i] = r[i];
        rs[i] = r[i] / rnorm;
      }
      alpha_n = rnorm;
      res->restarts++;
    } else {
      double bet = an_new / (alpha_d * omega);
      for (i = 0; i < n; i++) p[i] = fma(bet, fma(-omega, v[i], p[i]), r[i]);
      alpha_n = an_new;
    }
  }
  res->iters = k;
  res->rel_res = sqrt(beta) / sqrt(bb);
  res->true_rel_res = true_rel_res(n, rp, col, val, b, x, bb);
  free(r);
  free(rs);
  free(p);
  free(v);
  free(s);
  free(t);
  return res->status;
}

/* ------------------------------------------------------------------------ */
/* Mixed-precision iterative refinement around CG.  Not in the paper (it is  */
/* FP64 throughout, Section 4.1); the outer loop is classical iterative      */
/* refinement, the inner solve is the CG above on FP32 vectors.               */
/*   outer (FP64): r = b - A x, test, rn = ||r||, rh = (float)(r/rn),         */
/*                 inner solve A_lo d = rh, x = x + rn*d                      */
/*   inner (FP32 vectors and stored values, FP32 fma chains and updates;      */
/*          dot products exact and rounded to double, scalars in double and  */
/*          rounded to float where they scale a vector)                       */
/* val_lo holds the low-precision stored values (FP32, or FP16 values widened */
/* exactly to FP32).  The inner solve stops when its residual falls below     */
/* inner_rtol times its initial norm; max_iter caps the total number of inner */
/* iterations and max_outer the number of outer corrections.                  */
/* ------------------------------------------------------------------------ */
int orc_ir_cg(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
              const float *val_lo, const double *b, double *x, double rtol,
              int64_t max_iter, double inner_rtol, int64_t max_outer, orc_result *res) {
  double bb, thr2 = 0.0, rho = 0.0;
  int64_t i, outer, inner_total = 0;
  double *r;
  float *ri, *d, *p, *q;
  if (solve_prologue(n, b, x, rtol, &bb, &thr2, res)) return res->status;
  if (!(inner_rtol >= 0.0) || max_outer < 0) {
    res->status = ORC_E_INVALID;
    return res->status;
  }
  r = (double *)malloc(sizeof(double) * (size_t)n);
  ri = (float *)malloc(sizeof(float) * (size_t)n);
  d = (float *)malloc(sizeof(float) * (size_t)n);
  p = (float *)malloc(sizeof(float) * (size_t)n);
  q = (float *)malloc(sizeof(float) * (size_t)n);
  for (outer = 0;; outer++) {
    double rn, rho_i, ithr, ithr2;
    float beta32 = 0.0f;
    int64_t j;
    int broke = 0;
    residual(n, rp, col, val, b, x, r);
    rho = orc_dot(n, r, r);
    if (rho <= thr2) {
      res->status = ORC_OK;
      break;
    }
    if (!isfinite(rho)) {
      res->status = ORC_BREAKDOWN;
      break;
    }
    if (outer == max_outer || inner_total >= max_iter) {
      res->status = ORC_NOT_CONVERGED;
      break;
    }
    rn = sqrt(rho);
    for (i = 0; i < n; i++) {
      ri[i] = (float)(r[i] / rn);
      d[i] = 0.0f;
    }
    rho_i = orc_dot_f32(n, ri, ri);
    ithr = inner_rtol * sqrt(rho_i);
    ithr2 = ithr * ithr;
    for (j = 0;; j++) {
      double pq, alpha, rho_new;
      float a32;
      if (rho_i <= ithr2 || inner_total >= max_iter) break;
      if (j == 0)
        memcpy(p, ri, sizeof(float) * (size_t)n);
      else
        for (i = 0; i < n; i++) p[i] = fmaf(beta32, p[i], ri[i]);
      orc_spmv_f32(n, rp, col, val_lo, p, q);
      pq = orc_dot_f32(n, p, q);
      if (pq == 0.0 || !isfinite(pq)) {
        broke = 1;
        break;
      }
      alpha = rho_i / pq;
      a32 = (float)alpha;
      for (i = 0; i < n; i++) {
        d[i] = fmaf(a32, p[i], d[i]);
        ri[i] = fmaf(-a32, q[i], ri[i]);
      }
      rho_new = orc_dot_f32(n, ri, ri);
      beta32 = (float)(rho_new / rho_i);
      rho_i = rho_new;
      inner_total++;
    }
    if (broke) {
      res->status = ORC_BREAKDOWN;
      break;
    }
    for (i = 0; i < n; i++) x[i] = fma(rn, (double)d[i], x[i]);
  }
  res->iters = outer;
  res->inner_iters = inner_total;
  res->rel_res = sqrt(rho) / sqrt(bb);
  res->true_rel_res = res->rel_res;
  free(r);
  free(ri);
  free(d);
  free(p);
  free(q);
  return res->status;
}

/* ------------------------------------------------------------------------ */
/* Dense LU with partial pivoting (textbook Gaussian elimination), solving   */
/* a x = b in place (b is overwritten by x, a by its factors).  Used only to */
/* pin the iterative solvers on tiny grids.                                   */
/* ------------------------------------------------------------------------ */
int orc_lu_solve(int64_t n, double *a, double *b) {
  int64_t i, j, k;
  for (k = 0; k < n; k++) {
    int64_t piv = k;
    double amax = fabs(a[k * n + k]);
    for (i = k + 1; i < n; i++)
      if (fabs(a[i * n + k]) > amax) {
        amax = fabs(a[i * n + k]);
        piv = i;
      }
    if (amax == 0.0) return ORC_E_INVALID;
    if (piv != k) {
      for (j = 0; j < n; j++) {
        double t = a[k * n + j];
        a[k * n + j] = a[piv * n + j];
        a[piv * n + j] = t;
      }
      {
        double t = b[k];
        b[k] = b[piv];
        b[piv] = t;
      }
    }
    for (i = k + 1; i < n; i++) {
      double l = a[i * n + k] / a[k * n + k];
      a[i * n + k] = l;
      for (j = k + 1; j < n; j++) a[i * n + j] -= l * a[k * n + j];
      b[i] -= l * b[k];
    }
  }
  for (i = n - 1; i >= 0; i--) {
    double s = b[i];
    for (j = i + 1; j < n; j++) s -= a[i * n + j] * b[j];
    b[i] = s / a[i * n + i];
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Variable-coefficient diffusion (not in the paper, which uses constant     */
/* stencils; it is the operator of the differentiable solve).                */
/*                                                                           */
/* Cell-centred finite volumes on nx*ny*nz, row i + nx(j + ny k), per-cell   */
/* coefficient k_c > 0, homogeneous Dirichlet boundary:                      */
/*   (A x)_c = sum over the 6 faces f of c of k_f (x_c - x_nbr),            */
/* with x_nbr = 0 across the boundary.  An interior face between cells a and */
/* b (a the lower row index) has the harmonic mean k_f = 2 k_a k_b/(k_a+k_b) */
/* (flux continuity across two half-cells).  Reading: a boundary face has    */
/* k_f = k_c (a ghost cell with the same coefficient), so k = 1 gives the   */
/* (6, -1) Laplacian.  Roundings fixed here and matched by the GPU:          */
/*   face:  ((2 a) b) / (a + b), a the lower-index cell;                     */
/*   diagonal: 0 + f(z-1) + f(y-1) + f(x-1) + f(x+1) + f(y+1) + f(z+1),     */
/*             left to right, boundary faces included;                       */
/*   off-diagonal entry: -f; entries in ascending column order.             */
/* ------------------------------------------------------------------------ */
static double orc_face(double a, double b) { return (2.0 * a * b) / (a + b); }

int64_t orc_varcoef_csr(int32_t nx, int32_t ny, int32_t nz, const double *k, int64_t *rp,
                        int32_t *col, double *val) {
  const int64_t nxy = (int64_t)nx * ny, n = nxy * nz;
  int64_t i, at = 0;
  for (i = 0; i < n; i++) {
    const int64_t ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    /* faces in the order z-1, y-1, x-1, x+1, y+1, z+1 */
    const int64_t off[6] = {-nxy, -nx, -1, 1, nx, nxy};
    const int in[6] = {iz > 0, iy > 0, ix > 0, ix < nx - 1, iy < ny - 1, iz < nz - 1};
    double f[6], diag = 0.0;
    int o;
    for (o = 0; o < 6; o++) {
      if (!in[o])
        f[o] = k[i];
      else if (off[o] < 0)
        f[o] = orc_face(k[i + off[o]], k[i]);
      else
        f[o] = orc_face(k[i], k[i + off[o]]);
      diag = diag + f[o];
    }
    rp[i] = at;
    for (o = 0; o < 3; o++)
      if (in[o]) {
        col[at] = (int32_t)(i + off[o]);
        val[at++] = -f[o];
      }
    col[at] = (int32_t)i;
    val[at++] = diag;
    for (o = 3; o < 6; o++)
      if (in[o]) {
        col[at] = (int32_t)(i + off[o]);
        val[at++] = -f[o];
      }
  }
  rp[n] = at;
  return at;
}

/* Gradient of L(x(k)) with respect to k where A(k) x = b and lam solves     */
/* A^T lam = dL/dx (A is symmetric): dL/dk_c = -lam^T (dA/dk_c) x.  Face f of */
/* c with neighbour m contributes dk_f/dk_c (lam_c - lam_m)(x_c - x_m), with  */
/* dk_f/dk_c = 2 k_m^2/(k_c + k_m)^2; a boundary face (k_f = k_c, lam_m =     */
/* x_m = 0) contributes lam_c x_c.  Roundings (matched by the GPU):           */
/*   dk_f/dk_c = ((2 k_m) k_m) / ((k_c + k_m)(k_c + k_m));                    */
/*   term = (dk_f/dk_c (lam_c - lam_m)) (x_c - x_m);                          */
/*   dk_c = -(0 + term(z-1) + ... + term(z+1)), faces in the order above.     */
void orc_varcoef_grad(int32_t nx, int32_t ny, int32_t nz, const double *k, const double *x,
                      const double *lam, double *dk) {
  const int64_t nxy = (int64_t)nx * ny, n = nxy * nz;
  int64_t i;
  for (i = 0; i < n; i++) {
    const int64_t ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    const int64_t off[6] = {-nxy, -nx, -1, 1, nx, nxy};
    const int in[6] = {iz > 0, iy > 0, ix > 0, ix < nx - 1, iy < ny - 1, iz < nz - 1};
    double acc = 0.0;
    int o;
    for (o = 0; o < 6; o++) {
      double term;
      if (!in[o]) {
        term = lam[i] * x[i];
      } else {
        const int64_t m = i + off[o];
        const double s = k[i] + k[m];
        const double d = (2.0 * k[m] * k[m]) / (s * s);
        term = (d * (lam[i] - lam[m])) * (x[i] - x[m]);
      }
      acc = acc + term;
    }
    dk[i] = -acc;
  }
}
