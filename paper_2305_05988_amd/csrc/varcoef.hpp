// Variable-coefficient 7-point diffusion operator, matrix-free from a
// per-cell coefficient array, and the gradient of a loss with respect to
// those coefficients (see rowops.hpp for the row-sweep contract).
#pragma once

#include "brick.hpp"
#include "rowops.hpp"

namespace its {

// Cell-centred finite volumes on nx*ny*nz (row = i + nx(j + ny k)), per-cell
// coefficient k_c > 0, homogeneous Dirichlet boundary:
//   (A x)_c = sum over the 6 faces of c of k_f (x_c - x_nbr),  x_nbr = 0
// across the boundary.  An interior face between cells a < b (row order) has
// the harmonic mean k_f = ((2 k_a) k_b) / (k_a + k_b); a boundary face has
// k_f = k_c.  The diagonal is 0 + f(z-1) + f(y-1) + f(x-1) + f(x+1) + f(y+1)
// + f(z+1) in that order, off-diagonal entries are -k_f, and the chain runs
// in ascending column order, so the operator equals the CSR matrix built
// with the same roundings bit for bit.  A is symmetric (each face value is
// formed once, from its lower cell), so it is its own transpose.
struct VarCoefOp;
template <> struct GathersPairs<VarCoefOp> : std::false_type {};

struct VarCoefOp {
  int32_t nx, ny, nz, n;
  const double *__restrict__ k;
  int32_t nbx = 0, nby = 0, nbz = 0, zb = 1;

  // the brick sweep of brick.hpp, with the coefficients staged beside the
  // vector values
  struct Smem {
    double v[kBrickSlots][kBrickPlane];
    double kc[kBrickSlots][kBrickPlane];
  };

  void plan() {
    const BrickGeom g = brick_plan(nx, ny, nz);
    nbx = g.nbx;
    nby = g.nby;
    nbz = g.nbz;
    zb = g.zb;
  }
  __host__ __device__ BrickGeom geom() const { return {nx, ny, nz, nbx, nby, nbz, zb}; }
  int grid() const { return brick_grid(geom()); }

  __device__ static __forceinline__ double face(double a, double b) {
    return (2.0 * a * b) / (a + b);
  }

  // The rows a thread owns in rows(), in the same order: body(i).
  template <class Body>
  __device__ __forceinline__ void own_rows(Body &&body) const {
    brick_own_rows(geom(), body);
  }

  template <class Load, class Value, class Body>
  __device__ __forceinline__ void rows(Smem &sm, Load &&load, Value &&value, Body &&body) const {
    using Raw = decltype(load(0));
    struct Point {
      Raw v;
      double k;
    };
    const int32_t nxy = nx * ny;
    brick_march(
        geom(), [&](int32_t r) { return Point{load(r), k[r]}; },
        [&](int slot, int q, const Point &p) {
          sm.v[slot][q] = value(p.v);
          sm.kc[slot][q] = p.k;
        },
        [&](int32_t i, bool valid, int32_t gx, int32_t gy, int32_t z, int sm1, int s0, int sp1, int c0) {
          auto entries = [&](auto &&consume) {
            if (!valid) return;
            const double kc = sm.kc[s0][c0];
            const bool in[6] = {z > 0, gy > 0, gx > 0, gx < nx - 1, gy < ny - 1, z < nz - 1};
            const double kn[6] = {sm.kc[sm1][c0],     sm.kc[s0][c0 - kBrickCols], sm.kc[s0][c0 - 1],
                                  sm.kc[s0][c0 + 1], sm.kc[s0][c0 + kBrickCols], sm.kc[sp1][c0]};
            const double xv[7] = {sm.v[sm1][c0],     sm.v[s0][c0 - kBrickCols], sm.v[s0][c0 - 1],
                                  sm.v[s0][c0],      sm.v[s0][c0 + 1],          sm.v[s0][c0 + kBrickCols],
                                  sm.v[sp1][c0]};
            double f[6];
            double diag = 0.0;
#pragma unroll
            for (int o = 0; o < 6; ++o) {
              f[o] = !in[o] ? kc : (o < 3 ? face(kn[o], kc) : face(kc, kn[o]));
              diag = diag + f[o];
            }
            if (in[0]) consume(i - nxy, -f[0], xv[0]);
            if (in[1]) consume(i - nx, -f[1], xv[1]);
            if (in[2]) consume(i - 1, -f[2], xv[2]);
            consume(i, diag, xv[3]);
            if (in[3]) consume(i + 1, -f[3], xv[4]);
            if (in[4]) consume(i + nx, -f[4], xv[5]);
            if (in[5]) consume(i + nxy, -f[5], xv[6]);
          };
          auto own = [&]() -> double { return sm.v[s0][c0]; };
          body(i, valid, entries, own);
        });
  }
};

// dL/dk for A(k) x = b given x and the adjoint lam (A lam = dL/dx): face f of
// c with neighbour m contributes (dk_f/dk_c (lam_c - lam_m)) (x_c - x_m),
// dk_f/dk_c = ((2 k_m) k_m) / ((k_c + k_m)(k_c + k_m)); a boundary face
// contributes lam_c x_c; dk_c = -(0 + contributions in face order
// z-1, y-1, x-1, x+1, y+1, z+1).
__global__ void __launch_bounds__(kBlock) k_varcoef_grad(VarCoefOp A, const double *__restrict__ x,
                                                         const double *__restrict__ lam,
                                                         double *__restrict__ dk) {
  const int32_t nx = A.nx, ny = A.ny, nz = A.nz, nxy = nx * ny;
  for_rows(A.n, [&](int32_t i) {
    const int32_t t = i / nx, ix = i - t * nx, iz = t / ny, iy = t - iz * ny;
    const bool in[6] = {iz > 0, iy > 0, ix > 0, ix < nx - 1, iy < ny - 1, iz < nz - 1};
    const int32_t off[6] = {-nxy, -nx, -1, 1, nx, nxy};
    // unconditional gathers (outside the grid: the cell itself, unused)
    double km[6], xm[6], lm[6];
#pragma unroll
    for (int o = 0; o < 6; ++o) {
      const int32_t m = in[o] ? i + off[o] : i;
      km[o] = A.k[m];
      xm[o] = x[m];
      lm[o] = lam[m];
    }
    const double kc = A.k[i], xc = x[i], lc = lam[i];
    double acc = 0.0;
#pragma unroll
    for (int o = 0; o < 6; ++o) {
      double term;
      if (in[o]) {
        const double s = kc + km[o];
        const double d = (2.0 * km[o] * km[o]) / (s * s);
        term = (d * (lc - lm[o])) * (xc - xm[o]);
      } else {
        term = lc * xc;
      }
      acc = acc + term;
    }
    dk[i] = -acc;
  });
}

}  // namespace its
