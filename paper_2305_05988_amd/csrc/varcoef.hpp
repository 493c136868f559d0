// Variable-coefficient 7-point diffusion operator, matrix-free from a
// per-cell coefficient array, and the gradient of a loss with respect to
// those coefficients (see rowops.hpp for the row-sweep contract).
#pragma once

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
struct VarCoefOp {
  int32_t nx, ny, nz, n;
  const double *__restrict__ k;
  int32_t nbx = 0, nby = 0, nbz = 0, zb = 1;

  static constexpr int kTX = 64, kTY = kBlock / 64;
  static constexpr int kCols = kTX + 2, kTileRows = kTY + 2, kPlane = kCols * kTileRows;
  static constexpr int kSlots = 4;
  struct Smem {
    double v[kSlots][kPlane];
    double kc[kSlots][kPlane];
  };

  void plan() {
    nbx = (nx + kTX - 1) / kTX;
    nby = (ny + kTY - 1) / kTY;
    const int64_t nxy = int64_t(nbx) * nby;
    int64_t chunks = nxy > 0 ? (2048 + nxy - 1) / nxy : 1;
    if (chunks > nz) chunks = nz;
    if (chunks < 1) chunks = 1;
    zb = int32_t((nz + chunks - 1) / chunks);
    if (zb < 1) zb = 1;
    nbz = (nz + zb - 1) / zb;
  }
  int grid() const {
    int64_t b = int64_t(nbx) * nby * nbz;
    if (b < 1) b = 1;
    int g = int(b < kMaxGrid ? b : kMaxGrid);
    if (g >= 64) g -= g % kXcds;
    return g;
  }

  __device__ static __forceinline__ double face(double a, double b) {
    return (2.0 * a * b) / (a + b);
  }

  // The rows a thread owns in rows(), in the same order: body(i).
  template <class Body>
  __device__ __forceinline__ void own_rows(Body &&body) const {
    const int64_t nbricks = int64_t(nbx) * nby * nbz;
    const Sched sc = my_tiles(nbricks);
    const int t = threadIdx.x, lane = t & 63, wy = t >> 6;
    const int32_t nxy = nx * ny;
    for (int64_t bi = sc.begin; bi < sc.end; bi += sc.stride) {
      const int32_t bx = int32_t(bi % nbx), by = int32_t((bi / nbx) % nby);
      const int32_t bz = int32_t(bi / (int64_t(nbx) * nby));
      const int32_t gx = bx * kTX + lane, gy = by * kTY + wy;
      if (gx >= nx || gy >= ny) continue;
      const int32_t z0 = bz * zb, z1 = min(nz, z0 + zb);
      for (int32_t z = z0; z < z1; ++z) body(gx + nx * gy + nxy * z);
    }
  }

  // The 2.5-D sweep of the constant stencil, with the coefficients staged
  // beside the vector values.
  template <class Load, class Value, class Body>
  __device__ __forceinline__ void rows(Smem &sm, Load &&load, Value &&value, Body &&body) const {
    using Raw = decltype(load(0));
    constexpr int kPer = (kPlane + kBlock - 1) / kBlock;
    const int64_t nbricks = int64_t(nbx) * nby * nbz;
    const Sched sc = my_tiles(nbricks);
    const int t = threadIdx.x, lane = t & 63, wy = t >> 6;
    const int32_t nxy = nx * ny;
    for (int64_t bi = sc.begin; bi < sc.end; bi += sc.stride) {
      const int32_t bx = int32_t(bi % nbx), by = int32_t((bi / nbx) % nby);
      const int32_t bz = int32_t(bi / (int64_t(nbx) * nby));
      const int32_t x0 = bx * kTX, y0 = by * kTY, z0 = bz * zb, z1 = min(nz, z0 + zb);
      auto tile_row = [&](int q, int32_t z) -> int32_t {
        const int32_t gy = y0 - 1 + q / kCols, gx = x0 - 1 + q % kCols;
        if (q >= kPlane || z < 0 || z >= nz || gx < 0 || gx >= nx || gy < 0 || gy >= ny) return -1;
        return gx + nx * gy + nxy * z;
      };
      Raw rv[kPer];
      double rk[kPer];
      auto issue = [&](int32_t z) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
          const int32_t r = tile_row(t + u * kBlock, z);
          const int32_t rr = r >= 0 ? r : 0;
          rv[u] = load(rr);
          rk[u] = k[rr];
        }
      };
      auto put = [&](int32_t z) {
        double *dv = sm.v[z & (kSlots - 1)];
        double *dk = sm.kc[z & (kSlots - 1)];
#pragma unroll
        for (int u = 0; u < kPer; ++u)
          if (t + u * kBlock < kPlane) {
            dv[t + u * kBlock] = value(rv[u]);
            dk[t + u * kBlock] = rk[u];
          }
      };
      for (int32_t z = max(z0 - 1, 0); z <= min(z0 + 1, nz - 1); ++z) {
        issue(z);
        put(z);
      }
      __syncthreads();
      const int32_t gx = x0 + lane, gy = y0 + wy;
      const bool valid = gx < nx && gy < ny;
      const int c0 = (wy + 1) * kCols + lane + 1;
      for (int32_t z = z0; z < z1; ++z) {
        const int32_t zn = z + 2;
        const bool pf = zn <= z1 && zn < nz;
        if (pf) issue(zn);
        const int sm1 = (z - 1) & (kSlots - 1), s0 = z & (kSlots - 1), sp1 = (z + 1) & (kSlots - 1);
        const int32_t i = gx + nx * gy + nxy * z;
        auto entries = [&](auto &&consume) {
          if (!valid) return;
          const double kc = sm.kc[s0][c0];
          const bool in[6] = {z > 0, gy > 0, gx > 0, gx < nx - 1, gy < ny - 1, z < nz - 1};
          const double kn[6] = {sm.kc[sm1][c0], sm.kc[s0][c0 - kCols], sm.kc[s0][c0 - 1],
                                sm.kc[s0][c0 + 1], sm.kc[s0][c0 + kCols], sm.kc[sp1][c0]};
          const double xv[7] = {sm.v[sm1][c0], sm.v[s0][c0 - kCols], sm.v[s0][c0 - 1], sm.v[s0][c0],
                                sm.v[s0][c0 + 1], sm.v[s0][c0 + kCols], sm.v[sp1][c0]};
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
        if (pf) put(zn);
        __syncthreads();
      }
    }
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
