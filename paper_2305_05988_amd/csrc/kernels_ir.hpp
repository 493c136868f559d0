// Mixed-precision iterative refinement: outer scaling and update kernels.
#pragma once

#include "common.hpp"

namespace its {

// ------------------------------------------------- mixed-precision refinement
// Outer step: rh = (float)(r/rn), d = 0, rh.rh; then (after the inner CG)
// x += rn * d in double.

// rh is the first member of the inner {r, p} pairs (stride 2).
__global__ void __launch_bounds__(kBlock) k_ir_scale(int32_t n, const double *__restrict__ r,
                                                     float *__restrict__ rh, float *__restrict__ d,
                                                     Reduce *R, double rn) {
  Dot2 a;
  for_rows(n, [&](int32_t i) {
    const float v = float(r[i] / rn);
    rh[2 * int64_t(i)] = v;
    d[i] = 0.0f;
    a.add(double(v), double(v));
  });
  DD v[1] = {a.get()};
  block_partial<1>(v, R);
}

__global__ void __launch_bounds__(kBlock) k_ir_update(int32_t n, double *__restrict__ x,
                                                      const float *__restrict__ d, double rn) {
  for_rows(n, [&](int32_t i) { st_nt(x + i, fma(rn, double(ld_nt(d + i)), ld_nt(x + i))); });
}

}  // namespace its
