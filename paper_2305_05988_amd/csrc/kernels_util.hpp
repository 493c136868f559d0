// Utilities: value casts, the streaming copy probe, structure checks.
#pragma once

#include "common.hpp"

namespace its {

// ----------------------------------------------------------------- utilities

__global__ void __launch_bounds__(kBlock) k_cast_f32(int64_t n, const double *src, float *dst) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    dst[i] = float(src[i]);
}

// double -> IEEE half in one rounding (nearest-even), no float intermediate
__global__ void __launch_bounds__(kBlock) k_cast_f16(int64_t n, const double *src, _Float16 *dst) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    dst[i] = static_cast<_Float16>(src[i]);
}

// Streaming copy, 16 bytes per lane, non-temporal; launched with one tile
// of 256 lanes per block up to 2^20 blocks (measured: one tile per block
// streams faster than a grid-stride loop over fewer blocks).
__global__ void __launch_bounds__(kBlock) k_copy(int64_t n, const double *__restrict__ src,
                                                 double *__restrict__ dst) {
  const int64_t n2 = n / 2;
  const double2_t *s2 = reinterpret_cast<const double2_t *>(src);
  double2_t *d2 = reinterpret_cast<double2_t *>(dst);
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n2; i += stride)
    st_nt(d2 + i, ld_nt(s2 + i));
  if (blockIdx.x == 0 && threadIdx.x == 0 && (n & 1)) dst[n - 1] = src[n - 1];
}

// CSR structure check: counts bad rows into *bad.
__global__ void __launch_bounds__(kBlock) k_csr_check(int32_t n, int32_t nnz,
                                                      const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ col,
                                                      const double *__restrict__ val,
                                                      int32_t need_diag, uint32_t *bad) {
  for_rows(n, [&](int32_t i) {
    const int32_t b = rp[i], e = rp[i + 1];
    bool ok = (b <= e) && (b >= 0) && (e <= nnz) && (i != 0 || b == 0) && (i != n - 1 || e == nnz);
    bool diag = false;
    if (ok) {
      int32_t last = -1;
      for (int32_t k = b; k < e; ++k) {
        const int32_t c = col[k];
        if (c < 0 || c >= n || c <= last) ok = false;
        last = c;
        if (c == i && val[k] != 0.0) diag = true;
      }
    }
    if (!ok || (need_diag && !diag)) atomicAdd(bad, 1u);
  });
}

// Colouring check: colour in range, no off-diagonal entry couples two rows
// of the same colour.
__global__ void __launch_bounds__(kBlock) k_color_check(int32_t n, const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ col,
                                                        const uint8_t *__restrict__ color,
                                                        int32_t ncolors, uint32_t *bad) {
  for_rows(n, [&](int32_t i) {
    const int32_t ci = color[i];
    bool ok = ci < ncolors;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
      const int32_t c = col[k];
      if (c != i && color[c] == ci) ok = false;
    }
    if (!ok) atomicAdd(bad, 1u);
  });
}

}  // namespace its
