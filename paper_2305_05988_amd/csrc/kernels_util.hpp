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

// 64-bit row pointers narrowed to 32 bits: dst[i] = src[i] for i < count,
// counting into *bad the pointers outside [0, nnz] (their copy is
// meaningless and the caller refuses the matrix).
__global__ void __launch_bounds__(kBlock) k_narrow_rp(int64_t count, int64_t nnz,
                                                      const int64_t *__restrict__ src,
                                                      int32_t *__restrict__ dst, uint32_t *bad) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < count; i += int64_t(gridDim.x) * kBlock) {
    const int64_t v = src[i];
    const bool ok = v >= 0 && v <= nnz;
    dst[i] = ok ? int32_t(v) : 0;
    if (!ok) atomicAdd(bad, 1u);
  }
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

// ------------------------------------------------------ CSR transpose
// A^T of a validated CSR matrix (columns in range and strictly ascending per
// row), built in three steps: entries per column (the row lengths of A^T),
// a scatter that places each entry in its column's range through an atomic
// cursor (in whatever order the atomics serve), and a per-row sort of A^T by
// column index, which makes the result unique: row j of A^T lists A's rows
// with an entry in column j in ascending order, as CSR requires.
__global__ void __launch_bounds__(kBlock) k_tr_count(int32_t n, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ col,
                                                     int32_t *__restrict__ cnt) {
  for_rows(n, [&](int32_t i) {
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) atomicAdd(cnt + col[k], 1);
  });
}

__global__ void __launch_bounds__(kBlock) k_tr_scatter(int32_t n, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ col,
                                                       const double *__restrict__ val,
                                                       int32_t *__restrict__ cursor,
                                                       int32_t *__restrict__ colT,
                                                       double *__restrict__ valT) {
  for_rows(n, [&](int32_t i) {
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
      const int32_t p = atomicAdd(cursor + col[k], 1);
      colT[p] = i;
      valT[p] = val[k];
    }
  });
}

// Insertion sort of each row of A^T by column (the entries are distinct).
__global__ void __launch_bounds__(kBlock) k_tr_sort(int32_t n, const int32_t *__restrict__ rpT,
                                                    int32_t *__restrict__ colT,
                                                    double *__restrict__ valT) {
  for_rows(n, [&](int32_t j) {
    const int32_t b = rpT[j], e = rpT[j + 1];
    for (int32_t k = b + 1; k < e; ++k) {
      const int32_t c = colT[k];
      const double v = valT[k];
      int32_t m = k - 1;
      while (m >= b && colT[m] > c) {
        colT[m + 1] = colT[m];
        valT[m + 1] = valT[m];
        --m;
      }
      colT[m + 1] = c;
      valT[m + 1] = v;
    }
  });
}

// Gradient of a loss with respect to the stored values of A given the
// solution x and the adjoint lam (A^T lam = dL/dx): dL/da_ij = -lam_i x_j.
__global__ void __launch_bounds__(kBlock) k_csr_value_grad(int32_t n, const int32_t *__restrict__ rp,
                                                           const int32_t *__restrict__ col,
                                                           const double *__restrict__ x,
                                                           const double *__restrict__ lam,
                                                           double *__restrict__ dval) {
  for_rows(n, [&](int32_t i) {
    const double li = lam[i];
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) dval[k] = -(li * x[col[k]]);
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
