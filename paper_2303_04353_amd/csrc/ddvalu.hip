// Plain software double-double GEMM on the FP64 vector units: the "FP64x2
// arithmetic" triple loop the cascade is measured against (Sec. 5.2), tiled
// for the GPU.  Every output entry runs exactly the sequence
//   acc = 0; for p = 0..k-1: acc = dd_add(acc, dd_mul(a_ip, b_pj)); C = dd_add(C, acc)
// so results do not depend on the tiling.
//
// A workgroup of 256 threads owns a 64x64 tile of C; each thread owns a 4x4
// micro-tile (rows ty + 16*ii, columns tx + 16*jj).  Tiles of op(A) and op(B)
// (hi and lo, 16 inner indices at a time) are staged through LDS.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dd_device.hpp"
#include "kernels.hpp"

namespace ddk {

namespace {
constexpr int kT = 64;   // tile of C
constexpr int kK = 16;   // inner indices per LDS stage
}

__global__ void __launch_bounds__(256)
dd_valu_kernel(int64_t m, int64_t n, int64_t k,
               const double* __restrict__ Ahi, const double* __restrict__ Alo, int64_t a_si, int64_t a_sp,
               const double* __restrict__ Bhi, const double* __restrict__ Blo, int64_t b_sp, int64_t b_sj,
               double* __restrict__ Chi, double* __restrict__ Clo, int64_t ldc, int64_t tiles_n) {
  __shared__ double sAh[kK][kT + 1], sAl[kK][kT + 1];
  __shared__ double sBh[kK][kT + 1], sBl[kK][kT + 1];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int64_t tm = (int64_t)blockIdx.x / tiles_n;
  const int64_t tn = (int64_t)blockIdx.x - tm * tiles_n;
  const int64_t row0 = tm * kT, col0 = tn * kT;

  double acc_h[4][4], acc_l[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc_h[i][j] = acc_l[i][j] = 0.0;

  for (int64_t p0 = 0; p0 < k; p0 += kK) {
    // stage op(A)[row0:row0+64, p0:p0+16] and op(B)[p0:p0+16, col0:col0+64]
    for (int e = tid; e < kT * kK; e += 256) {
      int r = e % kT, pp = e / kT;
      int64_t i = row0 + r, p = p0 + pp;
      double h = 0.0, l = 0.0;
      if (i < m && p < k) { int64_t idx = i * a_si + p * a_sp; h = Ahi[idx]; l = Alo[idx]; }
      sAh[pp][r] = h; sAl[pp][r] = l;
      int64_t j = col0 + r;
      h = 0.0; l = 0.0;
      if (j < n && p < k) { int64_t idx = p * b_sp + j * b_sj; h = Bhi[idx]; l = Blo[idx]; }
      sBh[pp][r] = h; sBl[pp][r] = l;
    }
    __syncthreads();
    const int kk_end = (k - p0) < kK ? (int)(k - p0) : kK;
    for (int kk = 0; kk < kk_end; ++kk) {
      double ah[4], al[4], bh[4], bl[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) { ah[i] = sAh[kk][ty + 16 * i]; al[i] = sAl[kk][ty + 16 * i]; }
#pragma unroll
      for (int j = 0; j < 4; ++j) { bh[j] = sBh[kk][tx + 16 * j]; bl[j] = sBl[kk][tx + 16 * j]; }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          double ph, pl;
          dd_mul(ah[i], al[i], bh[j], bl[j], ph, pl);
          dd_add(acc_h[i][j], acc_l[i][j], ph, pl, acc_h[i][j], acc_l[i][j]);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t row = row0 + ty + 16 * i;
    if (row >= m) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = col0 + tx + 16 * j;
      if (col >= n) continue;
      const int64_t idx = row + col * ldc;
      double rh, rl;
      dd_add(Chi[idx], Clo[idx], acc_h[i][j], acc_l[i][j], rh, rl);
      Chi[idx] = rh;
      Clo[idx] = rl;
    }
  }
}

hipError_t launch_dd_valu(int64_t m, int64_t n, int64_t k,
                          const double* Ahi, const double* Alo, int64_t a_si, int64_t a_sp,
                          const double* Bhi, const double* Blo, int64_t b_sp, int64_t b_sj,
                          double* Chi, double* Clo, int64_t ldc, hipStream_t s) {
  const int64_t tiles_m = (m + kT - 1) / kT, tiles_n = (n + kT - 1) / kT;
  const int64_t tiles = tiles_m * tiles_n;
  if (tiles <= 0 || tiles > 0x7fffffff) return hipErrorInvalidValue;
  dd_valu_kernel<<<(unsigned)tiles, 256, 0, s>>>(m, n, k, Ahi, Alo, a_si, a_sp, Bhi, Blo, b_sp, b_sj,
                                                 Chi, Clo, ldc, tiles_n);
  return hipGetLastError();
}

}  // namespace ddk
