// FP64x2 vector kernels used around the GEMM: a dot product (the reduction
// of sum(Y o G) in the differentiation chain), a scaling y = alpha x with
// alpha in device memory, and an addition z = x + y (the accumulation of
// the gradients of a tensor used more than once).  All use the same
// double-double arithmetic as the comparator GEMM (TwoProd by FMA, accurate
// DD addition).
//
// dd_dot: pass 1, each of `nblk` workgroups accumulates a strided subset of
// the products in FP64x2 per thread and reduces its 256 partial sums in
// FP64x2 through LDS (fixed tree, so the result is deterministic); pass 2,
// one workgroup reduces the `nblk` block sums the same way.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dd_device.hpp"
#include "kernels.hpp"

namespace ddk {

namespace {

__device__ __forceinline__ void block_reduce_dd(double& h, double& l) {
  __shared__ double sh[256], sl[256];
  const int t = threadIdx.x;
  sh[t] = h;
  sl[t] = l;
  __syncthreads();
  for (int s = 128; s >= 1; s >>= 1) {
    if (t < s) {
      double rh, rl;
      dd_add(sh[t], sl[t], sh[t + s], sl[t + s], rh, rl);
      sh[t] = rh;
      sl[t] = rl;
    }
    __syncthreads();
  }
  h = sh[0];
  l = sl[0];
}

}  // namespace

__global__ void __launch_bounds__(256)
dd_dot_partial(int64_t n, const double* __restrict__ xh, const double* __restrict__ xl, int64_t incx,
               const double* __restrict__ yh, const double* __restrict__ yl, int64_t incy,
               double* __restrict__ part) {
  double h = 0.0, l = 0.0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    double ph, pl;
    dd_mul(xh[i * incx], xl[i * incx], yh[i * incy], yl[i * incy], ph, pl);
    dd_add(h, l, ph, pl, h, l);
  }
  block_reduce_dd(h, l);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = h;
    part[2 * blockIdx.x + 1] = l;
  }
}

__global__ void __launch_bounds__(256)
dd_dot_final(int nblk, const double* __restrict__ part, double* __restrict__ res) {
  double h = 0.0, l = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) dd_add(h, l, part[2 * i], part[2 * i + 1], h, l);
  block_reduce_dd(h, l);
  if (threadIdx.x == 0) {
    res[0] = h;
    res[1] = l;
  }
}

// alpha = (alpha[0], alpha[1]) is read from device memory, so a scale
// computed on the device needs no trip through the host.
__global__ void __launch_bounds__(256)
dd_scal_kernel(int64_t n, const double* __restrict__ alpha, const double* xh, const double* xl,
               int64_t incx, double* yh, double* yl, int64_t incy) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double rh, rl;
  dd_mul(alpha[0], alpha[1], xh[i * incx], xl[i * incx], rh, rl);
  yh[i * incy] = rh;
  yl[i * incy] = rl;
}

// z = x + y with the accurate FP64x2 addition; z may be x or y (each
// element is read before it is written, by the same thread).
__global__ void __launch_bounds__(256)
dd_add_kernel(int64_t n, const double* xh, const double* xl, int64_t incx, const double* yh,
              const double* yl, int64_t incy, double* zh, double* zl, int64_t incz) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double rh, rl;
  dd_add(xh[i * incx], xl[i * incx], yh[i * incy], yl[i * incy], rh, rl);
  zh[i * incz] = rh;
  zl[i * incz] = rl;
}

int dd_dot_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (int)(b < 1024 ? (b > 0 ? b : 1) : 1024);
}

hipError_t launch_dd_dot(int64_t n, const double* xh, const double* xl, int64_t incx,
                         const double* yh, const double* yl, int64_t incy,
                         double* part, double* res, hipStream_t s) {
  const int nblk = dd_dot_blocks(n);
  dd_dot_partial<<<nblk, 256, 0, s>>>(n, xh, xl, incx, yh, yl, incy, part);
  dd_dot_final<<<1, 256, 0, s>>>(nblk, part, res);
  return hipGetLastError();
}

hipError_t launch_dd_scal(int64_t n, const double* alpha, const double* xh, const double* xl, int64_t incx,
                          double* yh, double* yl, int64_t incy, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if ((n + 255) / 256 > 0x7fffffff) return hipErrorInvalidValue;
  dd_scal_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, alpha, xh, xl, incx, yh, yl, incy);
  return hipGetLastError();
}

hipError_t launch_dd_add(int64_t n, const double* xh, const double* xl, int64_t incx, const double* yh,
                         const double* yl, int64_t incy, double* zh, double* zl, int64_t incz, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if ((n + 255) / 256 > 0x7fffffff) return hipErrorInvalidValue;
  dd_add_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, xh, xl, incx, yh, yl, incy, zh, zl, incz);
  return hipGetLastError();
}

}  // namespace ddk
