// The paper's "simple" form of the cascade (Sec. 4.2): the ten products of
// eq. (Gemm10) as ten plain FP64 GEMM calls per rank-kc update, into four
// explicit bin matrices in HBM, then a combine pass per update and one
// epilogue.  The GEMMs are the vendor library's (rocBLAS); the split, the
// combine and the epilogue are this library's kernels.
//
// Bins 0-2 are exact whatever order the library sums in: every partial sum
// of a rank-kc block is an integer multiple of the block's grid below 2^53
// (the split widths of Sec. 3.3), so FMA or plain additions in any order
// give the same value.  Bin 3-6 is rounded, in the library's order.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <stdint.h>

#include <mutex>
#include <unordered_map>

#include "dd_device.hpp"
#include "kernels.hpp"
#include "layout.hpp"

namespace ddk {

namespace {

// acc += bin0 + (bin1 + (bin2 + bin36)) in FP64x2, the order of the fused
// kernel's combine (Sec. 3.6 fl_casc); bins are m x n, leading dimension m.
__global__ void __launch_bounds__(256)
combine_bins(const double* __restrict__ bins, int64_t mn, double* __restrict__ acc_h,
             double* __restrict__ acc_l) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= mn) return;
  double s, e;
  two_sum(bins[2 * mn + i], bins[3 * mn + i], s, e);
  dd_add_d(s, e, bins[mn + i], s, e);
  dd_add_d(s, e, bins[i], s, e);
  double h, l;
  dd_add(acc_h[i], acc_l[i], s, e, h, l);
  acc_h[i] = h;
  acc_l[i] = l;
}

// C := C + acc 2^(e_i + f_j), as the fused kernel's epilogue.
__global__ void __launch_bounds__(256)
simple_epilogue(const double* __restrict__ acc_h, const double* __restrict__ acc_l, int64_t m, int64_t n,
                const uint64_t* __restrict__ amax, const uint64_t* __restrict__ bmax,
                double* __restrict__ Chi, double* __restrict__ Clo, int64_t ldc) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= m * n) return;
  const int64_t i = t % m, j = t / m;
  const int sh = exp_of_bits(amax[i]) + exp_of_bits(bmax[j]);
  const double h = __builtin_ldexp(acc_h[t], sh), l = __builtin_ldexp(acc_l[t], sh);
  double rh, rl;
  dd_add(Chi[i + j * ldc], Clo[i + j * ldc], h, l, rh, rl);
  Chi[i + j * ldc] = rh;
  Clo[i + j * ldc] = rl;
}

__global__ void fill_f64(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

inline unsigned nblocks(int64_t n) { return (unsigned)((n + 255) / 256); }

std::mutex g_blas_mu;
std::unordered_map<int, rocblas_handle> g_blas;

}  // namespace

BlasLease blas_lease(hipStream_t s) {
  BlasLease r;
  r.lock = std::unique_lock<std::mutex>(g_blas_mu);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) { r.status = hipErrorInvalidDevice; return r; }
  auto it = g_blas.find(dev);
  if (it == g_blas.end()) {
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) { r.status = hipErrorNotInitialized; return r; }
    it = g_blas.emplace(dev, h).first;
  }
  r.h = it->second;
  if (rocblas_set_stream(r.h, s) != rocblas_status_success) r.status = hipErrorInvalidHandle;
  return r;
}

hipError_t run_simple_products(const CascadeLayout& L, char* ws, const uint64_t* amax, const uint64_t* bmax,
                               double* Chi, double* Clo, int64_t ldc, hipStream_t s) {
  const int64_t m = L.m, n = L.n, k = L.k, mn = m * n;
  if (m > 0x7fffffff || n > 0x7fffffff || k > 0x7fffffff) return hipErrorInvalidValue;
  const double* Ap = (const double*)(ws + L.off_aplain);   // 4 planes m x k, ld m
  const double* Bp = (const double*)(ws + L.off_bplain);   // 7 planes k x n, ld k
  double* bins = (double*)(ws + L.off_bins);               // 4 planes m x n, ld m
  double* acc_h = (double*)(ws + L.off_acc);
  double* acc_l = acc_h + mn;
  hipError_t e = launch_unpack((const double*)(ws + L.off_apack), 0, m, k, L.K4, (double*)Ap, s);
  if (e == hipSuccess) e = launch_unpack((const double*)(ws + L.off_bpack), 1, k, n, L.K4, (double*)Bp, s);
  if (e != hipSuccess) return e;
  fill_f64<<<nblocks(2 * mn), 256, 0, s>>>(acc_h, 2 * mn);
  e = hipGetLastError();
  if (e != hipSuccess) return e;

  BlasLease lease = blas_lease(s);
  if (lease.status != hipSuccess) return lease.status;
  rocblas_handle h = lease.h;

  // (bin, A plane, B plane) of the ten products, bin 3-6 with B4', B5', B6'
  static const int prod[10][3] = {{0, 0, 0}, {1, 0, 1}, {1, 1, 0}, {2, 0, 2}, {2, 1, 1},
                                  {2, 2, 0}, {3, 0, 3}, {3, 1, 4}, {3, 2, 5}, {3, 3, 6}};
  const double one = 1.0, zero = 0.0;
  const int64_t kc = L.kc;
  for (int64_t p0 = 0; p0 < k; p0 += kc) {
    const int64_t kb = p0 + kc < k ? kc : k - p0;
    bool started[4] = {false, false, false, false};
    for (const auto& q : prod) {
      const int b = q[0];
      const double* A = Ap + (int64_t)q[1] * m * k + p0 * m;
      const double* B = Bp + (int64_t)q[2] * k * n + p0;
      const rocblas_status st = rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, (rocblas_int)m,
                                              (rocblas_int)n, (rocblas_int)kb, &one, A, (rocblas_int)m, B,
                                              (rocblas_int)k, started[b] ? &one : &zero, bins + b * mn,
                                              (rocblas_int)m);
      if (st != rocblas_status_success) return hipErrorLaunchFailure;
      started[b] = true;
    }
    combine_bins<<<nblocks(mn), 256, 0, s>>>(bins, mn, acc_h, acc_l);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  simple_epilogue<<<nblocks(mn), 256, 0, s>>>(acc_h, acc_l, m, n, amax, bmax, Chi, Clo, ldc);
  return hipGetLastError();
}

}  // namespace ddk
