// Device-side FP64x2 arithmetic and the Appendix A split, shared by the HIP
// kernels of this library.  Everything is compiled with -ffp-contract=off:
// a*b+c is never fused unless written as __builtin_fma, and (v + K) - K is
// evaluated with two roundings as the split requires.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ddk {

typedef double d4 __attribute__((ext_vector_type(4)));

struct dd { double hi, lo; };

// Knuth's TwoSum: s + e == a + b exactly, s = fl(a + b).
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Dekker's Fast/QuickTwoSum, exact when |a| >= |b| (or a == 0).
__device__ __forceinline__ void quick_two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  e = b - (s - a);
}

// FP64x2 + FP64.
__device__ __forceinline__ void dd_add_d(double xh, double xl, double y, double& rh, double& rl) {
  double s, e;
  two_sum(xh, y, s, e);
  e = e + xl;
  quick_two_sum(s, e, rh, rl);
}

// FP64x2 + FP64x2, the accurate variant (both words summed with TwoSum).
__device__ __forceinline__ void dd_add(double xh, double xl, double yh, double yl,
                                       double& rh, double& rl) {
  double s, e, t, f;
  two_sum(xh, yh, s, e);
  two_sum(xl, yl, t, f);
  e = e + t;
  quick_two_sum(s, e, s, e);
  e = e + f;
  quick_two_sum(s, e, rh, rl);
}

// FP64x2 * FP64x2: TwoProd of the high words by FMA, the two cross products
// added to its error, one renormalisation (lo*lo is below the FP64x2 grid).
__device__ __forceinline__ void dd_mul(double ah, double al, double bh, double bl,
                                       double& rh, double& rl) {
  double p = ah * bh;
  double e = __builtin_fma(ah, bh, -p);
  double t = ah * bl;
  double u = al * bh;
  double v = t + u;
  e = e + v;
  quick_two_sum(p, e, rh, rl);
}

// Split widths and the constants of Appendix A for one rank-kc update.
struct SplitParams {
  double K[3];    // 2^(53-c_t) + 2^(52-c_t): adding and subtracting K rounds to 2^(1-c_t)
  double P[3];    // 2^c_t: moves the remainder up to the next digit
  double sig[4];  // 1, sigma_1, sigma_2, sigma_3: weights of the pre-weighted planes
};

// Digits of one FP64 value v (|v| < 1 after scaling): d0..d2 are v rounded to
// the grid 2^(1-c_t) at each level, d3 the exact remainder (Appendix A).
__device__ __forceinline__ void split4(double v, const SplitParams& sp, double d[4]) {
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    double r = (v + sp.K[t]) - sp.K[t];
    v = (v - r) * sp.P[t];
    d[t] = r;
  }
  d[3] = v;
}

// Pre-weighted digits of the FP64x2 entry (hi, lo) scaled by 2^-e: the two
// words are split separately and added digit by digit (exact for d0..d2, the
// fourth digit rounds once).  Also returns the scaled words.
__device__ __forceinline__ void split_entry(double hi, double lo, int e, const SplitParams& sp,
                                            double w[4], double& xh, double& xl) {
  xh = __builtin_ldexp(hi, -e);
  xl = __builtin_ldexp(lo, -e);
  double dh[4], dl[4];
  split4(xh, sp, dh);
  split4(xl, sp, dl);
#pragma unroll
  for (int t = 0; t < 4; ++t) w[t] = (dh[t] + dl[t]) * sp.sig[t];
}

// Workgroups are dealt to the 8 XCDs round robin (block b runs on XCD b % 8)
// and each XCD has its own L2.  Give every XCD a contiguous range of tiles
// and walk that range in groups of kGroupM tile rows, so the workgroups that
// run together on one XCD share a few A and B strips in its L2.  For T
// blocks (b < T), XCD x runs ceil((T - x) / 8) of them; its range starts
// after those of XCDs 0..x-1, so b -> L is a bijection on [0, T) for any T.
constexpr int64_t kXcds = 8;
constexpr int64_t kGroupM = 8;

__device__ __forceinline__ void tile_of_block(int64_t b, int64_t tiles_m, int64_t tiles_n,
                                              int64_t& tm, int64_t& tn) {
  const int64_t T = tiles_m * tiles_n;
  const int64_t per_xcd = T / kXcds, extra = T % kXcds, x = b % kXcds;
  const int64_t L = x * per_xcd + (x < extra ? x : extra) + b / kXcds;
  const int64_t per_group = kGroupM * tiles_n;
  const int64_t g = L / per_group;
  const int64_t first_m = g * kGroupM;
  const int64_t gm = tiles_m - first_m < kGroupM ? tiles_m - first_m : kGroupM;
  const int64_t r = L - g * per_group;
  tm = first_m + r % gm;
  tn = r / gm;
}

// frexp exponent of a non-negative double held as its bit pattern (0 -> 0).
__device__ __forceinline__ int exp_of_bits(uint64_t bits) {
  return __builtin_amdgcn_frexp_exp(__builtin_bit_cast(double, bits));
}

}  // namespace ddk
