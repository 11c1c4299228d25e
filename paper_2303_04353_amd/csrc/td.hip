// FP64x3 (triple-word) GEMM by the cascade with six FP64 digits (the case
// Sec. 6.2 names: FP64x3 in terms of FP64).  Unfused: this library's split
// into column-major digit panels, per rank-kc update the 21 products as six
// plain FP64 GEMMs of the vendor library (rocBLAS), one per bin (the
// products of a bin stacked along the inner dimension), this library's
// combine into a triple-word accumulator, and its epilogue.
//
// Layout per rank-kc block b (kb columns of op(A), kb rows of op(B)):
//  * A: the six m x kb digit panels side by side in descending order,
//    [A_5' | A_4' | ... | A_0'] (ld m), at b * 6 kc m;
//  * B: the six kb x n digit panels stacked in ascending order,
//    [B_0'; B_1'; ...; B_5'] (ld 6 kb), at b * 6 kc n; and the suffix sums
//    stacked the same way, [U_0'; ...; U_5'] (U_5' = B_5'), after all of B.
// Bin L <= 4 is then [A_L' | ... | A_0'] times [B_0'; ...; B_L'], one GEMM of
// inner dimension (L+1) kb, and the tail bin [A_5' | ... | A_0'] times
// [U_0'; ...; U_5'].  Bins 0..4 stay exact in any summation order: the
// widths rule bounds the sum of the magnitudes of all their products.
//
// Steps:
//  * widths c0..c4 for a rank-kc block: the largest (in total, then in
//    order) for which bins 0..4 are exact with digits of up to 3 level units
//    (three words each contribute at most one);
//  * Sigma / T from the largest |x0| per row of op(A) / column of op(B);
//  * each scaled word cut as in Appendix A into five digits and a
//    remainder, digits added level by level, remainders rounded in order;
//    planes pre-weighted by 2^-D_(t-1);
//  * bins L = 0..4: sum over i + j = L of A_i' B_j' (exact); tail bin: sum
//    over i of A_i' U_(5-i)', U the suffix sums of B's planes (each
//    addition rounded once, from the last plane up to U_0');
//  * triple words from bins, accumulator and C by a fixed sequence of
//    error-free transforms: three VecSum passes (Ogita, Rump and Oishi), the
//    last element the first word, two more passes for the second, the plain
//    sum of the rest the third, one renormalising TwoSum chain.  It is a
//    faithful stand-in for rounding the exact sum to three words (a few
//    units of 2^-158 relative, plus 2^-200 of the terms' magnitudes).
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <stdint.h>

#include <array>
#include <cmath>
#include <mutex>
#include <unordered_map>

#include "dd_device.hpp"
#include "kernels.hpp"
#include "layout.hpp"

namespace ddk {

namespace {

constexpr int kD = 53;

struct Widths3 {
  int c[5];
  double K[5];       // 2^(53-c) + 2^(52-c)
  double P[5];       // 2^c
  double w[6];       // weights 1, 2^-D0, ..., 2^-D4
};

// One level-by-level split of a scaled word into d[0..5].
__device__ __forceinline__ void split6(double v, const Widths3& W, double d[6]) {
#pragma unroll
  for (int t = 0; t < 5; ++t) {
    const double r = (v + W.K[t]) - W.K[t];
    v = (v - r) * W.P[t];
    d[t] = r;
  }
  d[5] = v;
}

// Planes of op(X) entry (r, c) at X[r*sr + c*sc] scaled by 2^-e: out[t] =
// pre-weighted level t (levels 0..4 exact sums, level 5 rounded in order)
// and the three scaled words.
__device__ __forceinline__ void split_entry3(double x0, double x1, double x2, int e, const Widths3& W,
                                             double out[6], double ys[3]) {
  ys[0] = __builtin_ldexp(x0, -e);
  ys[1] = __builtin_ldexp(x1, -e);
  ys[2] = __builtin_ldexp(x2, -e);
  double a[6], b[6], c[6];
  split6(ys[0], W, a);
  split6(ys[1], W, b);
  split6(ys[2], W, c);
#pragma unroll
  for (int t = 0; t < 5; ++t) out[t] = ((a[t] + b[t]) + c[t]) * W.w[t];
  out[5] = ((a[5] + b[5]) + c[5]) * W.w[5];
}

// Block of inner index p (blocks of kc, the last one kb = k - b kc wide).
struct BlockPos {
  int64_t b, pl, kb;
};
__device__ __forceinline__ BlockPos block_pos(int64_t p, int64_t k, int64_t kc) {
  const int64_t b = p / kc, first = b * kc;
  return {b, p - first, k - first < kc ? k - first : kc};
}

// op(A) entries (i, p) into the descending digit panels of their block.
__global__ void __launch_bounds__(256)
td_split_a(const double* __restrict__ X0, const double* __restrict__ X1, const double* __restrict__ X2,
           int64_t si, int64_t sp, int64_t m, int64_t k, int64_t kc, const uint64_t* __restrict__ amax, Widths3 W,
           double* __restrict__ panels) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= m * k) return;
  const int64_t i = t % m, p = t / m, idx = i * si + p * sp;
  double out[6], ys[3];
  split_entry3(X0[idx], X1[idx], X2[idx], exp_of_bits(amax[i]), W, out, ys);
  const BlockPos q = block_pos(p, k, kc);
  double* base = panels + q.b * 6 * kc * m + q.pl * m + i;
#pragma unroll
  for (int l = 0; l < 6; ++l) base[(5 - l) * q.kb * m] = out[l];
}

// op(B) entries (p, j) into the ascending digit panels of their block and
// the suffix sums U_5' = B_5', U_t' = B_t' + U_(t+1)' (from the last plane
// up to U_0') into the U panels, which start at `upanels`.
__global__ void __launch_bounds__(256)
td_split_b(const double* __restrict__ X0, const double* __restrict__ X1, const double* __restrict__ X2,
           int64_t sp, int64_t sj, int64_t k, int64_t n, int64_t kc, const uint64_t* __restrict__ bmax, Widths3 W,
           double* __restrict__ panels, double* __restrict__ upanels) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= k * n) return;
  const int64_t p = t % k, j = t / k, idx = p * sp + j * sj;
  double out[6], ys[3];
  split_entry3(X0[idx], X1[idx], X2[idx], exp_of_bits(bmax[j]), W, out, ys);
  const BlockPos q = block_pos(p, k, kc);
  const int64_t off = q.b * 6 * kc * n + j * 6 * q.kb + q.pl;
  double* base = panels + off;
  double* ub = upanels + off;
#pragma unroll
  for (int l = 0; l < 6; ++l) base[l * q.kb] = out[l];
  double u = out[5];
  ub[5 * q.kb] = u;
#pragma unroll
  for (int l = 4; l >= 0; --l) {
    u = out[l] + u;
    ub[l * q.kb] = u;
  }
}

__device__ __forceinline__ void vec_sum6(double a[6]) {
#pragma unroll
  for (int i = 1; i < 6; ++i) two_sum(a[i], a[i - 1], a[i], a[i - 1]);
}
__device__ __forceinline__ void vec_sum5(double a[5]) {
#pragma unroll
  for (int i = 1; i < 5; ++i) two_sum(a[i], a[i - 1], a[i], a[i - 1]);
}

// The triple word of six terms, least significant first.
__device__ __forceinline__ void td_from6(double a[6], double& r0, double& r1, double& r2) {
  vec_sum6(a);
  vec_sum6(a);
  vec_sum6(a);
  r0 = a[5];
  double rest[5] = {a[0], a[1], a[2], a[3], a[4]};
  vec_sum5(rest);
  vec_sum5(rest);
  r1 = rest[4];
  r2 = ((rest[0] + rest[1]) + rest[2]) + rest[3];
  two_sum(r1, r2, r1, r2);
  two_sum(r0, r1, r0, r1);
  two_sum(r1, r2, r1, r2);
}

// acc := acc + TD(bins), bins six m x n planes (bins 0..4, tail).
__global__ void __launch_bounds__(256)
td_combine(const double* __restrict__ bins, int64_t mn, double* __restrict__ acc) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= mn) return;
  double t[6] = {bins[5 * mn + i], bins[4 * mn + i], bins[3 * mn + i], bins[2 * mn + i], bins[mn + i], bins[i]};
  double b0, b1, b2;
  td_from6(t, b0, b1, b2);
  double u[6] = {acc[2 * mn + i], b2, acc[mn + i], b1, acc[i], b0};
  td_from6(u, b0, b1, b2);
  acc[i] = b0;
  acc[mn + i] = b1;
  acc[2 * mn + i] = b2;
}

// C := C + acc 2^(e_i + f_j).
__global__ void __launch_bounds__(256)
td_epilogue(const double* __restrict__ acc, int64_t m, int64_t n, const uint64_t* __restrict__ amax,
            const uint64_t* __restrict__ bmax, double* __restrict__ C0, double* __restrict__ C1,
            double* __restrict__ C2, int64_t ldc) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t mn = m * n;
  if (t >= mn) return;
  const int64_t i = t % m, j = t / m, c = i + j * ldc;
  const int sh = exp_of_bits(amax[i]) + exp_of_bits(bmax[j]);
  double u[6] = {C2[c], __builtin_ldexp(acc[2 * mn + t], sh), C1[c], __builtin_ldexp(acc[mn + t], sh),
                 C0[c], __builtin_ldexp(acc[t], sh)};
  double r0, r1, r2;
  td_from6(u, r0, r1, r2);
  C0[c] = r0;
  C1[c] = r1;
  C2[c] = r2;
}

__global__ void td_fill(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }


}  // namespace

// The exactness rule for widths c0..c4 (all quantities are sums of a few
// powers of two times 9: exact in double).
bool td_widths_ok(const int c[5], int64_t kc) {
  int Dc[5], Dm[5];
  int acc = 0;
  for (int t = 0; t < 5; ++t) { Dm[t] = acc; acc += c[t]; Dc[t] = acc; }
  for (int L = 0; L < 5; ++L) {
    int fine = 1 << 30;
    for (int i = 0; i <= L; ++i) fine = std::min(fine, 2 - Dc[i] - Dc[L - i]);
    double total = 0.0;
    for (int i = 0; i <= L; ++i) total += std::ldexp(9.0 * (double)kc, -Dm[i] - Dm[L - i] - fine);
    if (total >= std::ldexp(1.0, 53)) return false;
  }
  return true;
}

// Largest total, then lexicographically largest widths in [14, 26].  The
// search takes some 20 ms on the host, so its result is kept per kc.
void td_widths(int64_t kc, int c[5]) {
  static std::mutex mu;
  static std::unordered_map<int64_t, std::array<int, 5>> cache;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(kc);
    if (it != cache.end()) {
      for (int t = 0; t < 5; ++t) c[t] = it->second[t];
      return;
    }
  }
  int best[5] = {0, 0, 0, 0, 0}, best_sum = -1;
  int w[5];
  for (w[0] = 26; w[0] >= 14; --w[0])
    for (w[1] = 26; w[1] >= 14; --w[1])
      for (w[2] = 26; w[2] >= 14; --w[2])
        for (w[3] = 26; w[3] >= 14; --w[3])
          for (w[4] = 26; w[4] >= 14; --w[4]) {
            if (!td_widths_ok(w, kc)) continue;
            const int s = w[0] + w[1] + w[2] + w[3] + w[4];
            bool better = s > best_sum;
            if (s == best_sum) {
              for (int t = 0; t < 5; ++t)
                if (w[t] != best[t]) { better = w[t] > best[t]; break; }
            }
            if (better) { best_sum = s; for (int t = 0; t < 5; ++t) best[t] = w[t]; }
            break;
          }
  std::array<int, 5> r;
  for (int t = 0; t < 5; ++t) c[t] = r[t] = best[t];
  std::lock_guard<std::mutex> lk(mu);
  cache[kc] = r;
}

size_t td_workspace_bytes(int64_t m, int64_t n, int64_t k, TdOffsets* off) {
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = (size_t)round_up((int64_t)(o + bytes), 256); return r; };
  TdOffsets t{};
  t.amax = take(sizeof(uint64_t) * (size_t)m);
  t.bmax = take(sizeof(uint64_t) * (size_t)n);
  t.aplanes = take(sizeof(double) * 6 * (size_t)m * (size_t)k);
  t.bplanes = take(sizeof(double) * 12 * (size_t)k * (size_t)n);   // digit panels, then U panels
  t.bins = take(sizeof(double) * 6 * (size_t)m * (size_t)n);
  t.acc = take(sizeof(double) * 3 * (size_t)m * (size_t)n);
  if (off) *off = t;
  return o;
}

hipError_t run_td(int64_t m, int64_t n, int64_t k, int64_t kc_in, const double* A0, const double* A1,
                  const double* A2, int64_t a_si, int64_t a_sp, const double* B0, const double* B1,
                  const double* B2, int64_t b_sp, int64_t b_sj, double* C0, double* C1, double* C2,
                  int64_t ldc, char* ws, hipStream_t s) {
  if (m > 0x7fffffff || n > 0x7fffffff || k > 0x7fffffff) return hipErrorInvalidValue;
  TdOffsets off;
  td_workspace_bytes(m, n, k, &off);
  uint64_t* amax = (uint64_t*)(ws + off.amax);
  uint64_t* bmax = (uint64_t*)(ws + off.bmax);
  double* Ap = (double*)(ws + off.aplanes);
  double* Bp = (double*)(ws + off.bplanes);
  double* bins = (double*)(ws + off.bins);
  double* acc = (double*)(ws + off.acc);
  const int64_t kc = k < kc_in ? k : kc_in;
  Widths3 W;
  td_widths(kc, W.c);
  int D = 0;
  W.w[0] = 1.0;
  for (int t = 0; t < 5; ++t) {
    W.K[t] = std::ldexp(1.0, kD - W.c[t]) + std::ldexp(1.0, kD - 1 - W.c[t]);
    W.P[t] = std::ldexp(1.0, W.c[t]);
    D += W.c[t];
    W.w[t + 1] = std::ldexp(1.0, -D);
  }
  hipError_t e = launch_fill_u64(amax, m, 0, s);
  if (e == hipSuccess) e = launch_fill_u64(bmax, n, 0, s);
  if (e == hipSuccess) e = launch_max_abs_bits(A0, m, k, a_si, a_sp, amax, s);
  if (e == hipSuccess) e = launch_max_abs_bits(B0, n, k, b_sj, b_sp, bmax, s);
  if (e != hipSuccess) return e;
  double* Up = Bp + 6 * k * n;
  td_split_a<<<nblk(m * k), 256, 0, s>>>(A0, A1, A2, a_si, a_sp, m, k, kc, amax, W, Ap);
  td_split_b<<<nblk(k * n), 256, 0, s>>>(B0, B1, B2, b_sp, b_sj, k, n, kc, bmax, W, Bp, Up);
  const int64_t mn = m * n;
  td_fill<<<nblk(3 * mn), 256, 0, s>>>(acc, 3 * mn);
  e = hipGetLastError();
  if (e != hipSuccess) return e;

  BlasLease lease = blas_lease(s);
  if (lease.status != hipSuccess) return lease.status;
  rocblas_handle h = lease.h;

  const double one = 1.0, zero = 0.0;
  for (int64_t p0 = 0; p0 < k; p0 += kc) {
    const int64_t kb = p0 + kc < k ? kc : k - p0;
    const double* Ablk = Ap + p0 * 6 * m;   // [A_5' | ... | A_0'], each m x kb
    const double* Bblk = Bp + p0 * 6 * n;   // [B_0'; ...; B_5'], ld 6 kb
    const double* Ublk = Up + p0 * 6 * n;   // [U_0'; ...; U_5'], ld 6 kb
    // bin L <= 4: [A_L' | ... | A_0'] [B_0'; ...; B_L']; tail: all six A
    // panels times the U panels
    for (int L = 0; L < 6; ++L) {
      const int64_t np = L < 5 ? L + 1 : 6;
      const double* A = Ablk + (6 - np) * kb * m;
      const double* B = L < 5 ? Bblk : Ublk;
      const rocblas_status st = rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, (rocblas_int)m,
                                              (rocblas_int)n, (rocblas_int)(np * kb), &one, A, (rocblas_int)m, B,
                                              (rocblas_int)(6 * kb), &zero, bins + L * mn, (rocblas_int)m);
      if (st != rocblas_status_success) return hipErrorLaunchFailure;
    }
    td_combine<<<nblk(mn), 256, 0, s>>>(bins, mn, acc);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  td_epilogue<<<nblk(mn), 256, 0, s>>>(acc, m, n, amax, bmax, C0, C1, C2, ldc);
  return hipGetLastError();
}

}  // namespace ddk
