// FP64x3 (triple-word) GEMM by the cascade with six FP64 digits (the case
// Sec. 6.2 names: FP64x3 in terms of FP64), products fused on the FP64
// matrix cores.
//
// Phase one (HBM bound):
//  * widths c0..c4 for a rank-kc block: the largest (in total, then in
//    order) for which bins 0..4 are exact with digits of up to 3 level units
//    (three words each contribute at most one);
//  * Sigma / T from the largest |x0| per row of op(A) / column of op(B);
//  * each scaled word cut as in Appendix A into five digits and a
//    remainder, digits added level by level, remainders rounded in order;
//    planes pre-weighted by 2^-D_(t-1) and packed for v_mfma_f64_4x4x4_4b_f64
//    as the FP64x2 planes are: A per 16-row block and group of 4 inner
//    indices, the six planes A_0'..A_5', position s*16 + kk*4 + i within a
//    plane; B per 16-column block the six planes B_0'..B_5', lane kk*16 + c.
//
// Phases two and three (FP64 MFMA bound), one kernel: a workgroup of 8
// waves (two per SIMD) owns a 64x64 tile of C, each wave 16x32.  Per group
// of 4 inner indices the 21 products: bin L = 0..4 takes A_i' B_j' with
// i + j = L (exact, by the widths rule), the tail bin A_i' U_(5-i)' with the
// suffix sums U_5' = B_5', U_t' = B_t' + U_(t+1)' formed in registers just
// before they are used (the same roundings, in the same order, as the
// oracle's).  The products go by plane of A (A_0' with six planes of B,
// A_1' with five, ...), ordered so that the same bin is updated at most
// every other product.  Per rank-kc block the six bins become a triple word
// by a fixed sequence of error-free transforms and are added to the
// triple-word accumulator the same way; Sigma / T and C at the end.
//
// Operand staging: one LDS stage per group of 4 inner indices (24 KiB: six
// planes of four 16-row blocks of A and four 16-column blocks of B), three
// stage buffers.  Each group runs in two halves around one barrier: the
// first half (products of A_0', A_1') writes the next stage, which was
// loaded into registers during the previous group; the second half (A_2'
// .. A_5') reads the next group's B planes and A_0' from the stage just
// written and loads the stage after it.  With three buffers the stage
// written in a first half is one whose last reads ended before the
// previous barrier.
//
// Triple words: three VecSum passes (Ogita, Rump and Oishi) over the terms,
// roughly least significant first, the last element the first word, two
// more passes over the rest for the second word, the plain sum of what
// remains the third, one renormalising TwoSum chain.  It stands in for
// rounding the exact sum to three words, within a few units of 2^-158 of
// the sum plus 2^-200 of the terms' magnitudes.  Per rank-kc block one such
// sum takes the six bins and the accumulator's three words (nine terms); the
// epilogue takes the result and the three words of C (six).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <array>
#include <cmath>
#include <mutex>
#include <type_traits>
#include <unordered_map>

#include "dd_device.hpp"
#include "kernels.hpp"
#include "layout.hpp"

namespace ddk {

namespace {

constexpr int kD = 53;
constexpr int kP3 = 6;                        // digit planes per operand
constexpr int kWaves3 = 8;
constexpr int kFrag3 = kP3 * kLanes;          // doubles per block and group (384)
constexpr int kAStage3 = 4 * kFrag3;          // A part of an LDS stage: four 16-row blocks
constexpr int kStage3 = 2 * kAStage3;         // doubles per stage (24 KiB)
constexpr int kNBuf3 = 3;
constexpr int kPieces3 = kStage3 / 128;       // 1 KiB pieces per stage (24), three per wave
static_assert(kPieces3 == 3 * kWaves3, "every wave stages three 1 KiB pieces of a stage");

// Packed planes of one 16-row (16-column) block are contiguous over k; the
// blocks are 4 KiB + 256 B further apart than their size (L2 sets).
constexpr int64_t td_block_stride(int64_t K4) { return K4 * kFrag3 + kBlockPad; }

typedef double d2 __attribute__((ext_vector_type(2)));

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

// Pre-weighted levels of an entry (x0, x1, x2) scaled by 2^-e: levels 0..4
// exact sums of the three words' digits, level 5 the remainders rounded in
// order.
__device__ __forceinline__ void split_entry3(double x0, double x1, double x2, int e, const Widths3& W,
                                             double out[6]) {
  double a[6], b[6], c[6];
  split6(__builtin_ldexp(x0, -e), W, a);
  split6(__builtin_ldexp(x1, -e), W, b);
  split6(__builtin_ldexp(x2, -e), W, c);
#pragma unroll
  for (int t = 0; t < 6; ++t) out[t] = ((a[t] + b[t]) + c[t]) * W.w[t];
}

// One wave per 64-lane fragment (16-row block rb, group kq) of op(A),
// op(A)(i, p) = X[i*si + p*sp]; zero outside m, k.
__global__ void __launch_bounds__(256)
td_pack_a(const double* __restrict__ X0, const double* __restrict__ X1, const double* __restrict__ X2,
          int64_t si, int64_t sp, int64_t m, int64_t k, int64_t K4, int64_t nfrag,
          const uint64_t* __restrict__ amax, Widths3 W, double* __restrict__ Apack) {
  const int64_t frag = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (frag >= nfrag) return;
  const int lane = threadIdx.x & 63;
  const int64_t rb = frag / K4, kq = frag - rb * K4;
  const int64_t i = rb * 16 + (lane >> 4) * 4 + (lane & 3), p = kq * 4 + ((lane >> 2) & 3);
  double out[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (i < m && p < k) {
    const int64_t idx = i * si + p * sp;
    split_entry3(X0[idx], X1[idx], X2[idx], exp_of_bits(amax[i]), W, out);
  }
  double* dst = Apack + rb * td_block_stride(K4) + kq * kFrag3 + lane;
#pragma unroll
  for (int t = 0; t < kP3; ++t) dst[t * kLanes] = out[t];
}

// One wave per fragment (16-column block cb, group kq) of op(B),
// op(B)(p, j) = X[p*sp + j*sj].
__global__ void __launch_bounds__(256)
td_pack_b(const double* __restrict__ X0, const double* __restrict__ X1, const double* __restrict__ X2,
          int64_t sp, int64_t sj, int64_t k, int64_t n, int64_t K4, int64_t nfrag,
          const uint64_t* __restrict__ bmax, Widths3 W, double* __restrict__ Bpack) {
  const int64_t frag = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (frag >= nfrag) return;
  const int lane = threadIdx.x & 63;
  const int64_t cb = frag / K4, kq = frag - cb * K4;
  const int64_t j = cb * 16 + (lane & 15), p = kq * 4 + (lane >> 4);
  double out[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (j < n && p < k) {
    const int64_t idx = p * sp + j * sj;
    split_entry3(X0[idx], X1[idx], X2[idx], exp_of_bits(bmax[j]), W, out);
  }
  double* dst = Bpack + cb * td_block_stride(K4) + kq * kFrag3 + lane;
#pragma unroll
  for (int t = 0; t < kP3; ++t) dst[t * kLanes] = out[t];
}

template <int N>
__device__ __forceinline__ void vec_sum_n(double (&a)[N]) {
#pragma unroll
  for (int i = 1; i < N; ++i) two_sum(a[i], a[i - 1], a[i], a[i - 1]);
}

// The triple word of N terms given roughly least significant first: three
// VecSum passes, the last element the first word; two more passes over the
// rest, its last element the second word; the plain sum of what remains the
// third; one renormalising TwoSum chain.
template <int N>
__device__ __forceinline__ void td_from_n(double (&a)[N], double& r0, double& r1, double& r2) {
  vec_sum_n(a);
  vec_sum_n(a);
  vec_sum_n(a);
  r0 = a[N - 1];
  double rest[N - 1];
#pragma unroll
  for (int i = 0; i < N - 1; ++i) rest[i] = a[i];
  vec_sum_n(rest);
  vec_sum_n(rest);
  r1 = rest[N - 2];
  r2 = rest[0];
#pragma unroll
  for (int i = 1; i < N - 2; ++i) r2 = r2 + rest[i];
  two_sum(r1, r2, r1, r2);
  two_sum(r0, r1, r0, r1);
  two_sum(r1, r2, r1, r2);
}

__device__ __forceinline__ double mfma4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ void lds_barrier() { asm volatile("s_barrier" ::: "memory"); }
__device__ __forceinline__ void lds_reads_done() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

constexpr int kSub3 = 4;   // 4-row sub-blocks per wave
constexpr int kCG3 = 2;    // 16-column groups per wave
constexpr int kTail = 5;   // index of the tail bin

struct Bins3 {
  double b[6][kSub3][kCG3];   // bins 0..4, tail
};

// One product: 8 independent MFMAs into bin `L`.
__device__ __forceinline__ void product(Bins3& B, int L, const double (&a)[kSub3], const double (&b)[kCG3]) {
#pragma unroll
  for (int s = 0; s < kSub3; ++s)
#pragma unroll
    for (int g = 0; g < kCG3; ++g) B.b[L][s][g] = mfma4(a[s], b[g], B.b[L][s][g]);
}

__device__ __forceinline__ void read_a(double (&a)[kSub3], const double* sA, int t) {
#pragma unroll
  for (int s = 0; s < kSub3; ++s) a[s] = sA[t * kLanes + s * 16];
}

__device__ __forceinline__ void read_b(double (&b)[kP3][kCG3], const double* sB) {
#pragma unroll
  for (int t = 0; t < kP3; ++t)
#pragma unroll
    for (int g = 0; g < kCG3; ++g) b[t][g] = sB[g * kFrag3 + t * kLanes];
}

__device__ __forceinline__ void add_u(double (&u)[kCG3], const double (&b)[kCG3]) {
#pragma unroll
  for (int g = 0; g < kCG3; ++g) u[g] = b[g] + u[g];
}

// Where the memory instructions of a group go among its 168 MFMAs.  Each
// plane of A is read during the products of the plane before it, and the
// next group's operands only once A_2' and A_3' are no longer needed, which
// bounds the registers in flight.
// First half, 88 MFMAs (A_0': 48, A_1': 40): reads of A_1', the three LDS
// writes of the next stage, reads of A_2'.
__device__ __forceinline__ void interleave_first_half() {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // DS read (A_1')
    __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);   // MFMA
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);   // DS write (next stage)
    __builtin_amdgcn_sched_group_barrier(0x008, 10, 0);
  }
  __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // DS read (A_2')
    __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
  }
  __builtin_amdgcn_sched_group_barrier(0x008, 24, 0);
}

// Second half, 80 MFMAs (A_2': 32, A_3': 24, A_4': 16, A_5': 8): the three
// global loads of the stage after next, reads of A_3', A_4', A_5', then the
// next group's B planes and A_0' (16 reads).
__device__ __forceinline__ void interleave_second_half() {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);   // VMEM read
    __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // DS read (A_3')
    __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
  }
  __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // DS read (A_4', A_5')
    __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // DS read (next B planes, A_0')
    __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
  }
}

// Bins of a rank-kc block added to the triple-word accumulator; bins reset.
__device__ __forceinline__ void combine3(Bins3& B, double (&r0)[kSub3][kCG3], double (&r1)[kSub3][kCG3],
                                         double (&r2)[kSub3][kCG3]) {
#pragma unroll
  for (int s = 0; s < kSub3; ++s)
#pragma unroll
    for (int g = 0; g < kCG3; ++g) {
      // the block's six bins and the accumulator's three words in one sum,
      // roughly by magnitude
      double t[9] = {B.b[kTail][s][g], r2[s][g], B.b[4][s][g], B.b[3][s][g], r1[s][g],
                     B.b[2][s][g],     B.b[1][s][g], B.b[0][s][g], r0[s][g]};
      td_from_n(t, r0[s][g], r1[s][g], r2[s][g]);
#pragma unroll
      for (int L = 0; L < 6; ++L) B.b[L][s][g] = 0.0;
    }
}

__global__ void __launch_bounds__(kWaves3 * 64)
td_cascade_kernel(const double* __restrict__ Apack, const double* __restrict__ Bpack,
                  const uint64_t* __restrict__ amax, const uint64_t* __restrict__ bmax, int64_t K4, int32_t kcq,
                  int64_t m, int64_t n, int64_t tiles_m, int64_t tiles_n, double* __restrict__ C0,
                  double* __restrict__ C1, double* __restrict__ C2, int64_t ldc) {
  __shared__ __attribute__((aligned(16))) double lds[kNBuf3 * kStage3];
  int64_t tm, tn;
  tile_of_block(blockIdx.x, tiles_m, tiles_n, tm, tn);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave >> 1, wn = wave & 1;     // 16-row block wm, 32-column half wn
  const int64_t rb0 = tm * 4 + wm, cb0 = tn * 4 + wn * kCG3;

  Bins3 bins;
  double r0[kSub3][kCG3], r1[kSub3][kCG3], r2[kSub3][kCG3];
#pragma unroll
  for (int s = 0; s < kSub3; ++s)
#pragma unroll
    for (int g = 0; g < kCG3; ++g) {
#pragma unroll
      for (int L = 0; L < 6; ++L) bins.b[L][s][g] = 0.0;
      r0[s][g] = r1[s][g] = r2[s][g] = 0.0;
    }

  // Piece d of a stage (d = wave, wave + 8, wave + 16): d < 12 is chunk d%3
  // of 16-row block d/3 of A, else chunk e%3 of 16-column block e/3 of B
  // (e = d - 12).  A block's group is 384 contiguous doubles, 3 pieces.
  // A piece's source and LDS place are the same for all lanes of the wave
  // (scalar registers); each lane adds its own 16 bytes.  Vector
  // instructions in the loop take issue cycles from the matrix cores.
  __builtin_assume(wave >= 0 && wave < kWaves3);
  const double* pbase[3];
  int pdst[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int d = wave + c * kWaves3;
    if (d < 12) {
      const int blk = d / 3, i = d % 3;
      pbase[c] = Apack + (tm * 4 + blk) * td_block_stride(K4) + i * 128;
      pdst[c] = blk * kFrag3 + i * 128;
    } else {
      const int e = d - 12, blk = e / 3, i = e % 3;
      pbase[c] = Bpack + (tn * 4 + blk) * td_block_stride(K4) + i * 128;
      pdst[c] = kAStage3 + blk * kFrag3 + i * 128;
    }
  }
  d2 stg[3];
  const int64_t last = K4 - 1;
  auto load_stage = [&](int64_t st) {
#pragma unroll
    for (int c = 0; c < 3; ++c) stg[c] = *(const d2*)(pbase[c] + st * kFrag3 + lane * 2);
  };
  auto store_stage = [&](int buf) {
    // every piece starts on a 16-byte boundary: say so, or the 16-byte
    // writes get split into two 8-byte ones, which conflict in the LDS banks
    double* dst = lds + buf * kStage3 + lane * 2;
#pragma unroll
    for (int c = 0; c < 3; ++c)
      *(d2*)__builtin_assume_aligned(dst + pdst[c], 16) = stg[c];
  };
  const int aoff = wm * kFrag3 + (lane >> 4) * 4 + (lane & 3);
  const int boff = kAStage3 + wn * kCG3 * kFrag3 + lane;

  // Prologue: stage 0 in buffer 0, stage 1 in the staging registers; the
  // first group's B planes and A_0' in registers.
  load_stage(0);
  store_stage(0);
  load_stage(last > 0 ? 1 : 0);
  lds_reads_done();
  lds_barrier();
  double bx[kP3][kCG3], by[kP3][kCG3], ax0[kSub3], ay0[kSub3];
  read_b(bx, lds + boff);
  read_a(ax0, lds + aoff, 0);

  int32_t inblk = 0;
  // One group: bc / ac0 hold its B planes and A_0'; bn / an0 receive the
  // next group's.  The last group reads and loads in-bounds copies that are
  // not used.
  // The buffer of a group is a template constant: the loop below runs six
  // groups (two rounds of the three buffers) at a time, so every LDS
  // address is a fixed offset from the lane's own.
  auto group = [&](auto curc, int64_t st, double (&bc)[kP3][kCG3], double (&ac0)[kSub3], double (&bn)[kP3][kCG3],
                   double (&an0)[kSub3]) {
    constexpr int cur = decltype(curc)::value;
    constexpr int nxt = cur == kNBuf3 - 1 ? 0 : cur + 1;
    const double* sA = lds + cur * kStage3 + aoff;
    double a1[kSub3], a2[kSub3], a3[kSub3], a4[kSub3], a5[kSub3];
    double u[kCG3];
    // first half: A_0' with B_0'..B_4' and U_5' = B_5', A_1' with B_0'..B_3' and U_4'
    read_a(a1, sA, 1);
    product(bins, 0, ac0, bc[0]);
    product(bins, 1, ac0, bc[1]);
    product(bins, 2, ac0, bc[2]);
    product(bins, 3, ac0, bc[3]);
    product(bins, 4, ac0, bc[4]);
    u[0] = bc[5][0];
    u[1] = bc[5][1];
    product(bins, kTail, ac0, u);
    read_a(a2, sA, 2);
    store_stage(nxt);
    product(bins, 1, a1, bc[0]);
    product(bins, 2, a1, bc[1]);
    add_u(u, bc[4]);                           // U_4'
    product(bins, kTail, a1, u);
    product(bins, 3, a1, bc[2]);
    product(bins, 4, a1, bc[3]);
    interleave_first_half();
    lds_reads_done();
    lds_barrier();
    // second half: A_2'..A_5'; the next group's operands from the stage
    // just written, the stage after it from memory
    // group numbers fit in 32 bits; the 32-bit compare is a scalar one
    const int32_t s2 = (int32_t)st + 2;
    load_stage(s2 <= (int32_t)last ? s2 : (int32_t)last);
    read_a(a3, sA, 3);
    read_a(a4, sA, 4);
    read_a(a5, sA, 5);
    product(bins, 2, a2, bc[0]);
    add_u(u, bc[3]);                           // U_3'
    product(bins, kTail, a2, u);
    product(bins, 3, a2, bc[1]);
    product(bins, 4, a2, bc[2]);
    product(bins, 3, a3, bc[0]);
    add_u(u, bc[2]);                           // U_2'
    product(bins, kTail, a3, u);
    product(bins, 4, a3, bc[1]);
    add_u(u, bc[1]);                           // U_1'
    product(bins, kTail, a4, u);
    product(bins, 4, a4, bc[0]);
    add_u(u, bc[0]);                           // U_0'
    product(bins, kTail, a5, u);
    read_b(bn, lds + nxt * kStage3 + boff);
    read_a(an0, lds + nxt * kStage3 + aoff, 0);
    interleave_second_half();
    if (++inblk == kcq) {
      inblk = 0;
      combine3(bins, r0, r1, r2);
    }
  };
  using B0 = std::integral_constant<int, 0>;
  using B1 = std::integral_constant<int, 1>;
  using B2 = std::integral_constant<int, 2>;
  int64_t st = 0;
  for (; st + 6 <= K4; st += 6) {
    group(B0{}, st, bx, ax0, by, ay0);
    group(B1{}, st + 1, by, ay0, bx, ax0);
    group(B2{}, st + 2, bx, ax0, by, ay0);
    group(B0{}, st + 3, by, ay0, bx, ax0);
    group(B1{}, st + 4, bx, ax0, by, ay0);
    group(B2{}, st + 5, by, ay0, bx, ax0);
  }
  // K4 is even: 0, 2 or 4 groups remain, starting again in buffer 0
  if (st < K4) {
    group(B0{}, st, bx, ax0, by, ay0);
    group(B1{}, st + 1, by, ay0, bx, ax0);
    if (st + 2 < K4) {
      group(B2{}, st + 2, bx, ax0, by, ay0);
      group(B0{}, st + 3, by, ay0, bx, ax0);
    }
  }
  if (inblk != 0) combine3(bins, r0, r1, r2);

  // Epilogue: C + acc 2^(e_i + f_j) as triple words.
#pragma unroll
  for (int s = 0; s < kSub3; ++s) {
    const int64_t row = rb0 * 16 + s * 4 + (lane >> 4);
    if (row >= m) continue;
    const int er = exp_of_bits(amax[row]);
#pragma unroll
    for (int g = 0; g < kCG3; ++g) {
      const int64_t col = (cb0 + g) * 16 + (lane & 15);
      if (col >= n) continue;
      const int sh = er + exp_of_bits(bmax[col]);
      const int64_t c = row + col * ldc;
      double u[6] = {C2[c], __builtin_ldexp(r2[s][g], sh), C1[c], __builtin_ldexp(r1[s][g], sh), C0[c],
                     __builtin_ldexp(r0[s][g], sh)};
      double w0, w1, w2;
      td_from_n(u, w0, w1, w2);
      C0[c] = w0;
      C1[c] = w1;
      C2[c] = w2;
    }
  }
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

// Padded sizes: m, n to the 64x64 tile, k to whole pairs of groups (8).
static void td_sizes(int64_t m, int64_t n, int64_t k, int64_t* mpad, int64_t* npad, int64_t* K4) {
  *mpad = round_up(m > 0 ? m : 1, 64);
  *npad = round_up(n > 0 ? n : 1, 64);
  *K4 = round_up(k > 0 ? k : 1, 8) / 4;
}

size_t td_workspace_bytes(int64_t m, int64_t n, int64_t k, TdOffsets* off) {
  int64_t mpad, npad, K4;
  td_sizes(m, n, k, &mpad, &npad, &K4);
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = (size_t)round_up((int64_t)(o + bytes), 256); return r; };
  TdOffsets t{};
  t.amax = take(sizeof(uint64_t) * (size_t)mpad);
  t.bmax = take(sizeof(uint64_t) * (size_t)npad);
  t.aplanes = take(sizeof(double) * (size_t)(mpad / 16) * (size_t)td_block_stride(K4));
  t.bplanes = take(sizeof(double) * (size_t)(npad / 16) * (size_t)td_block_stride(K4));
  if (off) *off = t;
  return o;
}

hipError_t run_td(int64_t m, int64_t n, int64_t k, int64_t kc_in, const double* A0, const double* A1,
                  const double* A2, int64_t a_si, int64_t a_sp, const double* B0, const double* B1,
                  const double* B2, int64_t b_sp, int64_t b_sj, double* C0, double* C1, double* C2,
                  int64_t ldc, char* ws, hipStream_t s) {
  int64_t mpad, npad, K4;
  td_sizes(m, n, k, &mpad, &npad, &K4);
  const int64_t tiles = (mpad / 64) * (npad / 64);
  if (tiles <= 0 || tiles > 0x7fffffff) return hipErrorInvalidValue;
  TdOffsets off;
  td_workspace_bytes(m, n, k, &off);
  uint64_t* amax = (uint64_t*)(ws + off.amax);
  uint64_t* bmax = (uint64_t*)(ws + off.bmax);
  double* Ap = (double*)(ws + off.aplanes);
  double* Bp = (double*)(ws + off.bplanes);
  // one block when k <= kc (padding included), else blocks of kc (a multiple of 4)
  const int64_t kc = k < kc_in ? k : kc_in;
  const int32_t kcq = (int32_t)(k <= kc_in ? K4 : kc_in / 4);
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
  hipError_t e = launch_fill_u64(amax, mpad, 0, s);
  if (e == hipSuccess) e = launch_fill_u64(bmax, npad, 0, s);
  if (e == hipSuccess) e = launch_max_abs_bits(A0, m, k, a_si, a_sp, amax, s);
  if (e == hipSuccess) e = launch_max_abs_bits(B0, n, k, b_sj, b_sp, bmax, s);
  if (e != hipSuccess) return e;
  const int64_t nfa = (mpad / 16) * K4, nfb = (npad / 16) * K4;
  td_pack_a<<<(unsigned)((nfa + 3) / 4), 256, 0, s>>>(A0, A1, A2, a_si, a_sp, m, k, K4, nfa, amax, W, Ap);
  td_pack_b<<<(unsigned)((nfb + 3) / 4), 256, 0, s>>>(B0, B1, B2, b_sp, b_sj, k, n, K4, nfb, bmax, W, Bp);
  td_cascade_kernel<<<(unsigned)tiles, kWaves3 * 64, 0, s>>>(Ap, Bp, amax, bmax, K4, kcq, m, n, mpad / 64,
                                                              npad / 64, C0, C1, C2, ldc);
  return hipGetLastError();
}

}  // namespace ddk
