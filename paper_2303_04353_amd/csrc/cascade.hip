// Phases two and three of the cascade (Sec. 4), fused: the ten FP64 digit
// products of eq. (Gemm10) on the FP64 matrix cores, accumulated per rank-kc
// update into bins 0, 1, 2 and 3-6 (bins 0-2 exact, Sec. 3.3), the bins added
// in FP64x2 from the least significant one (Sec. 3.3, 3.6), the rank-kc
// results accumulated in FP64x2, Sigma and T applied and C added last.
//
// Work decomposition (gfx950): a workgroup of 8 waves (two per SIMD) owns a
// 64x64 tile of C, each wave a 16x32 piece.  The products use
// v_mfma_f64_4x4x4_4b_f64, which runs at the full FP64 matrix rate on gfx950
// (the 16x16x4 form does not): one instruction multiplies a 4-row sub-block
// of A (the same 16 values in all four MFMA blocks) by a 16-column group of B
// (four 4-column blocks).  A wave holds, per group of 4 inner indices, 4 A
// registers per plane and 2 B registers per plane, and 4 bins x 4 x 2
// accumulator registers; with two waves per SIMD one wave's products cover
// the other's LDS reads.
//
// Operand staging: per LDS stage (2 groups of 4 inner indices) the
// workgroup's 64 rows of A (4 planes) and 64 columns of B (5 stored planes)
// are copied from the packed planes into LDS with global_load_lds_dwordx4,
// 36 copies of 1 KiB dealt round robin to the 8 waves.  Four stage buffers
// rotate, three stages in flight while one is multiplied.  Copies are waited
// for with explicit vmcnt counts and a plain s_barrier.  FP64 vector work
// does not overlap the matrix cores on gfx950, so the loop keeps vector
// instructions to the two additions that form B4' and B5'.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dd_device.hpp"
#include "kernels.hpp"
#include "layout.hpp"

namespace ddk {

namespace {

constexpr int kWaves = 8;               // waves per workgroup
constexpr int kWaveCB = 2;              // 16-column groups per wave
constexpr int kSub = 4;                 // 4-row sub-blocks per wave (one 16-row block)
constexpr int kTile = 64;               // workgroup tile (rows and columns)

// LDS stage: A [16-row block 0..3][group h][plane 4][64], B [16-col block][h][plane 5][64]
constexpr int kStageQ = 2;                                 // groups of 4 inner indices per stage
constexpr int kNStage = 4;                                 // stage buffers in LDS
constexpr int kAStage = 4 * kStageQ * kFragA * kLanes;     // doubles
constexpr int kBStage = 4 * kStageQ * kFragB * kLanes;
constexpr int kStage = kAStage + kBStage;                  // 36 KiB
constexpr int kDmaA = 4 * kStageQ * kFragA * kLanes / 128; // 1 KiB copies per stage, A (16)
constexpr int kDmaB = 4 * kStageQ * kFragB * kLanes / 128; // and B (20)
constexpr int kDma = kDmaA + kDmaB;                        // 36, copy d goes to wave d % 8
constexpr int kDmaHi = (kDma + kWaves - 1) / kWaves;       // copies of waves 0..3
constexpr int kDmaLo = kDma / kWaves;                      // copies of waves 4..7
static_assert(kDma % kWaves == 4 && kDmaHi == 5 && kDmaLo == 4, "copy split assumed below");

typedef __attribute__((address_space(3))) void lds_void;

__device__ __forceinline__ double mfma4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void dma_1k(const double* src, double* lds_dst) {
  __builtin_amdgcn_global_load_lds((const void*)src, (lds_void*)lds_dst, 16, 0, 0);
}

// Waits until at most `ahead` stages of this wave's copies are outstanding
// (vector memory operations complete in order); `hi` selects 5 or 4 copies
// per stage.
__device__ __forceinline__ void wait_stages(int ahead, bool hi) {
  if (hi) {
    if (ahead >= 3) asm volatile("s_waitcnt vmcnt(15)" ::: "memory");
    else if (ahead == 2) asm volatile("s_waitcnt vmcnt(10)" ::: "memory");
    else if (ahead == 1) asm volatile("s_waitcnt vmcnt(5)" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  } else {
    if (ahead >= 3) asm volatile("s_waitcnt vmcnt(12)" ::: "memory");
    else if (ahead == 2) asm volatile("s_waitcnt vmcnt(8)" ::: "memory");
    else if (ahead == 1) asm volatile("s_waitcnt vmcnt(4)" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  }
}

__device__ __forceinline__ void lds_barrier() { asm volatile("s_barrier" ::: "memory"); }

// Operands of one group of 4 inner indices.  A register (sub-block s, plane
// t) of lane 16k + 4b + i holds position s*16 + k*4 + i of the wave's 16-row
// block; B registers hold the planes B0'..B6' (B4', B5' formed here).
struct Ops {
  double a[4][kSub];
  double b[7][kWaveCB];
};

__device__ __forceinline__ void read_ops(Ops& o, const double* sA, const double* sB, int h) {
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int s = 0; s < kSub; ++s) o.a[t][s] = sA[h * (kFragA * kLanes) + t * kLanes + s * 16];
#pragma unroll
  for (int g = 0; g < kWaveCB; ++g) {
    const double* b = sB + (g * kStageQ + h) * (kFragB * kLanes);
    o.b[0][g] = b[0 * kLanes];
    o.b[1][g] = b[1 * kLanes];
    o.b[2][g] = b[2 * kLanes];
    o.b[3][g] = b[3 * kLanes];
    o.b[6][g] = b[4 * kLanes];
  }
}

__device__ __forceinline__ void derive_b(Ops& o) {
#pragma unroll
  for (int g = 0; g < kWaveCB; ++g) {
    o.b[4][g] = o.b[2][g] + o.b[3][g];   // sigma_2 B4 = B2' + B3'
    o.b[5][g] = o.b[1][g] + o.b[4][g];   // sigma_1 B5 = B1' + B2' + B3'
  }
}

struct Bins {
  double b0[kSub][kWaveCB], b1[kSub][kWaveCB], b2[kSub][kWaveCB], b36[kSub][kWaveCB];
};

// The ten products of eq. (Gemm10) for one group of 4 inner indices; each
// product is 8 independent MFMAs.
__device__ __forceinline__ void ten_products(Bins& B, const Ops& o) {
#define DD_PRODUCT(BIN, TA, TB)                                 \
  _Pragma("unroll") for (int i = 0; i < kSub; ++i)              \
  _Pragma("unroll") for (int g = 0; g < kWaveCB; ++g)           \
      B.BIN[i][g] = mfma4(o.a[TA][i], o.b[TB][g], B.BIN[i][g]);
  DD_PRODUCT(b0, 0, 0)
  DD_PRODUCT(b1, 0, 1)
  DD_PRODUCT(b1, 1, 0)
  DD_PRODUCT(b2, 0, 2)
  DD_PRODUCT(b2, 1, 1)
  DD_PRODUCT(b2, 2, 0)
  DD_PRODUCT(b36, 0, 3)
  DD_PRODUCT(b36, 1, 4)
  DD_PRODUCT(b36, 2, 5)
  DD_PRODUCT(b36, 3, 6)
#undef DD_PRODUCT
}

// bin0 + (bin1 + (bin2 + bin36)) in FP64x2, added to the accumulator; bins reset.
__device__ __forceinline__ void combine(Bins& B, double (&acc_h)[kSub][kWaveCB],
                                        double (&acc_l)[kSub][kWaveCB]) {
#pragma unroll
  for (int i = 0; i < kSub; ++i)
#pragma unroll
    for (int g = 0; g < kWaveCB; ++g) {
      double s, e;
      two_sum(B.b2[i][g], B.b36[i][g], s, e);
      dd_add_d(s, e, B.b1[i][g], s, e);
      dd_add_d(s, e, B.b0[i][g], s, e);
      dd_add(acc_h[i][g], acc_l[i][g], s, e, acc_h[i][g], acc_l[i][g]);
      B.b0[i][g] = B.b1[i][g] = B.b2[i][g] = B.b36[i][g] = 0.0;
    }
}

// Workgroups are dealt to the 8 XCDs round robin (block b runs on XCD b % 8)
// and each XCD has its own L2.  Give every XCD a contiguous range of tiles
// and walk that range in groups of kGroupM tile rows, so the workgroups that
// run together on one XCD share a few A and B strips in its L2.
constexpr int64_t kXcds = 8;
constexpr int64_t kGroupM = 8;

__device__ __forceinline__ void tile_of_block(int64_t b, int64_t tiles_m, int64_t tiles_n,
                                              int64_t& tm, int64_t& tn) {
  const int64_t T = tiles_m * tiles_n;
  int64_t L = b;
  if (T % kXcds == 0) L = (b % kXcds) * (T / kXcds) + b / kXcds;
  const int64_t per_group = kGroupM * tiles_n;
  const int64_t g = L / per_group;
  const int64_t first_m = g * kGroupM;
  const int64_t gm = tiles_m - first_m < kGroupM ? tiles_m - first_m : kGroupM;
  const int64_t r = L - g * per_group;
  tm = first_m + r % gm;
  tn = r / gm;
}

__device__ __forceinline__ int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }

}  // namespace

__global__ void __launch_bounds__(kWaves * 64)
cascade_kernel(const double* __restrict__ Apack, const double* __restrict__ Bpack,
               const uint64_t* __restrict__ amax, const uint64_t* __restrict__ bmax,
               int64_t K4, int32_t kcq, int64_t m, int64_t n, int64_t tiles_m, int64_t tiles_n,
               double* __restrict__ Chi, double* __restrict__ Clo, int64_t ldc) {
  __shared__ __attribute__((aligned(16))) double lds[kNStage * kStage];

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave >> 1, wn = wave & 1;     // 16-row block wm, 32-column half wn
  int64_t tm, tn;
  tile_of_block(blockIdx.x, tiles_m, tiles_n, tm, tn);
  const int64_t rb0 = tm * 4 + wm;             // this wave's 16-row block
  const int64_t cb0 = tn * 4 + wn * kWaveCB;   // first 16-column group

  Bins bins;
  double acc_h[kSub][kWaveCB], acc_l[kSub][kWaveCB];
#pragma unroll
  for (int i = 0; i < kSub; ++i)
#pragma unroll
    for (int g = 0; g < kWaveCB; ++g) {
      bins.b0[i][g] = bins.b1[i][g] = bins.b2[i][g] = bins.b36[i][g] = 0.0;
      acc_h[i][g] = acc_l[i][g] = 0.0;
    }

  // Copy d of a stage (d = wave, wave + 8, ...): d < 16 is chunk d%4 of
  // 16-row block d/4 of A, otherwise chunk e%5 of 16-column block e/5 of B
  // (e = d - 16).  The packed planes of one block are contiguous over k.
  const bool hi = wave < (kDma % kWaves);
  const int ncopy = hi ? kDmaHi : kDmaLo;
  const int64_t nst = K4 / kStageQ;
  auto issue = [&](int64_t st) {
    double* buf = lds + (int)(st % kNStage) * kStage;
#pragma unroll
    for (int c = 0; c < kDmaHi; ++c) {
      if (c == kDmaHi - 1 && !hi) break;
      const int d = wave + c * kWaves;
      const double* src;
      double* dst;
      if (d < kDmaA) {
        const int blk = d >> 2, i = d & 3;
        src = Apack + (((tm * 4 + blk) * K4) + st * kStageQ) * (kFragA * kLanes) + i * 128;
        dst = buf + blk * (kStageQ * kFragA * kLanes) + i * 128;
      } else {
        const int e = d - kDmaA, blk = e / 5, i = e % 5;
        src = Bpack + (((tn * 4 + blk) * K4) + st * kStageQ) * (kFragB * kLanes) + i * 128;
        dst = buf + kAStage + blk * (kStageQ * kFragB * kLanes) + i * 128;
      }
      dma_1k(src + lane * 2, dst);
    }
  };
  (void)ncopy;

  auto a_ptr = [&](int64_t st) {
    return lds + (int)(st % kNStage) * kStage + wm * (kStageQ * kFragA * kLanes)
           + (lane >> 4) * 4 + (lane & 3);
  };
  auto b_ptr = [&](int64_t st) {
    return lds + (int)(st % kNStage) * kStage + kAStage + (wn * kWaveCB) * (kStageQ * kFragB * kLanes)
           + lane;
  };

  // Prologue: stages 0..2 in flight.
#pragma unroll
  for (int st = 0; st < kNStage - 1; ++st)
    if (st < nst) issue(st);

  int32_t inblk = 0;
  Ops ox, oy;
  for (int64_t st = 0; st < nst; ++st) {
    const int64_t last = nst - 1;
    wait_stages((int)(last - st < kNStage - 2 ? last - st : kNStage - 2), hi);
    lds_barrier();  // stage st is in LDS for every wave; stage st-1 is no longer read
    if (st + kNStage - 1 < nst) issue(st + kNStage - 1);
    const double* sA = a_ptr(st);
    const double* sB = b_ptr(st);
    read_ops(ox, sA, sB, 0);
    read_ops(oy, sA, sB, 1);
    derive_b(ox);
    ten_products(bins, ox);
    if (++inblk == kcq) { inblk = 0; combine(bins, acc_h, acc_l); }
    derive_b(oy);
    ten_products(bins, oy);
    if (++inblk == kcq) { inblk = 0; combine(bins, acc_h, acc_l); }
  }
  if (inblk != 0) combine(bins, acc_h, acc_l);

  // Epilogue: D lane 16i + 4b + j of (sub-block, group) holds row 4*sub + i,
  // column 16*group + 4b + j, i.e. row lane/16 and column lane%16.
#pragma unroll
  for (int i = 0; i < kSub; ++i) {
    const int64_t row = rb0 * 16 + i * 4 + (lane >> 4);
    if (row >= m) continue;
    const int er = exp_of_bits(amax[row]);
#pragma unroll
    for (int g = 0; g < kWaveCB; ++g) {
      const int64_t col = (cb0 + g) * 16 + (lane & 15);
      if (col >= n) continue;
      const int sh = er + exp_of_bits(bmax[col]);
      const double h = __builtin_ldexp(acc_h[i][g], sh);
      const double l = __builtin_ldexp(acc_l[i][g], sh);
      const int64_t idx = row + col * ldc;
      double rh, rl;
      dd_add(Chi[idx], Clo[idx], h, l, rh, rl);
      Chi[idx] = rh;
      Clo[idx] = rl;
    }
  }
}

hipError_t launch_cascade(const CascadeLayout& L, const double* Apack, const double* Bpack,
                          const uint64_t* amax, const uint64_t* bmax,
                          double* Chi, double* Clo, int64_t ldc, hipStream_t s) {
  if (L.tile_m != kTile || L.tile_n != kTile || L.K4 % kStageQ != 0) return hipErrorInvalidValue;
  const int64_t tiles_m = L.mpad / kTile, tiles_n = L.npad / kTile;
  const int64_t tiles = tiles_m * tiles_n;
  if (tiles <= 0 || tiles > 0x7fffffff) return hipErrorInvalidValue;
  cascade_kernel<<<(unsigned)tiles, kWaves * 64, 0, s>>>(Apack, Bpack, amax, bmax, L.K4, L.kcq, L.m, L.n,
                                                 tiles_m, tiles_n, Chi, Clo, ldc);
  return hipGetLastError();
}

}  // namespace ddk
