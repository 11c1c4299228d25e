// Phases two and three of the cascade (Sec. 4), fused: the ten FP64 digit
// products of eq. (Gemm10) on the FP64 matrix cores, accumulated per rank-kc
// update into bins 0, 1, 2 and 3-6 (bins 0-2 exact, Sec. 3.3), the bins added
// in FP64x2 from the least significant one (Sec. 3.3, 3.6), the rank-kc
// results accumulated in FP64x2, Sigma and T applied and C added last.
//
// Work decomposition (gfx950): a workgroup of 4 waves owns a 64x64 tile of C,
// each wave a 32x32 quarter.  The products use v_mfma_f64_4x4x4_4b_f64, which
// runs at the full FP64 matrix rate on gfx950 (the 16x16x4 form does not):
// one instruction multiplies a 4-row sub-block of A (the same 16 values in
// all four MFMA blocks) by a 16-column group of B (four 4-column blocks).  A
// wave therefore holds, per group of 4 inner indices, 8 A registers and
// 2 B registers per plane, and 4 bins x 8 x 2 accumulator registers.
// Operand staging: per LDS stage (2 groups of 4 inner indices) the
// workgroup's 64 rows of A (4 planes) and 64 columns of B (5 stored planes)
// are copied from the packed planes into LDS with global_load_lds_dwordx4
// (each wave moves one 16-row block of A and one 16-column block of B), four
// stages deep, so three stages are in flight while the matrix cores work on
// one.  The copies are waited for with explicit vmcnt counts and a plain
// s_barrier; waves then read their operands from LDS.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dd_device.hpp"
#include "kernels.hpp"
#include "layout.hpp"

namespace ddk {

namespace {

constexpr int kWaveRB = 2;              // 16-row blocks per wave
constexpr int kWaveCB = 2;              // 16-column groups per wave
constexpr int kSub = 4 * kWaveRB;       // 4-row sub-blocks per wave
constexpr int kTile = 64;               // workgroup tile (rows and columns)

__device__ __forceinline__ double mfma4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

struct Frags {
  double a[4][kSub];      // plane, 4-row sub-block
  double b[7][kWaveCB];   // plane B0'..B6', 16-column group
};

// LDS stage: A [16-row block 0..3][group h][plane 4][64], B [16-col block][h][plane 5][64]
constexpr int kStageQ = 2;                                 // groups of 4 inner indices per stage
constexpr int kNStage = 4;                                 // stages resident in LDS
constexpr int kAStage = 4 * kStageQ * kFragA * kLanes;     // doubles
constexpr int kBStage = 4 * kStageQ * kFragB * kLanes;
constexpr int kStage = kAStage + kBStage;                  // 36 KiB
constexpr int kDmaA = kStageQ * kFragA * kLanes / 128;     // 1 KiB copies per wave per stage
constexpr int kDmaB = kStageQ * kFragB * kLanes / 128;
constexpr int kDmaPerStage = kDmaA + kDmaB;

typedef __attribute__((address_space(3))) void lds_void;

__device__ __forceinline__ void dma_1k(const double* src, double* lds_dst) {
  __builtin_amdgcn_global_load_lds((const void*)src, (lds_void*)lds_dst, 16, 0, 0);
}

// Waits until at most `ahead` stages of this wave's copies are outstanding.
__device__ __forceinline__ void wait_stages(int ahead) {
  static_assert(kNStage == 4 && kDmaPerStage == 9, "vmcnt immediates assume 4 stages of 9 copies");
  if (ahead >= 2) asm volatile("s_waitcnt vmcnt(18)" ::: "memory");
  else if (ahead == 1) asm volatile("s_waitcnt vmcnt(9)" ::: "memory");
  else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

__device__ __forceinline__ void lds_barrier() { asm volatile("s_barrier" ::: "memory"); }

// Operands of group h of a stage, from LDS.  A register (sub-block i = 4r+s,
// plane t) of lane 16k + 4b + i' holds position s*16 + k*4 + i' of its block.
__device__ __forceinline__ void read_frags(Frags& f, const double* sA, const double* sB, int h) {
#pragma unroll
  for (int r = 0; r < kWaveRB; ++r) {
    const double* a = sA + (r * kStageQ + h) * (kFragA * kLanes);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int s = 0; s < 4; ++s) f.a[t][r * 4 + s] = a[t * kLanes + s * 16];
  }
#pragma unroll
  for (int g = 0; g < kWaveCB; ++g) {
    const double* b = sB + (g * kStageQ + h) * (kFragB * kLanes);
    f.b[0][g] = b[0 * kLanes];
    f.b[1][g] = b[1 * kLanes];
    f.b[2][g] = b[2 * kLanes];
    f.b[3][g] = b[3 * kLanes];
    f.b[6][g] = b[4 * kLanes];
    f.b[4][g] = f.b[2][g] + f.b[3][g];   // sigma_2 B4 = B2' + B3'
    f.b[5][g] = f.b[1][g] + f.b[4][g];   // sigma_1 B5 = B1' + B2' + B3'
  }
}

struct Bins {
  double b0[kSub][kWaveCB], b1[kSub][kWaveCB], b2[kSub][kWaveCB], b36[kSub][kWaveCB];
};

// The ten products of eq. (Gemm10) for one group of 4 inner indices.  Each
// product is 16 independent MFMAs, so consecutive updates of one accumulator
// are 16 instructions apart.
__device__ __forceinline__ void ten_products(Bins& B, const Frags& f) {
#define DD_PRODUCT(BIN, TA, TB)                                 \
  _Pragma("unroll") for (int i = 0; i < kSub; ++i)              \
  _Pragma("unroll") for (int g = 0; g < kWaveCB; ++g)           \
      B.BIN[i][g] = mfma4(f.a[TA][i], f.b[TB][g], B.BIN[i][g]);
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

}  // namespace

__global__ void __launch_bounds__(256)
cascade_kernel(const double* __restrict__ Apack, const double* __restrict__ Bpack,
               const uint64_t* __restrict__ amax, const uint64_t* __restrict__ bmax,
               int64_t K4, int32_t kcq, int64_t m, int64_t n, int64_t tiles_m, int64_t tiles_n,
               double* __restrict__ Chi, double* __restrict__ Clo, int64_t ldc) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  int64_t tm, tn;
  tile_of_block(blockIdx.x, tiles_m, tiles_n, tm, tn);
  const int64_t rb0 = tm * 4 + wm * kWaveRB;   // first 16-row block of this wave
  const int64_t cb0 = tn * 4 + wn * kWaveCB;   // first 16-column group

  __shared__ __attribute__((aligned(16))) double lds[kNStage * kStage];

  Bins bins;
  double acc_h[kSub][kWaveCB], acc_l[kSub][kWaveCB];
#pragma unroll
  for (int i = 0; i < kSub; ++i)
#pragma unroll
    for (int g = 0; g < kWaveCB; ++g) {
      bins.b0[i][g] = bins.b1[i][g] = bins.b2[i][g] = bins.b36[i][g] = 0.0;
      acc_h[i][g] = acc_l[i][g] = 0.0;
    }

  // This wave copies 16-row block tm*4 + wave of A and 16-column block
  // tn*4 + wave of B; the packed planes of one block are contiguous over k.
  const double* gA = Apack + ((tm * 4 + wave) * K4) * (kFragA * kLanes) + lane * 2;
  const double* gB = Bpack + ((tn * 4 + wave) * K4) * (kFragB * kLanes) + lane * 2;
  const int64_t nst = K4 / kStageQ;
  auto issue = [&](int64_t st) {
    double* dA = lds + (int)(st % kNStage) * kStage + wave * (kStageQ * kFragA * kLanes);
    double* dB = lds + (int)(st % kNStage) * kStage + kAStage + wave * (kStageQ * kFragB * kLanes);
    const double* sA = gA + st * (kStageQ * kFragA * kLanes);
    const double* sB = gB + st * (kStageQ * kFragB * kLanes);
#pragma unroll
    for (int i = 0; i < kDmaA; ++i) dma_1k(sA + i * 128, dA + i * 128);
#pragma unroll
    for (int i = 0; i < kDmaB; ++i) dma_1k(sB + i * 128, dB + i * 128);
  };
#pragma unroll
  for (int st = 0; st < kNStage - 1; ++st)
    if (st < nst) issue(st);

  Frags fx;
  int32_t inblk = 0;
  for (int64_t st = 0; st < nst; ++st) {
    const int64_t last = nst - 1;
    wait_stages((int)((last - st) < (kNStage - 2) ? (last - st) : (kNStage - 2)));
    lds_barrier();  // stage st is in LDS for every wave; stage st-1 is no longer read
    if (st + kNStage - 1 < nst) issue(st + kNStage - 1);
    const double* sA = lds + (int)(st % kNStage) * kStage + (wm * kWaveRB) * (kStageQ * kFragA * kLanes)
                       + (lane >> 4) * 4 + (lane & 3);
    const double* sB = lds + (int)(st % kNStage) * kStage + kAStage
                       + (wn * kWaveCB) * (kStageQ * kFragB * kLanes) + lane;
#pragma unroll
    for (int h = 0; h < kStageQ; ++h) {
      read_frags(fx, sA, sB, h);
      ten_products(bins, fx);
      if (++inblk == kcq) { inblk = 0; combine(bins, acc_h, acc_l); }
    }
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
  if (L.tile_m != kTile || L.tile_n != kTile) return hipErrorInvalidValue;
  const int64_t tiles_m = L.mpad / kTile, tiles_n = L.npad / kTile;
  const int64_t tiles = tiles_m * tiles_n;
  if (tiles <= 0 || tiles > 0x7fffffff) return hipErrorInvalidValue;
  cascade_kernel<<<(unsigned)tiles, 256, 0, s>>>(Apack, Bpack, amax, bmax, L.K4, L.kcq, L.m, L.n,
                                                 tiles_m, tiles_n, Chi, Clo, ldc);
  return hipGetLastError();
}

}  // namespace ddk
