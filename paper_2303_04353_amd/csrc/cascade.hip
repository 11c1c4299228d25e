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
// workgroup's 64 rows of A (4 planes) and 64 columns of B (7 planes), 44
// KiB, are loaded from the packed planes into registers (16-byte loads, 44
// pieces of 1 KiB dealt round robin to the 8 waves; a wave with five pieces
// moves its first one twice, so every wave runs the same branch-free code),
// then written to the other of two LDS buffers; one barrier per
// stage.  (Direct global-to-LDS copies would save the registers, but their
// completion is tracked with the LDS counter as well, so every wait for an
// operand read would also wait for the copies in flight.)  Every memory
// instruction is issued between MFMAs: group 0's MFMAs carry the reads of
// group 1 and, at their end, the LDS writes of the next stage; group 1's
// MFMAs carry, first, the global loads of the stage after that, then the
// reads of the next stage's group 0.  Both waves of a SIMD meet at the
// barrier, so nothing but the wait for the writes is left there.  Vector
// instructions, integer ones included, do not overlap the matrix cores on
// gfx950, so the loop has next to none: B4' and B5' are stored planes
// rather than sums formed here, staging addresses are wave-uniform (scalar)
// bases plus the lane's 16 bytes, and the loop takes two stages at a time
// so LDS buffer offsets are constants.  Batched plans, whose short-k tiles
// gain less from this than their packing pays for two more planes, and the
// split-on-load kernel store five B planes and form B4' and B5' with two
// additions per column group.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "dd_device.hpp"
#include "kernels.hpp"
#include "layout.hpp"

namespace ddk {

namespace {

constexpr int kWaves = 8;               // waves per workgroup
constexpr int kSub = 4;                 // 4-row sub-blocks per wave (one 16-row block)
constexpr int kStageQ = 2;              // groups of 4 inner indices per LDS stage
constexpr int kNBuf = 2;                // stage buffers in LDS

// A workgroup tile of TM x TN outputs (64 x 64, 32 x 64 or 64 x 32): the
// 16-row blocks and 16-column groups are dealt to the 8 waves, 16 rows by
// kWaveCB column groups each (two for 64 x 64, one otherwise).  LDS stage:
// A [16-row block][group h][plane 4][64], B [16-col block][h][plane FB][64],
// FB the stored B planes (7, or 5 in batched plans: B4', B5' formed here).
template <int TM, int TN, int FB = kFragB>
struct Shape {
  static constexpr int kFB = FB;
  static constexpr int kRB = TM / 16;                        // 16-row blocks
  static constexpr int kCB = TN / 16;                        // 16-column groups
  static constexpr int kWaveCB = kRB * kCB / kWaves;         // column groups per wave
  static constexpr int kWavesN = kCB / kWaveCB;              // waves along a row of the tile
  static constexpr int kAStage = kRB * kStageQ * kFragA * kLanes;   // doubles
  static constexpr int kBStage = kCB * kStageQ * FB * kLanes;
  static constexpr int kStage = kAStage + kBStage;
  static constexpr int kPieceA = kRB * 4;                    // 1 KiB pieces per stage
  static constexpr int kPieceB = kCB * FB;
  static constexpr int kPieces = kPieceA + kPieceB;          // piece d goes to wave d % 8
  static constexpr int kPiecesMax = (kPieces + kWaves - 1) / kWaves;
  static_assert(kWaveCB >= 1 && kRB * kCB == kWaves * kWaveCB, "8 waves cover the tile");
};
using Shape64x64 = Shape<64, 64>;
using Shape32x64 = Shape<32, 64>;
using Shape64x32 = Shape<64, 32>;
using BShape64x64 = Shape<64, 64, kFragBBatched>;   // batched plans
using BShape32x64 = Shape<32, 64, kFragBBatched>;
using BShape64x32 = Shape<64, 32, kFragBBatched>;
constexpr int kLdsBatched = kNBuf * BShape64x64::kStage;    // 72 KiB, the largest batched shape's

typedef double d2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double mfma4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void lds_barrier() { asm volatile("s_barrier" ::: "memory"); }
__device__ __forceinline__ void lds_reads_done() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// The scheduler's order for the MFMAs of one group (80 with two column
// groups per wave, 40 with one) and the memory instructions issued among
// them (the LDS reads of the next operand set are 15 two-word reads, or 12,
// with 7 stored B planes; 13 or 11 with 5).
// Group 0: the reads of the next operands, then the LDS writes of the staged
// stage, spread over the MFMAs.
template <int CB, int NP, int FB>
__device__ __forceinline__ void interleave_reads_writes() {
  constexpr int R = CB == 2 ? (FB == 7 ? 15 : 13) : (FB == 7 ? 12 : 11), MR = CB == 2 ? 4 : 2;
  constexpr int MW = FB == 7 ? 3 : (CB == 2 ? 5 : 4);
#pragma unroll
  for (int i = 0; i < R; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // DS read
    __builtin_amdgcn_sched_group_barrier(0x008, MR, 0);  // MFMA
  }
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);   // DS write
    __builtin_amdgcn_sched_group_barrier(0x008, MW, 0);  // MFMA
  }
}

// Group 1: the global loads of a later stage, then the reads.
template <int CB, int NP, int FB>
__device__ __forceinline__ void interleave_reads_loads() {
  constexpr int R = CB == 2 ? (FB == 7 ? 15 : 13) : (FB == 7 ? 12 : 11), ML = CB == 2 ? 3 : 2;
  constexpr int MR = CB == 2 ? (FB == 7 ? 4 : 5) : 2;
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);   // VMEM read
    __builtin_amdgcn_sched_group_barrier(0x008, ML, 0);  // MFMA
  }
#pragma unroll
  for (int i = 0; i < R; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // DS read
    __builtin_amdgcn_sched_group_barrier(0x008, MR, 0);  // MFMA
  }
}

// Operands of one group of 4 inner indices.  A register (sub-block s, plane
// t) of lane 16k + 4b + i holds position s*16 + k*4 + i of the wave's 16-row
// block; B registers hold the planes B0'..B6' (with 5 stored planes, B4'
// and B5' formed by derive_b).
template <int CB>
struct Ops {
  double a[4][kSub];
  double b[7][CB];
};

template <int CB, int FB>
__device__ __forceinline__ void read_ops(Ops<CB>& o, const double* sA, const double* sB, int h) {
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int s = 0; s < kSub; ++s) o.a[t][s] = sA[h * (kFragA * kLanes) + t * kLanes + s * 16];
#pragma unroll
  for (int g = 0; g < CB; ++g) {
    const double* b = sB + (g * kStageQ + h) * (FB * kLanes);
    if constexpr (FB == 7) {
#pragma unroll
      for (int t = 0; t < 7; ++t) o.b[t][g] = b[t * kLanes];
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t) o.b[t][g] = b[t * kLanes];
      o.b[6][g] = b[4 * kLanes];
    }
  }
}

// B4' and B5' of operands read from 5 stored planes.
template <int CB, int FB>
__device__ __forceinline__ void derive_b(Ops<CB>& o) {
  if constexpr (FB == 5) {
#pragma unroll
    for (int g = 0; g < CB; ++g) {
      o.b[4][g] = o.b[2][g] + o.b[3][g];   // sigma_2 B4 = B2' + B3'
      o.b[5][g] = o.b[1][g] + o.b[4][g];   // sigma_1 B5 = B1' + B2' + B3'
    }
  }
}

template <int CB>
struct Bins {
  double b0[kSub][CB], b1[kSub][CB], b2[kSub][CB], b36[kSub][CB];
};

// The ten products of eq. (Gemm10) for one group of 4 inner indices; each
// product is 4 CB independent MFMAs.  The products are ordered so that no
// two consecutive ones update the same bin: an MFMA then depends on one
// issued at least 8 CB instructions earlier, which keeps the matrix core busy.
template <int CB>
__device__ __forceinline__ void ten_products(Bins<CB>& B, const Ops<CB>& o) {
#define DD_PRODUCT(BIN, TA, TB)                                 \
  _Pragma("unroll") for (int i = 0; i < kSub; ++i)              \
  _Pragma("unroll") for (int g = 0; g < CB; ++g)                \
      B.BIN[i][g] = mfma4(o.a[TA][i], o.b[TB][g], B.BIN[i][g]);
  DD_PRODUCT(b36, 0, 3)
  DD_PRODUCT(b2, 0, 2)
  DD_PRODUCT(b36, 1, 4)
  DD_PRODUCT(b2, 1, 1)
  DD_PRODUCT(b36, 2, 5)
  DD_PRODUCT(b1, 0, 1)
  DD_PRODUCT(b36, 3, 6)
  DD_PRODUCT(b1, 1, 0)
  DD_PRODUCT(b2, 2, 0)
  DD_PRODUCT(b0, 0, 0)
#undef DD_PRODUCT
}

// bin0 + (bin1 + (bin2 + bin36)) in FP64x2, added to the accumulator; bins reset.
// With kFlags, bit (i * CB + g) of `flg` is set when this block's bin 0
// is zero while a lower bin is not (cancellation, Sec. 3.7 and Sec. 4.4).
// With kPanel, the block's result is first scaled by its own Sigma and T,
// 2^(ea[4 i] + fb[16 g]) (exact), so the accumulator holds unscaled values.
template <bool kFlags, bool kPanel, int CB>
__device__ __forceinline__ void combine(Bins<CB>& B, double (&acc_h)[kSub][CB], double (&acc_l)[kSub][CB],
                                        uint32_t& flg, const int32_t* __restrict__ ea,
                                        const int32_t* __restrict__ fb) {
  int fc[CB];
  if constexpr (kPanel) {
#pragma unroll
    for (int g = 0; g < CB; ++g) fc[g] = fb[g * 16];
  }
#pragma unroll
  for (int i = 0; i < kSub; ++i) {
    int er = 0;
    if constexpr (kPanel) er = ea[i * 4];
#pragma unroll
    for (int g = 0; g < CB; ++g) {
      if constexpr (kFlags) {
        const bool lower = B.b1[i][g] != 0.0 || B.b2[i][g] != 0.0 || B.b36[i][g] != 0.0;
        if (B.b0[i][g] == 0.0 && lower) flg |= 1u << (i * CB + g);
      }
      double s, e;
      two_sum(B.b2[i][g], B.b36[i][g], s, e);
      dd_add_d(s, e, B.b1[i][g], s, e);
      dd_add_d(s, e, B.b0[i][g], s, e);
      if constexpr (kPanel) {
        s = __builtin_ldexp(s, er + fc[g]);
        e = __builtin_ldexp(e, er + fc[g]);
      }
      dd_add(acc_h[i][g], acc_l[i][g], s, e, acc_h[i][g], acc_l[i][g]);
      B.b0[i][g] = B.b1[i][g] = B.b2[i][g] = B.b36[i][g] = 0.0;
    }
  }
}

__device__ __forceinline__ int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }

}  // namespace

// One TM x TN output tile (tile row tm, tile column tn) of one GEMM,
// computed by the whole workgroup.  `lds` is the workgroup's staging memory.
// With kFlags, entries at risk of cancellation get their bit set in the m x n
// column-major bitmap `flags` (bit i + j*m).  With kPanel, the exponents of
// Sigma and T of rank-kc block b are aexp[b * astride + i] and
// bexp[b * bstride + j] and are applied to each block's result; otherwise
// the maxima amax[i], bmax[j] give the exponents that scale the sum.  The
// arithmetic of every output entry is the same for every tile shape.
template <bool kFlags, bool kPanel, class SH, bool kBuf = false>
__device__ __forceinline__ void cascade_tile(double* __restrict__ lds, const double* __restrict__ Apack,
                                             const double* __restrict__ Bpack,
                                             const uint64_t* __restrict__ amax,
                                             const uint64_t* __restrict__ bmax, int64_t K4, int32_t kcq,
                                             int64_t m, int64_t n, int64_t tm, int64_t tn,
                                             double* __restrict__ Chi, double* __restrict__ Clo,
                                             int64_t ldc, uint32_t* __restrict__ flags,
                                             const int32_t* __restrict__ aexp = nullptr,
                                             const int32_t* __restrict__ bexp = nullptr,
                                             int64_t astride = 0, int64_t bstride = 0) {
  constexpr int CB = SH::kWaveCB, FB = SH::kFB;
  constexpr int kPiecesMax = SH::kPiecesMax, kPieceA = SH::kPieceA, kAStage = SH::kAStage;
  constexpr int kStage = SH::kStage;
  uint32_t flg = 0;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave / SH::kWavesN, wn = wave % SH::kWavesN;   // 16-row block, column-group set
  const int64_t rb0 = tm * SH::kRB + wm;       // this wave's 16-row block
  const int64_t cb0 = tn * SH::kCB + wn * CB;  // its first 16-column group

  Bins<CB> bins;
  double acc_h[kSub][CB], acc_l[kSub][CB];
#pragma unroll
  for (int i = 0; i < kSub; ++i)
#pragma unroll
    for (int g = 0; g < CB; ++g) {
      bins.b0[i][g] = bins.b1[i][g] = bins.b2[i][g] = bins.b36[i][g] = 0.0;
      acc_h[i][g] = acc_l[i][g] = 0.0;
    }

  // Piece d of a stage (d = wave, wave + 8, ...): d < kPieceA is chunk d%4
  // of 16-row block d/4 of A, otherwise chunk e%5 of 16-column block e/5 of
  // B (e = d - kPieceA).  The packed planes of one block are contiguous over k.
  // Every wave moves kPiecesMax pieces; a wave with fewer repeats piece 0
  // (the same data to the same place), so the code has no branch.  A
  // piece's source, stride and LDS place are the same for all lanes of the
  // wave (scalar registers); each lane adds its own 16 bytes.  Vector
  // instructions in this loop take issue cycles from the matrix cores, so
  // the per-stage address work is kept scalar.
  constexpr int kRem = SH::kPieces % kWaves;
  __builtin_assume(wave >= 0 && wave < kWaves);   // 8 waves per workgroup
  const int npiece = (kRem == 0 || wave < kRem) ? kPiecesMax : kPiecesMax - 1;
  const int64_t strideA = kStageQ * kFragA * kLanes, strideB = kStageQ * FB * kLanes;
  const double* pbase[kPiecesMax];
  int64_t pstride[kPiecesMax];
  int pdst[kPiecesMax];
#pragma unroll
  for (int c = 0; c < kPiecesMax; ++c) {
    const int d = c < npiece ? wave + c * kWaves : wave;   // unused slots repeat piece 0
    if (d < kPieceA) {
      const int blk = d >> 2, i = d & 3;
      pbase[c] = Apack + (tm * SH::kRB + blk) * a_block_stride(K4) + i * 128;
      pstride[c] = strideA;
      pdst[c] = blk * (kStageQ * kFragA * kLanes) + i * 128;
    } else {
      const int e = d - kPieceA, blk = e / FB, i = e % FB;
      pbase[c] = Bpack + (tn * SH::kCB + blk) * b_block_stride(K4, FB) + i * 128;
      pstride[c] = strideB;
      pdst[c] = kAStage + blk * (kStageQ * FB * kLanes) + i * 128;
    }
  }
  d2 stg[kPiecesMax];
  auto load_stage = [&](int64_t st) {
#pragma unroll
    for (int c = 0; c < kPiecesMax; ++c) stg[c] = *(const d2*)(pbase[c] + st * pstride[c] + lane * 2);
  };
  // With kBuf the loop loads through buffer resources over the tile's A and
  // B blocks: the piece's offset, stage included, is scalar and the lane's
  // 16 bytes are the only vector part, so no vector instruction forms an
  // address (32-bit offsets: the host takes this form while the tile's
  // blocks span less than 2 GiB).
  const char* tileA = (const char*)(Apack + tm * SH::kRB * a_block_stride(K4));
  const char* tileB = (const char*)(Bpack + tn * SH::kCB * b_block_stride(K4, FB));
  // dword 3 of a raw buffer resource on gfx9 parts: 32-bit data, no swizzle
  const __amdgpu_buffer_rsrc_t rA = __builtin_amdgcn_make_buffer_rsrc(
      (void*)tileA, (short)0, kBuf ? (int)(SH::kRB * a_block_stride(K4) * 8) : 0, 0x00020000);
  const __amdgpu_buffer_rsrc_t rB = __builtin_amdgcn_make_buffer_rsrc(
      (void*)tileB, (short)0, kBuf ? (int)(SH::kCB * b_block_stride(K4, FB) * 8) : 0, 0x00020000);
  bool isA[kPiecesMax];
  uint32_t poff[kPiecesMax];   // byte offset of the piece's stage-0 chunk in its tile
#pragma unroll
  for (int c = 0; c < kPiecesMax; ++c) {
    isA[c] = pstride[c] == strideA;
    poff[c] = kBuf ? (uint32_t)((const char*)pbase[c] - (isA[c] ? tileA : tileB)) : 0u;
  }
  const uint32_t loff = (uint32_t)lane * 16u;
  auto load_stage_buf = [&](int32_t st) {
#pragma unroll
    for (int c = 0; c < kPiecesMax; ++c) {
      const uint32_t so = poff[c] + (uint32_t)st * (uint32_t)(pstride[c] * 8);
      stg[c] = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(isA[c] ? rA : rB, loff, so, 0));
    }
  };
  auto store_buf = [&](int b) {   // into stage buffer b
    double* buf = lds + b * kStage + lane * 2;
#pragma unroll
    for (int c = 0; c < kPiecesMax; ++c) *(d2*)(buf + pdst[c]) = stg[c];
  };
  auto store_stage = [&](int64_t st) { store_buf((int)(st % kNBuf)); };

  auto a_ptr = [&](int64_t st) {
    return lds + (int)(st % kNBuf) * kStage + wm * (kStageQ * kFragA * kLanes)
           + (lane >> 4) * 4 + (lane & 3);
  };
  auto b_ptr = [&](int64_t st) {
    return lds + (int)(st % kNBuf) * kStage + kAStage + (wn * CB) * (kStageQ * FB * kLanes)
           + lane;
  };

  // Prologue: stage 0 into LDS, stage 1 into the staging registers.
  const int64_t nst = K4 / kStageQ;
  const int64_t last = nst - 1;
  load_stage(0);
  store_stage(0);
  load_stage(nst > 1 ? 1 : 0);
  lds_reads_done();
  lds_barrier();
  Ops<CB> ox, oy;
  read_ops<CB, FB>(ox, a_ptr(0), b_ptr(0), 0);

  // Per stage st: group 0's products (ox) run while group 1 is read into oy
  // and stage st+1 (staged in registers) is written to the other buffer,
  // whose last reads ended before the previous barrier; after the barrier
  // group 1's products (oy) run while group 0 of stage st+1 is read into ox
  // and stage st+2 is loaded.  The last iteration writes, reads and loads
  // in-bounds copies that are not used.  The loop takes two stages at a
  // time (nst is even), so each stage's buffer is known at compile time and
  // every LDS address is a fixed offset from the lane's own.
  int32_t inblk = 0, blk = 0;
  auto block_done = [&]() {
    const int32_t* ea = nullptr;
    const int32_t* fb = nullptr;
    if constexpr (kPanel) {
      int l = threadIdx.x & 63;
      asm volatile("" : "+v"(l));
      ea = aexp + blk * astride + rb0 * 16 + (l >> 4);
      fb = bexp + blk * bstride + cb0 * 16 + (l & 15);
    }
    combine<kFlags, kPanel, CB>(bins, acc_h, acc_l, flg, ea, fb);
    ++blk;
  };
  const double* a0 = a_ptr(0);
  const double* b0 = b_ptr(0);
  auto one_stage = [&](int64_t st, int b) {   // stage st, in buffer b
    read_ops<CB, FB>(oy, a0 + b * kStage, b0 + b * kStage, 1);
    derive_b<CB, FB>(ox);
    store_buf(b ^ 1);
    ten_products(bins, ox);
    interleave_reads_writes<CB, kPiecesMax, FB>();
    if (++inblk == kcq) { inblk = 0; block_done(); }
    derive_b<CB, FB>(oy);
    lds_reads_done();
    lds_barrier();
    read_ops<CB, FB>(ox, a0 + (b ^ 1) * kStage, b0 + (b ^ 1) * kStage, 0);
    // stage numbers fit in 32 bits (the planes of 2^31 stages would not fit
    // in memory), and the 32-bit compare is a scalar one
    const int32_t s2 = (int32_t)st + 2;
    if constexpr (kBuf) {
      load_stage_buf(s2 <= (int32_t)last ? s2 : (int32_t)last);
    } else {
      load_stage(s2 <= (int32_t)last ? s2 : (int32_t)last);
    }
    ten_products(bins, oy);
    interleave_reads_loads<CB, kPiecesMax, FB>();
    if (++inblk == kcq) { inblk = 0; block_done(); }
  };
  for (int64_t st = 0; st < nst; st += 2) {
    one_stage(st, 0);
    one_stage(st + 1, 1);
  }
  if (inblk != 0) block_done();

  // Epilogue: Sigma and T (unless applied per block), then C + result.
#pragma unroll
  for (int i = 0; i < kSub; ++i) {
    const int64_t row = rb0 * 16 + i * 4 + (lane >> 4);
    if (row >= m) continue;
    const int er = kPanel ? 0 : exp_of_bits(amax[row]);
#pragma unroll
    for (int g = 0; g < CB; ++g) {
      const int64_t col = (cb0 + g) * 16 + (lane & 15);
      if (col >= n) continue;
      const int sh = kPanel ? 0 : er + exp_of_bits(bmax[col]);
      const double h = __builtin_ldexp(acc_h[i][g], sh);
      const double l = __builtin_ldexp(acc_l[i][g], sh);
      const int64_t idx = row + col * ldc;
      double rh, rl;
      dd_add(Chi[idx], Clo[idx], h, l, rh, rl);
      Chi[idx] = rh;
      Clo[idx] = rl;
      if constexpr (kFlags) {
        if (flg & (1u << (i * CB + g))) {
          const int64_t bit = row + col * m;
          atomicOr(&flags[bit >> 5], 1u << (bit & 31));
        }
      }
    }
  }
}

// Split on load (the paper cascades while it packs, Sec. 4.3): the same
// product loop over one 64x64 tile, but the operands come straight from
// the caller's hi/lo planes.  Per stage of 8 inner indices each thread
// loads one entry of op(A) and one of op(B) (consecutive threads take
// consecutive addresses: rows of A or inner indices of B when those are
// contiguous), splits them as phase one's packing does (Appendix A, the
// same operations) and writes the digits to the LDS stage in the packed
// fragment order, so every product and every bit of the result equal the
// packed path's.  No digit planes exist in memory; the split is redone by
// every workgroup that stages an operand tile, on the vector units, which
// do not overlap the FP64 matrix cores.
template <bool kFlags>
__device__ __forceinline__ void cascade_tile_onload(double* __restrict__ lds, const double* __restrict__ Ahi,
                                                    const double* __restrict__ Alo, int64_t a_si, int64_t a_sp,
                                                    const double* __restrict__ Bhi, const double* __restrict__ Blo,
                                                    int64_t b_sp, int64_t b_sj, const uint64_t* __restrict__ amax,
                                                    const uint64_t* __restrict__ bmax, int c0, int c1, int c2,
                                                    int64_t K4, int32_t kcq, int64_t m, int64_t n, int64_t k,
                                                    int64_t tm, int64_t tn, double* __restrict__ Chi,
                                                    double* __restrict__ Clo, int64_t ldc,
                                                    uint32_t* __restrict__ flags) {
  // five B planes in LDS, B4' and B5' formed from them (registers are short here)
  using SH = BShape64x64;
  constexpr int CB = SH::kWaveCB, kStage = SH::kStage, kAStage = SH::kAStage, FB = SH::kFB;
  uint32_t flg = 0;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int wm = wave / SH::kWavesN, wn = wave % SH::kWavesN;
  const int64_t rb0 = tm * SH::kRB + wm, cb0 = tn * SH::kCB + wn * CB;

  Bins<CB> bins;
  double acc_h[kSub][CB], acc_l[kSub][CB];
#pragma unroll
  for (int i = 0; i < kSub; ++i)
#pragma unroll
    for (int g = 0; g < CB; ++g) {
      bins.b0[i][g] = bins.b1[i][g] = bins.b2[i][g] = bins.b36[i][g] = 0.0;
      acc_h[i][g] = acc_l[i][g] = 0.0;
    }

  // This thread's entry of each stage: row ia and inner index 8 st + pa of
  // op(A); inner index 8 st + pb and column jb of op(B).
  const bool a_rows = a_si == 1, b_inner = b_sp == 1;
  const int ia = a_rows ? (t & 63) : (t >> 3), pa = a_rows ? (t >> 6) : (t & 7);
  const int pb = b_inner ? (t & 7) : (t >> 6), jb = b_inner ? (t >> 3) : (t & 63);
  const int64_t row = tm * 64 + ia, col = tn * 64 + jb;
  const int ea = row < m ? exp_of_bits(amax[row]) : 0;
  const int eb = col < n ? exp_of_bits(bmax[col]) : 0;
  // LDS positions of the digits: A block ia/16, group pa/4, plane p at
  // p*64 + s*16 + kk*4 + ii (ia%16 = 4s + ii, kk = pa%4); B block jb/16,
  // group pb/4, plane p at p*64 + kk*16 + c (c = jb%16, kk = pb%4)
  const int adst = (ia >> 4) * (kStageQ * kFragA * kLanes) + (pa >> 2) * (kFragA * kLanes)
                   + ((ia & 15) >> 2) * 16 + (pa & 3) * 4 + (ia & 3);
  const int bdst = kAStage + (jb >> 4) * (kStageQ * FB * kLanes) + (pb >> 2) * (FB * kLanes)
                   + (pb & 3) * 16 + (jb & 15);
  SplitParams sp;
  {
    const int c[3] = {c0, c1, c2};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      sp.K[q] = __builtin_ldexp(1.0, 53 - c[q]) + __builtin_ldexp(1.0, 52 - c[q]);
      sp.P[q] = __builtin_ldexp(1.0, c[q]);
    }
    sp.sig[0] = 1.0;
    sp.sig[1] = __builtin_ldexp(1.0, -c0);
    sp.sig[2] = __builtin_ldexp(1.0, -(c0 + c1));
    sp.sig[3] = __builtin_ldexp(1.0, -(c0 + c1 + c2));
  }
  double rah = 0.0, ral = 0.0, rbh = 0.0, rbl = 0.0;   // raw entries of the staged stage
  auto load_stage = [&](int64_t st) {
    const int64_t p1 = st * 8 + pa, p2 = st * 8 + pb;
    const bool va = row < m && p1 < k, vb = col < n && p2 < k;
    const int64_t ai = va ? row * a_si + p1 * a_sp : 0, bi = vb ? p2 * b_sp + col * b_sj : 0;
    rah = va ? Ahi[ai] : 0.0;
    ral = va ? Alo[ai] : 0.0;
    rbh = vb ? Bhi[bi] : 0.0;
    rbl = vb ? Blo[bi] : 0.0;
  };
  auto store_stage = [&](int64_t st) {
    double* buf = lds + (int)(st % kNBuf) * kStage;
    double w[4], xh, xl;
    split_entry(rah, ral, ea, sp, w, xh, xl);   // zeros give zero digits
#pragma unroll
    for (int q = 0; q < 4; ++q) buf[adst + q * kLanes] = w[q];
    double v[4], yh, yl;
    split_entry(rbh, rbl, eb, sp, v, yh, yl);
    buf[bdst + 0 * kLanes] = v[0];
    buf[bdst + 1 * kLanes] = v[1];
    buf[bdst + 2 * kLanes] = v[2];
    buf[bdst + 3 * kLanes] = v[3];
    buf[bdst + 4 * kLanes] = yh + yl;               // B6': the scaled entry, rounded once
  };
  auto a_ptr = [&](int64_t st) {
    return lds + (int)(st % kNBuf) * kStage + wm * (kStageQ * kFragA * kLanes) + (lane >> 4) * 4 + (lane & 3);
  };
  auto b_ptr = [&](int64_t st) {
    return lds + (int)(st % kNBuf) * kStage + kAStage + (wn * CB) * (kStageQ * FB * kLanes) + lane;
  };

  const int64_t nst = K4 / kStageQ;
  const int64_t last = nst - 1;
  load_stage(0);
  store_stage(0);
  load_stage(nst > 1 ? 1 : 0);
  lds_reads_done();
  lds_barrier();
  Ops<CB> ox, oy;
  read_ops<CB, FB>(ox, a_ptr(0), b_ptr(0), 0);
  int32_t inblk = 0;
  auto block_done = [&]() { combine<kFlags, false, CB>(bins, acc_h, acc_l, flg, nullptr, nullptr); };
  for (int64_t st = 0; st < nst; ++st) {
    read_ops<CB, FB>(oy, a_ptr(st), b_ptr(st), 1);
    derive_b<CB, FB>(ox);
    store_stage(st + 1);
    ten_products(bins, ox);
    interleave_reads_writes<CB, kFragA + FB, FB>();
    if (++inblk == kcq) { inblk = 0; block_done(); }
    derive_b<CB, FB>(oy);
    lds_reads_done();
    lds_barrier();
    read_ops<CB, FB>(ox, a_ptr(st + 1), b_ptr(st + 1), 0);
    load_stage(st + 2 <= last ? st + 2 : last);
    ten_products(bins, oy);
    interleave_reads_loads<CB, 4, FB>();
    if (++inblk == kcq) { inblk = 0; block_done(); }
  }
  if (inblk != 0) block_done();

#pragma unroll
  for (int i = 0; i < kSub; ++i) {
    const int64_t r = rb0 * 16 + i * 4 + (lane >> 4);
    if (r >= m) continue;
    const int er = exp_of_bits(amax[r]);
#pragma unroll
    for (int g = 0; g < CB; ++g) {
      const int64_t c = (cb0 + g) * 16 + (lane & 15);
      if (c >= n) continue;
      const int sh = er + exp_of_bits(bmax[c]);
      const double h = __builtin_ldexp(acc_h[i][g], sh);
      const double l = __builtin_ldexp(acc_l[i][g], sh);
      const int64_t idx = r + c * ldc;
      double rh, rl;
      dd_add(Chi[idx], Clo[idx], h, l, rh, rl);
      Chi[idx] = rh;
      Clo[idx] = rl;
      if constexpr (kFlags) {
        if (flg & (1u << (i * CB + g))) {
          const int64_t bit = r + c * m;
          atomicOr(&flags[bit >> 5], 1u << (bit & 31));
        }
      }
    }
  }
}

template <bool kFlags>
__global__ void __launch_bounds__(kWaves * 64)
cascade_onload_kernel(const double* __restrict__ Ahi, const double* __restrict__ Alo, int64_t a_si, int64_t a_sp,
                      const double* __restrict__ Bhi, const double* __restrict__ Blo, int64_t b_sp, int64_t b_sj,
                      const uint64_t* __restrict__ amax, const uint64_t* __restrict__ bmax, int c0, int c1, int c2,
                      int64_t K4, int32_t kcq, int64_t m, int64_t n, int64_t k, int64_t tiles_m, int64_t tiles_n,
                      double* __restrict__ Chi, double* __restrict__ Clo, int64_t ldc, uint32_t* __restrict__ flags) {
  __shared__ __attribute__((aligned(16))) double lds[kNBuf * BShape64x64::kStage];
  int64_t tm, tn;
  tile_of_block(blockIdx.x, tiles_m, tiles_n, tm, tn);
  cascade_tile_onload<kFlags>(lds, Ahi, Alo, a_si, a_sp, Bhi, Blo, b_sp, b_sj, amax, bmax, c0, c1, c2, K4, kcq, m,
                              n, k, tm, tn, Chi, Clo, ldc, flags);
}

hipError_t launch_cascade_onload(const CascadeLayout& L, const double* Ahi, const double* Alo, int64_t a_si,
                                 int64_t a_sp, const double* Bhi, const double* Blo, int64_t b_sp, int64_t b_sj,
                                 const uint64_t* amax, const uint64_t* bmax, double* Chi, double* Clo, int64_t ldc,
                                 uint32_t* flags, hipStream_t s) {
  if (L.K4 % kStageQ != 0 || L.npanel != 1 || L.balance) return hipErrorInvalidValue;
  const int64_t tiles_m = (L.m + 63) / 64, tiles_n = (L.n + 63) / 64;
  const int64_t tiles = tiles_m * tiles_n;
  if (tiles <= 0 || tiles > 0x7fffffff) return hipErrorInvalidValue;
  if (flags) {
    cascade_onload_kernel<true><<<(unsigned)tiles, kWaves * 64, 0, s>>>(
        Ahi, Alo, a_si, a_sp, Bhi, Blo, b_sp, b_sj, amax, bmax, L.c[0], L.c[1], L.c[2], L.K4, L.kcq, L.m, L.n, L.k,
        tiles_m, tiles_n, Chi, Clo, ldc, flags);
  } else {
    cascade_onload_kernel<false><<<(unsigned)tiles, kWaves * 64, 0, s>>>(
        Ahi, Alo, a_si, a_sp, Bhi, Blo, b_sp, b_sj, amax, bmax, L.c[0], L.c[1], L.c[2], L.K4, L.kcq, L.m, L.n, L.k,
        tiles_m, tiles_n, Chi, Clo, ldc, nullptr);
  }
  return hipGetLastError();
}

template <bool kFlags, bool kPanel, class SH, bool kBuf>
__global__ void __launch_bounds__(kWaves * 64)
cascade_kernel(const double* __restrict__ Apack, const double* __restrict__ Bpack,
               const uint64_t* __restrict__ amax, const uint64_t* __restrict__ bmax,
               int64_t K4, int32_t kcq, int64_t m, int64_t n, int64_t tiles_m, int64_t tiles_n,
               double* __restrict__ Chi, double* __restrict__ Clo, int64_t ldc, uint32_t* __restrict__ flags,
               const int32_t* __restrict__ aexp, const int32_t* __restrict__ bexp, int64_t mpad, int64_t npad) {
  __shared__ __attribute__((aligned(16))) double lds[kNBuf * SH::kStage];
  int64_t tm, tn;
  tile_of_block(blockIdx.x, tiles_m, tiles_n, tm, tn);
  cascade_tile<kFlags, kPanel, SH, kBuf>(lds, Apack, Bpack, amax, bmax, K4, kcq, m, n, tm, tn, Chi, Clo, ldc,
                                         flags, aexp, bexp, mpad, npad);
}

// Persistent form for a batch of GEMMs: every workgroup takes tiles from the
// list (in list order: the list is sorted by decreasing cost) until none is
// left, either with a fixed stride or from an atomic counter.  Each tile
// carries its shape (all tiles of one problem have the same).  With kFlags,
// problem p's cancellation bits go to its bitmap at flags + off_flags.
// kBuf: stage through buffer loads (every problem's blocks span < 2 GiB).
template <bool kFlags, bool kBuf>
__global__ void __launch_bounds__(kWaves * 64)
cascade_batched_kernel(const BatchDesc* __restrict__ desc, const BatchTile* __restrict__ tiles,
                       int64_t ntiles, double* const* __restrict__ Chi, double* const* __restrict__ Clo,
                       const char* __restrict__ ws, unsigned long long* __restrict__ counter, int dynamic,
                       uint32_t* __restrict__ flags) {
  __shared__ __attribute__((aligned(16))) double lds[kLdsBatched];
  __shared__ unsigned long long next;
  int64_t w = blockIdx.x;
  for (;;) {
    if (dynamic) {
      if (threadIdx.x == 0) next = atomicAdd(counter, 1ull);
      __syncthreads();
      w = (int64_t)next;
      __syncthreads();
    }
    if (w >= ntiles) break;
    const BatchTile t = tiles[w];
    const BatchDesc d = desc[t.p];
    const double* Ap = (const double*)(ws + d.off_apack);
    const double* Bp = (const double*)(ws + d.off_bpack);
    const uint64_t* am = (const uint64_t*)(ws + d.off_amax);
    const uint64_t* bm = (const uint64_t*)(ws + d.off_bmax);
    uint32_t* fl = kFlags ? flags + d.off_flags : nullptr;
    if (t.shape == kTile32x64) {
      cascade_tile<kFlags, false, BShape32x64, kBuf>(lds, Ap, Bp, am, bm, d.K4, d.kcq, d.m, d.n, t.tm, t.tn, Chi[t.p],
                                              Clo[t.p], d.ldc, fl);
    } else if (t.shape == kTile64x32) {
      cascade_tile<kFlags, false, BShape64x32, kBuf>(lds, Ap, Bp, am, bm, d.K4, d.kcq, d.m, d.n, t.tm, t.tn, Chi[t.p],
                                              Clo[t.p], d.ldc, fl);
    } else {
      cascade_tile<kFlags, false, BShape64x64, kBuf>(lds, Ap, Bp, am, bm, d.K4, d.kcq, d.m, d.n, t.tm, t.tn, Chi[t.p],
                                              Clo[t.p], d.ldc, fl);
    }
    __syncthreads();  // the next tile reuses the staging buffers
    if (!dynamic) w += gridDim.x;
  }
}

hipError_t launch_cascade_batched(const BatchDesc* desc, const BatchTile* tiles, int64_t ntiles,
                                  double* const* Chi, double* const* Clo, const char* ws,
                                  uint32_t* counter, int grid, bool dynamic, uint32_t* flags, bool buf,
                                  hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (grid < 1) return hipErrorInvalidValue;
  if (dynamic) {
    hipError_t e = launch_fill_u64((uint64_t*)counter, 1, 0, s);
    if (e != hipSuccess) return e;
  }
  auto go = [&](auto fl, auto bf) {
    cascade_batched_kernel<decltype(fl)::value, decltype(bf)::value><<<grid, kWaves * 64, 0, s>>>(
        desc, tiles, ntiles, Chi, Clo, ws, (unsigned long long*)counter, dynamic ? 1 : 0, flags);
  };
  using T = std::true_type;
  using F = std::false_type;
  if (flags) {
    if (buf) go(T{}, T{});
    else go(T{}, F{});
  } else {
    if (buf) go(F{}, T{});
    else go(F{}, F{});
  }
  return hipGetLastError();
}

bool buffer_staging_fits(int64_t K4) {
  return 4 * a_block_stride(K4) * 8 < (int64_t(1) << 31) &&
         4 * b_block_stride(K4, kFragBBatched) * 8 < (int64_t(1) << 31);
}

namespace {

template <class SH>
hipError_t launch_shape(const CascadeLayout& L, const double* Apack, const double* Bpack, const uint64_t* amax,
                        const uint64_t* bmax, double* Chi, double* Clo, int64_t ldc, uint32_t* flags,
                        hipStream_t s, const int32_t* aexp, const int32_t* bexp) {
  constexpr int64_t TM = SH::kRB * 16, TN = SH::kCB * 16;
  // tiles that hold output entries (the planes are padded to 64 anyway)
  const int64_t tiles_m = (L.m + TM - 1) / TM, tiles_n = (L.n + TN - 1) / TN;
  const int64_t tiles = tiles_m * tiles_n;
  if (tiles <= 0 || tiles > 0x7fffffff) return hipErrorInvalidValue;
  const unsigned g = (unsigned)tiles;
  const bool panel = L.npanel > 1;
  // the buffer-load form while a tile's A and B blocks span less than 2 GiB
  const bool buf = SH::kRB * a_block_stride(L.K4) * 8 < (int64_t(1) << 31) &&
                   SH::kCB * b_block_stride(L.K4) * 8 < (int64_t(1) << 31);
  auto go = [&](auto fl, auto pn, auto bf) {
    cascade_kernel<decltype(fl)::value, decltype(pn)::value, SH, decltype(bf)::value><<<g, kWaves * 64, 0, s>>>(
        Apack, Bpack, amax, bmax, L.K4, L.kcq, L.m, L.n, tiles_m, tiles_n, Chi, Clo, ldc,
        decltype(fl)::value ? flags : nullptr, aexp, bexp, L.mpad, L.npad);
  };
  using T = std::true_type;
  using F = std::false_type;
  if (buf) {
    if (flags && panel) go(T{}, T{}, T{});
    else if (flags) go(T{}, F{}, T{});
    else if (panel) go(F{}, T{}, T{});
    else go(F{}, F{}, T{});
  } else {
    if (flags && panel) go(T{}, T{}, F{});
    else if (flags) go(T{}, F{}, F{});
    else if (panel) go(F{}, T{}, F{});
    else go(F{}, F{}, F{});
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_cascade(const CascadeLayout& L, const double* Apack, const double* Bpack,
                          const uint64_t* amax, const uint64_t* bmax,
                          double* Chi, double* Clo, int64_t ldc, uint32_t* flags, hipStream_t s,
                          const int32_t* aexp, const int32_t* bexp, int shape) {
  if (L.tile_m != 64 || L.tile_n != 64 || L.K4 % kStageQ != 0) return hipErrorInvalidValue;
  if (L.npanel > 1 && (!aexp || !bexp)) return hipErrorInvalidValue;
  switch (shape) {
    case kTile32x64: return launch_shape<Shape32x64>(L, Apack, Bpack, amax, bmax, Chi, Clo, ldc, flags, s, aexp, bexp);
    case kTile64x32: return launch_shape<Shape64x32>(L, Apack, Bpack, amax, bmax, Chi, Clo, ldc, flags, s, aexp, bexp);
    case kTile64x64: return launch_shape<Shape64x64>(L, Apack, Bpack, amax, bmax, Chi, Clo, ldc, flags, s, aexp, bexp);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ddk
