// The narrow-slice variants: FP64x2 GEMM from BF16 / FP16 / INT8 matrix-core
// products with exact level sums (the bfloat16 cascade of Sec. 6.2 carried
// to FP64x2, with equal-width splits and the product triangle of Sec. 6.1;
// the INT8 form is the "FP64x2 in terms of INT8" case of Sec. 6.2).
//
//  * slices_split: per entry of op(A) (op(B)), scaled by the power of two of
//    its row (column), s slices of w bits: the running remainder, an
//    unevaluated FP64 pair, is rounded to the grid u_t = 2^-((t+1)w-1) with
//    (r + K) - K and renormalised by TwoSum.  Each slice a_t = d_t / u_t is an
//    integer with |a_t| <= 2^(w-1), stored exactly as BF16, FP16 or INT8 and
//    packed as MFMA operands (one 16-byte chunk per lane and slice).
//  * slices_product: one 64 x 64 output tile per workgroup, a 32 x 32 block
//    per wave.  For every step of the inner dimension (16 deep for BF16/FP16,
//    32 for INT8), the products A_i B_j with i + j = L < s go to the
//    accumulator of level L (v_mfma_f32_32x32x16_{bf16,f16} or
//    v_mfma_i32_32x32x32_i8).  All operands are integers: FP32 sums are exact
//    while below 2^24, so a BF16/FP16 level is flushed to its FP64 group every
//    2^n steps with 16 * 2^n * (L+1) * 2^(2w-2) <= 2^24; INT32 sums are exact
//    over the whole chunk and are converted once.  Groups of three levels
//    share one FP64 accumulator (the lower levels shifted up by w and 2w
//    bits; exact below 2^53, which bounds the inner-dimension chunk).  The
//    epilogue adds the groups in FP64x2 from the least significant, applies
//    the row and column powers of two and adds C.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "dd_device.hpp"
#include "kernels.hpp"
#include "layout.hpp"

namespace ddk {

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x16 __attribute__((ext_vector_type(16)));

constexpr int kBF16 = kSliceBF16, kF16 = kSliceF16, kI8 = kSliceI8;
constexpr int kGroup = 3;     // levels per FP64 accumulator
constexpr int kXcds = 8;      // XCDs of the MI355X; workgroups go round-robin over them
constexpr int kGroupM = 8;    // tile rows per group of the tile order

__device__ __forceinline__ void tile_order(int64_t b, int64_t tiles_m, int64_t tiles_n, int64_t& tm,
                                           int64_t& tn) {
  // consecutive workgroups of one XCD take neighbouring tiles (shared L2)
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

// Inner indices one lane holds per operand: 8 two-byte values or 16 bytes.
template <int FMT>
constexpr int kPerLane = FMT == kI8 ? 16 : 8;

// Exact pattern of an integer-valued double with |a| <= 2^8 (BF16), 2^11
// (FP16) or 127 (INT8).  Non-finite values map to NaN/Inf in the floating
// formats and to 0 in INT8 (the epilogue marks those rows and columns NaN).
template <int FMT>
__device__ __forceinline__ uint32_t slice_bits(double a) {
  if constexpr (FMT == kI8) {
    const bool finite = __builtin_isfinite(a);
    return (uint32_t)(uint8_t)(int8_t)(finite ? (int)a : 0);
  } else {
    const float f = (float)a;
    if constexpr (FMT == kF16) {
      return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)f);
    } else {
      return __builtin_bit_cast(uint32_t, f) >> 16;
    }
  }
}

// One thread per (outer index o, group rg of kPerLane packed inner indices):
// packed index rg * kPerLane + e lies in chunk c at offset r (chunks are
// cpk = chunk_q * kstep packed indices apart), so it holds the entry
// X(o, c * chunk + r) = X[o*so + (c*chunk + r)*sr], or zero past the end of
// the chunk or of the inner dimension.  The entries are split and written
// as one 16-byte piece per slice.
template <int FMT>
__global__ void __launch_bounds__(256)
slices_split(const double* __restrict__ Xhi, const double* __restrict__ Xlo, int64_t so, int64_t sr,
             int64_t outer, int64_t red, int64_t opad, int64_t Q, int S, int w, int64_t chunk, int64_t cpk,
             const uint64_t* __restrict__ maxbits, u32x4* __restrict__ pack) {
  constexpr int E = kPerLane<FMT>;
  constexpr int PER_WORD = FMT == kI8 ? 4 : 2;     // values per 32-bit word
  const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (u >= opad * Q * 2) return;
  const int64_t o = u % opad, rg = u / opad;
  // the kPerLane values of a thread share one step, hence one chunk
  const int64_t ch = (rg * E) / cpk, off0 = rg * E - ch * cpk;
  const int ex = o < outer ? exp_of_bits(maxbits[o]) : 0;
  uint32_t words[16][4];
#pragma unroll
  for (int t = 0; t < 16; ++t)
#pragma unroll
    for (int h = 0; h < 4; ++h) words[t][h] = 0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int64_t off = off0 + e, r = ch * chunk + off;
    double xh = 0.0, xl = 0.0;
    if (o < outer && off < chunk && r < red) {
      xh = __builtin_ldexp(Xhi[o * so + r * sr], -ex);
      xl = __builtin_ldexp(Xlo[o * so + r * sr], -ex);
    }
    double rem, rho;
    two_sum(xh, xl, rem, rho);
    for (int t = 0; t < S; ++t) {
      const double K = __builtin_ldexp(3.0, 52 - (t + 1) * w);
      const double d = (rem + K) - K;
      const uint32_t bits = slice_bits<FMT>(d * __builtin_ldexp(1.0, (t + 1) * w - 1));
      const double left = rem - d;
      two_sum(left, rho, rem, rho);
      // constant-index stores keep `words` in registers
#pragma unroll
      for (int tt = 0; tt < 16; ++tt)
        if (tt == t) words[tt][e / PER_WORD] |= bits << ((32 / PER_WORD) * (e % PER_WORD));
    }
  }
  const int64_t rb = o / 32, q = rg / 2;
  const int lane = (int)(o % 32) + 32 * (int)(rg % 2);
  u32x4* dst = pack + rb * slices_block_stride(Q, S) + (q * S) * 64 + lane;
#pragma unroll
  for (int t = 0; t < 16; ++t)
    if (t < S) dst[t * 64] = u32x4{words[t][0], words[t][1], words[t][2], words[t][3]};
}

template <int FMT>
using acc_t = std::conditional_t<FMT == kI8, i32x16, f32x16>;

template <int FMT>
__device__ __forceinline__ acc_t<FMT> mma(u32x4 a, u32x4 b, acc_t<FMT> c) {
  if constexpr (FMT == kI8) {
    return __builtin_amdgcn_mfma_i32_32x32x32_i8(__builtin_bit_cast(i32x4, a), __builtin_bit_cast(i32x4, b),
                                                  c, 0, 0, 0);
  } else if constexpr (FMT == kF16) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b),
                                                   c, 0, 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                    c, 0, 0, 0);
  }
}

// A scheduling group of n MFMAs (n is a constant once the loops are unrolled).
template <int N>
__device__ __forceinline__ void mfma_group_n() {
  __builtin_amdgcn_sched_group_barrier(0x008, N, 0);
}
__device__ __forceinline__ void mfma_group(int n) {
  switch (n) {
    case 1: mfma_group_n<1>(); break;
    case 2: mfma_group_n<2>(); break;
    case 3: mfma_group_n<3>(); break;
    case 4: mfma_group_n<4>(); break;
    case 5: mfma_group_n<5>(); break;
    case 6: mfma_group_n<6>(); break;
    case 7: mfma_group_n<7>(); break;
    case 8: mfma_group_n<8>(); break;
    case 9: mfma_group_n<9>(); break;
    case 10: mfma_group_n<10>(); break;
    case 11: mfma_group_n<11>(); break;
    case 12: mfma_group_n<12>(); break;
    case 13: mfma_group_n<13>(); break;
    case 14: mfma_group_n<14>(); break;
    case 15: mfma_group_n<15>(); break;
    case 16: mfma_group_n<16>(); break;
    default: break;
  }
}

// A scheduling group of n vector-memory reads (n in 1..10).
__device__ __forceinline__ void vmem_group(int n) {
  switch (n) {
    case 1: __builtin_amdgcn_sched_group_barrier(0x020, 1, 0); break;
    case 2: __builtin_amdgcn_sched_group_barrier(0x020, 2, 0); break;
    case 3: __builtin_amdgcn_sched_group_barrier(0x020, 3, 0); break;
    case 4: __builtin_amdgcn_sched_group_barrier(0x020, 4, 0); break;
    case 5: __builtin_amdgcn_sched_group_barrier(0x020, 5, 0); break;
    case 6: __builtin_amdgcn_sched_group_barrier(0x020, 6, 0); break;
    case 7: __builtin_amdgcn_sched_group_barrier(0x020, 7, 0); break;
    case 8: __builtin_amdgcn_sched_group_barrier(0x020, 8, 0); break;
    case 9: __builtin_amdgcn_sched_group_barrier(0x020, 9, 0); break;
    case 10: __builtin_amdgcn_sched_group_barrier(0x020, 10, 0); break;
    default: break;
  }
}

// Next-step B slices loaded per iteration of a step: B_j goes out in
// iteration j / BPER, so the last one has most of the step to arrive.  The
// final pass (levels 0..8, few products per step) loads them sooner than
// the upper pass, whose longer steps already cover the wait.
constexpr int kBPerLower = 4, kBPerUpper = 2;

struct ProductArgs {
  const u32x4* Apack;
  const u32x4* Bpack;
  const uint64_t* amax;
  const uint64_t* bmax;
  double* Chi;
  double* Clo;
  double* planes;    // FP64 group sums of the upper pass (NGU groups per wave and tile)
  int64_t ldc, m, n, tiles_m, tiles_n, Q;
  int32_t S, NG, NGU;  // slices (operand stride), groups in total, groups of the upper pass
  int32_t q0, q1, w;
};

// true if a max-|x| bit pattern is Inf or NaN
__device__ __forceinline__ bool nonfinite_bits(uint64_t b) {
  return (b & 0x7ff0000000000000ull) == 0x7ff0000000000000ull;
}

// Levels [LB, LE) of the product triangle for one 64 x 64 tile.  With LB == 0
// the epilogue combines every group (groups at or above LE/3 are read from
// `planes`) and updates C; otherwise it writes its groups to `planes`.
//
// BF16/FP16 flush schedule: level L goes to its FP64 group after the steps
// whose index (counted from q0) is congruent to L modulo P, and at the end.
// P divides 4 and every level's exact depth, so no FP32 sum passes 2^24;
// staggering the levels spreads the conversions over the steps.  A flushed
// accumulator is not cleared: the level's first product of the next step
// takes C = 0.  The step loop is unrolled by 4 so that this schedule is fixed
// at compile time.  The first step's "previous" flushes take the zero
// accumulators: harmless.  INT8 levels are converted once, after the chunk.
template <int LB, int LE, int P, int FMT>
__global__ void __launch_bounds__(256, 1) slices_product(const ProductArgs a) {
  static_assert(LB % kGroup == 0, "a pass owns whole level groups");
  static_assert(P == 1 || P == 4, "the flush period divides the unroll");
  constexpr bool kFlushes = FMT != kI8;
  constexpr int NL = LE - LB;
  constexpr int G0 = LB / kGroup, NGP = (LE + kGroup - 1) / kGroup - G0;   // groups of this pass
  constexpr int BPER = LB == 0 ? kBPerLower : kBPerUpper;
  static_assert(BPER >= 1 && BPER <= 9, "a scheduling group holds up to 10 loads");
  using Acc = acc_t<FMT>;
  // the wave index is uniform: operand addresses are formed on the scalar unit
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int64_t tm, tn;
  tile_order(blockIdx.x, a.tiles_m, a.tiles_n, tm, tn);
  const int64_t rb = tm * 2 + (wv >> 1), cb = tn * 2 + (wv & 1);
  const int64_t step = (int64_t)a.S * 64;
  const int64_t bstride = slices_block_stride(a.Q, a.S);
  const u32x4* Ap = a.Apack + rb * bstride + lane;   // not restrict: the loads stay where written
  const u32x4* Bp = a.Bpack + cb * bstride + lane;

  Acc acc[NL];
  double grp[NGP][16];
  const Acc zero = {};
#pragma unroll
  for (int L = 0; L < NL; ++L) acc[L] = zero;
#pragma unroll
  for (int g = 0; g < NGP; ++g)
#pragma unroll
    for (int v = 0; v < 16; ++v) grp[g][v] = 0.0;
  const double up1 = __builtin_ldexp(1.0, a.w), up2 = __builtin_ldexp(1.0, 2 * a.w);

  // slices 0 .. LE-1 of both operands take part (every one reaches level LE-1).
  // A_i is reloaded for the next step right after its products; B_0 is
  // needed until the end of a step, so B has two buffers: the next step's B
  // loads early in the current step, BPER slices per iteration.
  u32x4 fa[LE], fb0[LE], fb1[LE];
  {
    // same order as the loads inside the loop, so the waits there can count
    const int64_t base = (int64_t)a.q0 * step;
#pragma unroll
    for (int i = 0; i < LE; ++i) {
      fa[i] = Ap[base + i * 64];
#pragma unroll
      for (int j = i * BPER; j < (i + 1) * BPER && j < LE; ++j) fb0[j] = Bp[base + j * 64];
      asm volatile("" ::: "memory");
    }
  }

  // level L's sum `x` (values [v0, v1)) into its group (exact: an integer
  // times a power of two)
  auto flush_vals = [&](int L, const Acc& x, int v0, int v1) {
    const int g = L / kGroup - G0, shift = kGroup - 1 - L % kGroup;
    const double sc = shift == 2 ? up2 : (shift == 1 ? up1 : 1.0);
#pragma unroll
    for (int v = v0; v < v1; ++v) grp[g][v] = __builtin_fma((double)x[v], sc, grp[g][v]);
  };

  // With P = 4 a level's flush is deferred: at the start of the step after
  // its flush point its sum is copied to `held` (before the level restarts
  // from zero) and converted a few values per iteration, among the step's
  // products.  With P = 1 every level flushes at the end of every step.
  constexpr int NH = P == 4 ? (NL + 3) / 4 : 1;
  constexpr int kSpread = LE < 8 ? LE : 8;            // iterations that take a share
  constexpr int kShare = (16 + kSpread - 1) / kSpread;  // values per iteration
  Acc held[NH];

  // One step of phase PH (its index from q0, mod 4): the products with B
  // from `fb`, next step's A into fa and B into `fbn`, the flushes.
  auto run_step = [&](auto phase, const u32x4 (&fb)[LE], u32x4 (&fbn)[LE], int q) {
    constexpr int PH = decltype(phase)::value;
    constexpr int PREV = (PH + P - 1) % P;   // levels flushed after the previous step
    const int64_t nxt = (int64_t)(q + 1 < a.q1 ? q + 1 : q) * step;   // in bounds on the last step
    if constexpr (kFlushes && P == 4) {
      int h = 0;
#pragma unroll
      for (int L = LB; L < LE; ++L)
        if (L % 4 == PREV) held[h++] = acc[L - LB];
    }
    bool started[NL];
#pragma unroll
    for (int L = 0; L < NL; ++L) started[L] = false;
#pragma unroll
    for (int i = 0; i < LE; ++i) {
      // levels ascending: the one restarted last in iteration 0 is the top one
      int nm = 0;
#pragma unroll
      for (int j = (LB - i > 0 ? LB - i : 0); j <= LE - 1 - i; ++j, ++nm) {
        const int L = i + j - LB;
        // flushed after the previous step: start from zero
        const bool fresh = kFlushes && !started[L] && ((i + j) % P == PREV);
        acc[L] = mma<FMT>(fa[i], fb[j], fresh ? zero : acc[L]);
        started[L] = true;
      }
      // A_i is not needed again in this step; up to BPER of next step's B slices
      fa[i] = Ap[nxt + i * 64];
      int nl = 1;
#pragma unroll
      for (int j = i * BPER; j < (i + 1) * BPER && j < LE; ++j, ++nl) fbn[j] = Bp[nxt + j * 64];
      // keep the loads here (not sunk below the flushes)
      asm volatile("" ::: "memory");
      mfma_group(nm);                                      // this iteration's MFMAs,
      vmem_group(nl);                                      // then its loads
      if constexpr (kFlushes && P == 4) {
        if (i < kSpread) {
          const int v0 = i * kShare, v1 = v0 + kShare < 16 ? v0 + kShare : 16;
          int h = 0;
#pragma unroll
          for (int L = LB; L < LE; ++L)
            if (L % 4 == PREV) flush_vals(L, held[h++], v0, v1);
        }
      }
    }
    if constexpr (kFlushes && P == 1) {
#pragma unroll
      for (int L = LB; L < LE; ++L) flush_vals(L, acc[L - LB], 0, 16);
    }
  };
  using Ph0 = std::integral_constant<int, 0>;
  using Ph1 = std::integral_constant<int, 1>;
  using Ph2 = std::integral_constant<int, 2>;
  using Ph3 = std::integral_constant<int, 3>;
  // q1 - q0 is a multiple of 4 (the inner dimension is padded to 4 steps)
  for (int q = a.q0; q < a.q1; q += 4) {
    run_step(Ph0{}, fb0, fb1, q);
    run_step(Ph1{}, fb1, fb0, q + 1);
    run_step(Ph2{}, fb0, fb1, q + 2);
    run_step(Ph3{}, fb1, fb0, q + 3);
  }
  // what every level has gathered since its last flush (INT8: everything)
  if constexpr (!kFlushes || P == 4) {
#pragma unroll
    for (int L = LB; L < LE; ++L) flush_vals(L, acc[L - LB], 0, 16);
  }

  // group sums of the upper pass: per tile, wave, group and register, 64 lanes
  const int64_t tile = tm * a.tiles_n + tn;
  double* plane = a.planes + ((tile * 4 + wv) * (int64_t)a.NGU * 16) * 64 + lane;
  if constexpr (LB > 0) {
#pragma unroll
    for (int g = 0; g < NGP; ++g)
#pragma unroll
      for (int v = 0; v < 16; ++v) plane[(g * 16 + v) * 64] = grp[g][v];
    return;
  } else {
    // epilogue: lane holds rows 8*(v/4) + 4*(lane/32) + v%4, column lane%32 of its block
    const int64_t j = cb * 32 + (lane & 31);
    if (j >= a.n) return;
    const uint64_t bbits = a.bmax[j];
    const int fj = exp_of_bits(bbits);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t i = rb * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      if (i < a.m) {
        double h = 0.0, l = 0.0;
        for (int g = a.NG - 1; g >= NGP; --g) {
          const double W = __builtin_ldexp(1.0, 2 - (kGroup * g + kGroup + 1) * a.w);
          dd_add_d(h, l, plane[((g - NGP) * 16 + v) * 64] * W, h, l);
        }
#pragma unroll
        for (int g = NGP - 1; g >= 0; --g) {
          const double W = __builtin_ldexp(1.0, 2 - (kGroup * g + kGroup + 1) * a.w);
          dd_add_d(h, l, grp[g][v] * W, h, l);
        }
        const uint64_t abits = a.amax[i];
        const int sh = exp_of_bits(abits) + fj;
        h = __builtin_ldexp(h, sh);
        l = __builtin_ldexp(l, sh);
        if constexpr (FMT == kI8) {
          // integer slices carry no NaN: a non-finite row or column gives NaN here
          if (nonfinite_bits(abits) || nonfinite_bits(bbits)) h = l = __builtin_nan("");
        }
        double* ch = a.Chi + i + j * a.ldc;
        double* cl = a.Clo + i + j * a.ldc;
        double rh, rl;
        dd_add(*ch, *cl, h, l, rh, rl);
        *ch = rh;
        *cl = rl;
      }
    }
  }
}

template <int LB, int LE, int P, int FMT>
hipError_t launch_pass(const ProductArgs& a, int64_t blocks, hipStream_t s) {
  slices_product<LB, LE, P, FMT><<<(unsigned)blocks, 256, 0, s>>>(a);
  return hipGetLastError();
}

// Levels below kSplit run in the final pass; slice counts above it add an
// upper pass for levels kSplit .. S-1 that runs first.
constexpr int kSplit = kSlicesSplit;
static_assert(kSplit % kGroup == 0, "the passes split between level groups");

template <int P, int FMT>
hipError_t launch_lower(int S, const ProductArgs& a, int64_t blocks, hipStream_t s) {
  switch (S < kSplit ? S : kSplit) {
    case 1: return launch_pass<0, 1, P, FMT>(a, blocks, s);
    case 2: return launch_pass<0, 2, P, FMT>(a, blocks, s);
    case 3: return launch_pass<0, 3, P, FMT>(a, blocks, s);
    case 4: return launch_pass<0, 4, P, FMT>(a, blocks, s);
    case 5: return launch_pass<0, 5, P, FMT>(a, blocks, s);
    case 6: return launch_pass<0, 6, P, FMT>(a, blocks, s);
    case 7: return launch_pass<0, 7, P, FMT>(a, blocks, s);
    case 8: return launch_pass<0, 8, P, FMT>(a, blocks, s);
    case 9: return launch_pass<0, 9, P, FMT>(a, blocks, s);
    default: return hipErrorInvalidValue;
  }
}

template <int P, int FMT>
hipError_t launch_upper(int S, const ProductArgs& a, int64_t blocks, hipStream_t s) {
  switch (S) {
    case 10: return launch_pass<kSplit, 10, P, FMT>(a, blocks, s);
    case 11: return launch_pass<kSplit, 11, P, FMT>(a, blocks, s);
    case 12: return launch_pass<kSplit, 12, P, FMT>(a, blocks, s);
    case 13: return launch_pass<kSplit, 13, P, FMT>(a, blocks, s);
    case 14: return launch_pass<kSplit, 14, P, FMT>(a, blocks, s);
    case 15: return launch_pass<kSplit, 15, P, FMT>(a, blocks, s);
    case 16: return launch_pass<kSplit, 16, P, FMT>(a, blocks, s);
    default: return hipErrorInvalidValue;
  }
}

// The flush period of a BF16/FP16 pass: 4 steps if its top level (the one
// with the smallest exact depth) allows it, else every step (always exact).
inline int flush_period(const SlicesLayout& L, int top_level) {
  return L.flush_mask[top_level] + 1 >= 4 ? 4 : 1;
}

template <int FMT>
hipError_t launch_passes(const SlicesLayout& L, const ProductArgs& a, int64_t blocks, hipStream_t s) {
  if constexpr (FMT == kI8) {
    if (L.S > kSplit) {
      const hipError_t e = launch_upper<4, FMT>(L.S, a, blocks, s);
      if (e != hipSuccess) return e;
    }
    return launch_lower<4, FMT>(L.S, a, blocks, s);
  } else {
    if (L.S > kSplit) {
      const hipError_t e = flush_period(L, L.S - 1) == 4 ? launch_upper<4, FMT>(L.S, a, blocks, s)
                                                         : launch_upper<1, FMT>(L.S, a, blocks, s);
      if (e != hipSuccess) return e;
    }
    return flush_period(L, (L.S < kSplit ? L.S : kSplit) - 1) == 4 ? launch_lower<4, FMT>(L.S, a, blocks, s)
                                                                   : launch_lower<1, FMT>(L.S, a, blocks, s);
  }
}

// Diagnostic copy of packed slices into plain column-major 16-bit planes:
// element (o, r) of slice t goes to out[t*plane + o*oo + r*ro] (INT8 slices
// sign-extended to 16 bits).  Source index r sits at packed index
// (r / chunk) * cpk + r % chunk.
template <int FMT>
__global__ void __launch_bounds__(256)
slices_unpack(const uint8_t* __restrict__ pack, int64_t outer, int64_t red, int64_t Q, int S,
              int64_t chunk, int64_t cpk, int64_t oo, int64_t ro, uint16_t* __restrict__ out) {
  constexpr int E = kPerLane<FMT>;
  const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t plane = outer * red;
  if (u >= plane * S) return;
  const int t = (int)(u / plane);
  const int64_t rest = u - (int64_t)t * plane;
  const int64_t o = rest % outer, rs = rest / outer;
  const int64_t r = (rs / chunk) * cpk + rs % chunk;
  const int64_t rb = o / 32, q = r / (2 * E);
  const int lane = (int)(o % 32) + 32 * (int)((r % (2 * E)) / E);
  const int64_t at = (rb * slices_block_stride(Q, S) + (q * S + t) * 64 + lane) * 16;   // byte offset of the lane's piece
  uint16_t v;
  if constexpr (FMT == kI8) {
    v = (uint16_t)(int16_t)(int8_t)pack[at + (r % E)];
  } else {
    v = ((const uint16_t*)(pack + at))[r % E];
  }
  out[t * plane + o * oo + rs * ro] = v;
}

}  // namespace

hipError_t launch_slices_split(const double* Xhi, const double* Xlo, int64_t so, int64_t sr, int64_t outer,
                               int64_t red, int64_t opad, const SlicesLayout& L, const uint64_t* maxbits,
                               void* pack, hipStream_t s) {
  const int64_t units = opad * L.Q * 2;
  const unsigned blocks = (unsigned)((units + 255) / 256);
  const int64_t cpk = L.chunk_q * L.kstep;
  if (L.fmt == kI8) {
    slices_split<kI8><<<blocks, 256, 0, s>>>(Xhi, Xlo, so, sr, outer, red, opad, L.Q, L.S, L.w, L.chunk, cpk,
                                             maxbits, (u32x4*)pack);
  } else if (L.fmt == kF16) {
    slices_split<kF16><<<blocks, 256, 0, s>>>(Xhi, Xlo, so, sr, outer, red, opad, L.Q, L.S, L.w, L.chunk, cpk,
                                              maxbits, (u32x4*)pack);
  } else {
    slices_split<kBF16><<<blocks, 256, 0, s>>>(Xhi, Xlo, so, sr, outer, red, opad, L.Q, L.S, L.w, L.chunk, cpk,
                                               maxbits, (u32x4*)pack);
  }
  return hipGetLastError();
}

hipError_t launch_slices_unpack(const void* pack, int64_t outer, int64_t red, const SlicesLayout& L,
                                int64_t oo, int64_t ro, uint16_t* out, hipStream_t s) {
  const int64_t units = outer * red * L.S;
  const unsigned blocks = (unsigned)((units + 255) / 256);
  const int64_t cpk = L.chunk_q * L.kstep;
  if (L.fmt == kI8) {
    slices_unpack<kI8><<<blocks, 256, 0, s>>>((const uint8_t*)pack, outer, red, L.Q, L.S, L.chunk, cpk, oo, ro,
                                              out);
  } else {
    slices_unpack<kBF16><<<blocks, 256, 0, s>>>((const uint8_t*)pack, outer, red, L.Q, L.S, L.chunk, cpk, oo, ro,
                                                out);
  }
  return hipGetLastError();
}

hipError_t launch_slices_product(const SlicesLayout& L, const void* Apack, const void* Bpack,
                                 const uint64_t* amax, const uint64_t* bmax, double* planes, double* Chi,
                                 double* Clo, int64_t ldc, int64_t q0, int64_t q1, hipStream_t s) {
  ProductArgs a{};
  a.Apack = (const u32x4*)Apack;
  a.Bpack = (const u32x4*)Bpack;
  a.amax = amax;
  a.bmax = bmax;
  a.Chi = Chi;
  a.Clo = Clo;
  a.planes = planes;
  a.ldc = ldc;
  a.m = L.m;
  a.n = L.n;
  a.tiles_m = L.mpad / 64;
  a.tiles_n = L.npad / 64;
  a.Q = L.Q;
  a.S = L.S;
  a.NG = (L.S + kGroup - 1) / kGroup;
  a.NGU = L.S > kSplit ? a.NG - kSplit / kGroup : 0;
  a.q0 = (int32_t)q0;
  a.q1 = (int32_t)q1;
  a.w = L.w;
  if ((q1 - q0) % 4 != 0) return hipErrorInvalidValue;
  const int64_t blocks = a.tiles_m * a.tiles_n;
  if (L.fmt == kI8) return launch_passes<kI8>(L, a, blocks, s);
  if (L.fmt == kF16) return launch_passes<kF16>(L, a, blocks, s);
  return launch_passes<kBF16>(L, a, blocks, s);
}

}  // namespace ddk
