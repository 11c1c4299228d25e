// Workspace layout of one cascaded FP64x2 GEMM, shared by the host runtime
// and the kernels.
//
// Packed digit planes (the "cascaded" operands of Sec. 3.4, pre-weighted),
// laid out for v_mfma_f64_4x4x4_4b_f64 (four independent 4x4x4 blocks; A lane
// 16k+4b+i holds row i / inner index k of block b, B lane 16k+4b+j holds inner
// index k / column j, D lane 16i+4b+j holds row i / column j):
//   A: for each 16-row block rb and each group of 4 inner indices kq, the
//      four planes A0'..A3'; within a plane the 4-row sub-block s, inner
//      index kk and row i sit at s*16 + kk*4 + i (16 values per 4-row
//      sub-block, read by all four MFMA blocks at once):
//        Apack[rb*a_block_stride(K4) + (kq*4 + t)*64 + s*16 + kk*4 + i]
//   B: for each 16-column block cb, FB planes, one 64-lane operand each
//      (lane kk*16 + c holds inner index kk, column c).  Single GEMMs store
//      all seven, B0', ..., B6' (FB = 7: B4' = B2' + B3' and B5' = B1' + B4'
//      computed by the split); batched plans store B0', B1', B2', B3', B6'
//      (FB = 5), and their product loop forms B4' and B5' with the same two
//      FP64 additions:
//        Bpack[cb*b_block_stride(K4, FB) + (kq*FB + t)*64 + kk*16 + c]
// Rows/columns are padded with zeros up to the workgroup tile and the inner
// dimension up to a multiple of 16 (two LDS stages of the product kernel, 8
// inner indices each, which its main loop takes in pairs), so the product
// kernel needs no bounds checks in its main loop.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace ddk {

constexpr int kFragA = 4;   // planes of op(A)
constexpr int kFragB = 7;   // stored planes of op(B) for single GEMMs: B0', B1', ..., B6'
constexpr int kFragBBatched = 5;   // in batched plans: B0', B1', B2', B3', B6'
constexpr int kPlanesB = 7; // planes of op(B) in the products
constexpr int kLanes = 64;

// The packed planes of one 16-row block of op(A) (16-column block of op(B))
// are contiguous over k; consecutive blocks are KPAD doubles further apart
// than their size.  Without it the block stride is a multiple of 1 MiB for
// k a multiple of 2048, so the pieces a workgroup loads from its four
// blocks, and those of neighbouring tiles, fall on the same L2 sets.
constexpr int64_t kBlockPad = 544;   // 4 KiB + 256 B
constexpr int64_t a_block_stride(int64_t K4) { return K4 * kFragA * kLanes + kBlockPad; }
constexpr int64_t b_block_stride(int64_t K4, int fb = kFragB) { return K4 * fb * kLanes + kBlockPad; }

struct CascadeLayout {
  int64_t m, n, k;
  int64_t mpad, npad, kpad, K4;  // padded sizes, K4 = kpad / 4
  int64_t tile_m, tile_n;        // workgroup tile of the product kernel
  int32_t kc;                    // rank-kc block actually used (min(kc, k))
  int32_t kcq;                   // kc in groups of four inner indices
  int32_t c[3];                  // split widths c0, c1, c2
  int32_t npanel;                // exponent sets: 1, or one per rank-kc panel
  size_t off_amax, off_bmax, off_apack, off_bpack, bytes;
  size_t off_aexp, off_bexp;     // per-panel exponents as int32 (npanel > 1 only)
  bool balance;                  // diagonal balancing of the inner dimension
  size_t off_acol, off_brow;     // balance: column maxima of op(A), row maxima of op(B)
  size_t off_gexp;               // balance: int32 exponent g[p] per inner index
  // simple (unfused) form: plain column-major digit planes, bins, accumulator
  size_t off_aplain, off_bplain, off_bins, off_acc;
};

inline int64_t round_up(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

// One problem of a batch, as the batched kernels see it (device memory).
// Offsets are bytes into the batch's workspace, laid out per problem as in
// CascadeLayout.  Operand pointers come from the caller's device arrays.
struct BatchDesc {
  int64_t m, n, k, K4, mpad, npad, tiles_m, tiles_n;
  int64_t lda, ldb, ldc;
  int64_t off_amax, off_bmax, off_apack, off_bpack;
  int64_t off_flags;   // first word of this problem's cancellation bitmap
  int32_t kcq, c0, c1, c2;
};

// Fragments of packed planes one wave of the packing kernels fills (a
// batched plan's units are 4 waves' worth).
constexpr int kPackFragsPerWave = 4;

// Output tile shapes of the product kernel (rows x columns per workgroup);
// every shape computes every entry with the same arithmetic.
constexpr int kTile64x64 = 1, kTile32x64 = 2, kTile64x32 = 3;
inline int tile_rows(int shape) { return shape == kTile32x64 ? 32 : 64; }
inline int tile_cols(int shape) { return shape == kTile64x32 ? 32 : 64; }

// A tile of the persistent product kernel: problem p, tile row tm, column tn
// (in units of the tile shape), and the shape.
struct BatchTile {
  int32_t p, tm, tn, shape;
};

// ceil(log2 kc) and the widths of Sec. 3.3 (bins 0-2 exact for kc terms).
inline void split_widths(int64_t kc, int32_t c[3]) {
  int L = 0;
  while ((int64_t(1) << L) < kc) ++L;
  int c0 = (53 - L) / 2;
  int c1a = 53 - L - 1 - c0, c1b = (53 - L - 2) / 2;
  c[0] = c0;
  c[1] = c1a < c1b ? c1a : c1b;
  c[2] = 53 - L - 2 - c0;
}

// With `panels`, Sigma and T are taken per rank-kc panel (inner indices
// [4 kcq b, 4 kcq (b + 1))): the row maxima of op(A) are stored as npanel
// sets of mpad words (set b at b * mpad), the column maxima of op(B) as
// npanel sets of npad words.
// With `simple`, also room for the unfused form: A0'..A3' as m x k and
// B0'..B6' as k x n column-major planes, the four bins and the FP64x2
// accumulator as m x n planes.
inline CascadeLayout make_layout(int64_t m, int64_t n, int64_t k, int32_t kc,
                                 int64_t tile_m, int64_t tile_n, bool panels = false,
                                 bool balance = false, bool simple = false) {
  CascadeLayout L{};
  L.m = m; L.n = n; L.k = k;
  L.tile_m = tile_m; L.tile_n = tile_n;
  L.mpad = round_up(m > 0 ? m : 1, tile_m);
  L.npad = round_up(n > 0 ? n : 1, tile_n);
  L.kpad = round_up(k > 0 ? k : 1, 16);   // whole LDS stages (8 inner indices each), in pairs
  L.K4 = L.kpad / 4;
  int64_t kce = k < kc ? k : kc;
  if (kce < 1) kce = 1;
  L.kc = (int32_t)kce;
  // one block when k <= kc, padding included (no block of padding alone)
  L.kcq = (int32_t)(k <= kc ? L.K4 : (kce + 3) / 4);
  split_widths(kce, L.c);
  // panels are the runs of 4 kcq inner indices the product kernel combines
  L.npanel = panels ? (int32_t)((L.K4 + L.kcq - 1) / L.kcq) : 1;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = (size_t)round_up((int64_t)(off + bytes), 256); return o; };
  L.off_amax = take(sizeof(uint64_t) * (size_t)L.mpad * (size_t)L.npanel);
  L.off_bmax = take(sizeof(uint64_t) * (size_t)L.npad * (size_t)L.npanel);
  L.off_apack = take(sizeof(double) * (size_t)(L.mpad / 16) * (size_t)a_block_stride(L.K4));
  L.off_bpack = take(sizeof(double) * (size_t)(L.npad / 16) * (size_t)b_block_stride(L.K4));
  if (L.npanel > 1) {
    L.off_aexp = take(sizeof(int32_t) * (size_t)L.mpad * (size_t)L.npanel);
    L.off_bexp = take(sizeof(int32_t) * (size_t)L.npad * (size_t)L.npanel);
  }
  if (simple) {
    L.off_aplain = take(sizeof(double) * (size_t)kFragA * (size_t)m * (size_t)k);
    L.off_bplain = take(sizeof(double) * (size_t)kPlanesB * (size_t)k * (size_t)n);
    L.off_bins = take(sizeof(double) * 4 * (size_t)m * (size_t)n);
    L.off_acc = take(sizeof(double) * 2 * (size_t)m * (size_t)n);
  }
  L.balance = balance;
  if (balance) {
    L.off_acol = take(sizeof(uint64_t) * (size_t)L.kpad);
    L.off_brow = take(sizeof(uint64_t) * (size_t)L.kpad);
    L.off_gexp = take(sizeof(int32_t) * (size_t)L.kpad);
  }
  L.bytes = off;
  return L;
}

// Slice formats of the narrow-slice variants.
constexpr int kSliceBF16 = 0, kSliceF16 = 1, kSliceI8 = 2;

// Workspace of the narrow-slice variants.  Slices are integer-valued BF16 /
// FP16 numbers or INT8 integers packed for v_mfma_f32_32x32x16_{bf16,f16} /
// v_mfma_i32_32x32x32_i8: for each 32-row block rb of op(A) (32-column block
// of op(B)), each step q of the inner dimension (16 indices for BF16/FP16, 32
// for INT8) and each slice t, one 64-lane operand of 16 bytes per lane; lane
// l holds row (column) rb*32 + l%32 and the step's inner indices
// (l/32)*E .. (l/32)*E + E-1 (E = 8 two-byte or 16 one-byte values):
//   pack[rb*slices_block_stride(Q, S) + (q*S + t)*64 + l]   (in 16-byte units,
// blocks padded like the cascade's planes)
// Rows/columns are padded with zeros to the 64 x 64 workgroup tile.  The
// inner dimension is cut into chunks of `chunk` indices (one product pass
// each); every chunk starts a new step and is padded with zeros to whole
// blocks of four steps (64 or 128 indices), so packed inner index
// c * chunk_q * kstep + r holds source index c * chunk + r.
struct SlicesLayout {
  int64_t m, n, k;
  int64_t mpad, npad, kpad, Q;  // Q = kpad / kstep steps
  int32_t S, w, fmt, kstep;     // slice count, width, format, inner indices per step
  int64_t chunk;                // inner indices per chunk (every group sum exact), min(limit, k)
  int64_t chunk_q;              // packed steps per whole chunk: chunk padded to a multiple of 4 steps
  int32_t flush_mask[16];       // BF16/FP16: level L may go flush_mask[L] + 1 steps between flushes
  size_t off_amax, off_bmax, off_apack, off_bpack, off_planes, bytes;
};

// Slice counts above this run the levels from it upwards in a pass of their
// own, whose FP64 group sums go through the workspace.
constexpr int kSlicesSplit = 9;

// Largest chunk of the inner dimension keeping every FP64 level-group sum an
// exact integer, k s 2^(2w-2) (2^2w + 2^w + 1) <= 2^53, and for INT8 every
// level sum an INT32, k s 2^(2w-2) <= 2^31 - 1 (the exactness bounds alone;
// chunk c covers inner indices [c limit, (c + 1) limit)).  Integer division
// of 2^53 by the exact integer factor, so the limit is exact.
inline int64_t slices_chunk_limit(int w, int S, int fmt) {
  const unsigned __int128 per = (unsigned __int128)S * ((unsigned __int128)1 << (2 * w - 2)) *
                                (((unsigned __int128)1 << (2 * w)) + ((unsigned __int128)1 << w) + 1);
  const unsigned __int128 lim = ((unsigned __int128)1 << 53) / per;
  int64_t out = lim > (unsigned __int128)INT64_MAX ? INT64_MAX : (int64_t)lim;
  if (fmt == kSliceI8) {
    const int64_t l32 = ((int64_t(1) << 31) - 1) / ((int64_t)S << (2 * w - 2));
    out = out < l32 ? out : l32;
  }
  return out;
}

// (w, S) usable in the format: slices (|a| <= 2^(w-1)) exact in it, and for
// BF16/FP16 the FP32 sums of the top level exact over one 16-deep step.
inline bool slices_params_ok(int w, int S, int fmt) {
  if (w < 2 || S < 1 || S > 16) return false;
  const double maxmag = fmt == kSliceI8 ? 127.0 : (fmt == kSliceF16 ? 2048.0 : 256.0);
  if (__builtin_ldexp(1.0, w - 1) > maxmag) return false;
  if (fmt == kSliceI8) return true;
  return 16.0 * S * __builtin_ldexp(1.0, 2 * w - 2) <= __builtin_ldexp(1.0, 24);
}

// 16-byte units from one 32-row (32-column) block of packed slices to the
// next: the block plus 4 KiB + 256 B, so blocks loaded together do not share
// L2 sets.
constexpr int64_t kSlicePad = 272;
constexpr int64_t slices_block_stride(int64_t Q, int64_t S) { return Q * S * 64 + kSlicePad; }

inline SlicesLayout make_slices_layout(int64_t m, int64_t n, int64_t k, int S, int w, int fmt) {
  SlicesLayout L{};
  L.m = m; L.n = n; L.k = k;
  L.S = S; L.w = w; L.fmt = fmt;
  L.kstep = fmt == kSliceI8 ? 32 : 16;
  L.mpad = round_up(m > 0 ? m : 1, 64);
  L.npad = round_up(n > 0 ? n : 1, 64);
  const int64_t kk = k > 0 ? k : 1;
  const int64_t lim = slices_chunk_limit(w, S, fmt);
  L.chunk = lim < kk ? lim : kk;
  L.chunk_q = round_up(L.chunk, 4 * L.kstep) / L.kstep;
  const int64_t nchunk = (kk + L.chunk - 1) / L.chunk;
  const int64_t last = kk - (nchunk - 1) * L.chunk;   // indices of the last chunk
  L.Q = (nchunk - 1) * L.chunk_q + round_up(last, 4 * L.kstep) / L.kstep;
  L.kpad = L.Q * L.kstep;
  for (int lv = 0; lv < 16; ++lv) {
    // largest power-of-two number of steps with 16 * steps * (lv+1) * 2^(2w-2) <= 2^24
    int64_t steps = 1;
    while (2.0 * 16 * steps * (lv + 1) * __builtin_ldexp(1.0, 2 * w - 2) <= __builtin_ldexp(1.0, 24)) steps *= 2;
    L.flush_mask[lv] = (int32_t)(steps - 1);
  }
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = (size_t)round_up((int64_t)(off + bytes), 256); return o; };
  L.off_amax = take(sizeof(uint64_t) * (size_t)L.mpad);
  L.off_bmax = take(sizeof(uint64_t) * (size_t)L.npad);
  L.off_apack = take(16 * (size_t)(L.mpad / 32) * (size_t)slices_block_stride(L.Q, S));
  L.off_bpack = take(16 * (size_t)(L.npad / 32) * (size_t)slices_block_stride(L.Q, S));
  const int upper_groups = S > kSlicesSplit ? (S + 2) / 3 - kSlicesSplit / 3 : 0;
  L.off_planes = take(sizeof(double) * (size_t)upper_groups * (size_t)L.mpad * (size_t)L.npad);
  L.bytes = off;
  return L;
}

}  // namespace ddk
