// Phase one of the cascade (Sec. 4): Sigma and T, then the split of
// Appendix A into pre-weighted, MFMA-fragment-packed digit planes.
//
//  * max_abs_bits_*: per row of op(A) / column of op(B), the largest |hi| (or
//    |fl(hi + lo)| when the lo plane is given) as a bit pattern (non-negative
//    doubles order like their bits), reduced with atomicMax; the exponent
//    e = frexp_exp(max) is taken where it is used.
//  * pack_a / pack_b: four consecutive 64-lane fragments per wave, each lane
//    splits one entry of each and writes its 4 (A) or 5 (B: B0'..B3' and
//    B6'; B4' and B5' are formed in the product kernel) planes; zero padding
//    outside m, n, k.
//  * unpack_*: diagnostic copy of the packed planes into plain column-major
//    planes (used by dd_cascade_split).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dd_device.hpp"
#include "kernels.hpp"
#include "layout.hpp"

namespace ddk {

__global__ void fill_u64(uint64_t* p, int64_t n, uint64_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// With rscale, element (o, r) is first multiplied by 2^(rsign * rscale[r])
// (the diagonal balancing of the inner dimension).
// The reduced range is cut into chunks of `chunk` indices; chunk c (taken by
// blocks y = c, c + gridDim.y, ...) goes to out[o + c * ostride]: ostride = 0
// folds every chunk into one maximum, ostride > 0 keeps one per chunk (the
// per-panel maxima, chunk = the panel length).

// Element (o, r) at X[o + r*ld]: consecutive threads take consecutive o.
__global__ void __launch_bounds__(256)
max_abs_bits_outer_contig(const double* __restrict__ X, const double* __restrict__ Xlo, int64_t outer,
                          int64_t red, int64_t ld, int64_t chunk, int64_t ostride,
                          uint64_t* __restrict__ out, const int32_t* __restrict__ rscale, int rsign) {
  int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (o >= outer) return;
  const int64_t nchunk = (red + chunk - 1) / chunk;
  for (int64_t c = blockIdx.y; c < nchunk; c += gridDim.y) {
    int64_t r0 = c * chunk;
    int64_t r1 = r0 + chunk < red ? r0 + chunk : red;
    uint64_t mx = 0;
#pragma unroll 8
    for (int64_t r = r0; r < r1; ++r) {
      double v = Xlo ? X[o + r * ld] + Xlo[o + r * ld] : X[o + r * ld];
      if (rscale) v = __builtin_ldexp(v, rsign * rscale[r]);
      uint64_t b = __builtin_bit_cast(uint64_t, v) & 0x7fffffffffffffffull;
      mx = b > mx ? b : mx;
    }
    atomicMax((unsigned long long*)&out[o + c * ostride], (unsigned long long)mx);
  }
}

// Element (o, r) at X[r + o*ld]: one wave per o, lanes stride over r.
__global__ void __launch_bounds__(256)
max_abs_bits_red_contig(const double* __restrict__ X, const double* __restrict__ Xlo, int64_t outer,
                        int64_t red, int64_t ld, int64_t chunk, int64_t ostride,
                        uint64_t* __restrict__ out, const int32_t* __restrict__ rscale, int rsign) {
  int64_t o = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (o >= outer) return;
  const double* col = X + o * ld;
  const double* col_lo = Xlo ? Xlo + o * ld : nullptr;
  const int64_t nchunk = (red + chunk - 1) / chunk;
  for (int64_t c = blockIdx.y; c < nchunk; c += gridDim.y) {
    int64_t r0 = c * chunk;
    int64_t r1 = r0 + chunk < red ? r0 + chunk : red;
    uint64_t mx = 0;
#pragma unroll 4
    for (int64_t r = r0 + lane; r < r1; r += 64) {
      double v = col_lo ? col[r] + col_lo[r] : col[r];
      if (rscale) v = __builtin_ldexp(v, rsign * rscale[r]);
      uint64_t b = __builtin_bit_cast(uint64_t, v) & 0x7fffffffffffffffull;
      mx = b > mx ? b : mx;
    }
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
      uint64_t y = __shfl_xor(mx, s, 64);
      mx = y > mx ? y : mx;
    }
    if (lane == 0) atomicMax((unsigned long long*)&out[o + c * ostride], (unsigned long long)mx);
  }
}

__device__ __forceinline__ SplitParams make_params(int c0, int c1, int c2) {
  SplitParams sp;
  int c[3] = {c0, c1, c2};
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    sp.K[t] = __builtin_ldexp(1.0, 53 - c[t]) + __builtin_ldexp(1.0, 52 - c[t]);
    sp.P[t] = __builtin_ldexp(1.0, c[t]);
  }
  sp.sig[0] = 1.0;
  sp.sig[1] = __builtin_ldexp(1.0, -c0);
  sp.sig[2] = __builtin_ldexp(1.0, -(c0 + c1));
  sp.sig[3] = __builtin_ldexp(1.0, -(c0 + c1 + c2));
  return sp;
}

// Packed A planes, F consecutive 64-lane fragments per wave: op(A)(i, p) =
// A[i*si + p*sp_].  The exponent of entry (i, p) is amax[i] (pstride = 0),
// or with per-panel Sigma amax[i + (p / plen) * pstride]; likewise for B.
// With gexp, the entry is first multiplied by 2^gexp[p] (A) or 2^-gexp[p]
// (B): the diagonal balancing of the inner dimension.  Every load of the F
// fragments is issued before the first split, so a lane has 2F loads in
// flight (one fragment's two would leave HBM half idle).  Fragments at or
// past nfrag are skipped.
template <int F>
__device__ __forceinline__ void pack_a_frags(const double* __restrict__ Ahi, const double* __restrict__ Alo,
                                             int64_t si, int64_t sp_, int64_t m, int64_t k, int64_t K4,
                                             int64_t frag0, int64_t nfrag, int lane,
                                             const uint64_t* __restrict__ amax, int c0, int c1, int c2,
                                             double* __restrict__ Apack, int64_t plen = 1, int64_t pstride = 0,
                                             const int32_t* __restrict__ gexp = nullptr) {
  double h[F], l[F];
  uint64_t mb[F];
  int g[F];
#pragma unroll
  for (int f = 0; f < F; ++f) {
    const int64_t frag = frag0 + f;
    const int64_t rb = frag / K4, kq = frag - rb * K4;
    // position lane = s*16 + kk*4 + ii holds row rb*16 + s*4 + ii, inner index kq*4 + kk
    const int64_t i = rb * 16 + (lane >> 4) * 4 + (lane & 3), p = kq * 4 + ((lane >> 2) & 3);
    h[f] = l[f] = 0.0;
    mb[f] = 0;
    g[f] = 0;
    if (frag < nfrag && i < m && p < k) {
      const int64_t idx = i * si + p * sp_;
      h[f] = Ahi[idx];
      l[f] = Alo[idx];
      mb[f] = amax[i + (p / plen) * pstride];
      if (gexp) g[f] = gexp[p];
    }
  }
  const SplitParams spar = make_params(c0, c1, c2);
#pragma unroll
  for (int f = 0; f < F; ++f) {
    const int64_t frag = frag0 + f;
    if (frag >= nfrag) break;
    const int64_t rb = frag / K4, kq = frag - rb * K4;
    const int64_t i = rb * 16 + (lane >> 4) * 4 + (lane & 3), p = kq * 4 + ((lane >> 2) & 3);
    double w[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < m && p < k) {
      double xh, xl;
      split_entry(__builtin_ldexp(h[f], g[f]), __builtin_ldexp(l[f], g[f]), exp_of_bits(mb[f]), spar, w, xh, xl);
    }
    double* dst = Apack + rb * a_block_stride(K4) + kq * (kFragA * kLanes) + lane;
#pragma unroll
    for (int t = 0; t < 4; ++t) dst[t * kLanes] = w[t];
  }
}

// Packed B planes, F consecutive fragments per wave: op(B)(p, j) = B[p*sp_ + j*sj].
// FB stored planes per fragment: 7 (B0'..B6') or 5 (B0'..B3', B6').
template <int F, int FB = kFragB>
__device__ __forceinline__ void pack_b_frags(const double* __restrict__ Bhi, const double* __restrict__ Blo,
                                             int64_t sp_, int64_t sj, int64_t k, int64_t n, int64_t K4,
                                             int64_t frag0, int64_t nfrag, int lane,
                                             const uint64_t* __restrict__ bmax, int c0, int c1, int c2,
                                             double* __restrict__ Bpack, int64_t plen = 1, int64_t pstride = 0,
                                             const int32_t* __restrict__ gexp = nullptr) {
  double h[F], l[F];
  uint64_t mb[F];
  int g[F];
#pragma unroll
  for (int f = 0; f < F; ++f) {
    const int64_t frag = frag0 + f;
    const int64_t cb = frag / K4, kq = frag - cb * K4;
    const int64_t j = cb * 16 + (lane & 15), p = kq * 4 + (lane >> 4);
    h[f] = l[f] = 0.0;
    mb[f] = 0;
    g[f] = 0;
    if (frag < nfrag && j < n && p < k) {
      const int64_t idx = p * sp_ + j * sj;
      h[f] = Bhi[idx];
      l[f] = Blo[idx];
      mb[f] = bmax[j + (p / plen) * pstride];
      if (gexp) g[f] = gexp[p];   // negated where it is used: no wait here
    }
  }
  const SplitParams spar = make_params(c0, c1, c2);
#pragma unroll
  for (int f = 0; f < F; ++f) {
    const int64_t frag = frag0 + f;
    if (frag >= nfrag) break;
    const int64_t cb = frag / K4, kq = frag - cb * K4;
    const int64_t j = cb * 16 + (lane & 15), p = kq * 4 + (lane >> 4);
    double w[kFragB] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (j < n && p < k) {
      double yh, yl;
      split_entry(__builtin_ldexp(h[f], -g[f]), __builtin_ldexp(l[f], -g[f]), exp_of_bits(mb[f]), spar, w, yh, yl);
      w[4] = w[2] + w[3];   // sigma_2 B4 = B2' + B3'
      w[5] = w[1] + w[4];   // sigma_1 B5 = B1' + B2' + B3'
      w[6] = yh + yl;       // B6: the scaled entry itself, rounded once
    }
    double* dst = Bpack + cb * b_block_stride(K4, FB) + kq * (FB * kLanes) + lane;
    if constexpr (FB == kFragB) {
#pragma unroll
      for (int t = 0; t < kFragB; ++t) dst[t * kLanes] = w[t];
    } else {
      static_assert(FB == kFragBBatched, "5 or 7 stored planes");
#pragma unroll
      for (int t = 0; t < 4; ++t) dst[t * kLanes] = w[t];
      dst[4 * kLanes] = w[6];
    }
  }
}

constexpr int kPF = kPackFragsPerWave;

// kPF consecutive fragments (rb, kq) per wave.
__global__ void __launch_bounds__(256)
pack_a(const double* __restrict__ Ahi, const double* __restrict__ Alo, int64_t si, int64_t sp_,
       int64_t m, int64_t k, int64_t K4, int64_t nfrag, const uint64_t* __restrict__ amax,
       int c0, int c1, int c2, double* __restrict__ Apack, int64_t plen, int64_t pstride,
       const int32_t* __restrict__ gexp) {
  const int64_t frag0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * kPF;
  if (frag0 >= nfrag) return;
  pack_a_frags<kPF>(Ahi, Alo, si, sp_, m, k, K4, frag0, nfrag, threadIdx.x & 63, amax, c0, c1, c2, Apack, plen,
                    pstride, gexp);
}

// kPF consecutive fragments (cb, kq) per wave.
__global__ void __launch_bounds__(256)
pack_b(const double* __restrict__ Bhi, const double* __restrict__ Blo, int64_t sp_, int64_t sj,
       int64_t k, int64_t n, int64_t K4, int64_t nfrag, const uint64_t* __restrict__ bmax,
       int c0, int c1, int c2, double* __restrict__ Bpack, int64_t plen, int64_t pstride,
       const int32_t* __restrict__ gexp) {
  const int64_t frag0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * kPF;
  if (frag0 >= nfrag) return;
  pack_b_frags<kPF>(Bhi, Blo, sp_, sj, k, n, K4, frag0, nfrag, threadIdx.x & 63, bmax, c0, c1, c2, Bpack, plen,
                    pstride, gexp);
}

// ------------------------------------------------------------ batched phase one
// Units of work of every problem are numbered consecutively; prefix[p] is the
// first unit of problem p (prefix[count] = total).  A block finds its problem
// by binary search.
__device__ __forceinline__ int find_problem(const int64_t* __restrict__ prefix, int count, int64_t u) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= u) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Units of A: (256-row block, 256-long inner chunk); of B: (4 columns, 4096-long chunk).
__global__ void __launch_bounds__(256)
batched_max_abs(const BatchDesc* __restrict__ desc, int count, const int64_t* __restrict__ prefA,
                const int64_t* __restrict__ prefB, const double* const* __restrict__ Ahi,
                const double* const* __restrict__ Bhi, char* __restrict__ ws) {
  const int64_t totA = prefA[count], tot = totA + prefB[count];
  for (int64_t u = blockIdx.x; u < tot; u += gridDim.x) {
    if (u < totA) {
      const int p = find_problem(prefA, count, u);
      const BatchDesc d = desc[p];
      const int64_t local = u - prefA[p];
      const int64_t nchunk = (d.k + 255) / 256;
      const int64_t rblk = local / nchunk, ch = local - rblk * nchunk;
      const int64_t o = rblk * 256 + threadIdx.x;
      if (o >= d.m) continue;
      const int64_t r0 = ch * 256, r1 = r0 + 256 < d.k ? r0 + 256 : d.k;
      uint64_t mx = 0;
      const double* X = Ahi[p];
      for (int64_t r = r0; r < r1; ++r) {
        uint64_t b = __builtin_bit_cast(uint64_t, X[o + r * d.lda]) & 0x7fffffffffffffffull;
        mx = b > mx ? b : mx;
      }
      atomicMax((unsigned long long*)((uint64_t*)(ws + d.off_amax) + o), (unsigned long long)mx);
    } else {
      const int64_t v = u - totA;
      const int p = find_problem(prefB, count, v);
      const BatchDesc d = desc[p];
      const int64_t local = v - prefB[p];
      const int64_t nchunk = (d.k + 4095) / 4096;
      const int64_t cgrp = local / nchunk, ch = local - cgrp * nchunk;
      const int lane = threadIdx.x & 63;
      const int64_t o = cgrp * 4 + (threadIdx.x >> 6);
      if (o >= d.n) continue;
      const int64_t r0 = ch * 4096, r1 = r0 + 4096 < d.k ? r0 + 4096 : d.k;
      uint64_t mx = 0;
      const double* col = Bhi[p] + o * d.ldb;
      for (int64_t r = r0 + lane; r < r1; r += 64) {
        uint64_t b = __builtin_bit_cast(uint64_t, col[r]) & 0x7fffffffffffffffull;
        mx = b > mx ? b : mx;
      }
#pragma unroll
      for (int sft = 32; sft >= 1; sft >>= 1) {
        uint64_t y = __shfl_xor(mx, sft, 64);
        mx = y > mx ? y : mx;
      }
      if (lane == 0) atomicMax((unsigned long long*)((uint64_t*)(ws + d.off_bmax) + o), (unsigned long long)mx);
    }
  }
}

// Units: 4 x kPF fragments (kPF consecutive ones per wave) of the packed A
// planes, then of B.
__global__ void __launch_bounds__(256)
batched_pack(const BatchDesc* __restrict__ desc, int count, const int64_t* __restrict__ prefA,
             const int64_t* __restrict__ prefB, const double* const* __restrict__ Ahi,
             const double* const* __restrict__ Alo, const double* const* __restrict__ Bhi,
             const double* const* __restrict__ Blo, char* __restrict__ ws) {
  const int64_t totA = prefA[count], tot = totA + prefB[count];
  const int lane = threadIdx.x & 63;
  for (int64_t u = blockIdx.x; u < tot; u += gridDim.x) {
    if (u < totA) {
      const int p = find_problem(prefA, count, u);
      const BatchDesc d = desc[p];
      const int64_t frag0 = ((u - prefA[p]) * 4 + (threadIdx.x >> 6)) * kPF, nfrag = (d.mpad / 16) * d.K4;
      if (frag0 >= nfrag) continue;
      pack_a_frags<kPF>(Ahi[p], Alo[p], 1, d.lda, d.m, d.k, d.K4, frag0, nfrag, lane,
                        (const uint64_t*)(ws + d.off_amax), d.c0, d.c1, d.c2, (double*)(ws + d.off_apack));
    } else {
      const int64_t v = u - totA;
      const int p = find_problem(prefB, count, v);
      const BatchDesc d = desc[p];
      const int64_t frag0 = ((v - prefB[p]) * 4 + (threadIdx.x >> 6)) * kPF, nfrag = (d.npad / 16) * d.K4;
      if (frag0 >= nfrag) continue;
      pack_b_frags<kPF, kFragBBatched>(Bhi[p], Blo[p], 1, d.ldb, d.k, d.n, d.K4, frag0, nfrag, lane,
                        (const uint64_t*)(ws + d.off_bmax), d.c0, d.c1, d.c2, (double*)(ws + d.off_bpack));
    }
  }
}

// Plain planes from the packed layout (diagnostics).  side 0: element (i, p)
// of a rows x cols = m x k operand; side 1: element (p, j) of k x n.
__global__ void __launch_bounds__(256)
unpack_planes(const double* __restrict__ pack, int side, int64_t rows, int64_t cols, int64_t K4,
              double* __restrict__ planes) {
  int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= rows * cols) return;
  int64_t r = idx % rows, cidx = idx / rows;
  const int64_t plane = rows * cols;
  if (side == 0) {
    int64_t blk = r / 16, q = cidx / 4, kk = cidx % 4;
    int64_t lanepos = ((r % 16) / 4) * 16 + kk * 4 + (r % 4);
    const double* src = pack + blk * a_block_stride(K4) + q * (int64_t)(kFragA * kLanes) + lanepos;
    for (int t = 0; t < kFragA; ++t) planes[t * plane + idx] = src[t * kLanes];
  } else {
    int64_t blk = cidx / 16, q = r / 4, kk = r % 4;
    const double* src = pack + blk * b_block_stride(K4) + q * (int64_t)(kFragB * kLanes) + kk * 16 + (cidx % 16);
    for (int t = 0; t < kFragB; ++t) planes[t * plane + idx] = src[t * kLanes];
  }
}

// Diagonal balancing: g[p] = floor((e_B(p) - e_A(p)) / 2) from the column
// maxima of op(A) and row maxima of op(B); 0 beyond k.
__global__ void balance_exps(const uint64_t* __restrict__ acol, const uint64_t* __restrict__ brow,
                             int64_t k, int64_t kpad, int32_t* __restrict__ g) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= kpad) return;
  g[p] = p < k ? (exp_of_bits(brow[p]) - exp_of_bits(acol[p])) >> 1 : 0;
}

__global__ void exps_from_bits(const uint64_t* __restrict__ bits, int64_t n, int32_t* __restrict__ e) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) e[i] = exp_of_bits(bits[i]);
}

// ------------------------------------------------------------------ launchers
static inline unsigned blocks_for(int64_t n, int64_t per) { return (unsigned)((n + per - 1) / per); }

hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  fill_u64<<<blocks_for(n, 256), 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  fill_u32<<<blocks_for(n, 256), 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}

// max |X(o, r)| bits over r for o < outer, X(o, r) = X[o*so + r*sr]; one of
// so, sr is 1.  out must be zero on entry.  With plen > 0, one maximum per
// run of plen consecutive r: out[o + (r / plen) * ostride].
hipError_t launch_max_abs_bits(const double* X, int64_t outer, int64_t red, int64_t so, int64_t sr,
                               uint64_t* out, hipStream_t s, const double* Xlo, int64_t plen,
                               int64_t ostride, const int32_t* rscale, int rsign) {
  if (outer <= 0 || red <= 0) return hipSuccess;
  if (plen > 0 && ostride < outer) return hipErrorInvalidValue;
  // Rows of r per block: for consecutive o (so == 1) each thread walks its
  // chunk of r alone, so small matrices get short chunks (down to 16) until
  // the grid has about 2048 blocks; one wave per o walks 4096 per block.
  int64_t step = 4096;
  if (so == 1) {
    const int64_t bx = (outer + 255) / 256;
    step = 256;
    while (step > 16 && bx * ((red + step - 1) / step) < 2048) step /= 2;
  }
  int64_t chunk = plen > 0 ? plen : step;
  int64_t gy = (red + chunk - 1) / chunk;
  if (plen <= 0) {
    while (gy > 65535) { chunk *= 2; gy = (red + chunk - 1) / chunk; }
    ostride = 0;
  } else if (gy > 65535) {
    gy = 65535;   // blocks loop over the panels
  }
  if (so == 1) {
    dim3 grid(blocks_for(outer, 256), (unsigned)gy);
    max_abs_bits_outer_contig<<<grid, 256, 0, s>>>(X, Xlo, outer, red, sr, chunk, ostride, out, rscale, rsign);
  } else {
    dim3 grid(blocks_for(outer, 4), (unsigned)gy);
    max_abs_bits_red_contig<<<grid, 256, 0, s>>>(X, Xlo, outer, red, so, chunk, ostride, out, rscale, rsign);
  }
  return hipGetLastError();
}

hipError_t launch_pack_a(const double* Ahi, const double* Alo, int64_t si, int64_t sp,
                         const CascadeLayout& L, const uint64_t* amax, double* Apack, hipStream_t s,
                         const int32_t* gexp) {
  int64_t nfrag = (L.mpad / 16) * L.K4;
  const int64_t plen = 4 * (int64_t)L.kcq, pstride = L.npanel > 1 ? L.mpad : 0;
  pack_a<<<blocks_for(nfrag, 4 * kPF), 256, 0, s>>>(Ahi, Alo, si, sp, L.m, L.k, L.K4, nfrag, amax,
                                              L.c[0], L.c[1], L.c[2], Apack, plen, pstride, gexp);
  return hipGetLastError();
}

hipError_t launch_pack_b(const double* Bhi, const double* Blo, int64_t sp, int64_t sj,
                         const CascadeLayout& L, const uint64_t* bmax, double* Bpack, hipStream_t s,
                         const int32_t* gexp) {
  int64_t nfrag = (L.npad / 16) * L.K4;
  const int64_t plen = 4 * (int64_t)L.kcq, pstride = L.npanel > 1 ? L.npad : 0;
  pack_b<<<blocks_for(nfrag, 4 * kPF), 256, 0, s>>>(Bhi, Blo, sp, sj, L.k, L.n, L.K4, nfrag, bmax,
                                              L.c[0], L.c[1], L.c[2], Bpack, plen, pstride, gexp);
  return hipGetLastError();
}

hipError_t launch_unpack(const double* pack, int side, int64_t rows, int64_t cols, int64_t K4,
                         double* planes, hipStream_t s) {
  if (rows * cols <= 0) return hipSuccess;
  unpack_planes<<<blocks_for(rows * cols, 256), 256, 0, s>>>(pack, side, rows, cols, K4, planes);
  return hipGetLastError();
}

hipError_t launch_batched_phase_one(const BatchDesc* desc, int count, const int64_t* prefExpA,
                                   const int64_t* prefExpB, int64_t units_exp, const int64_t* prefPackA,
                                   const int64_t* prefPackB, int64_t units_pack,
                                   const double* const* Ahi, const double* const* Alo,
                                   const double* const* Bhi, const double* const* Blo,
                                   char* ws, uint64_t* exps, int64_t nexps, hipStream_t s) {
  hipError_t e = launch_fill_u64(exps, nexps, 0, s);
  if (e != hipSuccess) return e;
  const unsigned ge = (unsigned)(units_exp < 65536 ? (units_exp > 0 ? units_exp : 1) : 65536);
  batched_max_abs<<<ge, 256, 0, s>>>(desc, count, prefExpA, prefExpB, Ahi, Bhi, ws);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned gp = (unsigned)(units_pack < 65536 ? (units_pack > 0 ? units_pack : 1) : 65536);
  batched_pack<<<gp, 256, 0, s>>>(desc, count, prefPackA, prefPackB, Ahi, Alo, Bhi, Blo, ws);
  return hipGetLastError();
}

hipError_t launch_balance_exps(const uint64_t* acol, const uint64_t* brow, int64_t k, int64_t kpad,
                               int32_t* g, hipStream_t s) {
  if (kpad <= 0) return hipSuccess;
  balance_exps<<<blocks_for(kpad, 256), 256, 0, s>>>(acol, brow, k, kpad, g);
  return hipGetLastError();
}

hipError_t launch_exps(const uint64_t* bits, int64_t n, int32_t* e, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  exps_from_bits<<<blocks_for(n, 256), 256, 0, s>>>(bits, n, e);
  return hipGetLastError();
}

}  // namespace ddk
