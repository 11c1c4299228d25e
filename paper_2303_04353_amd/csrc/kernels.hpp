// Host-side launchers of the library's kernels (each defined next to its
// kernel in a .hip file).  All launches are asynchronous on `s` and return
// the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <stdint.h>

#include <mutex>

#include "layout.hpp"

namespace ddk {

hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s);
// Largest |X| (|fl(X + Xlo)| if Xlo is given) per outer index, as bits.
hipError_t launch_max_abs_bits(const double* X, int64_t outer, int64_t red, int64_t so, int64_t sr,
                               uint64_t* out, hipStream_t s, const double* Xlo = nullptr,
                               int64_t plen = 0, int64_t ostride = 0, const int32_t* rscale = nullptr,
                               int rsign = 1);
hipError_t launch_balance_exps(const uint64_t* acol, const uint64_t* brow, int64_t k, int64_t kpad,
                               int32_t* g, hipStream_t s);
hipError_t launch_pack_a(const double* Ahi, const double* Alo, int64_t si, int64_t sp,
                         const CascadeLayout& L, const uint64_t* amax, double* Apack, hipStream_t s,
                         const int32_t* gexp = nullptr);
hipError_t launch_pack_b(const double* Bhi, const double* Blo, int64_t sp, int64_t sj,
                         const CascadeLayout& L, const uint64_t* bmax, double* Bpack, hipStream_t s,
                         const int32_t* gexp = nullptr);
hipError_t launch_unpack(const double* pack, int side, int64_t rows, int64_t cols, int64_t K4,
                         double* planes, hipStream_t s);
hipError_t launch_exps(const uint64_t* bits, int64_t n, int32_t* e, hipStream_t s);

// Phase one of a batch: zero the exponent words, reduce max |hi| per row of
// every A and column of every B, then split all operands.  Units of work are
// numbered through the prefix arrays (prefix[count] = total).
hipError_t launch_batched_phase_one(const BatchDesc* desc, int count, const int64_t* prefExpA,
                                   const int64_t* prefExpB, int64_t units_exp, const int64_t* prefPackA,
                                   const int64_t* prefPackB, int64_t units_pack,
                                   const double* const* Ahi, const double* const* Alo,
                                   const double* const* Bhi, const double* const* Blo,
                                   char* ws, uint64_t* exps, int64_t nexps, hipStream_t s);

// The product kernel over a list of tiles of a batch, `grid` persistent
// workgroups; `dynamic` takes tiles from an atomic counter (zeroed here)
// instead of a fixed stride.  `flags` (may be null): the cancellation
// bitmaps of all problems, problem p's from word desc[p].off_flags, zeroed
// by the caller.
hipError_t launch_cascade_batched(const BatchDesc* desc, const BatchTile* tiles, int64_t ntiles,
                                  double* const* Chi, double* const* Clo, const char* ws,
                                  uint32_t* counter, int grid, bool dynamic, uint32_t* flags, bool buf,
                                  hipStream_t s);
// Whether the packed blocks of a 64 x 64 tile at this K4 span less than the
// 2 GiB that the product kernels' buffer-load staging addresses.
bool buffer_staging_fits(int64_t K4);

// The fused product kernel: ten FP64 MFMA products per rank-kc block, bins
// combined in FP64x2, Sigma/T applied, C := C + result.  `flags` (may be
// null): m x n bitmap, zeroed by the caller, of entries at risk of
// cancellation (a block's bin 0 zero while a lower bin is not).
// With L.npanel > 1, aexp / bexp are the per-panel exponents (int32, set b
// at b * mpad / b * npad) and Sigma, T are applied per rank-kc block.
// `shape` is the output tile shape (kTile64x64, kTile32x64, kTile64x32).
hipError_t launch_cascade(const CascadeLayout& L, const double* Apack, const double* Bpack,
                          const uint64_t* amax, const uint64_t* bmax,
                          double* Chi, double* Clo, int64_t ldc, uint32_t* flags, hipStream_t s,
                          const int32_t* aexp = nullptr, const int32_t* bexp = nullptr,
                          int shape = kTile64x64);
// The product kernel with the split done while staging (64 x 64 tiles,
// global Sigma / T): operands from the caller's planes, op(A)(i, p) at
// A[i*a_si + p*a_sp], op(B)(p, j) at B[p*b_sp + j*b_sj]; amax / bmax from
// launch_max_abs_bits.  Gives the same bits as launch_cascade.
hipError_t launch_cascade_onload(const CascadeLayout& L, const double* Ahi, const double* Alo, int64_t a_si,
                                 int64_t a_sp, const double* Bhi, const double* Blo, int64_t b_sp, int64_t b_sj,
                                 const uint64_t* amax, const uint64_t* bmax, double* Chi, double* Clo, int64_t ldc,
                                 uint32_t* flags, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);

// FP64x3: workspace offsets (bytes: row/column maxima, packed digit planes)
// and the whole product (maxima, split, the fused product kernel).
struct TdOffsets {
  size_t amax, bmax, aplanes, bplanes;
};
size_t td_workspace_bytes(int64_t m, int64_t n, int64_t k, TdOffsets* off);
hipError_t run_td(int64_t m, int64_t n, int64_t k, int64_t kc, const double* A0, const double* A1,
                  const double* A2, int64_t a_si, int64_t a_sp, const double* B0, const double* B1,
                  const double* B2, int64_t b_sp, int64_t b_sj, double* C0, double* C1, double* C2,
                  int64_t ldc, char* ws, hipStream_t s);
void td_widths(int64_t kc, int c[5]);

// The unfused form (after the split into L's packed planes): plain planes,
// ten library GEMMs and a combine per rank-kc block, then the epilogue.
// The vendor BLAS handle of the current device (created on first use) with
// its stream set to `s`.  The lock is held until the lease ends, so calls on
// several host threads do not change the stream under each other.
struct BlasLease {
  std::unique_lock<std::mutex> lock;
  rocblas_handle h = nullptr;
  hipError_t status = hipSuccess;
};
BlasLease blas_lease(hipStream_t s);

hipError_t run_simple_products(const CascadeLayout& L, char* ws, const uint64_t* amax, const uint64_t* bmax,
                               double* Chi, double* Clo, int64_t ldc, hipStream_t s);

// Plain software double-double GEMM on the vector units.
hipError_t launch_dd_valu(int64_t m, int64_t n, int64_t k,
                          const double* Ahi, const double* Alo, int64_t a_si, int64_t a_sp,
                          const double* Bhi, const double* Blo, int64_t b_sp, int64_t b_sj,
                          double* Chi, double* Clo, int64_t ldc, hipStream_t s);

// FP64x2 dot product (two passes; `part` holds 2*dd_dot_blocks(n) doubles),
// scaling y = alpha x (alpha: two doubles in device memory) and addition
// z = x + y.
int dd_dot_blocks(int64_t n);
hipError_t launch_dd_dot(int64_t n, const double* xh, const double* xl, int64_t incx,
                         const double* yh, const double* yl, int64_t incy,
                         double* part, double* res, hipStream_t s);
hipError_t launch_dd_scal(int64_t n, const double* alpha, const double* xh, const double* xl, int64_t incx,
                          double* yh, double* yl, int64_t incy, hipStream_t s);
hipError_t launch_dd_add(int64_t n, const double* xh, const double* xl, int64_t incx, const double* yh,
                         const double* yl, int64_t incy, double* zh, double* zl, int64_t incz, hipStream_t s);

// The narrow-slice variant: split of op(A) (outer = m) or op(B) (outer = n)
// into packed BF16/FP16 slices, X(o, r) at X[o*so + r*sr] (r the inner index;
// maxbits from launch_max_abs_bits with the lo plane); the product passes
// for inner steps [q0, q1) (16 indices each), C := C + result; and a
// diagnostic unpack of packed slices into plain 16-bit planes.
hipError_t launch_slices_split(const double* Xhi, const double* Xlo, int64_t so, int64_t sr, int64_t outer,
                               int64_t red, int64_t opad, const SlicesLayout& L, const uint64_t* maxbits,
                               void* pack, hipStream_t s);
hipError_t launch_slices_product(const SlicesLayout& L, const void* Apack, const void* Bpack,
                                 const uint64_t* amax, const uint64_t* bmax, double* planes, double* Chi,
                                 double* Clo, int64_t ldc, int64_t q0, int64_t q1, hipStream_t s);
hipError_t launch_slices_unpack(const void* pack, int64_t outer, int64_t red, const SlicesLayout& L,
                                int64_t oo, int64_t ro, uint16_t* out, hipStream_t s);

}  // namespace ddk
