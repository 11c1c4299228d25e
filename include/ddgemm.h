/*
 * ddgemm -- double-double (FP64x2) GEMM for AMD Instinct MI355X (gfx950),
 * computed as a cascade of FP64 matrix products.
 *
 * Method: Parikh, van de Geijn, Henry, "Cascading GEMM: High Precision from
 * Low Precision" (arXiv 2303.04353).  An FP64x2 number is the unevaluated sum
 * hi + lo of two FP64 numbers (Sec. 3.1, eq. doubledouble).  Each row of A and
 * each column of B is scaled by a power of two and cut into four FP64 digits
 * of bounded width (Sec. 3.3-3.4, Appendix A); the ten digit products of
 * eq. (Gemm10) are accumulated in four FP64 bins per rank-kc update, bins 0-2
 * exactly (Sec. 3.3, exactness constraints), and the bins are added in FP64x2
 * from the least significant one (Sec. 3.3, 3.6).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Matrices are column-major (BLAS) with a leading dimension; an FP64x2
 *   matrix is two separate FP64 arrays ("planes") hi and lo with the same
 *   leading dimension.  The value of entry (i, j) is hi[i + j*ld] + lo[i + j*ld]
 *   taken exactly; the pair need not be normalised.
 * - All matrix pointers are DEVICE pointers owned by the caller; the library
 *   never frees them.  A and B are read only, C is read and written.  C must
 *   not overlap A or B.
 * - Every call is stream ordered and asynchronous on `stream` (NULL = the
 *   default stream).  Argument errors are detected on the host and returned
 *   before anything is launched; a launch error is returned as DD_ERR_HIP.
 *   A leading dimension for which the matrix's extent in bytes would not fit
 *   in int64 is invalid like one below the row count.
 *   No C++ exception and no process exit crosses this interface.
 * - Non-finite inputs: an output entry whose row of op(A) or column of op(B)
 *   holds an Inf or NaN becomes NaN (the split has no finite digits for it).
 *   Entries whose inputs are finite are unaffected.
 * - The library runs on gfx950 only; other devices get DD_ERR_UNSUPPORTED.
 */
#ifndef DDGEMM_H
#define DDGEMM_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* 0 = success; a negative value -i means that argument i (1-based, in the
 * order of the prototype) is invalid, LAPACK "info" style. */
typedef int32_t dd_status;
#define DD_OK 0
#define DD_ERR_HIP 1          /* a HIP runtime call or kernel launch failed      */
#define DD_ERR_WORKSPACE 2    /* workspace too small, or device memory exhausted */
#define DD_ERR_UNSUPPORTED 3  /* the current device is not gfx950                */
#define DD_ERR_INTERNAL 4     /* internal invariant violated (a library bug)     */

/* Operation codes (the transa / transb / trans arguments, taken as int32_t
 * so that any value can be passed and rejected). */
typedef enum { DD_OP_N = 0, DD_OP_T = 1 } dd_op;

typedef enum {
  /* The paper's method: four FP64 digits per operand, ten FP64 products on
   * the FP64 matrix cores, bins combined in FP64x2 (Sec. 3.4, eq. Gemm10). */
  DD_ALGO_CASCADE_F64 = 0,
  /* Plain software double-double GEMM on the FP64 vector units: the "FP64x2
   * arithmetic" triple loop the paper compares against (Sec. 5.2); per entry
   * acc += a*b in DD arithmetic, inner index ascending, C added last. */
  DD_ALGO_DD_VALU = 1,
  /* Narrow slices on the BF16 / FP16 matrix cores (the bfloat16 cascade of
   * Sec. 6.2 carried to FP64x2 with equal-width splits and the product
   * triangle of Sec. 6.1).  Each row of A and column of B is scaled by the
   * power of two of its largest |fl(hi + lo)| and cut into `slices` integer
   * slices of `slice_bits` bits (round to nearest on a fixed grid, the
   * remainder carried as an FP64 pair), stored exactly in BF16 or FP16.  The
   * s(s+1)/2 products A_i B_j with i + j < s are summed per level i + j on
   * v_mfma_f32_32x32x16 with FP32 accumulation, flushed to FP64 before any
   * partial sum could exceed 2^24, so every level sum is exact; level sums
   * are gathered in FP64 groups of three (exact below 2^53, which bounds a
   * chunk of the inner dimension) and the groups are added in FP64x2 from
   * the least significant.  Accuracy: the dropped products and slice
   * remainders are below (s+1) 2^-(s w) per inner index relative to the row
   * and column scales. */
  DD_ALGO_SLICES_BF16 = 2,
  DD_ALGO_SLICES_F16 = 3,
  /* The same computation with INT8 slices on v_mfma_i32_32x32x32_i8 (the
   * "FP64x2 in terms of INT8" case of Sec. 6.2): level sums in INT32 are exact
   * over a whole chunk of the inner dimension, so no flushes; the chunk is
   * bounded by k s 2^(2w-2) <= 2^31 - 1 as well.  Slices need |a| <= 127,
   * i.e. w <= 7; defaults w = 7, s = 16 (111 bits, 136 products).  Results
   * equal DD_ALGO_SLICES_BF16 at the same (w, s) while k fits one chunk. */
  DD_ALGO_SLICES_I8 = 4,
  /* The paper's simple form of the cascade (Sec. 4.2): the same split, then
   * per rank-kc update ten plain FP64 GEMMs of the vendor library (rocBLAS)
   * into four bin matrices in device memory, a combine pass, and the same
   * epilogue.  Bins 0-2 are exact as in the fused form; bin 3-6 is summed in
   * the library's order, so results differ from DD_ALGO_CASCADE_F64 only
   * there.  A comparator for the fused kernel; not for use under graph
   * capture (the library may allocate).  kc applies; flags and scaling do
   * not. */
  DD_ALGO_SIMPLE_UNFUSED = 5,
  /* The cascade with the split done while operands are staged (the paper
   * cascades while it packs, Sec. 4.3): after the row and column maxima,
   * one kernel reads the caller's hi/lo planes, splits each staged entry as
   * Appendix A does and runs the ten products from there.  No digit planes
   * are stored, so the workspace is only the maxima (8 (mpad + npad)
   * bytes); every workgroup splits the operand tiles it stages, so the
   * split runs n/64 (m/64) times per entry, on the vector units, which do
   * not overlap the FP64 matrix cores.  Bit-identical to
   * DD_ALGO_CASCADE_F64.  kc and flags apply; scaling must be global, tile
   * 0 or DD_TILE_64x64. */
  DD_ALGO_CASCADE_ON_LOAD = 6
} dd_algo;

/* Where the cascade takes its powers of two Sigma (rows of op(A)) and T
 * (columns of op(B)) from (Sec. 3.3-3.4, Appendix A). */
typedef enum {
  /* One exponent per row and per column, from the largest |hi| over the
   * whole inner dimension; Sigma and T are applied once at the end. */
  DD_SCALING_GLOBAL = 0,
  /* One exponent per row and per column for every rank-kc panel (inner
   * indices [b kc, (b + 1) kc)): each panel is split with its own powers of
   * two and its FP64x2 result is scaled by them (exactly) before it is
   * accumulated.  The same result as DD_SCALING_GLOBAL when k <= kc; keeps
   * FP64x2 accuracy relative to |A||B| when the scale of a row or column
   * changes from panel to panel (the paper splits one kc panel at a time,
   * Sec. 4.3).  Workspace: 12 (mpad + npad) bytes per panel. */
  DD_SCALING_PANEL = 1,
  /* Flag, may be OR-ed with either of the above: a power-of-two diagonal
   * balancing F of the inner dimension first (Sec. 6, scaling and
   * balancing: A B = (A F)(F^-1 B)).  Column p of op(A) is multiplied by
   * 2^g_p and row p of op(B) by 2^-g_p, g_p = floor((e_B(p) - e_A(p)) / 2)
   * with e_A(p), e_B(p) the exponents (as for Sigma and T) of the column's
   * and the row's largest |hi|.  The product is unchanged (exactly, barring
   * underflow); the split then sees operands whose scale does not hinge on
   * a few skewed inner indices.  The result does not change when A and B
   * are given as A F0, F0^-1 B for any power-of-two diagonal F0.
   * Workspace: 20 kpad bytes more. */
  DD_SCALING_BALANCE = 2
} dd_scaling;

/* Output tile shapes of the cascade's product kernel (rows x columns of C
 * per workgroup).  Every shape computes every entry with the same
 * arithmetic, so results do not depend on the shape; smaller tiles give
 * more workgroups to small problems and less padding to ragged ones. */
typedef enum { DD_TILE_AUTO = 0, DD_TILE_64x64 = 1, DD_TILE_32x64 = 2, DD_TILE_64x32 = 3 } dd_tile;

/* Options of dd_gemm_ex / dd_gemm_batched.  A NULL pointer means all zero. */
typedef struct {
  int32_t algo;        /* dd_algo                                                  */
  int32_t kc;          /* cascade: inner block of one rank-kc update (Sec. 3.5);
                          0 = 256.  Must be a multiple of 4 in [4, 4096].  The
                          split widths follow from min(kc, k) by the constraints
                          of Sec. 3.3.  Must be 0 for the slices variants.      */
  int32_t tile;        /* cascade: dd_tile; DD_TILE_AUTO = 64 x 64, or the shape
                          dd_tune recorded for this problem when use_tuned = 1.
                          Must be 0 for the other algorithms and the batched
                          calls (a batched plan chooses per problem).           */
  int32_t slices;      /* slices variants: s in [1, 16]; 0 = 14 (BF16, FP16) or
                          16 (INT8)                                              */
  int32_t slice_bits;  /* slices variants: w; 0 = 8 (BF16, FP16) or 7 (INT8).
                          Needs 2^(w-1) <= 256 (BF16), 2048 (FP16) or 127 (INT8),
                          and for BF16/FP16 16 s 2^(2w-2) <= 2^24.  With w <= 8
                          every level is flushed every 4 steps (the fast
                          schedule); wider slices flush every step.  Both must
                          be 0 for the other algorithms.                         */
  int32_t scaling;     /* cascade: DD_SCALING_GLOBAL or DD_SCALING_PANEL, OR-ed
                          with DD_SCALING_BALANCE or not; must be 0 for the
                          other algorithms and for the batched calls.           */
  uint32_t* flags_out; /* cascade only, may be NULL: device bitmap of ceil(m n / 32)
                          words, bit (i + j m) for entry (i, j) of C.  The call
                          zeroes it (also when k = 0), then sets the bit of
                          every entry at risk of cancellation: in some rank-kc
                          block the exact bin 0 (the leading digits' product,
                          Sec. 3.7 and Sec. 4.4) is zero while a lower bin of
                          that block is not.  No correction is applied.  Must
                          be NULL for the other algorithms.  Batched calls: one
                          bitmap for all problems, problem p's from word
                          sum over q < p of ceil(m_q n_q / 32); every execution
                          zeroes all of it (a plan keeps the pointer given at
                          its creation).                                        */
  int32_t use_tuned;   /* cascade, 0 or 1: with tile = DD_TILE_AUTO, take the tile
                          shape dd_tune recorded for (m, n, k, kc, scaling), if
                          any (must be 0 for the other algorithms)              */
} dd_gemm_opts;

/*
 * C := A*B + C  (Sec. 1 problem statement; C added last, Sec. 6).
 * A is m x k (lda >= max(1, m)), B is k x n (ldb >= max(1, k)), C is m x n
 * (ldc >= max(1, m)), all FP64x2 as hi/lo planes.  Uses the cascade with
 * kc = 256 and a workspace that the library allocates and keeps per device
 * and stream (grown on demand; calls that overlap on one stream are ordered
 * by the stream).  m = 0 or n = 0 is a no-op; k = 0 leaves C unchanged.
 * Graph capture: a call on a stream being captured uses the cached
 * workspace if it is large enough (make one call of the largest size on
 * that stream first) and returns DD_ERR_WORKSPACE otherwise, since it can
 * neither allocate nor wait.  A buffer handed to a captured call is never
 * freed, so replays of the graph stay valid when later calls grow the
 * cache.  Calls issued on one stream from several host threads at once
 * must be ordered by the caller (a call may replace the stream's buffer).
 */
dd_status dd_gemm(int64_t m, int64_t n, int64_t k,
                  const double* A_hi, const double* A_lo, int64_t lda,
                  const double* B_hi, const double* B_lo, int64_t ldb,
                  double* C_hi, double* C_lo, int64_t ldc,
                  hipStream_t stream);

/* Bytes of device workspace dd_gemm_ex needs for this problem and options
 * (0 for DD_ALGO_DD_VALU).  Returns 0 as well for invalid arguments.
 * DD_ALGO_SIMPLE_UNFUSED needs, besides the cascade's, 8 (4 m k + 7 k n +
 * 6 m n) bytes of plain planes, bins and accumulator.
 * The cascade needs 32 mpad kpad + 56 npad kpad bytes of packed digit planes
 * (mpad, npad rounded up to 64, kpad to 16) plus 4352 bytes of padding per
 * 16 rows and columns.  The slices variants need b s (mpad + npad) kpad
 * bytes of packed slices (b = 2 for BF16/FP16, 1 for INT8; kpad rounded up
 * to 64 for BF16/FP16 and to 128 for INT8) plus 4352 bytes per 32 rows and
 * columns, and, for s > 9, 8 mpad npad (ceil(s/3) - 3) bytes of FP64 group
 * sums.  Both add the row and column maxima.  DD_ALGO_CASCADE_ON_LOAD needs
 * the maxima only. */
size_t dd_gemm_workspace_size(int32_t transa, int32_t transb,
                              int64_t m, int64_t n, int64_t k,
                              const dd_gemm_opts* opts);

/*
 * C := op(A)*op(B) + C with op(X) = X or X^T.  op(A) is m x k, op(B) is k x n.
 * lda >= max(1, rows of A as stored), likewise ldb; ldc >= max(1, m).
 * `workspace` is caller-owned device memory of at least
 * dd_gemm_workspace_size(...) bytes, 256-byte aligned; passing NULL with
 * ws_bytes = 0 makes the library use its own cached workspace, as dd_gemm
 * does (under graph capture only if it is already large enough).  The
 * workspace is in use until the call's work on `stream` has finished.
 */
dd_status dd_gemm_ex(int32_t transa, int32_t transb,
                     int64_t m, int64_t n, int64_t k,
                     const double* A_hi, const double* A_lo, int64_t lda,
                     const double* B_hi, const double* B_lo, int64_t ldb,
                     double* C_hi, double* C_lo, int64_t ldc,
                     void* workspace, size_t ws_bytes,
                     const dd_gemm_opts* opts, hipStream_t stream);

/*
 * The tuner of the cascade's output tile shape (the blocking parameters the
 * paper leaves to the machine, Sec. 4.3): for each of the `count` shapes
 * (host arrays m, n, k; op(A) = A, op(B) = B) it times the cascade with
 * every tile shape, `repeats` times each after a warm-up, on zero operands
 * it allocates itself (so not for graph capture; the time of the kernels
 * does not depend on the values), and records the fastest for (m, n, k,
 * kc, scaling) of `opts` (cascade only; tile 0, flags_out NULL).  Records
 * are kept for the process and appended, as lines "s m n k kc scaling
 * shape", to the file named by DDGEMM_TUNE_CACHE (read at first use), so a
 * later process finds them too.  Calls with use_tuned = 1 then use them.
 * shapes_out (host, may be NULL) receives the chosen dd_tile per shape (0
 * for an empty one).  Synchronous.
 */
dd_status dd_tune(int32_t count, const int64_t* m, const int64_t* n, const int64_t* k,
                  const dd_gemm_opts* opts, int32_t repeats, int32_t* shapes_out, hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): dd_gemm_ex
 * without a workspace argument.  The workspace is a fixed array of
 * DD_NOALLOC_SCRATCH_BYTES bytes inside the library, one per device, held
 * from the library's first use on that device until the process ends.  The
 * call allocates nothing (no hipMalloc, hipFree, events or library handles)
 * and launches the same kernels as dd_gemm_ex, so results are bit-identical
 * to it.  Arguments as for dd_gemm_ex (opts is argument 15, stream 16);
 * DD_ALGO_SIMPLE_UNFUSED is rejected (-15).  A problem whose
 * dd_gemm_workspace_size exceeds DD_NOALLOC_SCRATCH_BYTES is rejected with
 * DD_ERR_WORKSPACE before anything is launched: 1024 x 1024 x 1024 with the
 * cascade needs about 89 MiB; square cascades fit up to m = n = k = 1216.
 * Every call on one device shares that device's array and leaves its
 * contents behind (each call clears what must start at zero), so calls that
 * overlap on one device, on any streams, race on it: order them on one
 * stream, or with events.  The first call on a device looks the array's
 * address up (hipGetSymbolAddress, which may load the library's device
 * code); make that call before any graph capture.
 */
#define DD_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
dd_status dd_gemm_noalloc(int32_t transa, int32_t transb, int64_t m, int64_t n, int64_t k,
                          const double* A_hi, const double* A_lo, int64_t lda,
                          const double* B_hi, const double* B_lo, int64_t ldb,
                          double* C_hi, double* C_lo, int64_t ldc,
                          const dd_gemm_opts* opts, hipStream_t stream);

/*
 * Batches of independent GEMMs of uneven shapes, C_p := A_p B_p + C_p for
 * p < count (each as dd_gemm, no transposes; kc from opts as in dd_gemm_ex).
 * The cascade is the one of dd_gemm; the whole batch runs as one phase-one
 * pass and one persistent product launch over all output tiles (Sec. 3.5:
 * the number of products is independent of the shapes, so uneven problems
 * mix freely in one launch).
 *
 * A plan fixes count and the shapes (host arrays m, n, k, lda, ldb, ldc) and
 * owns the device memory for descriptors, tile list and packed operands
 * (dd_batched_plan_info reports its size).  Creating a plan allocates and
 * uploads (synchronously).  dd_gemm_batched_exec then launches three
 * kernels on `stream`, allocates nothing and may be captured in a HIP
 * graph; A_hi .. C_lo are DEVICE arrays of `count` device pointers, read
 * when the kernels run.  Calls of one plan that overlap (on different
 * streams) race on its workspace.  Problems with m, n or k = 0 are no-ops.
 *
 * Tiles: a problem's output tiles are 64 x 64, or 32 x 64 / 64 x 32 when
 * that shape's padded area is smaller, as the tile policy says: 0, always
 * 64 x 64; 1, the smaller shape for problems with k >= 256; 2, the smaller
 * shape wherever it cuts the padding.  Every shape gives the same bits.
 * Schedule of the persistent kernel: tiles in decreasing cost (LPT: inner
 * dimension times tile area) or problem order, taken with a fixed stride or
 * from an atomic counter.  The default is policy 0, LPT with a counter,
 * unless the tuning cache (file named by DDGEMM_TUNE_CACHE) holds a choice
 * for these shapes.  dd_batched_plan_tune times every combination (3
 * policies x 4 schedules) `repeats` times with the given operands (C is
 * updated by every run!), keeps the fastest and appends it to the cache.
 */
typedef struct dd_batched_plan_s* dd_batched_plan;
dd_status dd_batched_plan_create(int32_t count, const int64_t* m, const int64_t* n, const int64_t* k,
                                 const int64_t* lda, const int64_t* ldb, const int64_t* ldc,
                                 const dd_gemm_opts* opts, dd_batched_plan* plan);
dd_status dd_gemm_batched_exec(dd_batched_plan plan,
                               const double* const* A_hi, const double* const* A_lo,
                               const double* const* B_hi, const double* const* B_lo,
                               double* const* C_hi, double* const* C_lo, hipStream_t stream);
dd_status dd_batched_plan_tune(dd_batched_plan plan,
                               const double* const* A_hi, const double* const* A_lo,
                               const double* const* B_hi, const double* const* B_lo,
                               double* const* C_hi, double* const* C_lo, int32_t repeats,
                               hipStream_t stream);
/* Sets the schedule and tiles directly (dynamic: 1 = atomic counter, lpt:
 * 1 = decreasing cost, tile_policy 0..2 as above). */
dd_status dd_batched_plan_schedule(dd_batched_plan plan, int32_t dynamic, int32_t lpt, int32_t tile_policy,
                                   hipStream_t stream);
dd_status dd_batched_plan_info(dd_batched_plan plan, int64_t* ntiles, int32_t* dynamic, int32_t* lpt,
                               int32_t* tile_policy, size_t* device_bytes);
/* Waits for the device, then frees the plan and its memory. */
dd_status dd_batched_plan_destroy(dd_batched_plan plan);

/*
 * One-shot form.  m, n, k, lda, ldb, ldc are host arrays, A_hi .. C_lo
 * device arrays of device pointers, as for a plan; opts as for a plan.
 *  - workspace = NULL, ws_bytes = 0: plan, execute, wait, free
 *    (allocates; synchronous).
 *  - workspace = caller-owned device memory, 256-byte aligned, of at least
 *    dd_gemm_batched_workspace_size(count, m, n, k, opts) bytes: the call
 *    launches its kernels on `stream` and returns (asynchronous; the
 *    workspace is in use until they finish).  The plan's tables
 *    (descriptors and tile list, a few hundred bytes per problem and 16 per
 *    tile) are built and uploaded at the first call with these shapes on a
 *    device and kept by the library until the process ends; later calls
 *    with the same shapes allocate nothing and may be captured in a HIP
 *    graph.  On a stream being captured, shapes seen for the first time
 *    give DD_ERR_WORKSPACE and nothing is launched.  A workspace smaller
 *    than needed gives DD_ERR_WORKSPACE.
 */
dd_status dd_gemm_batched(int32_t count, const int64_t* m, const int64_t* n, const int64_t* k,
                          const double* const* A_hi, const double* const* A_lo, const int64_t* lda,
                          const double* const* B_hi, const double* const* B_lo, const int64_t* ldb,
                          double* const* C_hi, double* const* C_lo, const int64_t* ldc,
                          void* workspace, size_t ws_bytes, const dd_gemm_opts* opts, hipStream_t stream);

/* Bytes of workspace dd_gemm_batched needs for these shapes (host arrays) and
 * options: an atomic counter, the row and column exponents and the packed
 * planes of every problem.  0 for invalid arguments. */
size_t dd_gemm_batched_workspace_size(int32_t count, const int64_t* m, const int64_t* n, const int64_t* k,
                                      const dd_gemm_opts* opts);

/*
 * The split of Appendix A on its own (phase one of Sec. 4), for inspection
 * and testing.  `side` = 0: X is op(A), rows x cols = m x k, one exponent per
 * row, 4 planes A0'..A3'.  `side` = 1: X is op(B), rows x cols = k x n, one
 * exponent per column, 7 planes B0'..B6'.  Planes are pre-weighted
 * (A_t' = sigma_t A_t, B4' = B2' + B3', B5' = B1' + B4', B6' = the scaled
 * entry rounded to FP64) and written column-major, plane t at
 * planes + t*rows*cols with leading dimension rows.  exps receives e (int32)
 * with max |hi| of the row/column in [2^(e-1), 2^e), 0 for an all-zero one.
 * kc has the meaning of dd_gemm_opts.kc, with the inner size k = cols
 * (side 0) or rows (side 1).  exps and planes are device pointers.
 */
dd_status dd_cascade_split(int32_t side, int32_t trans, int64_t rows, int64_t cols,
                           const double* X_hi, const double* X_lo, int64_t ldx,
                           int32_t kc, int32_t* exps, double* planes,
                           hipStream_t stream);

/*
 * The slice split of the slices variants on its own, for inspection and
 * testing.  `side` = 0: X is op(A), rows x cols = m x k, one exponent per
 * row; `side` = 1: X is op(B), rows x cols = k x n, one per column.  exps
 * receives e (int32) with max |fl(hi + lo)| of the row/column in
 * [2^(e-1), 2^e) (0 for an all-zero or non-finite one); `out` receives the
 * slices as 16-bit values: BF16 (fmt = 0) or FP16 (fmt = 1) patterns, or
 * INT8 integers sign-extended to 16 bits (fmt = 2), slice t at
 * out + t*rows*cols, column-major with leading dimension rows.  slices /
 * slice_bits as in dd_gemm_opts (0 = the format's default).  exps and out
 * are device pointers.
 */
dd_status dd_slices_split(int32_t side, int32_t trans, int64_t rows, int64_t cols,
                          const double* X_hi, const double* X_lo, int64_t ldx,
                          int32_t fmt, int32_t slices, int32_t slice_bits,
                          int32_t* exps, uint16_t* out, hipStream_t stream);

/*
 * FP64x2 dot product: result[0] + result[1] = sum_i x_i y_i, computed in
 * double-double arithmetic (each product by TwoProd with FMA plus the two
 * cross terms, sums by the accurate FP64x2 addition, a fixed reduction tree:
 * the result does not change between runs).  x and y are FP64x2 vectors of
 * n entries with strides incx, incy >= 1 (elements); `result` is device
 * memory for two doubles, written (not accumulated).  Uses the library's
 * cached per-stream scratch of 16 KiB.  n = 0 gives 0.
 */
dd_status dd_dot(int64_t n, const double* x_hi, const double* x_lo, int64_t incx,
                 const double* y_hi, const double* y_lo, int64_t incy,
                 double* result, hipStream_t stream);

/*
 * y := alpha * x in FP64x2, entry by entry with the double-double product
 * (TwoProd of the high words by FMA plus the two cross products, one
 * renormalisation).  alpha is a DEVICE pointer to two doubles, alpha[0] +
 * alpha[1], read when the kernel runs, so a scale the device has just
 * computed (the seed of a backward pass) needs no host synchronisation.
 * y may equal x (same pointers and stride); otherwise they must not overlap.
 */
dd_status dd_scal(int64_t n, const double* alpha,
                  const double* x_hi, const double* x_lo, int64_t incx,
                  double* y_hi, double* y_lo, int64_t incy, hipStream_t stream);

/*
 * z := x + y in FP64x2, entry by entry with the accurate double-double
 * addition (TwoSum of the high words and of the low words, two
 * renormalisations; relative error below 3 2^-106, Sec. 3.1 arithmetic of
 * FP64x2 numbers).  Used to accumulate the gradients of an FP64x2 tensor
 * that feeds several products.  z may equal x or y (same pointers and
 * stride); otherwise it must overlap neither.  Strides >= 1, in elements.
 */
dd_status dd_add(int64_t n, const double* x_hi, const double* x_lo, int64_t incx,
                 const double* y_hi, const double* y_lo, int64_t incy,
                 double* z_hi, double* z_lo, int64_t incz, hipStream_t stream);

/*
 * Phase timing (Fig. breakdown of Sec. 5.1 measures the same split).  While
 * enabled, every cascaded GEMM records HIP events on its own stream before
 * phase one (exponents and split), between the phases, and after the fused
 * product kernel (phases two and three).  dd_phase_times waits for those
 * events and returns the milliseconds summed since the last call (or since
 * enabling) and the number of GEMMs they cover, then starts a new sum.  Any
 * pointer may be NULL.  Enabling costs two event records per call; it is
 * meant for measurement, not production.  Not thread safe against
 * concurrent GEMM calls.
 */
dd_status dd_profile_enable(int32_t enable);
dd_status dd_phase_times(double* split_ms, double* product_ms, int64_t* calls);

/* Short English description of a status code (static storage). */
const char* dd_status_string(dd_status status);

/* Library version, major*10000 + minor*100 + patch. */
int32_t dd_version(void);

/* ------------------------------------------------------------------------
 * FP64x3 (triple-word) GEMM: C := op(A) op(B) + C with every entry the sum
 * of three doubles (x0 + x1 + x2, about 159 bits when |x1| <= ulp(x0) and
 * |x2| <= ulp(x1)), by the cascade with six FP64 digits (the case Sec. 6.2
 * names).  Per rank-kc block the widths c0..c4 are the largest for which
 * bins 0..4 are exact (about 156 bits in all at kc = 256), Sigma / T come
 * from the largest |x0| per row / column, and the 21 products run on the
 * FP64 matrix cores in one fused kernel of this library: bins 0..4 exact,
 * a tail bin over the suffix sums of B's planes, the six bins turned into a
 * triple word per block by a fixed error-free summation and accumulated
 * the same way, C added last.  Planes x0, x1, x2 of each operand share one
 * leading dimension; all device pointers, column-major.  kc: 0 = 256, else
 * a multiple of 4 in [4, 4096].  Status and quick returns as for
 * dd_gemm_ex; argument i invalid gives -i.  The workspace holds the row and
 * column maxima and 48 (mpad + npad) kpad bytes of packed digit planes
 * (mpad, npad rounded up to 64, kpad to 8), plus 4352 bytes per 16 rows and
 * columns; workspace NULL with ws_bytes 0 uses the library's cached one
 * (which may allocate, so not under graph capture).
 * ------------------------------------------------------------------------ */
size_t td_gemm_workspace_size(int32_t transa, int32_t transb, int64_t m, int64_t n, int64_t k, int32_t kc);

dd_status td_gemm_ex(int32_t transa, int32_t transb, int64_t m, int64_t n, int64_t k,
                     const double* A0, const double* A1, const double* A2, int64_t lda,
                     const double* B0, const double* B1, const double* B2, int64_t ldb,
                     double* C0, double* C1, double* C2, int64_t ldc,
                     void* workspace, size_t ws_bytes, int32_t kc, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* DDGEMM_H */
