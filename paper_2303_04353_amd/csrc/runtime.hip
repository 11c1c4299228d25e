// Host runtime and C ABI of the library: argument checks, workspace, and the
// launch sequence of the cascade (phase one: Sigma/T and split; phases two
// and three: the fused product/combine kernel) or of the plain double-double
// kernel.  See include/ddgemm.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/ddgemm.h"
#include "kernels.hpp"
#include "layout.hpp"

namespace {

using ddk::CascadeLayout;

constexpr int64_t kTileM = 64, kTileN = 64;
constexpr int32_t kDefaultKc = 256;

// ------------------------------------------------------------ device checks
std::mutex g_mu;
std::map<int, int> g_arch_ok;  // device -> 1 gfx950, 0 other

dd_status check_device(int* dev_out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return DD_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_arch_ok.find(dev);
  if (it == g_arch_ok.end()) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return DD_ERR_HIP;
    int ok = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 0;
    it = g_arch_ok.emplace(dev, ok).first;
  }
  if (dev_out) *dev_out = dev;
  return it->second ? DD_OK : DD_ERR_UNSUPPORTED;
}

// ------------------------------------------------------ cached workspaces
struct WsKey { int dev; hipStream_t stream; bool operator<(const WsKey& o) const {
  return dev != o.dev ? dev < o.dev : (uintptr_t)stream < (uintptr_t)o.stream; } };
// `captured`: the buffer was handed to a call made while its stream was
// being captured into a HIP graph.  Replays of that graph read it at any
// later time, so it is never freed: when the cache grows past it, it is
// kept (g_ws_kept) until the process ends.
struct WsBuf { void* ptr = nullptr; size_t bytes = 0; bool captured = false; };
std::map<WsKey, WsBuf> g_ws;
std::vector<void*> g_ws_kept;

dd_status cached_workspace(int dev, hipStream_t stream, size_t bytes, void** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) != hipSuccess) {
    (void)hipGetLastError();
    return DD_ERR_HIP;
  }
  const bool capturing = cs != hipStreamCaptureStatusNone;
  WsBuf& b = g_ws[WsKey{dev, stream}];
  if (b.bytes < bytes) {
    // a stream being captured can neither wait nor take a new allocation:
    // the caller warms the cache up before capturing, or passes a workspace
    if (capturing) return DD_ERR_WORKSPACE;
    if (b.ptr) {
      if (b.captured) {
        g_ws_kept.push_back(b.ptr);
      } else {
        // earlier work on this stream may still use the old buffer
        if (hipStreamSynchronize(stream) != hipSuccess) return DD_ERR_HIP;
        (void)hipFree(b.ptr);
      }
      b.ptr = nullptr;
      b.bytes = 0;
      b.captured = false;
    }
    size_t want = bytes + bytes / 8;
    if (hipMalloc(&b.ptr, want) != hipSuccess) {
      (void)hipGetLastError();
      b.ptr = nullptr;
      return DD_ERR_WORKSPACE;
    }
    b.bytes = want;
  }
  if (capturing) b.captured = true;
  *out = b.ptr;
  return DD_OK;
}

}  // namespace

// ------------------------------------------------------ no-alloc scratch
// Workspace of dd_gemm_noalloc: a fixed array in this file's code object.
// Every device the library runs on holds its own copy, at its own address,
// until the process ends.  In host code `scratch` only names the symbol; its
// device address comes from hipGetSymbolAddress (scratch_address below).
static __device__ __align__(256) unsigned char scratch[DD_NOALLOC_SCRATCH_BYTES];

namespace {

std::map<int, char*> g_scratch;  // device -> address of its copy of `scratch`

// Called with `dev` current (the device the call runs on).
dd_status scratch_address(int dev, char** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_scratch.find(dev);
  if (it == g_scratch.end()) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
      (void)hipGetLastError();
      return DD_ERR_HIP;
    }
    it = g_scratch.emplace(dev, (char*)ptr).first;
  }
  *out = it->second;
  return DD_OK;
}

// ------------------------------------------------------------ phase timing
struct PhaseEvents { hipEvent_t e0, e1, e2; };
bool g_prof = false;
std::vector<PhaseEvents> g_prof_events;

// Events around the two phases of one call while timing is enabled: `split`
// marks the end of phase one, `done` the end of the product and keeps the
// events for dd_phase_times.  A call that returns without `done` (an error)
// destroys them.
class PhaseTimer {
 public:
  PhaseTimer(hipStream_t s, bool allowed) : s_(s) {
    if (!allowed) return;
    {
      std::lock_guard<std::mutex> lk(g_mu);
      if (!g_prof) return;
    }
    hipEvent_t e[3] = {nullptr, nullptr, nullptr};
    for (hipEvent_t& x : e)
      if (hipEventCreate(&x) != hipSuccess) {
        (void)hipGetLastError();
        for (hipEvent_t y : e)
          if (y) (void)hipEventDestroy(y);
        return;
      }
    pe_ = PhaseEvents{e[0], e[1], e[2]};
    (void)hipEventRecord(pe_.e0, s_);
  }
  PhaseTimer(const PhaseTimer&) = delete;
  PhaseTimer& operator=(const PhaseTimer&) = delete;
  ~PhaseTimer() {
    if (!pe_.e0) return;
    (void)hipEventDestroy(pe_.e0);
    (void)hipEventDestroy(pe_.e1);
    (void)hipEventDestroy(pe_.e2);
  }
  void split() {
    if (pe_.e1) (void)hipEventRecord(pe_.e1, s_);
  }
  void done() {
    if (!pe_.e2) return;
    (void)hipEventRecord(pe_.e2, s_);
    std::lock_guard<std::mutex> lk(g_mu);
    g_prof_events.push_back(pe_);
    pe_ = PhaseEvents{nullptr, nullptr, nullptr};
  }

 private:
  hipStream_t s_;
  PhaseEvents pe_{nullptr, nullptr, nullptr};
};

// ------------------------------------------------------------ arguments
struct Problem {
  int transa, transb;
  int64_t m, n, k;
  const double *Ahi, *Alo; int64_t lda;
  const double *Bhi, *Blo; int64_t ldb;
  double *Chi, *Clo; int64_t ldc;
};

// Which logical argument failed; mapped to the position in each prototype.
enum Arg { ARG_OK = 0, ARG_TRANSA, ARG_TRANSB, ARG_M, ARG_N, ARG_K, ARG_AHI, ARG_ALO, ARG_LDA,
           ARG_BHI, ARG_BLO, ARG_LDB, ARG_CHI, ARG_CLO, ARG_LDC, ARG_OPTS };

bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
  uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
  return a0 < b0 + bbytes && b0 < a0 + abytes;
}

size_t span_bytes(int64_t rows, int64_t cols, int64_t ld) {
  if (rows <= 0 || cols <= 0) return 0;
  return (size_t)((cols - 1) * ld + rows) * sizeof(double);
}

// The bytes a rows x cols matrix with leading dimension ld (>= rows) spans
// fit in an int64 (false for leading dimensions no allocation can have).
bool span_fits(int64_t rows, int64_t cols, int64_t ld) {
  if (rows <= 0 || cols <= 1) return true;
  const int64_t lim = INT64_MAX / (int64_t)sizeof(double);
  return ld <= (lim - rows) / (cols - 1);
}

Arg validate(const Problem& p) {
  if (p.transa != DD_OP_N && p.transa != DD_OP_T) return ARG_TRANSA;
  if (p.transb != DD_OP_N && p.transb != DD_OP_T) return ARG_TRANSB;
  if (p.m < 0) return ARG_M;
  if (p.n < 0) return ARG_N;
  if (p.k < 0) return ARG_K;
  const int64_t arows = p.transa ? p.k : p.m, acols = p.transa ? p.m : p.k;
  const int64_t brows = p.transb ? p.n : p.k, bcols = p.transb ? p.k : p.n;
  if (p.lda < (arows > 1 ? arows : 1)) return ARG_LDA;
  if (p.ldb < (brows > 1 ? brows : 1)) return ARG_LDB;
  if (p.ldc < (p.m > 1 ? p.m : 1)) return ARG_LDC;
  if (!span_fits(arows, acols, p.lda)) return ARG_LDA;
  if (!span_fits(brows, bcols, p.ldb)) return ARG_LDB;
  if (!span_fits(p.m, p.n, p.ldc)) return ARG_LDC;
  if (p.m == 0 || p.n == 0) return ARG_OK;
  if (!p.Chi) return ARG_CHI;
  if (!p.Clo) return ARG_CLO;
  if (p.k == 0) return ARG_OK;
  if (!p.Ahi) return ARG_AHI;
  if (!p.Alo) return ARG_ALO;
  if (!p.Bhi) return ARG_BHI;
  if (!p.Blo) return ARG_BLO;
  const size_t cb = span_bytes(p.m, p.n, p.ldc);
  const size_t ab = span_bytes(arows, acols, p.lda), bb = span_bytes(brows, bcols, p.ldb);
  if (overlaps(p.Chi, cb, p.Clo, cb)) return ARG_CLO;
  for (const double* c : {(const double*)p.Chi, (const double*)p.Clo}) {
    const Arg which = c == p.Chi ? ARG_CHI : ARG_CLO;
    if (overlaps(c, cb, p.Ahi, ab) || overlaps(c, cb, p.Alo, ab) ||
        overlaps(c, cb, p.Bhi, bb) || overlaps(c, cb, p.Blo, bb)) return which;
  }
  return ARG_OK;
}

// Strides of op(A)(i, p) and op(B)(p, j) in elements.
void strides(const Problem& p, int64_t& a_si, int64_t& a_sp, int64_t& b_sp, int64_t& b_sj) {
  if (p.transa) { a_si = p.lda; a_sp = 1; } else { a_si = 1; a_sp = p.lda; }
  if (p.transb) { b_sp = p.ldb; b_sj = 1; } else { b_sp = 1; b_sj = p.ldb; }
}

bool valid_kc(int32_t kc) { return kc >= 4 && kc <= 4096 && kc % 4 == 0; }

dd_status hip_status(hipError_t e) {
  if (e == hipSuccess) return DD_OK;
  if (e == hipErrorOutOfMemory) return DD_ERR_WORKSPACE;
  return DD_ERR_HIP;
}

#define DD_TRY(expr) do { dd_status st_ = hip_status(expr); if (st_ != DD_OK) return st_; } while (0)

// Phase one into the workspace described by L.
dd_status run_split(const Problem& p, const CascadeLayout& L, char* ws, hipStream_t s) {
  int64_t a_si, a_sp, b_sp, b_sj;
  strides(p, a_si, a_sp, b_sp, b_sj);
  uint64_t* amax = (uint64_t*)(ws + L.off_amax);
  uint64_t* bmax = (uint64_t*)(ws + L.off_bmax);
  DD_TRY(ddk::launch_fill_u64(amax, L.mpad * L.npanel, 0, s));
  DD_TRY(ddk::launch_fill_u64(bmax, L.npad * L.npanel, 0, s));
  // diagonal balancing: column maxima of op(A) and row maxima of op(B) give
  // g[p]; every entry is then seen as A(i, p) 2^g[p], B(p, j) 2^-g[p]
  const int32_t* gexp = nullptr;
  if (L.balance) {
    uint64_t* acol = (uint64_t*)(ws + L.off_acol);
    uint64_t* brow = (uint64_t*)(ws + L.off_brow);
    DD_TRY(ddk::launch_fill_u64(acol, L.kpad, 0, s));
    DD_TRY(ddk::launch_fill_u64(brow, L.kpad, 0, s));
    DD_TRY(ddk::launch_max_abs_bits(p.Ahi, p.k, p.m, a_sp, a_si, acol, s));
    DD_TRY(ddk::launch_max_abs_bits(p.Bhi, p.k, p.n, b_sp, b_sj, brow, s));
    DD_TRY(ddk::launch_balance_exps(acol, brow, p.k, L.kpad, (int32_t*)(ws + L.off_gexp), s));
    gexp = (const int32_t*)(ws + L.off_gexp);
  }
  // rows of op(A): outer i, reduced p;  columns of op(B): outer j, reduced p;
  // with per-panel Sigma and T one maximum per run of 4 kcq inner indices
  const int64_t plen = L.npanel > 1 ? 4 * (int64_t)L.kcq : 0;
  DD_TRY(ddk::launch_max_abs_bits(p.Ahi, p.m, p.k, a_si, a_sp, amax, s, nullptr, plen, L.mpad, gexp, 1));
  DD_TRY(ddk::launch_max_abs_bits(p.Bhi, p.n, p.k, b_sj, b_sp, bmax, s, nullptr, plen, L.npad, gexp, -1));
  DD_TRY(ddk::launch_pack_a(p.Ahi, p.Alo, a_si, a_sp, L, amax, (double*)(ws + L.off_apack), s, gexp));
  DD_TRY(ddk::launch_pack_b(p.Bhi, p.Blo, b_sp, b_sj, L, bmax, (double*)(ws + L.off_bpack), s, gexp));
  if (L.npanel > 1) {
    DD_TRY(ddk::launch_exps(amax, L.mpad * L.npanel, (int32_t*)(ws + L.off_aexp), s));
    DD_TRY(ddk::launch_exps(bmax, L.npad * L.npanel, (int32_t*)(ws + L.off_bexp), s));
  }
  return DD_OK;
}

// Options after validation.
struct Opts {
  int32_t algo = DD_ALGO_CASCADE_F64;
  int32_t kc = kDefaultKc;
  int32_t S = 0, w = 0;   // slices variants
  uint32_t* flags = nullptr;   // cascade: cancellation bitmap (may be null)
  bool panels = false;         // cascade: Sigma and T per rank-kc panel
  bool balance = false;        // cascade: diagonal balancing of the inner dimension
  int32_t tile = 0;            // cascade: output tile shape, 0 = the library's choice
  bool use_tuned = false;      // cascade: take the shape recorded by dd_tune, if any
  int32_t scaling = 0;
  bool slices() const {
    return algo == DD_ALGO_SLICES_BF16 || algo == DD_ALGO_SLICES_F16 || algo == DD_ALGO_SLICES_I8;
  }
  int fmt() const {
    return algo == DD_ALGO_SLICES_I8 ? ddk::kSliceI8 : (algo == DD_ALGO_SLICES_F16 ? ddk::kSliceF16 : ddk::kSliceBF16);
  }
};

// Slice count and width with the format's defaults filled in (BF16/FP16:
// 14 slices of 8 bits; INT8: 16 slices of 7 bits); false if unusable.
bool slice_params(int fmt, int32_t slices, int32_t bits, int32_t* S, int32_t* w) {
  *S = slices ? slices : (fmt == ddk::kSliceI8 ? 16 : 14);
  *w = bits ? bits : (fmt == ddk::kSliceI8 ? 7 : 8);
  return ddk::slices_params_ok(*w, *S, fmt);
}

ddk::SlicesLayout slices_layout(const Problem& p, const Opts& o) {
  return ddk::make_slices_layout(p.m, p.n, p.k, o.S, o.w, o.fmt());
}

// Phase one of the slices variant: exponents from max |fl(hi + lo)|, then the split.
dd_status run_slices_split(const Problem& p, const ddk::SlicesLayout& L, char* ws, hipStream_t s) {
  int64_t a_si, a_sp, b_sp, b_sj;
  strides(p, a_si, a_sp, b_sp, b_sj);
  uint64_t* amax = (uint64_t*)(ws + L.off_amax);
  uint64_t* bmax = (uint64_t*)(ws + L.off_bmax);
  DD_TRY(ddk::launch_fill_u64(amax, L.mpad, 0, s));
  DD_TRY(ddk::launch_fill_u64(bmax, L.npad, 0, s));
  DD_TRY(ddk::launch_max_abs_bits(p.Ahi, p.m, p.k, a_si, a_sp, amax, s, p.Alo));
  DD_TRY(ddk::launch_max_abs_bits(p.Bhi, p.n, p.k, b_sj, b_sp, bmax, s, p.Blo));
  DD_TRY(ddk::launch_slices_split(p.Ahi, p.Alo, a_si, a_sp, p.m, p.k, L.mpad, L, amax, ws + L.off_apack, s));
  DD_TRY(ddk::launch_slices_split(p.Bhi, p.Blo, b_sj, b_sp, p.n, p.k, L.npad, L, bmax, ws + L.off_bpack, s));
  return DD_OK;
}

// The product passes, one inner-dimension chunk after another.
dd_status run_slices_product(const Problem& p, const ddk::SlicesLayout& L, char* ws, hipStream_t s) {
  for (int64_t q0 = 0; q0 < L.Q; q0 += L.chunk_q) {
    const int64_t q1 = q0 + L.chunk_q < L.Q ? q0 + L.chunk_q : L.Q;
    DD_TRY(ddk::launch_slices_product(L, ws + L.off_apack, ws + L.off_bpack, (const uint64_t*)(ws + L.off_amax),
                                      (const uint64_t*)(ws + L.off_bmax), (double*)(ws + L.off_planes), p.Chi,
                                      p.Clo, p.ldc, q0, q1, s));
  }
  return DD_OK;
}

// ------------------------------------------------------ tuned tile shapes
// Output tile shapes recorded by dd_tune, per (m, n, k, kc, scaling); kept
// in memory and, when DDGEMM_TUNE_CACHE names a file, appended to it as
// lines "s <m> <n> <k> <kc> <scaling> <shape>" (read once, at first use).
struct TuneKey {
  int64_t m, n, k;
  int32_t kc, scaling;
  bool operator<(const TuneKey& o) const {
    if (m != o.m) return m < o.m;
    if (n != o.n) return n < o.n;
    if (k != o.k) return k < o.k;
    if (kc != o.kc) return kc < o.kc;
    return scaling < o.scaling;
  }
};
std::map<TuneKey, int32_t> g_tuned;
bool g_tuned_loaded = false;

void load_tuned_locked() {
  if (g_tuned_loaded) return;
  g_tuned_loaded = true;
  const char* path = std::getenv("DDGEMM_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[256];
  while (std::fgets(line, sizeof(line), f)) {
    long long m, n, k;
    int kc, sc, sh;
    if (std::sscanf(line, "s %lld %lld %lld %d %d %d", &m, &n, &k, &kc, &sc, &sh) == 6 &&
        sh >= ddk::kTile64x64 && sh <= ddk::kTile64x32)
      g_tuned[TuneKey{m, n, k, kc, sc}] = sh;
  }
  std::fclose(f);
}

void record_tuned(const TuneKey& key, int32_t shape) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_tuned_locked();
  g_tuned[key] = shape;
  const char* path = std::getenv("DDGEMM_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "s %lld %lld %lld %d %d %d\n", (long long)key.m, (long long)key.n, (long long)key.k, key.kc,
               key.scaling, shape);
  std::fclose(f);
}

// The output tile shape of a cascade: the one asked for, else the tuned one
// (with use_tuned), else 64 x 64.
int32_t tile_shape(const Problem& p, const Opts& o) {
  if (o.tile != 0) return o.tile;
  if (o.use_tuned) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_tuned_locked();
    auto it = g_tuned.find(TuneKey{p.m, p.n, p.k, o.kc, o.scaling});
    if (it != g_tuned.end()) return it->second;
  }
  return ddk::kTile64x64;
}

// One GEMM after validation.  With `fixed` the workspace is the caller's (or
// the scratch array) and the call creates nothing: no phase-timing events
// either.
dd_status run(const Problem& p, const Opts& o, void* workspace, size_t ws_bytes, bool internal_ws,
              hipStream_t s, bool fixed = false) {
  const int32_t algo = o.algo, kc = o.kc;
  if (p.m == 0 || p.n == 0) return DD_OK;   // quick return: no device needed
  if (p.k == 0) {
    // C stays as it is; a cancellation bitmap is still cleared (no entry is at risk)
    if (!o.flags) return DD_OK;
    int dev = 0;
    const dd_status st = check_device(&dev);
    if (st != DD_OK) return st;
    return hip_status(ddk::launch_fill_u32(o.flags, (p.m * p.n + 31) / 32, 0u, s));
  }
  int dev = 0;
  dd_status st = check_device(&dev);
  if (st != DD_OK) return st;
  if (algo == DD_ALGO_DD_VALU) {
    int64_t a_si, a_sp, b_sp, b_sj;
    strides(p, a_si, a_sp, b_sp, b_sj);
    return hip_status(ddk::launch_dd_valu(p.m, p.n, p.k, p.Ahi, p.Alo, a_si, a_sp, p.Bhi, p.Blo,
                                          b_sp, b_sj, p.Chi, p.Clo, p.ldc, s));
  }
  if (o.slices()) {
    const ddk::SlicesLayout L = slices_layout(p, o);
    char* ws = (char*)workspace;
    if (internal_ws) {
      void* w = nullptr;
      st = cached_workspace(dev, s, L.bytes, &w);
      if (st != DD_OK) return st;
      ws = (char*)w;
    } else if (ws_bytes < L.bytes || ((uintptr_t)ws & 255u) != 0) {
      return DD_ERR_WORKSPACE;
    }
    PhaseTimer timer(s, !fixed);
    st = run_slices_split(p, L, ws, s);
    if (st != DD_OK) return st;
    timer.split();
    st = run_slices_product(p, L, ws, s);
    if (st == DD_OK) timer.done();
    return st;
  }
  if (algo == DD_ALGO_CASCADE_ON_LOAD) {
    // the row and column maxima, then the product kernel that splits as it stages
    const CascadeLayout L = ddk::make_layout(p.m, p.n, p.k, kc, kTileM, kTileN);
    const size_t need = L.off_apack;   // the maxima come first in the layout
    char* ws = (char*)workspace;
    if (internal_ws) {
      void* w = nullptr;
      st = cached_workspace(dev, s, need, &w);
      if (st != DD_OK) return st;
      ws = (char*)w;
    } else if (ws_bytes < need || ((uintptr_t)ws & 255u) != 0) {
      return DD_ERR_WORKSPACE;
    }
    int64_t a_si, a_sp, b_sp, b_sj;
    strides(p, a_si, a_sp, b_sp, b_sj);
    uint64_t* amax = (uint64_t*)(ws + L.off_amax);
    uint64_t* bmax = (uint64_t*)(ws + L.off_bmax);
    PhaseTimer timer(s, !fixed);
    DD_TRY(ddk::launch_fill_u64(amax, L.mpad, 0, s));
    DD_TRY(ddk::launch_fill_u64(bmax, L.npad, 0, s));
    DD_TRY(ddk::launch_max_abs_bits(p.Ahi, p.m, p.k, a_si, a_sp, amax, s));
    DD_TRY(ddk::launch_max_abs_bits(p.Bhi, p.n, p.k, b_sj, b_sp, bmax, s));
    timer.split();
    if (o.flags) DD_TRY(ddk::launch_fill_u32(o.flags, (p.m * p.n + 31) / 32, 0u, s));
    st = hip_status(ddk::launch_cascade_onload(L, p.Ahi, p.Alo, a_si, a_sp, p.Bhi, p.Blo, b_sp, b_sj, amax, bmax,
                                               p.Chi, p.Clo, p.ldc, o.flags, s));
    if (st == DD_OK) timer.done();
    return st;
  }
  const bool simple = algo == DD_ALGO_SIMPLE_UNFUSED;
  const CascadeLayout L = ddk::make_layout(p.m, p.n, p.k, kc, kTileM, kTileN, o.panels, o.balance, simple);
  char* ws = (char*)workspace;
  if (internal_ws) {
    void* w = nullptr;
    st = cached_workspace(dev, s, L.bytes, &w);
    if (st != DD_OK) return st;
    ws = (char*)w;
  } else if (ws_bytes < L.bytes || ((uintptr_t)ws & 255u) != 0) {
    return DD_ERR_WORKSPACE;
  }
  PhaseTimer timer(s, !fixed);
  st = run_split(p, L, ws, s);
  if (st != DD_OK) return st;
  timer.split();
  if (simple) {
    st = hip_status(ddk::run_simple_products(L, ws, (const uint64_t*)(ws + L.off_amax),
                                             (const uint64_t*)(ws + L.off_bmax), p.Chi, p.Clo, p.ldc, s));
    if (st == DD_OK) timer.done();
    return st;
  }
  if (o.flags) {
    st = hip_status(ddk::launch_fill_u32(o.flags, (p.m * p.n + 31) / 32, 0u, s));
    if (st != DD_OK) return st;
  }
  st = hip_status(ddk::launch_cascade(L, (const double*)(ws + L.off_apack),
                                      (const double*)(ws + L.off_bpack),
                                      (const uint64_t*)(ws + L.off_amax),
                                      (const uint64_t*)(ws + L.off_bmax), p.Chi, p.Clo, p.ldc, o.flags, s,
                                      (const int32_t*)(ws + L.off_aexp), (const int32_t*)(ws + L.off_bexp),
                                      tile_shape(p, o)));
  if (st == DD_OK) timer.done();
  return st;
}

}  // namespace

extern "C" {

dd_status dd_gemm(int64_t m, int64_t n, int64_t k,
                  const double* A_hi, const double* A_lo, int64_t lda,
                  const double* B_hi, const double* B_lo, int64_t ldb,
                  double* C_hi, double* C_lo, int64_t ldc, hipStream_t stream) {
  static const int pos[] = {0, 0, 0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 0};
  Problem p{DD_OP_N, DD_OP_N, m, n, k, A_hi, A_lo, lda, B_hi, B_lo, ldb, C_hi, C_lo, ldc};
  Arg a = validate(p);
  if (a != ARG_OK) return -pos[a];
  return run(p, Opts{}, nullptr, 0, true, stream);
}

static bool read_opts(const dd_gemm_opts* o, Opts* out) {
  *out = Opts{};
  if (!o) return true;
  if (o->algo < DD_ALGO_CASCADE_F64 || o->algo > DD_ALGO_CASCADE_ON_LOAD) return false;
  if (o->tile < 0 || o->tile > DD_TILE_64x32) return false;
  if (o->tile != 0 && o->algo != DD_ALGO_CASCADE_F64 &&
      !(o->algo == DD_ALGO_CASCADE_ON_LOAD && o->tile == DD_TILE_64x64)) return false;
  if (o->use_tuned != 0 && o->use_tuned != 1) return false;
  if (o->use_tuned && o->algo != DD_ALGO_CASCADE_F64) return false;
  if (o->scaling < 0 || o->scaling > (DD_SCALING_PANEL | DD_SCALING_BALANCE)) return false;
  out->algo = o->algo;
  const bool fused = o->algo == DD_ALGO_CASCADE_F64 || o->algo == DD_ALGO_CASCADE_ON_LOAD;
  if (o->flags_out && !fused) return false;
  if (o->scaling != DD_SCALING_GLOBAL && o->algo != DD_ALGO_CASCADE_F64) return false;
  out->flags = o->flags_out;
  out->tile = o->tile;
  out->use_tuned = o->use_tuned != 0;
  out->scaling = o->scaling;
  out->panels = (o->scaling & DD_SCALING_PANEL) != 0;
  out->balance = (o->scaling & DD_SCALING_BALANCE) != 0;
  if (out->slices()) {
    if (o->kc != 0) return false;
    return slice_params(out->fmt(), o->slices, o->slice_bits, &out->S, &out->w);
  }
  if (o->slices != 0 || o->slice_bits != 0) return false;
  if (o->kc != 0 && !valid_kc(o->kc)) return false;
  if (o->kc != 0) out->kc = o->kc;
  return true;
}

// Workspace bytes of a problem with validated options (0 when nothing runs).
static size_t workspace_bytes(int64_t m, int64_t n, int64_t k, const Opts& o) {
  if (m <= 0 || n <= 0 || k <= 0 || o.algo == DD_ALGO_DD_VALU) return 0;
  if (o.slices()) return ddk::make_slices_layout(m, n, k, o.S, o.w, o.fmt()).bytes;
  if (o.algo == DD_ALGO_CASCADE_ON_LOAD) return ddk::make_layout(m, n, k, o.kc, kTileM, kTileN).off_apack;
  return ddk::make_layout(m, n, k, o.kc, kTileM, kTileN, o.panels, o.balance,
                         o.algo == DD_ALGO_SIMPLE_UNFUSED).bytes;
}

size_t dd_gemm_workspace_size(int32_t transa, int32_t transb, int64_t m, int64_t n, int64_t k,
                              const dd_gemm_opts* opts) {
  Opts o;
  if (!read_opts(opts, &o)) return 0;
  if ((transa != DD_OP_N && transa != DD_OP_T) || (transb != DD_OP_N && transb != DD_OP_T)) return 0;
  return workspace_bytes(m, n, k, o);
}

dd_status dd_gemm_ex(int32_t transa, int32_t transb, int64_t m, int64_t n, int64_t k,
                     const double* A_hi, const double* A_lo, int64_t lda,
                     const double* B_hi, const double* B_lo, int64_t ldb,
                     double* C_hi, double* C_lo, int64_t ldc,
                     void* workspace, size_t ws_bytes, const dd_gemm_opts* opts,
                     hipStream_t stream) {
  static const int pos[] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 17};
  Problem p{(int)transa, (int)transb, m, n, k, A_hi, A_lo, lda, B_hi, B_lo, ldb, C_hi, C_lo, ldc};
  Arg a = validate(p);
  if (a != ARG_OK) return -pos[a];
  Opts o;
  if (!read_opts(opts, &o)) return -17;
  const bool internal = workspace == nullptr && ws_bytes == 0;
  if (!internal && workspace == nullptr) return -15;
  return run(p, o, workspace, ws_bytes, internal, stream);
}

dd_status dd_gemm_noalloc(int32_t transa, int32_t transb, int64_t m, int64_t n, int64_t k,
                          const double* A_hi, const double* A_lo, int64_t lda,
                          const double* B_hi, const double* B_lo, int64_t ldb,
                          double* C_hi, double* C_lo, int64_t ldc,
                          const dd_gemm_opts* opts, hipStream_t stream) {
  static const int pos[] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15};
  Problem p{(int)transa, (int)transb, m, n, k, A_hi, A_lo, lda, B_hi, B_lo, ldb, C_hi, C_lo, ldc};
  Arg a = validate(p);
  if (a != ARG_OK) return -pos[a];
  Opts o;
  if (!read_opts(opts, &o)) return -15;
  // the unfused form runs the vendor BLAS, whose handle and calls may allocate
  if (o.algo == DD_ALGO_SIMPLE_UNFUSED) return -15;
  if (m == 0 || n == 0 || k == 0) return DD_OK;
  int dev = 0;
  dd_status st = check_device(&dev);
  if (st != DD_OK) return st;
  if (workspace_bytes(m, n, k, o) > (size_t)DD_NOALLOC_SCRATCH_BYTES) return DD_ERR_WORKSPACE;
  char* ws = nullptr;
  st = scratch_address(dev, &ws);
  if (st != DD_OK) return st;
  return run(p, o, ws, (size_t)DD_NOALLOC_SCRATCH_BYTES, false, stream, true);
}

dd_status dd_tune(int32_t count, const int64_t* m, const int64_t* n, const int64_t* k,
                  const dd_gemm_opts* opts, int32_t repeats, int32_t* shapes_out, hipStream_t stream) {
  if (count < 0) return -1;
  if (count > 0 && !m) return -2;
  if (count > 0 && !n) return -3;
  if (count > 0 && !k) return -4;
  Opts o;
  if (!read_opts(opts, &o) || o.algo != DD_ALGO_CASCADE_F64 || o.tile != 0 || o.flags) return -5;
  if (repeats < 1) return -6;
  for (int32_t i = 0; i < count; ++i)
    if (m[i] < 0 || n[i] < 0 || k[i] < 0) return -2;
  int dev = 0;
  dd_status st = check_device(&dev);
  if (st != DD_OK) return st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipGetLastError();
    if (e0) (void)hipEventDestroy(e0);
    return DD_ERR_HIP;
  }
  for (int32_t i = 0; i < count && st == DD_OK; ++i) {
    if (shapes_out) shapes_out[i] = 0;
    if (m[i] == 0 || n[i] == 0 || k[i] == 0) continue;
    // operands of the shape (zeros: the kernels' time does not depend on the values)
    const size_t a = sizeof(double) * (size_t)m[i] * (size_t)k[i], b = sizeof(double) * (size_t)k[i] * (size_t)n[i];
    const size_t c = sizeof(double) * (size_t)m[i] * (size_t)n[i];
    const CascadeLayout L = ddk::make_layout(m[i], n[i], k[i], o.kc, kTileM, kTileN, o.panels, o.balance);
    char* buf = nullptr;
    const size_t wso = 2 * (a + b + c) + 1024, total = wso + L.bytes + 256;
    if (hipMalloc(&buf, total) != hipSuccess) {
      (void)hipGetLastError();
      st = DD_ERR_WORKSPACE;
      break;
    }
    if (hipMemsetAsync(buf, 0, wso, stream) != hipSuccess) st = DD_ERR_HIP;
    Problem p{DD_OP_N, DD_OP_N, m[i], n[i], k[i],
              (const double*)buf, (const double*)(buf + a), m[i],
              (const double*)(buf + 2 * a), (const double*)(buf + 2 * a + b), k[i],
              (double*)(buf + 2 * (a + b)), (double*)(buf + 2 * (a + b) + c), m[i]};
    char* ws = buf + ddk::round_up((int64_t)wso, 256);
    float best = 1e30f;
    int32_t best_shape = ddk::kTile64x64;
    for (int32_t shape = ddk::kTile64x64; shape <= ddk::kTile64x32 && st == DD_OK; ++shape) {
      Opts q = o;
      q.tile = shape;
      st = run(p, q, ws, L.bytes, false, stream, true);   // warm-up
      std::vector<float> t;
      for (int32_t r = 0; r < repeats && st == DD_OK; ++r) {
        (void)hipEventRecord(e0, stream);
        st = run(p, q, ws, L.bytes, false, stream, true);
        (void)hipEventRecord(e1, stream);
        if (hipEventSynchronize(e1) != hipSuccess) { st = DD_ERR_HIP; break; }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        t.push_back(ms);
      }
      if (st != DD_OK) break;
      std::sort(t.begin(), t.end());
      if (t[t.size() / 2] < best) { best = t[t.size() / 2]; best_shape = shape; }
    }
    if (hipStreamSynchronize(stream) != hipSuccess && st == DD_OK) st = DD_ERR_HIP;
    (void)hipFree(buf);
    if (st != DD_OK) break;
    record_tuned(TuneKey{m[i], n[i], k[i], o.kc, o.scaling}, best_shape);
    if (shapes_out) shapes_out[i] = best_shape;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

dd_status dd_cascade_split(int32_t side, int32_t trans, int64_t rows, int64_t cols,
                           const double* X_hi, const double* X_lo, int64_t ldx,
                           int32_t kc, int32_t* exps, double* planes, hipStream_t stream) {
  if (side != 0 && side != 1) return -1;
  if (trans != DD_OP_N && trans != DD_OP_T) return -2;
  if (rows < 0) return -3;
  if (cols < 0) return -4;
  const int64_t srows = trans ? cols : rows;
  if (ldx < (srows > 1 ? srows : 1)) return -7;
  if (kc != 0 && !valid_kc(kc)) return -8;
  if (rows == 0 || cols == 0) return DD_OK;
  if (!X_hi) return -5;
  if (!X_lo) return -6;
  if (!exps) return -9;
  if (!planes) return -10;
  int dev = 0;
  dd_status st = check_device(&dev);
  if (st != DD_OK) return st;
  // Present X as op(A) (side 0, m x k = rows x cols) or op(B) (side 1, k x n).
  Problem p{};
  p.transa = p.transb = (int)trans;
  int64_t m = 1, n = 1, k;
  if (side == 0) { m = rows; k = cols; p.Ahi = X_hi; p.Alo = X_lo; p.lda = ldx; }
  else { k = rows; n = cols; p.Bhi = X_hi; p.Blo = X_lo; p.ldb = ldx; }
  p.m = m; p.n = n; p.k = k;
  const CascadeLayout L = ddk::make_layout(m, n, k, kc ? kc : kDefaultKc, kTileM, kTileN);
  void* w = nullptr;
  st = cached_workspace(dev, stream, L.bytes, &w);
  if (st != DD_OK) return st;
  char* ws = (char*)w;
  int64_t a_si, a_sp, b_sp, b_sj;
  strides(p, a_si, a_sp, b_sp, b_sj);
  if (side == 0) {
    uint64_t* amax = (uint64_t*)(ws + L.off_amax);
    DD_TRY(ddk::launch_fill_u64(amax, L.mpad, 0, stream));
    DD_TRY(ddk::launch_max_abs_bits(p.Ahi, m, k, a_si, a_sp, amax, stream));
    DD_TRY(ddk::launch_pack_a(p.Ahi, p.Alo, a_si, a_sp, L, amax, (double*)(ws + L.off_apack), stream));
    DD_TRY(ddk::launch_unpack((const double*)(ws + L.off_apack), 0, m, k, L.K4, planes, stream));
    DD_TRY(ddk::launch_exps(amax, m, exps, stream));
  } else {
    uint64_t* bmax = (uint64_t*)(ws + L.off_bmax);
    DD_TRY(ddk::launch_fill_u64(bmax, L.npad, 0, stream));
    DD_TRY(ddk::launch_max_abs_bits(p.Bhi, n, k, b_sj, b_sp, bmax, stream));
    DD_TRY(ddk::launch_pack_b(p.Bhi, p.Blo, b_sp, b_sj, L, bmax, (double*)(ws + L.off_bpack), stream));
    DD_TRY(ddk::launch_unpack((const double*)(ws + L.off_bpack), 1, k, n, L.K4, planes, stream));
    DD_TRY(ddk::launch_exps(bmax, n, exps, stream));
  }
  return DD_OK;
}

dd_status dd_slices_split(int32_t side, int32_t trans, int64_t rows, int64_t cols,
                          const double* X_hi, const double* X_lo, int64_t ldx,
                          int32_t fmt, int32_t slices, int32_t slice_bits,
                          int32_t* exps, uint16_t* out, hipStream_t stream) {
  if (side != 0 && side != 1) return -1;
  if (trans != DD_OP_N && trans != DD_OP_T) return -2;
  if (rows < 0) return -3;
  if (cols < 0) return -4;
  const int64_t srows = trans ? cols : rows;
  if (ldx < (srows > 1 ? srows : 1)) return -7;
  if (fmt < 0 || fmt > 2) return -8;
  Opts o;
  o.algo = fmt == 2 ? DD_ALGO_SLICES_I8 : (fmt == 1 ? DD_ALGO_SLICES_F16 : DD_ALGO_SLICES_BF16);
  if (!slice_params(o.fmt(), slices, slice_bits, &o.S, &o.w)) return -9;
  if (rows == 0 || cols == 0) return DD_OK;
  if (!X_hi) return -5;
  if (!X_lo) return -6;
  if (!exps) return -11;
  if (!out) return -12;
  int dev = 0;
  dd_status st = check_device(&dev);
  if (st != DD_OK) return st;
  // X as op(A) (side 0: outer = rows) or op(B) (side 1: outer = cols); inner = the other
  Problem p{};
  p.transa = p.transb = (int)trans;
  if (side == 0) { p.m = rows; p.n = 1; p.k = cols; p.Ahi = X_hi; p.Alo = X_lo; p.lda = ldx; }
  else { p.m = 1; p.n = cols; p.k = rows; p.Bhi = X_hi; p.Blo = X_lo; p.ldb = ldx; }
  const ddk::SlicesLayout L = slices_layout(p, o);
  void* w = nullptr;
  st = cached_workspace(dev, stream, L.bytes, &w);
  if (st != DD_OK) return st;
  char* ws = (char*)w;
  int64_t a_si, a_sp, b_sp, b_sj;
  strides(p, a_si, a_sp, b_sp, b_sj);
  if (side == 0) {
    uint64_t* amax = (uint64_t*)(ws + L.off_amax);
    DD_TRY(ddk::launch_fill_u64(amax, L.mpad, 0, stream));
    DD_TRY(ddk::launch_max_abs_bits(p.Ahi, rows, cols, a_si, a_sp, amax, stream, p.Alo));
    DD_TRY(ddk::launch_slices_split(p.Ahi, p.Alo, a_si, a_sp, rows, cols, L.mpad, L, amax, ws + L.off_apack, stream));
    DD_TRY(ddk::launch_slices_unpack(ws + L.off_apack, rows, cols, L, 1, rows, out, stream));
    DD_TRY(ddk::launch_exps(amax, rows, exps, stream));
  } else {
    uint64_t* bmax = (uint64_t*)(ws + L.off_bmax);
    DD_TRY(ddk::launch_fill_u64(bmax, L.npad, 0, stream));
    DD_TRY(ddk::launch_max_abs_bits(p.Bhi, cols, rows, b_sj, b_sp, bmax, stream, p.Blo));
    DD_TRY(ddk::launch_slices_split(p.Bhi, p.Blo, b_sj, b_sp, cols, rows, L.npad, L, bmax, ws + L.off_bpack, stream));
    DD_TRY(ddk::launch_slices_unpack(ws + L.off_bpack, cols, rows, L, rows, 1, out, stream));
    DD_TRY(ddk::launch_exps(bmax, cols, exps, stream));
  }
  return DD_OK;
}

dd_status dd_dot(int64_t n, const double* x_hi, const double* x_lo, int64_t incx,
                 const double* y_hi, const double* y_lo, int64_t incy,
                 double* result, hipStream_t stream) {
  if (n < 0) return -1;
  if (n > 0 && !x_hi) return -2;
  if (n > 0 && !x_lo) return -3;
  if (incx < 1) return -4;
  if (n > 0 && !y_hi) return -5;
  if (n > 0 && !y_lo) return -6;
  if (incy < 1) return -7;
  if (!result) return -8;
  int dev = 0;
  dd_status st = check_device(&dev);
  if (st != DD_OK) return st;
  void* part = nullptr;
  st = cached_workspace(dev, stream, sizeof(double) * 2 * 1024, &part);
  if (st != DD_OK) return st;
  return hip_status(ddk::launch_dd_dot(n, x_hi, x_lo, incx, y_hi, y_lo, incy, (double*)part, result, stream));
}

// The output (zh, zl, incz) of an elementwise FP64x2 operation either is one
// of the inputs (same pointers and stride) or overlaps none of them; its two
// planes never overlap each other.  Returns 0, or 1 for the output's high
// plane, 2 for its low plane.
static int output_overlap(int64_t n, const double* zh, const double* zl, int64_t incz,
                          const double* const* in_h, const double* const* in_l, const int64_t* inc, int nin) {
  const size_t zb = (size_t)((n - 1) * incz + 1) * sizeof(double);
  if (overlaps(zl, zb, zh, zb)) return 2;
  for (int v = 0; v < nin; ++v) {
    if (zh == in_h[v] && zl == in_l[v] && incz == inc[v]) continue;
    const size_t xb = (size_t)((n - 1) * inc[v] + 1) * sizeof(double);
    if (overlaps(zh, zb, in_h[v], xb) || overlaps(zh, zb, in_l[v], xb)) return 1;
    if (overlaps(zl, zb, in_h[v], xb) || overlaps(zl, zb, in_l[v], xb)) return 2;
  }
  return 0;
}

dd_status dd_scal(int64_t n, const double* alpha,
                  const double* x_hi, const double* x_lo, int64_t incx,
                  double* y_hi, double* y_lo, int64_t incy, hipStream_t stream) {
  if (n < 0) return -1;
  if (n == 0) return DD_OK;
  if (!alpha) return -2;
  if (!x_hi) return -3;
  if (!x_lo) return -4;
  if (incx < 1) return -5;
  if (!y_hi) return -6;
  if (!y_lo) return -7;
  if (incy < 1) return -8;
  const double* ih[1] = {x_hi};
  const double* il[1] = {x_lo};
  const int64_t inc[1] = {incx};
  const int ov = output_overlap(n, y_hi, y_lo, incy, ih, il, inc, 1);
  if (ov) return ov == 1 ? -6 : -7;
  dd_status st = check_device(nullptr);
  if (st != DD_OK) return st;
  return hip_status(ddk::launch_dd_scal(n, alpha, x_hi, x_lo, incx, y_hi, y_lo, incy, stream));
}

dd_status dd_add(int64_t n, const double* x_hi, const double* x_lo, int64_t incx,
                 const double* y_hi, const double* y_lo, int64_t incy,
                 double* z_hi, double* z_lo, int64_t incz, hipStream_t stream) {
  if (n < 0) return -1;
  if (n == 0) return DD_OK;
  if (!x_hi) return -2;
  if (!x_lo) return -3;
  if (incx < 1) return -4;
  if (!y_hi) return -5;
  if (!y_lo) return -6;
  if (incy < 1) return -7;
  if (!z_hi) return -8;
  if (!z_lo) return -9;
  if (incz < 1) return -10;
  const double* ih[2] = {x_hi, y_hi};
  const double* il[2] = {x_lo, y_lo};
  const int64_t inc[2] = {incx, incy};
  const int ov = output_overlap(n, z_hi, z_lo, incz, ih, il, inc, 2);
  if (ov) return ov == 1 ? -8 : -9;
  dd_status st = check_device(nullptr);
  if (st != DD_OK) return st;
  return hip_status(ddk::launch_dd_add(n, x_hi, x_lo, incx, y_hi, y_lo, incy, z_hi, z_lo, incz, stream));
}

dd_status dd_profile_enable(int32_t enable) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_prof = enable != 0;
  return DD_OK;
}

dd_status dd_phase_times(double* split_ms, double* product_ms, int64_t* calls) {
  std::vector<PhaseEvents> evs;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    evs.swap(g_prof_events);
  }
  double a = 0.0, b = 0.0;
  dd_status st = DD_OK;
  for (const PhaseEvents& pe : evs) {
    float t1 = 0.f, t2 = 0.f;
    if (hipEventSynchronize(pe.e2) != hipSuccess ||
        hipEventElapsedTime(&t1, pe.e0, pe.e1) != hipSuccess ||
        hipEventElapsedTime(&t2, pe.e1, pe.e2) != hipSuccess) st = DD_ERR_HIP;
    a += t1;
    b += t2;
    (void)hipEventDestroy(pe.e0);
    (void)hipEventDestroy(pe.e1);
    (void)hipEventDestroy(pe.e2);
  }
  if (split_ms) *split_ms = a;
  if (product_ms) *product_ms = b;
  if (calls) *calls = (int64_t)evs.size();
  return st;
}

const char* dd_status_string(dd_status s) {
  switch (s) {
    case DD_OK: return "success";
    case DD_ERR_HIP: return "HIP runtime error or kernel launch failure";
    case DD_ERR_WORKSPACE: return "workspace too small, misaligned, or device memory exhausted";
    case DD_ERR_UNSUPPORTED: return "unsupported device (the library runs on gfx950 only)";
    case DD_ERR_INTERNAL: return "internal error";
    default: return s < 0 ? "invalid argument (-status is its 1-based position)" : "unknown status";
  }
}

int32_t dd_version(void) { return 100; }

// ------------------------------------------------------------------ FP64x3
size_t td_gemm_workspace_size(int32_t transa, int32_t transb, int64_t m, int64_t n, int64_t k, int32_t kc) {
  if ((transa != DD_OP_N && transa != DD_OP_T) || (transb != DD_OP_N && transb != DD_OP_T)) return 0;
  if (m <= 0 || n <= 0 || k <= 0) return 0;
  if (kc != 0 && !valid_kc(kc)) return 0;
  return ddk::td_workspace_bytes(m, n, k, nullptr);
}

dd_status td_gemm_ex(int32_t transa, int32_t transb, int64_t m, int64_t n, int64_t k,
                     const double* A0, const double* A1, const double* A2, int64_t lda,
                     const double* B0, const double* B1, const double* B2, int64_t ldb,
                     double* C0, double* C1, double* C2, int64_t ldc,
                     void* workspace, size_t ws_bytes, int32_t kc, hipStream_t stream) {
  if (transa != DD_OP_N && transa != DD_OP_T) return -1;
  if (transb != DD_OP_N && transb != DD_OP_T) return -2;
  if (m < 0) return -3;
  if (n < 0) return -4;
  if (k < 0) return -5;
  const int64_t arows = transa ? k : m, acols = transa ? m : k;
  const int64_t brows = transb ? n : k, bcols = transb ? k : n;
  if (lda < (arows > 1 ? arows : 1)) return -9;
  if (ldb < (brows > 1 ? brows : 1)) return -13;
  if (ldc < (m > 1 ? m : 1)) return -17;
  if (!span_fits(arows, acols, lda)) return -9;
  if (!span_fits(brows, bcols, ldb)) return -13;
  if (!span_fits(m, n, ldc)) return -17;
  if (kc != 0 && !valid_kc(kc)) return -20;
  const bool internal = workspace == nullptr && ws_bytes == 0;
  if (!internal && workspace == nullptr) return -18;
  if (m == 0 || n == 0) return DD_OK;
  double* Cw[3] = {C0, C1, C2};
  for (int w = 0; w < 3; ++w)
    if (!Cw[w]) return -(14 + w);
  if (k == 0) return DD_OK;
  const double* Aw[3] = {A0, A1, A2};
  const double* Bw[3] = {B0, B1, B2};
  for (int w = 0; w < 3; ++w) {
    if (!Aw[w]) return -(6 + w);
    if (!Bw[w]) return -(10 + w);
  }
  const size_t cb = span_bytes(m, n, ldc), ab = span_bytes(arows, acols, lda), bb = span_bytes(brows, bcols, ldb);
  for (int w = 0; w < 3; ++w) {
    for (int v = w + 1; v < 3; ++v)
      if (overlaps(Cw[w], cb, Cw[v], cb)) return -(14 + v);
    for (int v = 0; v < 3; ++v)
      if (overlaps(Cw[w], cb, Aw[v], ab) || overlaps(Cw[w], cb, Bw[v], bb)) return -(14 + w);
  }
  int dev = 0;
  dd_status st = check_device(&dev);
  if (st != DD_OK) return st;
  const size_t need = ddk::td_workspace_bytes(m, n, k, nullptr);
  char* ws = (char*)workspace;
  if (internal) {
    void* w = nullptr;
    st = cached_workspace(dev, stream, need, &w);
    if (st != DD_OK) return st;
    ws = (char*)w;
  } else if (ws_bytes < need || ((uintptr_t)ws & 255u) != 0) {
    return DD_ERR_WORKSPACE;
  }
  const int64_t a_si = transa ? lda : 1, a_sp = transa ? 1 : lda;
  const int64_t b_sp = transb ? ldb : 1, b_sj = transb ? 1 : ldb;
  return hip_status(ddk::run_td(m, n, k, kc ? kc : kDefaultKc, A0, A1, A2, a_si, a_sp, B0, B1, B2, b_sp, b_sj,
                                C0, C1, C2, ldc, ws, stream));
}

}  // extern "C"
