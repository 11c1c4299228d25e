// Batches of independent cascaded FP64x2 GEMMs of uneven shapes, run as one
// phase-one pass and one persistent product launch.
//
// A plan fixes the shapes: it numbers the units of work of every problem
// (prefix sums), lists the output tiles of all problems in decreasing cost
// (LPT order), lays out one workspace for all packed operands and uploads
// all of it once.  Executing a plan launches three kernels and allocates
// nothing, so it can be captured in a HIP graph.  Tiles are 64 x 64, or
// 32 x 64 / 64 x 32 for a problem whose padded area that shrinks, as the
// tile policy says (never; for inner dimensions of 256 or more; always).
// The policy and the schedule of the persistent kernel (fixed stride or
// atomic counter, LPT or problem order) are chosen by timing the
// candidates (dd_batched_plan_tune); choices are kept in a small cache file
// keyed by the shapes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ddgemm.h"
#include "kernels.hpp"
#include "layout.hpp"

using ddk::BatchDesc;
using ddk::BatchTile;

struct dd_batched_plan_s {
  int device = -1;
  int32_t count = 0;
  int32_t kc = 256;
  std::vector<BatchDesc> desc;
  std::vector<int32_t> small_shape;   // per problem: the smaller tile that cuts padding, or 0
  std::vector<BatchTile> tiles_lpt, tiles_natural;
  int64_t max_tiles = 0;              // over the tile policies
  uint64_t key = 0;
  char* dmem = nullptr;          // one device allocation for everything below
  size_t dmem_bytes = 0;
  size_t ws_bytes = 0;           // exponent words and packed planes of all problems
  bool own_ws = true;            // false: d_counter and d_ws come with each call
  uint32_t* flags = nullptr;     // cancellation bitmaps (opts.flags_out), or null
  int64_t flag_words = 0;        // words of all problems' bitmaps
  BatchDesc* d_desc = nullptr;
  int64_t *d_pexpA = nullptr, *d_pexpB = nullptr, *d_ppackA = nullptr, *d_ppackB = nullptr;
  BatchTile* d_tiles = nullptr;
  uint32_t* d_counter = nullptr;
  char* d_ws = nullptr;
  int64_t nexps = 0, units_exp = 0, units_pack = 0, ntiles = 0;
  int grid = 256;
  int dynamic = 1;
  int lpt = 1;
  int policy = 0;                     // tile policy, 0..2
  bool buf = true;                    // every problem's tiles take the buffer-load staging
};

namespace {

constexpr int64_t kTile = 64;

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

uint64_t fnv1a(const void* data, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* p = (const unsigned char*)data;
  for (size_t i = 0; i < n; ++i) { h ^= p[i]; h *= 1099511628211ull; }
  return h;
}

std::mutex g_cache_mu;

std::string cache_path() {
  const char* e = std::getenv("DDGEMM_TUNE_CACHE");
  return e ? std::string(e) : std::string();
}

// Cache file lines of batched plans: "b <key hex> <dynamic> <lpt> <policy>"
// (single GEMMs keep "s ..." lines in the same file).
bool cache_lookup(uint64_t key, int* dynamic, int* lpt, int* policy) {
  std::string path = cache_path();
  if (path.empty()) return false;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return false;
  bool found = false;
  char line[256];
  while (std::fgets(line, sizeof(line), f)) {
    unsigned long long k;
    int d, l, q;
    if (std::sscanf(line, "b %llx %d %d %d", &k, &d, &l, &q) == 4 && k == key && d >= 0 && d <= 1 &&
        l >= 0 && l <= 1 && q >= 0 && q <= 2) {
      *dynamic = d; *lpt = l; *policy = q; found = true;
    }
  }
  std::fclose(f);
  return found;
}

void cache_store(uint64_t key, int dynamic, int lpt, int policy) {
  std::string path = cache_path();
  if (path.empty()) return;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  FILE* f = std::fopen(path.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "b %016llx %d %d %d\n", (unsigned long long)key, dynamic, lpt, policy);
  std::fclose(f);
}

dd_status hip_st(hipError_t e) {
  if (e == hipSuccess) return DD_OK;
  if (e == hipErrorOutOfMemory) return DD_ERR_WORKSPACE;
  return DD_ERR_HIP;
}

// Shape of problem p's tiles under a tile policy: 0, all 64 x 64; 1, the
// smaller tile where it cuts the padded area and k >= 256; 2, wherever it
// cuts the padded area.
int32_t tile_shape(const dd_batched_plan_s* P, int32_t p, int policy) {
  const int32_t small = P->small_shape[p];
  if (small == 0 || policy == 0 || (policy == 1 && P->desc[p].k < 256)) return ddk::kTile64x64;
  return small;
}

// The tile lists of a policy: problem order, and decreasing cost (inner
// dimension times tile area, stable).
void build_tiles(dd_batched_plan_s* P, int policy) {
  P->tiles_natural.clear();
  for (int32_t p = 0; p < P->count; ++p) {
    const BatchDesc& d = P->desc[p];
    if (d.m <= 0 || d.n <= 0 || d.k <= 0) continue;
    const int32_t sh = tile_shape(P, p, policy);
    const int64_t tm_n = cdiv(d.m, ddk::tile_rows(sh)), tn_n = cdiv(d.n, ddk::tile_cols(sh));
    for (int64_t tm = 0; tm < tm_n; ++tm)
      for (int64_t tn = 0; tn < tn_n; ++tn)
        P->tiles_natural.push_back(BatchTile{p, (int32_t)tm, (int32_t)tn, sh});
  }
  P->ntiles = (int64_t)P->tiles_natural.size();
  P->tiles_lpt = P->tiles_natural;
  auto cost = [&](const BatchTile& t) {
    return P->desc[t.p].K4 * (int64_t)ddk::tile_rows(t.shape) * ddk::tile_cols(t.shape);
  };
  std::stable_sort(P->tiles_lpt.begin(), P->tiles_lpt.end(),
                   [&](const BatchTile& a, const BatchTile& b) { return cost(a) > cost(b); });
  P->policy = policy;
}

dd_status upload_tiles(dd_batched_plan_s* P, hipStream_t s) {
  const std::vector<BatchTile>& t = P->lpt ? P->tiles_lpt : P->tiles_natural;
  if (t.empty()) return DD_OK;
  return hip_st(hipMemcpyAsync(P->d_tiles, t.data(), t.size() * sizeof(BatchTile), hipMemcpyHostToDevice, s));
}

// Options a batch accepts (the cascade with global scaling and the library's
// tiles; kc and the cancellation flags may be set); kc out.
bool batched_opts(const dd_gemm_opts* opts, int32_t* kc) {
  if (!opts) return true;
  if (opts->algo != DD_ALGO_CASCADE_F64 || opts->tile != 0 || opts->slices != 0 || opts->slice_bits != 0 ||
      opts->scaling != 0 || opts->use_tuned != 0)
    return false;
  if (opts->kc != 0) {
    if (opts->kc < 4 || opts->kc > 4096 || opts->kc % 4 != 0) return false;
    *kc = opts->kc;
  }
  return true;
}

// Argument checks of a plan (numbers as in dd_batched_plan_create); kc out.
dd_status check_plan_args(int32_t count, const int64_t* m, const int64_t* n, const int64_t* k,
                          const int64_t* lda, const int64_t* ldb, const int64_t* ldc, const dd_gemm_opts* opts,
                          int32_t* kc_out) {
  if (count < 0) return -1;
  if (count > 0 && (!m)) return -2;
  if (count > 0 && (!n)) return -3;
  if (count > 0 && (!k)) return -4;
  if (count > 0 && (!lda)) return -5;
  if (count > 0 && (!ldb)) return -6;
  if (count > 0 && (!ldc)) return -7;
  int32_t kc = 256;
  if (!batched_opts(opts, &kc)) return -8;
  for (int32_t p = 0; p < count; ++p) {
    if (m[p] < 0 || n[p] < 0 || k[p] < 0) return -2;
    if (lda[p] < std::max<int64_t>(1, m[p])) return -5;
    if (ldb[p] < std::max<int64_t>(1, k[p])) return -6;
    if (ldc[p] < std::max<int64_t>(1, m[p])) return -7;
  }
  *kc_out = kc;
  return DD_OK;
}

// Bytes of the exponent words and packed planes of a batch; fills the
// descriptors' layout fields when desc is given.
size_t batch_ws_bytes(int32_t count, const int64_t* m, const int64_t* n, const int64_t* k, int32_t kc,
                      BatchDesc* desc) {
  int64_t nexps = 0;
  for (int32_t p = 0; p < count; ++p) {
    const bool active = m[p] > 0 && n[p] > 0 && k[p] > 0;
    if (active) nexps += ddk::round_up(m[p], kTile) + ddk::round_up(n[p], kTile);
  }
  size_t off = (size_t)ddk::round_up(nexps * 8, 256);
  int64_t eoff = 0;
  for (int32_t p = 0; p < count; ++p) {
    if (!(m[p] > 0 && n[p] > 0 && k[p] > 0)) continue;
    const ddk::CascadeLayout L = ddk::make_layout(m[p], n[p], k[p], kc, kTile, kTile);
    BatchDesc tmp;
    BatchDesc& d = desc ? desc[p] : tmp;
    d.K4 = L.K4; d.mpad = L.mpad; d.npad = L.npad;
    d.tiles_m = L.mpad / kTile; d.tiles_n = L.npad / kTile;
    d.kcq = L.kcq; d.c0 = L.c[0]; d.c1 = L.c[1]; d.c2 = L.c[2];
    d.off_amax = eoff * 8; eoff += d.mpad;
    d.off_bmax = eoff * 8; eoff += d.npad;
    d.off_apack = (int64_t)off;
    off += (size_t)ddk::round_up((int64_t)(sizeof(double) * (d.mpad / 16) * ddk::a_block_stride(L.K4)), 256);
    d.off_bpack = (int64_t)off;
    off += (size_t)ddk::round_up((int64_t)(sizeof(double) * (d.npad / 16) * ddk::b_block_stride(L.K4, ddk::kFragBBatched)), 256);
  }
  return off;
}

// A plan of checked arguments.  With own_ws, its one device allocation also
// holds the atomic counter and the workspace; otherwise only the tables
// (descriptors, prefix sums, tiles), and each execution brings the rest.
dd_status plan_create(int32_t count, const int64_t* m, const int64_t* n, const int64_t* k,
                      const int64_t* lda, const int64_t* ldb, const int64_t* ldc, int32_t kc, bool own_ws,
                      uint32_t* flags, dd_batched_plan* plan) {
  *plan = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DD_ERR_HIP;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return DD_ERR_HIP;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return DD_ERR_UNSUPPORTED;

  dd_batched_plan_s* P = new (std::nothrow) dd_batched_plan_s();
  if (!P) return DD_ERR_WORKSPACE;
  P->device = dev;
  P->count = count;
  P->kc = kc;
  P->desc.resize(count);
  std::vector<int64_t> pexpA(count + 1, 0), pexpB(count + 1, 0), ppackA(count + 1, 0), ppackB(count + 1, 0);
  // workspace: all exponent words first (zeroed with one fill), then the packed planes
  int64_t fw = 0;
  for (int32_t p = 0; p < count; ++p) {
    BatchDesc& d = P->desc[p];
    std::memset(&d, 0, sizeof(d));
    d.m = m[p]; d.n = n[p]; d.k = k[p];
    d.lda = lda[p]; d.ldb = ldb[p]; d.ldc = ldc[p];
    d.off_flags = fw;
    fw += cdiv(m[p] * n[p], 32);
  }
  P->flags = flags;
  P->flag_words = fw;
  const size_t off = batch_ws_bytes(count, m, n, k, kc, P->desc.data());
  for (int32_t p = 0; p < count; ++p)
    if (m[p] > 0 && n[p] > 0 && k[p] > 0 && !ddk::buffer_staging_fits(P->desc[p].K4)) P->buf = false;
  int64_t eoff = 0;
  for (int32_t p = 0; p < count; ++p) {
    BatchDesc& d = P->desc[p];
    const bool active = m[p] > 0 && n[p] > 0 && k[p] > 0;
    if (active) eoff += d.mpad + d.npad;
    pexpA[p + 1] = pexpA[p] + (active ? cdiv(d.m, 256) * cdiv(d.k, 256) : 0);
    pexpB[p + 1] = pexpB[p] + (active ? cdiv(d.n, 4) * cdiv(d.k, 4096) : 0);
    ppackA[p + 1] = ppackA[p] + (active ? cdiv((d.mpad / 16) * d.K4, 4 * ddk::kPackFragsPerWave) : 0);
    ppackB[p + 1] = ppackB[p] + (active ? cdiv((d.npad / 16) * d.K4, 4 * ddk::kPackFragsPerWave) : 0);
    // the smaller tile (32 x 64 or 64 x 32) with the least padded area, if
    // that is less than the 64 x 64 tiles'
    int32_t small = 0;
    if (active) {
      const int64_t a64 = ddk::round_up(d.m, 64) * ddk::round_up(d.n, 64);
      const int64_t a3264 = ddk::round_up(d.m, 32) * ddk::round_up(d.n, 64);
      const int64_t a6432 = ddk::round_up(d.m, 64) * ddk::round_up(d.n, 32);
      if (std::min(a3264, a6432) < a64) small = a3264 <= a6432 ? ddk::kTile32x64 : ddk::kTile64x32;
    }
    P->small_shape.push_back(small);
  }
  P->nexps = eoff;
  P->units_exp = pexpA[count] + pexpB[count];
  P->units_pack = ppackA[count] + ppackB[count];
  for (int q = 2; q >= 0; --q) {               // policy 2 has the most tiles
    build_tiles(P, q);
    P->max_tiles = std::max(P->max_tiles, P->ntiles);
  }
  P->ws_bytes = off;
  P->own_ws = own_ws;

  // device memory: descriptors, prefix arrays, tiles (and counter, workspace)
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = (size_t)ddk::round_up((int64_t)(o + bytes), 256); return r; };
  const size_t o_desc = take(sizeof(BatchDesc) * std::max(count, 1));
  const size_t o_pa = take(sizeof(int64_t) * (count + 1)), o_pb = take(sizeof(int64_t) * (count + 1));
  const size_t o_qa = take(sizeof(int64_t) * (count + 1)), o_qb = take(sizeof(int64_t) * (count + 1));
  const size_t o_tiles = take(sizeof(BatchTile) * std::max<int64_t>(P->max_tiles, 1));
  const size_t o_ctr = own_ws ? take(sizeof(uint64_t)) : 0;
  const size_t o_ws = own_ws ? take(std::max<size_t>(P->ws_bytes, 256)) : 0;
  P->dmem_bytes = o;
  if (hipMalloc(&P->dmem, P->dmem_bytes) != hipSuccess) {
    (void)hipGetLastError();
    delete P;
    return DD_ERR_WORKSPACE;
  }
  P->d_desc = (BatchDesc*)(P->dmem + o_desc);
  P->d_pexpA = (int64_t*)(P->dmem + o_pa);
  P->d_pexpB = (int64_t*)(P->dmem + o_pb);
  P->d_ppackA = (int64_t*)(P->dmem + o_qa);
  P->d_ppackB = (int64_t*)(P->dmem + o_qb);
  P->d_tiles = (BatchTile*)(P->dmem + o_tiles);
  P->d_counter = own_ws ? (uint32_t*)(P->dmem + o_ctr) : nullptr;
  P->d_ws = own_ws ? P->dmem + o_ws : nullptr;

  // key of the tuning cache: device, kc and every shape
  uint64_t key = fnv1a(prop.gcnArchName, std::strlen(prop.gcnArchName));
  key = fnv1a(&kc, sizeof(kc), key);
  for (int32_t p = 0; p < count; ++p) {
    const int64_t s3[3] = {m[p], n[p], k[p]};
    key = fnv1a(s3, sizeof(s3), key);
  }
  P->key = key;
  P->grid = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  int dyn = 1, lpt = 1, policy = 0;
  if (cache_lookup(key, &dyn, &lpt, &policy)) { P->dynamic = dyn; P->lpt = lpt; }
  build_tiles(P, policy);

  dd_status st = DD_OK;
  if (count > 0) {
    st = hip_st(hipMemcpy(P->d_desc, P->desc.data(), sizeof(BatchDesc) * count, hipMemcpyHostToDevice));
    if (st == DD_OK) st = hip_st(hipMemcpy(P->d_pexpA, pexpA.data(), 8 * (count + 1), hipMemcpyHostToDevice));
    if (st == DD_OK) st = hip_st(hipMemcpy(P->d_pexpB, pexpB.data(), 8 * (count + 1), hipMemcpyHostToDevice));
    if (st == DD_OK) st = hip_st(hipMemcpy(P->d_ppackA, ppackA.data(), 8 * (count + 1), hipMemcpyHostToDevice));
    if (st == DD_OK) st = hip_st(hipMemcpy(P->d_ppackB, ppackB.data(), 8 * (count + 1), hipMemcpyHostToDevice));
    if (st == DD_OK) st = upload_tiles(P, nullptr);
    if (st == DD_OK) st = hip_st(hipDeviceSynchronize());
  }
  if (st != DD_OK) {
    (void)hipFree(P->dmem);
    delete P;
    return st;
  }
  *plan = P;
  return DD_OK;
}

// One execution with the given workspace and counter (argument numbers as
// in dd_gemm_batched_exec).
dd_status plan_exec(dd_batched_plan P, const double* const* A_hi, const double* const* A_lo,
                    const double* const* B_hi, const double* const* B_lo, double* const* C_hi,
                    double* const* C_lo, char* ws, uint32_t* counter, uint32_t* flags, hipStream_t stream) {
  if (flags && P->flag_words > 0) {
    // every problem's bitmap starts cleared, also those with nothing to compute
    const hipError_t e = ddk::launch_fill_u32(flags, P->flag_words, 0u, stream);
    if (e != hipSuccess) return hip_st(e);
  }
  if (P->ntiles == 0) return DD_OK;
  if (!A_hi) return -2;
  if (!A_lo) return -3;
  if (!B_hi) return -4;
  if (!B_lo) return -5;
  if (!C_hi) return -6;
  if (!C_lo) return -7;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return DD_ERR_HIP;
  if (dev != P->device) return DD_ERR_UNSUPPORTED;
  hipError_t e = ddk::launch_batched_phase_one(P->d_desc, P->count, P->d_pexpA, P->d_pexpB, P->units_exp,
                                               P->d_ppackA, P->d_ppackB, P->units_pack, A_hi, A_lo, B_hi, B_lo,
                                               ws, (uint64_t*)ws, P->nexps, stream);
  if (e != hipSuccess) return hip_st(e);
  return hip_st(ddk::launch_cascade_batched(P->d_desc, P->d_tiles, P->ntiles, C_hi, C_lo, ws, counter, P->grid,
                                            P->dynamic != 0, flags, P->buf, stream));
}

// Tables of the one-shot form with a caller workspace, kept per device, kc
// and shapes until the process ends (read-only once built).
struct TableKey {
  int dev;
  int32_t kc;
  std::vector<int64_t> shapes;   // m, n, k, lda, ldb, ldc of every problem
  bool operator<(const TableKey& o) const {
    if (dev != o.dev) return dev < o.dev;
    if (kc != o.kc) return kc < o.kc;
    return shapes < o.shapes;
  }
};
std::mutex g_tables_mu;
std::map<TableKey, dd_batched_plan_s*> g_tables;

}  // namespace

extern "C" {

dd_status dd_batched_plan_create(int32_t count, const int64_t* m, const int64_t* n, const int64_t* k,
                                 const int64_t* lda, const int64_t* ldb, const int64_t* ldc,
                                 const dd_gemm_opts* opts, dd_batched_plan* plan) {
  int32_t kc = 256;
  const dd_status st = check_plan_args(count, m, n, k, lda, ldb, ldc, opts, &kc);
  if (st != DD_OK) return st;
  if (!plan) return -9;
  return plan_create(count, m, n, k, lda, ldb, ldc, kc, true, opts ? opts->flags_out : nullptr, plan);
}

dd_status dd_gemm_batched_exec(dd_batched_plan P, const double* const* A_hi, const double* const* A_lo,
                               const double* const* B_hi, const double* const* B_lo,
                               double* const* C_hi, double* const* C_lo, hipStream_t stream) {
  if (!P) return -1;
  if (!P->own_ws) return -1;
  return plan_exec(P, A_hi, A_lo, B_hi, B_lo, C_hi, C_lo, P->d_ws, P->d_counter, P->flags, stream);
}

size_t dd_gemm_batched_workspace_size(int32_t count, const int64_t* m, const int64_t* n, const int64_t* k,
                                      const dd_gemm_opts* opts) {
  if (count < 0 || (count > 0 && (!m || !n || !k))) return 0;
  int32_t kc = 256;
  if (!batched_opts(opts, &kc)) return 0;
  for (int32_t p = 0; p < count; ++p)
    if (m[p] < 0 || n[p] < 0 || k[p] < 0) return 0;
  // the atomic counter, then the exponent words and packed planes
  return 256 + std::max<size_t>(batch_ws_bytes(count, m, n, k, kc, nullptr), 256);
}

dd_status dd_batched_plan_tune(dd_batched_plan P, const double* const* A_hi, const double* const* A_lo,
                               const double* const* B_hi, const double* const* B_lo,
                               double* const* C_hi, double* const* C_lo, int32_t repeats,
                               hipStream_t stream) {
  if (!P) return -1;
  if (repeats < 1) return -8;
  if (P->ntiles == 0) return DD_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipGetLastError();
    if (e0) (void)hipEventDestroy(e0);
    return DD_ERR_HIP;
  }
  float best = 1e30f;
  int best_dyn = P->dynamic, best_lpt = P->lpt, best_policy = P->policy;
  dd_status st = DD_OK;
  for (int policy = 0; policy <= 2 && st == DD_OK; ++policy) {
    build_tiles(P, policy);
    for (int lpt = 1; lpt >= 0 && st == DD_OK; --lpt) {
      P->lpt = lpt;
      st = upload_tiles(P, stream);
      for (int dyn = 1; dyn >= 0 && st == DD_OK; --dyn) {
        P->dynamic = dyn;
        st = dd_gemm_batched_exec(P, A_hi, A_lo, B_hi, B_lo, C_hi, C_lo, stream);  // warm-up
        std::vector<float> t;
        for (int r = 0; r < repeats && st == DD_OK; ++r) {
          (void)hipEventRecord(e0, stream);
          st = dd_gemm_batched_exec(P, A_hi, A_lo, B_hi, B_lo, C_hi, C_lo, stream);
          (void)hipEventRecord(e1, stream);
          if (hipEventSynchronize(e1) != hipSuccess) st = DD_ERR_HIP;
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          t.push_back(ms);
        }
        if (st != DD_OK) break;
        std::sort(t.begin(), t.end());
        const float med = t[t.size() / 2];
        if (med < best) { best = med; best_dyn = dyn; best_lpt = lpt; best_policy = policy; }
      }
    }
  }
  build_tiles(P, best_policy);
  P->dynamic = best_dyn;
  P->lpt = best_lpt;
  if (st == DD_OK) st = upload_tiles(P, stream);
  if (st == DD_OK) st = hip_st(hipStreamSynchronize(stream));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == DD_OK) cache_store(P->key, best_dyn, best_lpt, best_policy);
  return st;
}

dd_status dd_batched_plan_schedule(dd_batched_plan P, int32_t dynamic, int32_t lpt, int32_t tile_policy,
                                   hipStream_t stream) {
  if (!P) return -1;
  if (dynamic != 0 && dynamic != 1) return -2;
  if (lpt != 0 && lpt != 1) return -3;
  if (tile_policy < 0 || tile_policy > 2) return -4;
  build_tiles(P, tile_policy);
  P->dynamic = dynamic;
  P->lpt = lpt;
  return upload_tiles(P, stream);
}

dd_status dd_batched_plan_info(dd_batched_plan P, int64_t* ntiles, int32_t* dynamic, int32_t* lpt,
                               int32_t* tile_policy, size_t* device_bytes) {
  if (!P) return -1;
  if (ntiles) *ntiles = P->ntiles;
  if (dynamic) *dynamic = P->dynamic;
  if (lpt) *lpt = P->lpt;
  if (tile_policy) *tile_policy = P->policy;
  if (device_bytes) *device_bytes = P->dmem_bytes;
  return DD_OK;
}

dd_status dd_batched_plan_destroy(dd_batched_plan P) {
  if (!P) return DD_OK;
  dd_status st = DD_OK;
  if (P->dmem) {
    if (hipDeviceSynchronize() != hipSuccess) st = DD_ERR_HIP;
    if (hipFree(P->dmem) != hipSuccess) st = DD_ERR_HIP;
  }
  delete P;
  return st;
}

dd_status dd_gemm_batched(int32_t count, const int64_t* m, const int64_t* n, const int64_t* k,
                          const double* const* A_hi, const double* const* A_lo, const int64_t* lda,
                          const double* const* B_hi, const double* const* B_lo, const int64_t* ldb,
                          double* const* C_hi, double* const* C_lo, const int64_t* ldc,
                          void* workspace, size_t ws_bytes, const dd_gemm_opts* opts, hipStream_t stream) {
  // argument numbers of the plan calls mapped onto this prototype
  static const int pos[] = {0, 1, 2, 3, 4, 7, 10, 13, 16, 0};
  static const int pos2[] = {0, 0, 5, 6, 8, 9, 11, 12};
  if (count < 0) return -1;
  if (!workspace && ws_bytes != 0) return -15;
  if (workspace && ((uintptr_t)workspace & 255u) != 0) return -14;
  int32_t kc = 256;
  dd_status st = check_plan_args(count, m, n, k, lda, ldb, ldc, opts, &kc);
  if (st != DD_OK) return st < 0 && -st < 10 ? -pos[-st] : st;
  if (count == 0) return DD_OK;
  uint32_t* const flags = opts ? opts->flags_out : nullptr;
  if (!workspace) {
    dd_batched_plan P = nullptr;
    st = plan_create(count, m, n, k, lda, ldb, ldc, kc, true, flags, &P);
    if (st != DD_OK) return st;
    st = plan_exec(P, A_hi, A_lo, B_hi, B_lo, C_hi, C_lo, P->d_ws, P->d_counter, flags, stream);
    if (st < 0) st = -pos2[-st];
    const dd_status st2 = dd_batched_plan_destroy(P);  // waits for the work to finish
    return st != DD_OK ? st : st2;
  }
  // caller workspace: the tables of these shapes, built once per device
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return DD_ERR_HIP;
  TableKey key{dev, kc, {}};
  key.shapes.reserve((size_t)count * 6);
  for (int32_t p = 0; p < count; ++p) {
    const int64_t v[6] = {m[p], n[p], k[p], lda[p], ldb[p], ldc[p]};
    key.shapes.insert(key.shapes.end(), v, v + 6);
  }
  dd_batched_plan P = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_tables_mu);
    auto it = g_tables.find(key);
    if (it != g_tables.end()) {
      P = it->second;
    } else {
      // building them allocates and waits: not on a stream being captured
      hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
      if (hipStreamIsCapturing(stream, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return DD_ERR_HIP;
      }
      if (cs != hipStreamCaptureStatusNone) return DD_ERR_WORKSPACE;
      st = plan_create(count, m, n, k, lda, ldb, ldc, kc, false, nullptr, &P);
      if (st != DD_OK) return st;
      g_tables.emplace(std::move(key), P);
    }
  }
  if (ws_bytes < 256 + std::max<size_t>(P->ws_bytes, 256)) return DD_ERR_WORKSPACE;
  char* w = (char*)workspace;
  st = plan_exec(P, A_hi, A_lo, B_hi, B_lo, C_hi, C_lo, w + 256, (uint32_t*)w, flags, stream);
  return st < 0 ? -pos2[-st] : st;
}

}  // extern "C"
