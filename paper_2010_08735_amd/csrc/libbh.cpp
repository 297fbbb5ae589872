// libbh host side: contexts, resident resources, argument validation, per-view setup in
// FP64, kernel launches, batched launches under HIP graphs, autotuning and the serving
// scheduler.  Public API: include/bh.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <set>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "bh.h"
#include "bh_dev.h"
#include "bh_sched.h"

namespace bh {
hipError_t launch_precompute(float* D, float* Dt, int d_n, float* U, float* Ut, int u_ne,
                             int u_nphi, int mode, double band, double step, hipStream_t s);
hipError_t launch_band_lut(float4* lut, int n, float x0, float dx, hipStream_t s);
hipError_t launch_band_eval(const LutDev& L, const float* temps, int64_t n, float* out,
                            hipStream_t s);
hipError_t launch_star_build(const float* dirs, const float* inten, const float* temp, int64_t n,
                             int n0, int levels, const uint32_t* level_off_host, int* head,
                             int* next, float2* pos, float4* master, unsigned* maxbits,
                             float* scale, int fp16, void* out, hipStream_t s);
hipError_t launch_fill_int(int* p, int64_t n, int v, hipStream_t s);
hipError_t launch_star_hash(const float* dirs, const float* inten, const float* temp, int64_t n,
                            unsigned long long* acc, hipStream_t s);
hipError_t launch_star_occupancy(const void* tex, int n0, int levels, const uint32_t* level_off,
                                 const uint32_t* occ_off, int fp16, uint32_t* occ,
                                 hipStream_t s);
hipError_t launch_star_unpack(const void* in, int64_t count, float scale, int fp16, float4* out,
                              hipStream_t s);
hipError_t launch_star_build_bands(const float* dirs, const float* rgb, int64_t n, int n0,
                                   int levels, const uint32_t* level_off_host, int* head,
                                   int* next, float2* pos, float4* master, unsigned* maxbits,
                                   float* scale, int fp16, void* out, int* bad, hipStream_t s);
hipError_t launch_star_hash_bands(const float* dirs, const float* rgb, int64_t n,
                                  unsigned long long* acc, hipStream_t s);
hipError_t launch_star_occupancy_bands(const void* tex, int n0, int levels,
                                       const uint32_t* level_off, const uint32_t* occ_off,
                                       int fp16, uint32_t* occ, hipStream_t s);
hipError_t launch_star_unpack_bands(const void* in, int64_t count, float scale, int fp16,
                                    float4* out, hipStream_t s);
hipError_t launch_render(int cfg, const ViewDev& v, const TablesDev& T, const LutDev& L,
                         hipStream_t s);
hipError_t launch_area_build(const float* it, int n0, float2* tex, int* bad, hipStream_t s);
hipError_t launch_area_build_bands(const float* rgbx, int n0, float4* tex, int* bad,
                                   hipStream_t s);
hipError_t launch_cshift_build(const CshiftRule& q, double4* spec, float4* tab, hipStream_t s);
hipError_t launch_render_batch(int cfg, int persistent, int feat, const ViewDev* views,
                               const TileRun* runs, int nruns, int ntiles, int* counter,
                               const TablesDev& T, const LutDev& L, int grid, hipStream_t s);
hipError_t launch_trace_rays(const TablesDev& T, const float* rays, int64_t n, float4* out,
                             float4* out_time, hipStream_t s);
hipError_t launch_render_march(const ViewDev& v, const LutDev& L, hipStream_t s);
hipError_t launch_bloom(const float4* in, void* out, float4* P, float4* U, const BloomDev& B,
                        bool display, float exposure, hipStream_t s);
hipError_t launch_tonemap(const float4* in, uint32_t* out, int64_t n, float exposure,
                          hipStream_t s);
hipError_t launch_march_rays(const float* rays, int64_t n, int nsteps, float h, float4* out,
                             hipStream_t s);
hipError_t launch_render_count(const ViewDev& v, const TablesDev& T, const LutDev& L,
                               uint32_t* touched, int64_t words, unsigned long long* total,
                               unsigned long long* l2_bytes, hipStream_t s);
int tile_config_count();
void tile_config(int i, int* tw, int* th, int* waves, int* ppt);
// The tile configuration a context starts with: 8x8 tiles of one pixel per thread (index 3
// of render.hip's table), the fastest for the 1080p frame and for uneven batches.
constexpr int kDefaultTileCfg = 3;
hipError_t scratch_address(void** p);
hipError_t launch_l2_read(const float4* buf, int64_t n4, int per_wg, int grid, float* sink,
                          hipStream_t s);
}  // namespace bh

using namespace bh;

// ---- errors ------------------------------------------------------------------------------

static thread_local std::string g_err;

static bh_status fail(bh_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

// One kernel launch covers at most 2^32 - 1 work-items.  Images (width x height) and arrays
// of rays or temperatures are held to 2^31 elements, which keeps every launch below that
// bound with its tile padding.
constexpr int64_t kMaxElems = (int64_t)1 << 31;

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(BH_EDEVICE, std::string(#expr) + " failed: " + hipGetErrorString(e_));    \
  } while (0)

extern "C" const char* bh_last_error(const bh_ctx*) { return g_err.c_str(); }

// Live handles of every context, by address and type, so that bh_release can dispatch on any
// handle, and reject an address that is not one, without reading through it.
enum HandleKind { kTables, kStars, kParticles, kBloom, kArea };
static std::mutex g_handles_mu;
static std::unordered_map<const void*, HandleKind> g_handles;
static void handle_add(const void* h, HandleKind k) {
  std::lock_guard<std::mutex> g(g_handles_mu);
  g_handles[h] = k;
}
static void handle_drop(const void* h) {
  std::lock_guard<std::mutex> g(g_handles_mu);
  g_handles.erase(h);
}

// ---- resources -----------------------------------------------------------------------------

struct bh_tables {
  bh_ctx* ctx;
  bh_table_params p;
  std::string key;
  float* D = nullptr;
  float* U = nullptr;
  float* Dt = nullptr;  // time channels: e tau at the same texel centres
  float* Ut = nullptr;
  size_t bytes = 0;
  int refs = 1;
};

struct bh_particles {
  bh_ctx* ctx;
  float4* dev = nullptr;  // 2 records per particle, then the start table
  int n = 0;
  size_t bytes = 0;
  float scale = 0.0f;     // start-table bins per unit radius
};

// Radius bins of the start table: a crossing at radius r starts its particle loop at
// start[min(floor(r * scale), kPartBins)], the first particle whose radial reach
// (r_apo + 1) extends to the bin; no earlier particle can touch r.
constexpr int kPartBins = 256;

struct bh_bloom {
  bh_ctx* ctx;
  int width = 0, height = 0, levels = 0;
  float4* P = nullptr;  // levels 1..K of the image's box pyramid
  float4* U = nullptr;  // the U chain of the coarse levels (same offsets as P)
  size_t elems = 0;     // float4 elements of P and of U
  BloomDev B{};          // launch record (sizes, offsets; weights filled per call)
};

// Star maps are shared by content: (hash of the star arrays, star count, face size,
// texel format, band colours).
using StarKey = std::tuple<uint64_t, int64_t, int, int, int>;

struct bh_stars {
  bh_ctx* ctx;
  StarKey key;
  int n0, levels, fp16;
  int bands = 0;          // 1: band-colour texels (R, G, B, p_u, p_v), see stars.hip
  void* tex = nullptr;
  float* scale = nullptr;
  uint32_t* level_off_dev = nullptr;
  uint32_t* occ = nullptr;        // occupancy bits (see k_star_occupancy)
  uint32_t* occ_off_dev = nullptr;
  size_t occ_bytes = 0;
  std::vector<uint32_t> level_off, occ_off;
  size_t bytes = 0;
  int refs = 1;
};

struct bh_area {
  bh_ctx* ctx;
  void* tex = nullptr;    // all levels (see area.hip): float2 (I, I T), or float4 (R, G, B, 0)
  int n0 = 0, levels = 0;
  int bands = 0;
  size_t bytes = 0;
};

struct Staging {
  void* host = nullptr;   // pinned
  size_t cap = 0;
  hipEvent_t done = nullptr;  // last copy out of this buffer
  bool used = false;
};

struct ServeBackend;

struct bh_ctx {
  int device = 0;
  uint64_t budget = 0;
  std::atomic<uint64_t> used{0};
  int cus = 256;
  std::mutex mu;  // resources, tile config, batch staging
  std::map<std::string, bh_tables*> tables;
  std::map<StarKey, bh_stars*> stars;
  std::set<bh_particles*> particles;
  std::set<bh_area*> areas;
  std::set<bh_bloom*> blooms;
  float4* lut = nullptr;
  float4* ctab = nullptr;  // colour-shift table, built with the first band map
  int lut_n = 4096;
  float lut_x0 = 6.0f, lut_dx = 15.0f / 4095.0f;
  int tile_cfg = kDefaultTileCfg;
  int persistent = 0;  // batched launches: 1 = persistent workgroups, 0 = one per tile
  // batched launches
  ViewDev* b_views = nullptr;
  TileRun* b_runs = nullptr;
  int* b_counter = nullptr;
  size_t b_cap = 0;  // views and runs held by b_views / b_runs
  Staging b_stage[2];
  int b_next_stage = 0;
  hipEvent_t b_last = nullptr;  // completion of the last batch that used b_views/b_runs
  // allocation-free batched launches: the device address of the library's scratch array on
  // this device, and pinned staging for its records (set up by bh_create)
  void* scratch = nullptr;
  Staging na_stage;
  struct GraphEntry {
    hipGraphExec_t exec;
    hipStream_t stream;
  };
  // a captured batch launch holds its kernel arguments by value: the key is every one of
  // them that can change between calls (tables by all their pointers and sizes)
  using GraphKey = std::tuple<int, int, int, int, uintptr_t, const void*, const void*, const void*,
                              const void*, int, int, int>;
  std::map<GraphKey, GraphEntry> graphs;
  // serving: the scheduler (bh_sched.h), its HIP backend and thread; smu guards their lifetime
  std::mutex smu;
  std::unique_ptr<ServeBackend> serve_backend;
  std::unique_ptr<sched::Scheduler<ServeBackend>> sched;
  std::thread serve_thread;
};

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Reserves the bytes in the budget first (one atomic add, so concurrent callers cannot both
// pass the check), then allocates; both steps are undone on failure.
static bh_status dev_alloc(bh_ctx* c, size_t bytes, void** p) {
  const uint64_t before = c->used.fetch_add(bytes);
  if (c->budget && before + bytes > c->budget) {
    c->used -= bytes;
    return fail(BH_ENOMEM, "HBM budget exceeded: " + std::to_string(before + bytes) + " > " +
                               std::to_string(c->budget));
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    c->used -= bytes;
    *p = nullptr;
    return fail(BH_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  return BH_OK;
}

static void dev_free(bh_ctx* c, void* p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  c->used -= bytes;
}

static bh_status ensure_staging(Staging& s, size_t bytes) {
  if (s.cap >= bytes) return BH_OK;
  if (s.host) (void)hipHostFree(s.host);
  s.host = nullptr;
  s.cap = 0;
  size_t cap = std::max(bytes, (size_t)1 << 16);
  HIPCHK(hipHostMalloc(&s.host, cap, hipHostMallocDefault));
  s.cap = cap;
  if (!s.done) HIPCHK(hipEventCreateWithFlags(&s.done, hipEventDisableTiming));
  return BH_OK;
}

// ---- context -------------------------------------------------------------------------------

// Device address of the scratch array of the allocation-free batched launch, looked up once
// per device (with that device current) and kept for the life of the process.
static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch;

// Host records staged for one allocation-free launch: views, tile runs, launch order.
static size_t noalloc_staging_bytes() {
  return (size_t)BH_NOALLOC_MAX_VIEWS * (sizeof(ViewDev) + sizeof(TileRun) + sizeof(int));
}

static bh_status noalloc_setup(bh_ctx* c) {
  {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch.find(c->device);
    if (it == g_scratch.end()) {
      void* p = nullptr;
      hipError_t e = scratch_address(&p);
      if (e != hipSuccess || !p)
        return fail(BH_EDEVICE, std::string("scratch address: ") + hipGetErrorString(e));
      it = g_scratch.emplace(c->device, p).first;
    }
    c->scratch = it->second;
  }
  return ensure_staging(c->na_stage, noalloc_staging_bytes());
}

extern "C" bh_status bh_create(int device, uint64_t budget, bh_ctx** out) {
  if (!out) return fail(BH_EINVAL, "out is NULL");
  int n = 0;
  HIPCHK(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(BH_EINVAL, "no such device");
  HIPCHK(hipSetDevice(device));
  std::unique_ptr<bh_ctx> c(new bh_ctx);
  c->device = device;
  c->budget = budget;
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, device));
  c->cus = prop.multiProcessorCount;
  bh_status st = dev_alloc(c.get(), sizeof(float4) * c->lut_n, (void**)&c->lut);
  if (st) return st;
  hipError_t e = launch_band_lut(c->lut, c->lut_n, c->lut_x0, c->lut_dx, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) {
    st = dev_alloc(c.get(), sizeof(int) * 64, (void**)&c->b_counter);
  } else {
    st = fail(BH_EDEVICE, std::string("band table: ") + hipGetErrorString(e));
  }
  if (!st) st = noalloc_setup(c.get());
  if (st) {
    dev_free(c.get(), c->lut, sizeof(float4) * c->lut_n);
    dev_free(c.get(), c->b_counter, c->b_counter ? sizeof(int) * 64 : 0);
    if (c->na_stage.host) (void)hipHostFree(c->na_stage.host);
    if (c->na_stage.done) (void)hipEventDestroy(c->na_stage.done);
    return st;
  }
  *out = c.release();
  return BH_OK;
}

static void serve_stop(bh_ctx* c);

extern "C" void bh_destroy(bh_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  serve_stop(c);
  (void)hipDeviceSynchronize();
  for (auto& kv : c->graphs) {
    (void)hipGraphExecDestroy(kv.second.exec);
  }
  if (c->b_last) (void)hipEventDestroy(c->b_last);
  for (auto& kv : c->tables) {
    dev_free(c, kv.second->D, 0);
    dev_free(c, kv.second->U, 0);
    dev_free(c, kv.second->Dt, 0);
    dev_free(c, kv.second->Ut, 0);
    handle_drop(kv.second);
    delete kv.second;
  }
  for (auto& kv : c->stars) {
    dev_free(c, kv.second->tex, 0);
    dev_free(c, kv.second->scale, 0);
    dev_free(c, kv.second->level_off_dev, 0);
    dev_free(c, kv.second->occ, 0);
    dev_free(c, kv.second->occ_off_dev, 0);
    handle_drop(kv.second);
    delete kv.second;
  }
  for (bh_bloom* b : c->blooms) {
    dev_free(c, b->P, 0);
    dev_free(c, b->U, 0);
    handle_drop(b);
    delete b;
  }
  for (bh_area* a : c->areas) {
    dev_free(c, a->tex, 0);
    handle_drop(a);
    delete a;
  }
  for (bh_particles* p : c->particles) {
    dev_free(c, p->dev, 0);
    handle_drop(p);
    delete p;
  }
  dev_free(c, c->lut, 0);
  dev_free(c, c->ctab, 0);
  dev_free(c, c->b_counter, 0);
  dev_free(c, c->b_views, 0);
  dev_free(c, c->b_runs, 0);
  for (auto& s : c->b_stage) {
    if (s.host) (void)hipHostFree(s.host);
    if (s.done) (void)hipEventDestroy(s.done);
  }
  if (c->na_stage.host) (void)hipHostFree(c->na_stage.host);
  if (c->na_stage.done) (void)hipEventDestroy(c->na_stage.done);
  delete c;
}

extern "C" uint64_t bh_bytes_in_use(const bh_ctx* c) { return c ? c->used.load() : 0; }

// ---- tables --------------------------------------------------------------------------------

static std::string table_key(const bh_table_params& p) {
  char b[256];
  snprintf(b, sizeof b, "%d/%d/%d/%d/%.17g/%.17g", p.d_n, p.u_ne, p.u_nphi, p.precision,
           p.fp64_band, p.step);
  return b;
}

extern "C" bh_status bh_precompute_tables(bh_ctx* c, const bh_table_params* pin, void* stream,
                                          bh_tables** out) {
  if (!c || !pin || !out) return fail(BH_EINVAL, "NULL argument");
  bh_table_params p = *pin;
  if (p.step == 0.0) p.step = 2e-3;
  if (p.d_n < 8 || p.d_n % 2 || p.d_n > 16384) return fail(BH_EINVAL, "d_n must be even, 8..16384");
  if (p.u_ne < 4 || p.u_nphi < 4 || p.u_ne > 4096 || p.u_nphi > 4096)
    return fail(BH_EINVAL, "u_ne, u_nphi must be in 4..4096");
  if (p.precision < BH_TAB_FP32 || p.precision > BH_TAB_FP64_ALL)
    return fail(BH_EINVAL, "bad precision");
  if (!(p.fp64_band >= 0.0 && p.fp64_band < 1.0)) return fail(BH_EINVAL, "bad fp64_band");
  if (!(p.step > 1e-7 && p.step <= 0.05)) return fail(BH_EINVAL, "step must be in (1e-7, 0.05]");
  HIPCHK(hipSetDevice(c->device));
  std::lock_guard<std::mutex> g(c->mu);
  std::string key = table_key(p);
  auto it = c->tables.find(key);
  if (it != c->tables.end()) {
    it->second->refs++;
    *out = it->second;
    return BH_OK;
  }
  auto* t = new bh_tables;
  t->ctx = c;
  t->p = p;
  t->key = key;
  size_t bd = sizeof(float) * (size_t)p.d_n * p.d_n, bu = sizeof(float) * (size_t)p.u_ne * p.u_nphi;
  bh_status st = dev_alloc(c, bd, (void**)&t->D);
  if (!st) st = dev_alloc(c, bu, (void**)&t->U);
  if (!st) st = dev_alloc(c, bd, (void**)&t->Dt);
  if (!st) st = dev_alloc(c, bu, (void**)&t->Ut);
  if (st) {
    dev_free(c, t->D, t->D ? bd : 0);
    dev_free(c, t->U, t->U ? bu : 0);
    dev_free(c, t->Dt, t->Dt ? bd : 0);
    delete t;
    return st;
  }
  t->bytes = 2 * (bd + bu);
  hipStream_t s = (hipStream_t)stream;
  int mode = p.precision == BH_TAB_FP32 ? 0 : (p.precision == BH_TAB_FP64_BAND ? 1 : 2);
  hipError_t e = launch_precompute(t->D, t->Dt, p.d_n, t->U, t->Ut, p.u_ne, p.u_nphi, mode,
                                   p.fp64_band, p.step, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    dev_free(c, t->D, bd);
    dev_free(c, t->U, bu);
    dev_free(c, t->Dt, bd);
    dev_free(c, t->Ut, bu);
    delete t;
    return fail(BH_EDEVICE, std::string("precompute: ") + hipGetErrorString(e));
  }
  c->tables[key] = t;
  handle_add(t, kTables);
  *out = t;
  return BH_OK;
}

extern "C" bh_status bh_tables_download(const bh_tables* t, float* hD, float* hU) {
  if (!t) return fail(BH_EINVAL, "NULL tables");
  HIPCHK(hipSetDevice(t->ctx->device));
  if (hD) HIPCHK(hipMemcpy(hD, t->D, sizeof(float) * (size_t)t->p.d_n * t->p.d_n, hipMemcpyDeviceToHost));
  if (hU) HIPCHK(hipMemcpy(hU, t->U, sizeof(float) * (size_t)t->p.u_ne * t->p.u_nphi, hipMemcpyDeviceToHost));
  return BH_OK;
}

extern "C" bh_status bh_tables_download_time(const bh_tables* t, float* hDt, float* hUt) {
  if (!t) return fail(BH_EINVAL, "NULL tables");
  HIPCHK(hipSetDevice(t->ctx->device));
  if (hDt) HIPCHK(hipMemcpy(hDt, t->Dt, sizeof(float) * (size_t)t->p.d_n * t->p.d_n, hipMemcpyDeviceToHost));
  if (hUt) HIPCHK(hipMemcpy(hUt, t->Ut, sizeof(float) * (size_t)t->p.u_ne * t->p.u_nphi, hipMemcpyDeviceToHost));
  return BH_OK;
}

extern "C" bh_status bh_release_tables(bh_tables* t) {
  if (!t) return fail(BH_EINVAL, "NULL tables");
  bh_ctx* c = t->ctx;
  std::lock_guard<std::mutex> g(c->mu);
  if (--t->refs > 0) return BH_OK;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  // captured batch launches that read these tables must not be replayed on a later table
  // set that happens to reuse the freed addresses
  for (auto it = c->graphs.begin(); it != c->graphs.end();) {
    if (std::get<5>(it->first) == t->D) {
      (void)hipGraphExecDestroy(it->second.exec);
      it = c->graphs.erase(it);
    } else {
      ++it;
    }
  }
  c->tables.erase(t->key);
  dev_free(c, t->D, sizeof(float) * (size_t)t->p.d_n * t->p.d_n);
  dev_free(c, t->U, sizeof(float) * (size_t)t->p.u_ne * t->p.u_nphi);
  dev_free(c, t->Dt, sizeof(float) * (size_t)t->p.d_n * t->p.d_n);
  dev_free(c, t->Ut, sizeof(float) * (size_t)t->p.u_ne * t->p.u_nphi);
  handle_drop(t);
  delete t;
  return BH_OK;
}

// ---- disc particles (Appendix B) -------------------------------------------------------------

// complete elliptic integral of the first kind by the arithmetic-geometric mean (Gauss):
// K(kappa) = pi / (2 AGM(1, sqrt(1 - kappa^2)))
static double ellipk_agm(double kappa) {
  double a = 1.0, b = std::sqrt(1.0 - kappa * kappa);
  for (int it = 0; it < 40 && std::fabs(a - b) > 1e-16 * a; ++it) {
    double an = 0.5 * (a + b);
    b = std::sqrt(a * b);
    a = an;
  }
  return M_PI / (a + b);
}

extern "C" bh_status bh_create_particles(bh_ctx* c, const double* tr, int32_t n,
                                         bh_particles** out) {
  if (!c || !out || n < 0 || n > 65536 || (n > 0 && !tr)) return fail(BH_EINVAL, "bad arguments");
  std::vector<float4> rec(2 * (size_t)std::max(n, 1));
  for (int32_t j = 0; j < n; ++j) {
    double rp = tr[3 * j], ra = tr[3 * j + 1], ph0 = tr[3 * j + 2];
    if (!(std::isfinite(rp) && std::isfinite(ra) && std::isfinite(ph0)) || !(rp >= 3.0) ||
        !(ra >= rp) || ra > 1e6)
      return fail(BH_EINVAL, "particle " + std::to_string(j) + ": need 3 <= r_peri <= r_apo");
    double u1 = 1.0 / ra, u2 = 1.0 / rp, u3 = 1.0 - u1 - u2;
    double K = ellipk_agm(std::sqrt((u2 - u1) / (u3 - u1)));
    double ubar = 0.5 * (u1 + u2);
    rec[2 * j] = make_float4((float)u1, (float)(u2 - u1),
                             (float)(M_PI / (4.0 * K) * std::sqrt(u3 - u1)),
                             (float)std::sqrt(ubar * ubar * ubar / 2.0));
    rec[2 * j + 1] = make_float4((float)ph0, (float)(rp - 1.0), (float)(ra + 1.0), 0.0f);
  }
  // sorted by the inner end of their radial reach, so a crossing stops at the first
  // particle that starts beyond it
  std::vector<int> order(n);
  for (int32_t j = 0; j < n; ++j) order[j] = j;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return rec[2 * a + 1].y < rec[2 * b + 1].y; });
  std::vector<float4> sorted(rec.size());
  for (int32_t j = 0; j < n; ++j) {
    sorted[2 * j] = rec[2 * order[j]];
    sorted[2 * j + 1] = rec[2 * order[j] + 1];
  }
  rec.swap(sorted);
  // start table: prefix maxima of the outer reach are non-decreasing, so the first particle
  // reaching a bin's lower edge (less a hundredth of a bin) is found by binary search
  std::vector<float> reach(n);
  float rmax = 0.0f;
  for (int32_t j = 0; j < n; ++j) reach[j] = rmax = std::max(rmax, rec[2 * j + 1].z);
  const float scale = n > 0 ? (float)kPartBins / rmax : 0.0f;
  std::vector<int32_t> start(kPartBins + 1 + 3, n);  // padded to whole float4s
  for (int b = 0; b <= kPartBins && n > 0; ++b) {
    const float edge = ((float)b - 0.01f) / scale;
    start[b] = (int32_t)(std::lower_bound(reach.begin(), reach.end(), edge) - reach.begin());
  }
  const size_t rec_bytes = sizeof(float4) * rec.size();
  std::vector<char> blob(rec_bytes + sizeof(int32_t) * start.size());
  memcpy(blob.data(), rec.data(), rec_bytes);
  memcpy(blob.data() + rec_bytes, start.data(), sizeof(int32_t) * start.size());
  HIPCHK(hipSetDevice(c->device));
  std::lock_guard<std::mutex> g(c->mu);
  auto* p = new bh_particles;
  p->ctx = c;
  p->n = n;
  p->scale = scale;
  size_t bytes = blob.size();
  p->bytes = bytes;
  bh_status st = dev_alloc(c, bytes, (void**)&p->dev);
  if (st) {
    delete p;
    return st;
  }
  hipError_t e = hipMemcpy(p->dev, blob.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    dev_free(c, p->dev, bytes);
    delete p;
    return fail(BH_EDEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
  }
  c->particles.insert(p);
  handle_add(p, kParticles);
  *out = p;
  return BH_OK;
}

extern "C" bh_status bh_release_particles(bh_particles* p) {
  if (!p) return fail(BH_EINVAL, "NULL particles");
  bh_ctx* c = p->ctx;
  std::lock_guard<std::mutex> g(c->mu);
  if (!c->particles.erase(p)) return fail(BH_ENOTFOUND, "unknown particles");
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();  // launches may still read the records
  dev_free(c, p->dev, p->bytes);
  handle_drop(p);
  delete p;
  return BH_OK;
}

// ---- bloom (Section 3.4.3) -------------------------------------------------------------------

extern "C" bh_status bh_bloom_create(bh_ctx* c, int32_t width, int32_t height, int32_t levels,
                                     bh_bloom** out) {
  if (!c || !out) return fail(BH_EINVAL, "NULL argument");
  if (width < 1 || height < 1 || width > 65536 || height > 65536)
    return fail(BH_EINVAL, "bad image size");
  if (levels < 0 || levels > kBloomMaxLevels) return fail(BH_EINVAL, "levels must be in [0, 16]");
  auto* b = new bh_bloom;
  b->ctx = c;
  b->width = width;
  b->height = height;
  b->levels = levels;
  BloomDev& B = b->B;
  B.w[0] = width;
  B.h[0] = height;
  size_t e = 0;
  for (int k = 1; k <= levels; ++k) {
    B.w[k] = (B.w[k - 1] + 1) / 2;
    B.h[k] = (B.h[k - 1] + 1) / 2;
    B.off[k] = (int64_t)e;
    e += (size_t)B.w[k] * B.h[k];
  }
  B.levels = levels;
  B.tiles_x = (width + 63) / 64;
  B.tiles_y = (height + 63) / 64;
  b->elems = std::max(e, (size_t)1);
  HIPCHK(hipSetDevice(c->device));
  bh_status st = dev_alloc(c, sizeof(float4) * b->elems, (void**)&b->P);
  if (!st) st = dev_alloc(c, sizeof(float4) * b->elems, (void**)&b->U);
  if (st) {
    dev_free(c, b->P, b->P ? sizeof(float4) * b->elems : 0);
    dev_free(c, b->U, b->U ? sizeof(float4) * b->elems : 0);
    delete b;
    return st;
  }
  std::lock_guard<std::mutex> g(c->mu);
  c->blooms.insert(b);
  handle_add(b, kBloom);
  *out = b;
  return BH_OK;
}

static bh_status bloom_weights(const bh_bloom* b, const float* weights, BloomDev& B) {
  B = b->B;
  for (int k = 0; k <= b->levels; ++k) {
    if (!std::isfinite(weights[k])) return fail(BH_EINVAL, "non-finite bloom weight");
    B.wt[k] = weights[k];
  }
  return BH_OK;
}

static bool bad_exposure(float e) { return !(e > 0.0f) || !std::isfinite(e); }

// [a, a + na) and [b, b + nb) share a byte
static bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + nb && y < x + na;
}

extern "C" bh_status bh_bloom_apply(bh_bloom* b, const float* weights, const float* in,
                                    float* out, void* stream) {
  if (!b || !weights || !in || !out) return fail(BH_EINVAL, "NULL argument");
  BloomDev B;
  if (bh_status st = bloom_weights(b, weights, B)) return st;
  HIPCHK(hipSetDevice(b->ctx->device));
  HIPCHK(launch_bloom((const float4*)in, out, b->P, b->U, B, false, 1.0f, (hipStream_t)stream));
  return BH_OK;
}

extern "C" bh_status bh_bloom_apply_display(bh_bloom* b, const float* weights, float exposure,
                                            const float* in, uint32_t* out, void* stream) {
  if (!b || !weights || !in || !out) return fail(BH_EINVAL, "NULL argument");
  if (bad_exposure(exposure)) return fail(BH_EINVAL, "exposure must be finite and > 0");
  const size_t n = (size_t)b->width * b->height;
  if (overlaps(in, 16 * n, out, 4 * n)) return fail(BH_EINVAL, "output overlaps the input");
  BloomDev B;
  if (bh_status st = bloom_weights(b, weights, B)) return st;
  HIPCHK(hipSetDevice(b->ctx->device));
  HIPCHK(launch_bloom((const float4*)in, out, b->P, b->U, B, true, exposure, (hipStream_t)stream));
  return BH_OK;
}

extern "C" bh_status bh_tonemap(bh_ctx* c, const float* in, uint32_t* out, int32_t width,
                                int32_t height, float exposure, void* stream) {
  if (!c || !in || !out) return fail(BH_EINVAL, "NULL argument");
  if (width < 1 || height < 1 || width > 65536 || height > 65536 ||
      (int64_t)width * height > kMaxElems)
    return fail(BH_EINVAL, "bad image size");
  if (bad_exposure(exposure)) return fail(BH_EINVAL, "exposure must be finite and > 0");
  const size_t n = (size_t)width * height;
  if (overlaps(in, 16 * n, out, 4 * n)) return fail(BH_EINVAL, "output overlaps the input");
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(launch_tonemap((const float4*)in, out, (int64_t)n, exposure, (hipStream_t)stream));
  return BH_OK;
}

extern "C" bh_status bh_bloom_release(bh_bloom* b) {
  if (!b) return fail(BH_EINVAL, "NULL bloom");
  bh_ctx* c = b->ctx;
  std::lock_guard<std::mutex> g(c->mu);
  if (!c->blooms.erase(b)) return fail(BH_ENOTFOUND, "unknown bloom");
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();  // launches may still use the pyramid
  dev_free(c, b->P, sizeof(float4) * b->elems);
  dev_free(c, b->U, sizeof(float4) * b->elems);
  handle_drop(b);
  delete b;
  return BH_OK;
}

// ---- stars ---------------------------------------------------------------------------------

static bh_status ensure_cshift(bh_ctx* c, hipStream_t hs);

// (I, T) maps (bands = 0: intensity_dev and temperature_dev) or band-colour maps (bands = 1:
// rgb in intensity_dev, three floats per star, temperature_dev unused)
static bh_status build_stars(bh_ctx* c, const float* dir_xyz_dev, const float* intensity_dev,
                             const float* temperature_dev, int64_t n, int32_t face_size,
                             int32_t texel_format, int bands, void* stream, bh_stars** out) {
  if (!c || !out) return fail(BH_EINVAL, "NULL argument");
  if (n < 0 || (n > 0 && (!dir_xyz_dev || !intensity_dev || (!bands && !temperature_dev))))
    return fail(BH_EINVAL, "bad star arrays");
  if (n >= (int64_t)1 << 31) return fail(BH_EINVAL, "at most 2^31 - 1 stars");
  int n0 = face_size;
  if (n0 < 1 || n0 > 8192 || (n0 & (n0 - 1))) return fail(BH_EINVAL, "face_size must be a power of two <= 8192");
  if (texel_format != BH_TEXEL_FP16 && texel_format != BH_TEXEL_FP32)
    return fail(BH_EINVAL, "bad texel_format");
  HIPCHK(hipSetDevice(c->device));
  hipStream_t hs = (hipStream_t)stream;
  if (bands) {
    bh_status st = ensure_cshift(c, hs);  // band maps are received through the table
    if (st) return st;
  }
  // content hash of the arrays (ordered after the caller's work on the stream)
  uint64_t hash = 0;
  {
    unsigned long long* acc = nullptr;
    bh_status hst = dev_alloc(c, sizeof(unsigned long long), (void**)&acc);
    if (hst) return hst;
    hipError_t e = hipMemsetAsync(acc, 0, sizeof(unsigned long long), hs);
    if (e == hipSuccess)
      e = bands ? launch_star_hash_bands(dir_xyz_dev, intensity_dev, n, acc, hs)
                : launch_star_hash(dir_xyz_dev, intensity_dev, temperature_dev, n, acc, hs);
    unsigned long long h = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, acc, sizeof(h), hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    dev_free(c, acc, sizeof(unsigned long long));
    if (e != hipSuccess) return fail(BH_EDEVICE, std::string("star hash: ") + hipGetErrorString(e));
    hash = h;
  }
  std::lock_guard<std::mutex> g(c->mu);
  StarKey key{hash, n, n0, texel_format, bands};
  auto found = c->stars.find(key);
  if (found != c->stars.end()) {
    found->second->refs++;
    *out = found->second;
    return BH_OK;
  }
  int levels = 0;
  while ((n0 >> levels) >= 1) ++levels;
  std::vector<uint32_t> off(levels), ooff(levels);
  uint64_t total = 0, owords = 0;
  for (int l = 0; l < levels; ++l) {
    off[l] = (uint32_t)total;
    total += 6ull * (n0 >> l) * (n0 >> l);
    ooff[l] = (uint32_t)owords;
    const uint64_t nl = (uint64_t)(n0 >> l);
    owords += 12ull * nl * (((nl + 31) >> 5) + 1);  // every row paired with the next (stars.hip)
  }
  int fp16 = texel_format == BH_TEXEL_FP16;
  const size_t tsz = (fp16 ? 8 : 16) * (bands ? 2 : 1);
  auto* s = new bh_stars;
  s->ctx = c;
  s->key = key;
  s->n0 = n0;
  s->levels = levels;
  s->fp16 = fp16;
  s->bands = bands;
  s->level_off = off;
  s->occ_off = ooff;
  size_t btex = tsz * total, bsc = sizeof(float) * levels, boff = sizeof(uint32_t) * levels;
  size_t bocc = sizeof(uint32_t) * owords;
  bh_status st = dev_alloc(c, btex, &s->tex);
  if (!st) st = dev_alloc(c, bsc, (void**)&s->scale);
  if (!st) st = dev_alloc(c, boff, (void**)&s->level_off_dev);
  if (!st) st = dev_alloc(c, bocc, (void**)&s->occ);
  if (!st) st = dev_alloc(c, boff, (void**)&s->occ_off_dev);
  s->occ_bytes = bocc;
  // build scratch (freed below)
  int64_t ntex0 = 6ll * n0 * n0;
  size_t bhead = sizeof(int) * ntex0, bnext = sizeof(int) * std::max<int64_t>(n, 1),
         bpos = sizeof(float2) * std::max<int64_t>(n, 1),
         bmaster = sizeof(float4) * total * (bands ? 2 : 1), bmax = sizeof(unsigned) * 64;
  int* head = nullptr;
  int* next = nullptr;
  float2* pos = nullptr;
  float4* master = nullptr;
  unsigned* maxbits = nullptr;
  int* bad = nullptr;
  if (!st) st = dev_alloc(c, bhead, (void**)&head);
  if (!st) st = dev_alloc(c, bnext, (void**)&next);
  if (!st) st = dev_alloc(c, bpos, (void**)&pos);
  if (!st) st = dev_alloc(c, bmaster, (void**)&master);
  if (!st) st = dev_alloc(c, bmax, (void**)&maxbits);
  if (!st && bands) st = dev_alloc(c, sizeof(int), (void**)&bad);
  hipError_t e = hipSuccess;
  int hbad = 0;
  if (!st) {
    e = hipMemcpyAsync(s->level_off_dev, off.data(), boff, hipMemcpyHostToDevice, hs);
    if (e == hipSuccess)
      e = hipMemcpyAsync(s->occ_off_dev, ooff.data(), boff, hipMemcpyHostToDevice, hs);
    if (e == hipSuccess) e = launch_fill_int(head, ntex0, -1, hs);
    if (e == hipSuccess) e = launch_fill_int((int*)maxbits, 64, 0, hs);
    if (e == hipSuccess && bands) e = launch_fill_int(bad, 1, 0, hs);
    if (e == hipSuccess)
      e = bands ? launch_star_build_bands(dir_xyz_dev, intensity_dev, n, n0, levels, off.data(),
                                          head, next, pos, master, maxbits, s->scale, fp16,
                                          s->tex, bad, hs)
                : launch_star_build(dir_xyz_dev, intensity_dev, temperature_dev, n, n0, levels,
                                    off.data(), head, next, pos, master, maxbits, s->scale, fp16,
                                    s->tex, hs);
    if (e == hipSuccess)
      e = bands ? launch_star_occupancy_bands(s->tex, n0, levels, off.data(), ooff.data(), fp16,
                                              s->occ, hs)
                : launch_star_occupancy(s->tex, n0, levels, off.data(), ooff.data(), fp16,
                                        s->occ, hs);
    if (e == hipSuccess && bands)
      e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
  }
  dev_free(c, head, head ? bhead : 0);
  dev_free(c, next, next ? bnext : 0);
  dev_free(c, pos, pos ? bpos : 0);
  dev_free(c, master, master ? bmaster : 0);
  dev_free(c, maxbits, maxbits ? bmax : 0);
  dev_free(c, bad, bad ? sizeof(int) : 0);
  if (st || e != hipSuccess || hbad) {
    dev_free(c, s->tex, s->tex ? btex : 0);
    dev_free(c, s->scale, s->scale ? bsc : 0);
    dev_free(c, s->level_off_dev, s->level_off_dev ? boff : 0);
    dev_free(c, s->occ, s->occ ? bocc : 0);
    dev_free(c, s->occ_off_dev, s->occ_off_dev ? boff : 0);
    delete s;
    if (st) return st;
    if (e != hipSuccess)
      return fail(BH_EDEVICE, std::string("star build: ") + hipGetErrorString(e));
    return fail(BH_EINVAL, "star band values must be finite and >= 0");
  }
  s->bytes = btex + bsc + 2 * boff + bocc;
  c->stars[key] = s;
  handle_add(s, kStars);
  *out = s;
  return BH_OK;
}

extern "C" bh_status bh_build_stars(bh_ctx* c, const float* dir_xyz_dev,
                                    const float* intensity_dev, const float* temperature_dev,
                                    int64_t n, int32_t face_size, int32_t texel_format,
                                    void* stream, bh_stars** out) {
  return build_stars(c, dir_xyz_dev, intensity_dev, temperature_dev, n, face_size, texel_format,
                     0, stream, out);
}

extern "C" bh_status bh_build_star_bands(bh_ctx* c, const float* dir_xyz_dev,
                                         const float* rgb_dev, int64_t n, int32_t face_size,
                                         int32_t texel_format, void* stream, bh_stars** out) {
  return build_stars(c, dir_xyz_dev, rgb_dev, nullptr, n, face_size, texel_format, 1, stream,
                     out);
}

extern "C" bh_status bh_stars_download(const bh_stars* s, int32_t level, float* host) {
  if (!s || !host) return fail(BH_EINVAL, "NULL argument");
  if (level < 0 || level >= s->levels) return fail(BH_EINVAL, "bad level");
  bh_ctx* c = s->ctx;
  HIPCHK(hipSetDevice(c->device));
  int64_t cnt = 6ll * (s->n0 >> level) * (s->n0 >> level);
  float scale = 1.0f;
  HIPCHK(hipMemcpy(&scale, s->scale + level, sizeof(float), hipMemcpyDeviceToHost));
  float4* tmp = nullptr;
  const int per = s->bands ? 2 : 1;  // float4 records per texel
  HIPCHK(hipMalloc(&tmp, sizeof(float4) * cnt * per));
  const size_t tsz = (s->fp16 ? 8 : 16) * per;
  const void* lvl = (const char*)s->tex + tsz * s->level_off[level];
  hipError_t e = s->bands ? launch_star_unpack_bands(lvl, cnt, scale, s->fp16, tmp, nullptr)
                          : launch_star_unpack(lvl, cnt, scale, s->fp16, tmp, nullptr);
  if (e == hipSuccess)
    e = hipMemcpy(host, tmp, sizeof(float4) * cnt * per, hipMemcpyDeviceToHost);
  (void)hipFree(tmp);
  if (e != hipSuccess) return fail(BH_EDEVICE, hipGetErrorString(e));
  return BH_OK;
}

extern "C" bh_status bh_release_stars(bh_stars* s) {
  if (!s) return fail(BH_EINVAL, "NULL stars");
  bh_ctx* c = s->ctx;
  std::lock_guard<std::mutex> g(c->mu);
  if (--s->refs > 0) return BH_OK;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  c->stars.erase(s->key);
  const size_t tsz = (s->fp16 ? 8 : 16) * (s->bands ? 2 : 1);
  uint64_t total = 0;
  for (int l = 0; l < s->levels; ++l) total += 6ull * (s->n0 >> l) * (s->n0 >> l);
  dev_free(c, s->tex, tsz * total);
  dev_free(c, s->scale, sizeof(float) * s->levels);
  dev_free(c, s->level_off_dev, sizeof(uint32_t) * s->levels);
  dev_free(c, s->occ, s->occ_bytes);
  dev_free(c, s->occ_off_dev, sizeof(uint32_t) * s->levels);
  handle_drop(s);
  delete s;
  return BH_OK;
}

// ---- area sources ----------------------------------------------------------------------------

// 8-point Gauss-Legendre rule on [-1, 1]: the roots of P_8 by Newton's method from
// x = cos(pi (i + 3/4) / (n + 1/2)), weights 2 / ((1 - x^2) P_8'(x)^2)
static CshiftRule gauss_legendre8() {
  CshiftRule q;
  const int n = 8;
  for (int i = 0; i < n; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    q.x[i] = x;
    q.w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  return q;
}

// the colour-shift table of this context, built on first use (the caller holds no lock)
static bh_status ensure_cshift(bh_ctx* c, hipStream_t hs) {
  static std::mutex build_mu;  // one build at a time; later callers find it done
  std::lock_guard<std::mutex> lk(build_mu);
  {
    std::lock_guard<std::mutex> g(c->mu);
    if (c->ctab) return BH_OK;
  }
  const size_t bt = sizeof(float4) * kCshiftN * kCshiftN * kCshiftN;
  const size_t bs = sizeof(double4) * kCshiftN * kCshiftN;
  float4* tab = nullptr;
  double4* spec = nullptr;
  bh_status st = dev_alloc(c, bt, (void**)&tab);
  if (!st) st = dev_alloc(c, bs, (void**)&spec);
  hipError_t e = hipSuccess;
  if (!st) {
    e = launch_cshift_build(gauss_legendre8(), spec, tab, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
  }
  dev_free(c, spec, spec ? bs : 0);
  if (st || e != hipSuccess) {
    dev_free(c, tab, tab ? bt : 0);
    if (st) return st;
    return fail(BH_EDEVICE, std::string("colour-shift table: ") + hipGetErrorString(e));
  }
  std::lock_guard<std::mutex> g(c->mu);
  c->ctab = tab;
  return BH_OK;
}

static bh_status build_area(bh_ctx* c, const float* texels, int32_t n0, int bands, void* stream,
                            bh_area** out) {
  if (!c || !texels || !out) return fail(BH_EINVAL, "NULL argument");
  if (n0 < 1 || n0 > 4096 || (n0 & (n0 - 1)))
    return fail(BH_EINVAL, "face_size must be a power of two <= 4096");
  HIPCHK(hipSetDevice(c->device));
  hipStream_t hs = (hipStream_t)stream;
  if (bands) {
    bh_status st = ensure_cshift(c, hs);
    if (st) return st;
  }
  int levels = 0;
  while ((n0 >> levels) >= 1) ++levels;
  const size_t texels_all = 8ull * n0 * n0 - 2;  // 6 (n0^2 + (n0/2)^2 + ... + 1)
  auto* a = new bh_area;
  a->ctx = c;
  a->n0 = n0;
  a->levels = levels;
  a->bands = bands;
  a->bytes = (bands ? sizeof(float4) : sizeof(float2)) * texels_all;
  int* bad = nullptr;
  bh_status st = dev_alloc(c, a->bytes, &a->tex);
  if (!st) st = dev_alloc(c, sizeof(int), (void**)&bad);
  hipError_t e = hipSuccess;
  int hbad = 0;
  if (!st) {
    e = launch_fill_int(bad, 1, 0, hs);
    if (e == hipSuccess)
      e = bands ? launch_area_build_bands(texels, n0, (float4*)a->tex, bad, hs)
                : launch_area_build(texels, n0, (float2*)a->tex, bad, hs);
    if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
  }
  dev_free(c, bad, bad ? sizeof(int) : 0);
  if (st || e != hipSuccess || hbad) {
    dev_free(c, a->tex, a->tex ? a->bytes : 0);
    delete a;
    if (st) return st;
    if (e != hipSuccess) return fail(BH_EDEVICE, std::string("area build: ") + hipGetErrorString(e));
    return fail(BH_EINVAL, bands ? "band texels must be finite and >= 0"
                                 : "area texels must be finite with I >= 0 and T >= 0");
  }
  std::lock_guard<std::mutex> g(c->mu);
  c->areas.insert(a);
  handle_add(a, kArea);
  *out = a;
  return BH_OK;
}

extern "C" bh_status bh_build_area(bh_ctx* c, const float* texels, int32_t n0, void* stream,
                                   bh_area** out) {
  return build_area(c, texels, n0, 0, stream, out);
}

extern "C" bh_status bh_build_area_bands(bh_ctx* c, const float* rgbx, int32_t n0, void* stream,
                                         bh_area** out) {
  return build_area(c, rgbx, n0, 1, stream, out);
}

extern "C" bh_status bh_color_shift_table_download(bh_ctx* c, float* host) {
  if (!c || !host) return fail(BH_EINVAL, "NULL argument");
  HIPCHK(hipSetDevice(c->device));
  bh_status st = ensure_cshift(c, nullptr);
  if (st) return st;
  HIPCHK(hipMemcpy(host, c->ctab, sizeof(float4) * kCshiftN * kCshiftN * kCshiftN,
                   hipMemcpyDeviceToHost));
  return BH_OK;
}

extern "C" bh_status bh_area_download(const bh_area* a, int32_t level, float* host) {
  if (!a || !host) return fail(BH_EINVAL, "NULL argument");
  if (level < 0 || level >= a->levels) return fail(BH_EINVAL, "bad level");
  HIPCHK(hipSetDevice(a->ctx->device));
  const int64_t n0 = a->n0, nl = n0 >> level;
  const int64_t off = 8 * (n0 * n0 - nl * nl);
  const size_t tsz = a->bands ? sizeof(float4) : sizeof(float2);
  HIPCHK(hipMemcpy(host, (const char*)a->tex + tsz * off, tsz * 6 * nl * nl,
                   hipMemcpyDeviceToHost));
  return BH_OK;
}

extern "C" bh_status bh_release_area(bh_area* a) {
  if (!a) return fail(BH_EINVAL, "NULL area");
  bh_ctx* c = a->ctx;
  std::lock_guard<std::mutex> g(c->mu);
  if (!c->areas.erase(a)) return fail(BH_EINVAL, "unknown area map");
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  dev_free(c, a->tex, a->bytes);
  handle_drop(a);
  delete a;
  return BH_OK;
}

extern "C" bh_status bh_release(void* h) {
  HandleKind k;
  {
    std::lock_guard<std::mutex> g(g_handles_mu);
    auto it = g_handles.find(h);
    if (it == g_handles.end()) return fail(BH_EINVAL, "not a live handle");
    k = it->second;
  }
  switch (k) {
    case kTables: return bh_release_tables((bh_tables*)h);
    case kStars: return bh_release_stars((bh_stars*)h);
    case kParticles: return bh_release_particles((bh_particles*)h);
    case kBloom: return bh_bloom_release((bh_bloom*)h);
    case kArea: return bh_release_area((bh_area*)h);
  }
  return fail(BH_EINVAL, "not a live handle");
}

// ---- views ---------------------------------------------------------------------------------

static bool finite_all(const double* p, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// Validate a view and build its constant block in FP64 (Section 3.2, Appendix C: the
// camera basis is O B(v) R; here O is given directly as cam_rot in the boosted frame).
static bh_status make_view(const bh_view* v, float* out, float* aov, ViewDev* o) {
  if (!v) return fail(BH_EINVAL, "NULL view");
  double sc[] = {v->r_s, v->fov_y, v->disc_r_in, v->disc_r_out, v->disc_T0, v->disc_T_exp,
                 v->disc_opacity, v->k_disc, v->k_star};
  if (!finite_all(sc, 9) || !finite_all(v->cam_pos, 3) || !finite_all(v->cam_vel, 3) ||
      !finite_all(v->cam_rot, 9))
    return fail(BH_EINVAL, "non-finite view parameter");
  if (!(v->r_s > 0)) return fail(BH_EINVAL, "r_s must be > 0");
  double r = std::sqrt(v->cam_pos[0] * v->cam_pos[0] + v->cam_pos[1] * v->cam_pos[1] +
                       v->cam_pos[2] * v->cam_pos[2]) / v->r_s;
  if (!(r > 1.0)) return fail(BH_EINVAL, "camera must be outside the horizon (|cam_pos| > r_s)");
  double vm = std::sqrt(v->cam_vel[0] * v->cam_vel[0] + v->cam_vel[1] * v->cam_vel[1] +
                        v->cam_vel[2] * v->cam_vel[2]);
  if (!(vm < 1.0)) return fail(BH_EINVAL, "camera speed must be < c");
  if (!(v->fov_y > 0 && v->fov_y < M_PI)) return fail(BH_EINVAL, "fov_y must be in (0, pi)");
  if (v->width < 1 || v->height < 1 || v->width > 65536 || v->height > 65536 ||
      (int64_t)v->width * v->height > kMaxElems)
    return fail(BH_EINVAL, "bad image size");
  if (!(v->disc_r_in >= 3.0 * v->r_s * (1.0 - 1e-12)))
    return fail(BH_EINVAL, "disc_r_in must be >= 3 r_s (innermost stable circular orbit)");
  if (!(v->disc_r_out > v->disc_r_in)) return fail(BH_EINVAL, "disc_r_out must exceed disc_r_in");
  if (!(v->disc_opacity >= 0 && v->disc_opacity <= 1)) return fail(BH_EINVAL, "opacity must be in [0,1]");
  if (v->disc_T_law != BH_T_POWER && v->disc_T_law != BH_T_PAPER) return fail(BH_EINVAL, "bad T law");
  if (!(v->disc_T0 >= 0)) return fail(BH_EINVAL, "disc_T0 must be >= 0");
  if (v->disc_density != BH_DENSITY_UNIFORM && v->disc_density != BH_DENSITY_PARTICLES)
    return fail(BH_EINVAL, "bad disc_density");
  if (v->disc_density == BH_DENSITY_PARTICLES && (!v->particles || !std::isfinite(v->time)))
    return fail(BH_EINVAL, "a particle disc needs particles and a finite time");
  if (v->area && !std::isfinite(v->k_area)) return fail(BH_EINVAL, "k_area must be finite");
  const double* R = v->cam_rot;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double d = R[3 * i] * R[3 * j] + R[3 * i + 1] * R[3 * j + 1] + R[3 * i + 2] * R[3 * j + 2];
      if (std::fabs(d - (i == j ? 1.0 : 0.0)) > 1e-6) return fail(BH_EINVAL, "cam_rot is not orthonormal");
    }
  if (!out) return fail(BH_EINVAL, "NULL output");
  memset(o, 0, sizeof(*o));
  double u = 1.0 / r;
  double rh[3], vh[3];
  for (int i = 0; i < 3; ++i) {
    rh[i] = v->cam_pos[i] / (r * v->r_s);
    vh[i] = vm > 0 ? v->cam_vel[i] / vm : 0.0;
  }
  // a vector's radial component and its part transverse to rh, in FP64
  auto split = [&](const double* w, float* perp, float* radial) {
    const double c = w[0] * rh[0] + w[1] * rh[1] + w[2] * rh[2];
    for (int i = 0; i < 3; ++i) perp[i] = (float)(w[i] - c * rh[i]);
    *radial = (float)c;
  };
  split(R, o->ew, &o->er[0]);
  split(R + 3, o->eh, &o->er[1]);
  split(R + 6, o->ed, &o->er[2]);
  split(vh, o->vhat, &o->er[3]);
  for (int i = 0; i < 3; ++i) o->rhat[i] = (float)rh[i];
  o->sq1mu = (float)std::sqrt(1.0 - u);
  o->inv_sq1mu = (float)(1.0 / std::sqrt(1.0 - u));
  o->u_c = (float)u;
  o->f = (float)(0.5 * v->height / std::tan(0.5 * v->fov_y));
  o->gamma = (float)(1.0 / std::sqrt(1.0 - vm * vm));
  o->vmag = (float)vm;
  o->half_w = (float)(0.5 * v->width);
  o->half_h = (float)(0.5 * v->height);
  o->u_ic = (float)(v->r_s / v->disc_r_in);
  o->u_oc = (float)(v->r_s / v->disc_r_out);
  o->T0 = (float)v->disc_T0;
  o->T_exp = (float)v->disc_T_exp;
  o->T_law = v->disc_T_law;
  double pk = 6.0 / 7.0;  // maximum of s^6 (1 - s) / 27 at s = sqrt(3u) = 6/7
  o->T_norm = (float)(27.0 / (std::pow(pk, 6) * (1.0 - pk)));
  o->rho = (float)v->disc_opacity;
  o->k_disc = (float)v->k_disc;
  o->k_star = (float)v->k_star;
  o->width = v->width;
  o->height = v->height;
  if (v->disc_density == BH_DENSITY_PARTICLES) {
    o->density_mode = 1;
    o->time = (float)v->time;
    o->nparts = v->particles->n;
    o->parts = v->particles->dev;
    o->pstart = (const int*)(v->particles->dev + 2 * (size_t)std::max(v->particles->n, 1));
    o->pscale = v->particles->scale;
    o->pbins = kPartBins;
  }
  if (v->stars) {
    const bh_stars* s = v->stars;
    o->has_stars = 1;
    o->stars.tex = s->tex;
    o->stars.scale = s->scale;
    o->stars.level_off = s->level_off_dev;
    o->stars.occ = s->occ;
    o->stars.occ_off = s->occ_off_dev;
    o->stars.n0 = s->n0;
    o->stars.levels = s->levels;
    o->stars.fp16 = s->fp16;
    o->stars.one = 1.0f;
    o->stars.tw0 = 2.0f / (float)s->n0;
    o->stars.bands = s->bands;
    o->stars.ctab = s->bands ? s->ctx->ctab : nullptr;
  }
  if (v->area) {
    o->area.tex = v->area->tex;
    o->area.n0 = v->area->n0;
    o->area.levels = v->area->levels;
    o->area.k_area = (float)v->k_area;
    o->area.bands = v->area->bands;
    o->area.ctab = v->area->bands ? v->area->ctx->ctab : nullptr;
  }
  o->out = (float4*)out;
  o->aov = (float4*)aov;
  return BH_OK;
}

static TablesDev tables_dev(const bh_tables* t) {
  TablesDev T;
  T.D = t->D;
  T.U = t->U;
  T.Dt = t->Dt;
  T.Ut = t->Ut;
  T.d_n = t->p.d_n;
  T.u_ne = t->p.u_ne;
  T.u_nphi = t->p.u_nphi;
  T.pad = 0;
  return T;
}

static LutDev lut_dev(const bh_ctx* c) {
  LutDev L;
  L.lut = c->lut;
  L.n = c->lut_n;
  L.x0 = c->lut_x0;
  L.inv_dx = 1.0f / c->lut_dx;
  L.pad = 0;
  return L;
}

extern "C" bh_status bh_render(bh_ctx* c, const bh_tables* t, const bh_view* v, float* out,
                               float* aov, void* stream) {
  if (!c || !t) return fail(BH_EINVAL, "NULL context or tables");
  ViewDev vd;
  bh_status st = make_view(v, out, aov, &vd);
  if (st) return st;
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(launch_render(c->tile_cfg, vd, tables_dev(t), lut_dev(c), (hipStream_t)stream));
  return BH_OK;
}

// Ray marching in place of TraceRay (the ablation of Section 5): h = 2 pi / max_steps.
static bh_status check_march_steps(int32_t max_steps) {
  if (max_steps < 3 || max_steps > (1 << 20))
    return fail(BH_EINVAL, "max_steps must be in [3, 1048576]");
  return BH_OK;
}

extern "C" bh_status bh_render_march(bh_ctx* c, const bh_view* v, int32_t max_steps,
                                     float* out, float* aov, void* stream) {
  if (!c) return fail(BH_EINVAL, "NULL context");
  bh_status st = check_march_steps(max_steps);
  if (st) return st;
  ViewDev vd;
  st = make_view(v, out, aov, &vd);
  if (st) return st;
  if (vd.density_mode != 0)
    return fail(BH_EINVAL, "ray marching carries no time channels: the disc must be uniform");
  vd.march_steps = max_steps;
  vd.march_h = (float)(2.0 * M_PI / max_steps);
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(launch_render_march(vd, lut_dev(c), (hipStream_t)stream));
  return BH_OK;
}

// ---- batched launches ------------------------------------------------------------------------

extern "C" int32_t bh_tile_config_count(void) { return tile_config_count(); }

extern "C" bh_status bh_tile_config_get(int32_t i, bh_tile_config* o) {
  if (!o || i < 0 || i >= tile_config_count()) return fail(BH_EINVAL, "bad tile config index");
  tile_config(i, &o->tile_w, &o->tile_h, &o->waves, &o->ppt);
  return BH_OK;
}

extern "C" bh_status bh_set_tile_config(bh_ctx* c, int32_t i) {
  if (!c || i < -1 || i >= tile_config_count()) return fail(BH_EINVAL, "bad tile config index");
  std::lock_guard<std::mutex> g(c->mu);
  c->tile_cfg = i < 0 ? kDefaultTileCfg : i;
  return BH_OK;
}

extern "C" bh_status bh_set_batch_form(bh_ctx* c, int32_t persistent) {
  if (!c || (persistent != 0 && persistent != 1)) return fail(BH_EINVAL, "persistent must be 0 or 1");
  std::lock_guard<std::mutex> g(c->mu);
  c->persistent = persistent;
  return BH_OK;
}

// Workgroups (of 4 waves, each claiming tiles on its own) of a persistent batched launch:
// as many as fit at the kernel's 7 resident waves per SIMD, 4 SIMDs per CU (k_render_batch);
// fewer when the launch has fewer tiles than waves.
static int batch_grid(const bh_ctx* c, int cfg, int64_t ntiles) {
  (void)cfg;
  return (int)std::max<int64_t>(1, std::min<int64_t>((ntiles + 3) / 4, (int64_t)c->cus * 7));
}

// Upload view blocks and tile runs through a pinned staging buffer and enqueue one batched
// launch over `ntiles` tiles on stream s.  With a copy stream `cs`, the uploads run there
// (after `slot_free`, the end of the last launch that read dviews/druns) and s waits for
// them through `copied`, so they overlap the kernels already queued on s.  Caller holds
// c->mu.
static bh_status enqueue_batch(bh_ctx* c, int cfg, int pers, const TablesDev& T,
                               const std::vector<ViewDev>& vds,
                               const std::vector<TileRun>& runs, int ntiles, ViewDev* dviews,
                               TileRun* druns, int* counter, Staging& stg, hipStream_t s,
                               bool use_graph, hipStream_t cs = nullptr,
                               hipEvent_t slot_free = nullptr, hipEvent_t copied = nullptr) {
  size_t bv = sizeof(ViewDev) * vds.size(), br = sizeof(TileRun) * runs.size();
  bh_status st = ensure_staging(stg, bv + br);
  if (st) return st;
  if (stg.used) HIPCHK(hipEventSynchronize(stg.done));
  hipStream_t up = cs ? cs : s;
  if (cs && slot_free) HIPCHK(hipStreamWaitEvent(cs, slot_free, 0));
  memcpy(stg.host, vds.data(), bv);
  memcpy((char*)stg.host + bv, runs.data(), br);
  HIPCHK(hipMemcpyAsync(dviews, stg.host, bv, hipMemcpyHostToDevice, up));
  HIPCHK(hipMemcpyAsync(druns, (char*)stg.host + bv, br, hipMemcpyHostToDevice, up));
  HIPCHK(hipEventRecord(stg.done, up));
  stg.used = true;
  if (cs) {
    HIPCHK(hipEventRecord(copied, cs));
    HIPCHK(hipStreamWaitEvent(s, copied, 0));
  }
  int grid = batch_grid(c, cfg, ntiles);
  int nruns = (int)runs.size();
  int feat = 0;  // the union of the views' features selects the kernel
  for (const ViewDev& vd : vds) feat |= view_features(vd);
  LutDev L = lut_dev(c);
  if (!use_graph) {
    HIPCHK(launch_render_batch(cfg, pers, feat, dviews, druns, nruns, ntiles, counter, T, L,
                               grid, s));
    return BH_OK;
  }
  bh_ctx::GraphKey key{(cfg * 2 + pers) * 8 + feat, ntiles, nruns, grid, (uintptr_t)counter,
                       (const void*)T.D, (const void*)T.U, (const void*)T.Dt, (const void*)T.Ut,
                       T.d_n, T.u_ne, T.u_nphi};
  auto it = c->graphs.find(key);
  if (it == c->graphs.end()) {
    hipStream_t cap;
    HIPCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t graph;
    HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = launch_render_batch(cfg, pers, feat, dviews, druns, nruns, ntiles, counter,
                                       T, L, grid, cap);
    hipError_t e2 = hipStreamEndCapture(cap, &graph);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess || e2 != hipSuccess)
      return fail(BH_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    hipGraphExec_t exec;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(BH_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    it = c->graphs.emplace(key, bh_ctx::GraphEntry{exec, s}).first;
  }
  HIPCHK(hipGraphLaunch(it->second.exec, s));
  return BH_OK;
}

static void clear_graphs(bh_ctx* c) {
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second.exec);
  c->graphs.clear();
}

static bh_status ensure_batch_buffers(bh_ctx* c, size_t nviews) {
  if (c->b_cap >= nviews) return BH_OK;
  // captured graphs hold the old buffer addresses
  if (c->b_last) HIPCHK(hipEventSynchronize(c->b_last));
  clear_graphs(c);
  dev_free(c, c->b_views, sizeof(ViewDev) * c->b_cap);
  dev_free(c, c->b_runs, sizeof(TileRun) * c->b_cap);
  c->b_views = nullptr;
  c->b_runs = nullptr;
  c->b_cap = 0;
  size_t cap = std::max<size_t>(nviews, 64);
  bh_status st = dev_alloc(c, sizeof(ViewDev) * cap, (void**)&c->b_views);
  if (st) return st;
  st = dev_alloc(c, sizeof(TileRun) * cap, (void**)&c->b_runs);
  if (st) {
    dev_free(c, c->b_views, sizeof(ViewDev) * cap);
    c->b_views = nullptr;
    return st;
  }
  c->b_cap = cap;
  return BH_OK;
}

extern "C" bh_status bh_render_batch(bh_ctx* c, const bh_tables* t, const bh_view* views,
                                     int32_t n, float* const* outs, void* stream) {
  if (!c || !t || !views || !outs || n < 1) return fail(BH_EINVAL, "bad batch arguments");
  std::vector<ViewDev> vds(n);
  for (int i = 0; i < n; ++i) {
    bh_status st = make_view(&views[i], outs[i], nullptr, &vds[i]);
    if (st) return fail(st, "view " + std::to_string(i) + ": " + g_err);
  }
  HIPCHK(hipSetDevice(c->device));
  std::lock_guard<std::mutex> g(c->mu);
  int tw, th, waves, ppt;
  tile_config(c->tile_cfg, &tw, &th, &waves, &ppt);
  // largest views first so the persistent workgroups end together
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return (int64_t)views[a].width * views[a].height > (int64_t)views[b].width * views[b].height;
  });
  std::vector<TileRun> runs;
  int64_t ntiles = 0;
  for (int i : order) {
    int tx = (views[i].width + tw - 1) / tw, ty = (views[i].height + th - 1) / th;
    runs.push_back(TileRun{i, 0, (int)ntiles, tx});
    ntiles += (int64_t)tx * ty;
    // the one-workgroup-per-tile launch runs ntiles x (tile pixels / ppt) work-items
    if (ntiles * tw * th > kMaxElems * 2 - 1)
      return fail(BH_EINVAL, "batch too large: more than 2^32 - 1 pixels in its tiles");
  }
  bh_status st = ensure_batch_buffers(c, n);
  if (st) return st;
  Staging& stg = c->b_stage[c->b_next_stage];
  c->b_next_stage ^= 1;
  hipStream_t s = (hipStream_t)stream;
  // the view/work buffers are shared by every batched call on this context: order this
  // call after the previous one even when it was issued on another stream
  if (!c->b_last) HIPCHK(hipEventCreateWithFlags(&c->b_last, hipEventDisableTiming));
  else HIPCHK(hipStreamWaitEvent(s, c->b_last, 0));
  st = enqueue_batch(c, c->tile_cfg, c->persistent, tables_dev(t), vds, runs, (int)ntiles,
                     c->b_views, c->b_runs, c->b_counter, stg, s, true);
  if (st) return st;
  HIPCHK(hipEventRecord(c->b_last, s));
  return BH_OK;
}

// The allocation-free form of bh_render_batch: records in the library's scratch array,
// staged through the context's pinned buffer, kernels launched directly.  Calls no device
// or pinned allocation (the scratch address and the staging buffer come from bh_create).
extern "C" bh_status bh_render_batch_noalloc(bh_ctx* c, const bh_tables* t, const bh_view* views,
                                             int32_t n, float* const* outs, void* stream) {
  if (!c || !t || !views || !outs || n < 1) return fail(BH_EINVAL, "bad batch arguments");
  if (n > BH_NOALLOC_MAX_VIEWS)
    return fail(BH_EINVAL, "at most " + std::to_string(BH_NOALLOC_MAX_VIEWS) + " views per call");
  HIPCHK(hipSetDevice(c->device));
  std::lock_guard<std::mutex> g(c->mu);
  Staging& stg = c->na_stage;
  // the previous call's upload out of the staging buffer must have happened
  if (stg.used) HIPCHK(hipEventSynchronize(stg.done));
  ViewDev* hv = (ViewDev*)stg.host;
  TileRun* hr = (TileRun*)(hv + BH_NOALLOC_MAX_VIEWS);
  int* order = (int*)(hr + BH_NOALLOC_MAX_VIEWS);
  for (int i = 0; i < n; ++i) {
    bh_status st = make_view(&views[i], outs[i], nullptr, &hv[i]);
    if (st) return fail(st, "view " + std::to_string(i) + ": " + g_err);
  }
  const int cfg = c->tile_cfg;
  int tw, th, waves, ppt;
  tile_config(cfg, &tw, &th, &waves, &ppt);
  // largest views first (ties by index, as bh_render_batch orders them)
  for (int i = 0; i < n; ++i) order[i] = i;
  std::sort(order, order + n, [&](int a, int b) {
    const int64_t pa = (int64_t)views[a].width * views[a].height;
    const int64_t pb = (int64_t)views[b].width * views[b].height;
    return pa != pb ? pa > pb : a < b;
  });
  int64_t ntiles = 0;
  for (int k = 0; k < n; ++k) {
    const int i = order[k];
    const int tx = (views[i].width + tw - 1) / tw, ty = (views[i].height + th - 1) / th;
    hr[k] = TileRun{i, 0, (int)ntiles, tx};
    ntiles += (int64_t)tx * ty;
    if (ntiles * tw * th > kMaxElems * 2 - 1)
      return fail(BH_EINVAL, "batch too large: more than 2^32 - 1 pixels in its tiles");
  }
  hipStream_t s = (hipStream_t)stream;
  int* dcounter = (int*)c->scratch;
  ViewDev* dviews = (ViewDev*)((char*)c->scratch + 256);
  TileRun* druns = (TileRun*)(dviews + BH_NOALLOC_MAX_VIEWS);
  HIPCHK(hipMemcpyAsync(dviews, hv, sizeof(ViewDev) * n, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(druns, hr, sizeof(TileRun) * n, hipMemcpyHostToDevice, s));
  HIPCHK(hipEventRecord(stg.done, s));
  stg.used = true;
  int feat = 0;
  for (int i = 0; i < n; ++i) feat |= view_features(hv[i]);
  HIPCHK(launch_render_batch(cfg, c->persistent, feat, dviews, druns, n, (int)ntiles, dcounter,
                             tables_dev(t), lut_dev(c), batch_grid(c, cfg, ntiles), s));
  return BH_OK;
}

extern "C" bh_status bh_autotune(bh_ctx* c, const bh_tables* t, const bh_view* views, int32_t n,
                                 float* const* outs, int32_t reps, int32_t* best,
                                 float* ms_per_config) {
  if (!c || !t || !views || !outs || n < 1 || reps < 1) return fail(BH_EINVAL, "bad autotune arguments");
  HIPCHK(hipSetDevice(c->device));
  hipStream_t s;
  HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  int nc = tile_config_count(), bi = 0, bp = 0;
  float bms = 1e30f;
  bh_status st = BH_OK;
  for (int kk = 0; kk < 2 * nc && !st; ++kk) {
    int k = kk >> 1, pers = kk & 1;
    st = bh_set_tile_config(c, k);
    {
      std::lock_guard<std::mutex> g(c->mu);
      c->persistent = pers;
    }
    if (!st) st = bh_render_batch(c, t, views, n, outs, s);  // warm-up and graph build
    if (st) break;
    HIPCHK(hipEventRecord(e0, s));
    for (int r = 0; r < reps && !st; ++r) st = bh_render_batch(c, t, views, n, outs, s);
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    ms /= reps;
    if (ms_per_config) ms_per_config[kk] = ms;
    if (ms < bms) {
      bms = ms;
      bi = k;
      bp = pers;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  if (st) return st;
  bh_set_tile_config(c, bi);
  {
    std::lock_guard<std::mutex> g(c->mu);
    c->persistent = bp;
  }
  if (best) *best = 2 * bi + bp;
  return BH_OK;
}

// ---- unit-level entry points -------------------------------------------------------------------

extern "C" bh_status bh_trace_rays(bh_ctx* c, const bh_tables* t, const float* rays, int64_t n,
                                   float* out, void* stream) {
  if (!c || !t || (n > 0 && (!rays || !out)) || n < 0 || n > kMaxElems)
    return fail(BH_EINVAL, "bad arguments");
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(launch_trace_rays(tables_dev(t), rays, n, (float4*)out, nullptr, (hipStream_t)stream));
  return BH_OK;
}

extern "C" bh_status bh_march_rays(bh_ctx* c, const float* rays, int64_t n, int32_t max_steps,
                                   float* out, void* stream) {
  if (!c || (n > 0 && (!rays || !out)) || n < 0 || n > kMaxElems)
    return fail(BH_EINVAL, "bad arguments");
  bh_status st = check_march_steps(max_steps);
  if (st) return st;
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(launch_march_rays(rays, n, max_steps, (float)(2.0 * M_PI / max_steps), (float4*)out,
                           (hipStream_t)stream));
  return BH_OK;
}

extern "C" bh_status bh_trace_rays_timed(bh_ctx* c, const bh_tables* t, const float* rays,
                                         int64_t n, float* out, float* out_time, void* stream) {
  if (!c || !t || (n > 0 && (!rays || !out || !out_time)) || n < 0 || n > kMaxElems)
    return fail(BH_EINVAL, "bad arguments");
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(launch_trace_rays(tables_dev(t), rays, n, (float4*)out, (float4*)out_time,
                           (hipStream_t)stream));
  return BH_OK;
}

extern "C" bh_status bh_footprint_texels(bh_ctx* c, const bh_tables* t, const bh_view* v,
                                         float* out, uint64_t* texels, uint64_t* req_bytes) {
  if (!c || !t || !texels) return fail(BH_EINVAL, "NULL argument");
  if (!v || !v->stars) return fail(BH_EINVAL, "view without a star map");
  if (v->stars->bands) return fail(BH_EINVAL, "footprint counting reads (I, T) star maps only");
  ViewDev vd;
  bh_status st = make_view(v, out, nullptr, &vd);
  if (st) return st;
  HIPCHK(hipSetDevice(c->device));
  const bh_stars* s = v->stars;
  uint64_t total = 0;
  for (int l = 0; l < s->levels; ++l) total += 6ull * (s->n0 >> l) * (s->n0 >> l);
  int64_t words = (int64_t)((total + 31) / 32);
  uint32_t* bits = nullptr;
  unsigned long long* cnt = nullptr;  // [0] distinct texels, [1] requested bytes
  HIPCHK(hipMalloc(&bits, sizeof(uint32_t) * words));
  hipError_t e = hipMalloc(&cnt, 2 * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMemset(bits, 0, sizeof(uint32_t) * words);
  if (e == hipSuccess) e = hipMemset(cnt, 0, 2 * sizeof(unsigned long long));
  if (e == hipSuccess)
    e = launch_render_count(vd, tables_dev(t), lut_dev(c), bits, words, cnt, cnt + 1, nullptr);
  unsigned long long h[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpy(h, cnt, sizeof(h), hipMemcpyDeviceToHost);
  (void)hipFree(bits);
  if (cnt) (void)hipFree(cnt);
  if (e != hipSuccess) return fail(BH_EDEVICE, std::string("footprint count: ") + hipGetErrorString(e));
  *texels = h[0];
  if (req_bytes) *req_bytes = h[1];
  return BH_OK;
}

extern "C" bh_status bh_probe_l2_read(bh_ctx* c, int64_t window_bytes, int32_t reps,
                                      double* bytes_per_s) {
  if (!c || !bytes_per_s || reps < 1 || window_bytes < 4096 || window_bytes > (4 << 20) ||
      (window_bytes & (window_bytes - 1)))
    return fail(BH_EINVAL, "window_bytes must be a power of two in [4 KiB, 4 MiB], reps >= 1");
  HIPCHK(hipSetDevice(c->device));
  const int64_t n4 = window_bytes / 16;
  const int per_wg = 16384;          // 256 KiB per workgroup
  const int grid = c->cus * 8;       // 8 workgroups of 4 waves per CU
  float4* buf = nullptr;
  float* sink = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&buf, window_bytes);
  if (e == hipSuccess) e = hipMalloc(&sink, sizeof(float) * grid);
  if (e == hipSuccess) e = hipMemset(buf, 0, window_bytes);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  for (int w = 0; w < 3 && e == hipSuccess; ++w)  // bring the window into every L2
    e = launch_l2_read(buf, n4, per_wg, grid, sink, nullptr);
  if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_l2_read(buf, n4, per_wg, grid, sink, nullptr);
  if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (buf) (void)hipFree(buf);
  if (sink) (void)hipFree(sink);
  if (e != hipSuccess) return fail(BH_EDEVICE, std::string("L2 probe: ") + hipGetErrorString(e));
  *bytes_per_s = 16.0 * per_wg * (double)grid * reps / (ms * 1e-3);
  return BH_OK;
}

extern "C" bh_status bh_band_table_info(const bh_ctx* c, int32_t* n, float* x0, float* dx) {
  if (!c || !n || !x0 || !dx) return fail(BH_EINVAL, "NULL argument");
  *n = c->lut_n;
  *x0 = c->lut_x0;
  *dx = c->lut_dx;
  return BH_OK;
}

extern "C" bh_status bh_band_table_download(const bh_ctx* c, float* host) {
  if (!c || !host) return fail(BH_EINVAL, "NULL argument");
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipMemcpy(host, c->lut, sizeof(float4) * c->lut_n, hipMemcpyDeviceToHost));
  return BH_OK;
}

extern "C" bh_status bh_band_eval(bh_ctx* c, const float* temps, int64_t n, float* out,
                                  void* stream) {
  if (!c || n < 0 || n > kMaxElems || (n > 0 && (!temps || !out)))
    return fail(BH_EINVAL, "bad arguments");
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(launch_band_eval(lut_dev(c), temps, n, out, (hipStream_t)stream));
  return BH_OK;
}

// ---- serving ---------------------------------------------------------------------------------
// The policy (admission by budget, continuous batching, failure and cancellation) is the
// scheduler of bh_sched.h, run on its own thread; this is its HIP backend.  Launches go to
// the serving stream through maxin + 1 slots of device records (view blocks, tile runs,
// a claim counter), uploaded on a copy stream after the slot's previous launch; a launch is
// in flight until an event recorded after it completes.  Library images come from a
// stream-ordered memory pool on the serving stream, inside the context's HBM budget.
struct ServePayload {
  bh_view view;
  const bh_tables* tables;
};

struct ServeBackend {
  using Payload = ServePayload;
  struct Handle {
    hipEvent_t ev = nullptr;
  };
  using Pieces = std::vector<sched::Piece<Payload>>;

  bh_ctx* c;
  int cfg = 0, pers = 0;         // tile configuration and launch form, fixed at start
  int tw = 16, th = 16;
  int slots = 0, slot = 0;
  hipStream_t stream = nullptr, copy_stream = nullptr;
  hipMemPool_t img_pool = nullptr;
  std::vector<Staging> stg;
  std::vector<ViewDev*> dviews;
  std::vector<TileRun*> druns;
  std::vector<int*> dcounter;
  std::vector<size_t> rcap;
  std::vector<hipEvent_t> slot_free, copied, evpool;
  bool dev_ok = true;

  ServeBackend(bh_ctx* ctx, int maxin) : c(ctx), slots(maxin + 1) {
    cfg = c->tile_cfg;
    pers = c->persistent;
    int waves, ppt;
    tile_config(cfg, &tw, &th, &waves, &ppt);
    stg.resize(slots);
    dviews.assign(slots, nullptr);
    druns.assign(slots, nullptr);
    dcounter.assign(slots, nullptr);
    rcap.assign(slots, 0);
    slot_free.assign(slots, nullptr);
    copied.assign(slots, nullptr);
  }

  // streams, image pool, per-slot counters and events
  hipError_t init() {
    hipError_t e = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&copy_stream, hipStreamNonBlocking);
    if (e == hipSuccess) {
      hipMemPoolProps props = {};
      props.allocType = hipMemAllocationTypePinned;
      props.location.type = hipMemLocationTypeDevice;
      props.location.id = c->device;
      e = hipMemPoolCreate(&img_pool, &props);
    }
    if (e == hipSuccess) {
      uint64_t keep = UINT64_MAX;  // released images stay reserved for the next allocations
      e = hipMemPoolSetAttribute(img_pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    for (int k = 0; k < slots && e == hipSuccess; ++k) {
      e = hipMalloc(&dcounter[k], sizeof(int) * 16);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&slot_free[k], hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&copied[k], hipEventDisableTiming);
    }
    return e;
  }

  // after the scheduler is gone (its destructor returned every image through dealloc)
  ~ServeBackend() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (copy_stream) {
      (void)hipStreamSynchronize(copy_stream);
      (void)hipStreamDestroy(copy_stream);
    }
    for (int k = 0; k < slots; ++k) {
      if (slot_free[k]) (void)hipEventDestroy(slot_free[k]);
      if (copied[k]) (void)hipEventDestroy(copied[k]);
      if (dviews[k]) (void)hipFree(dviews[k]);
      if (druns[k]) (void)hipFree(druns[k]);
      if (dcounter[k]) (void)hipFree(dcounter[k]);
      if (stg[k].host) (void)hipHostFree(stg[k].host);
      if (stg[k].done) (void)hipEventDestroy(stg[k].done);
    }
    for (hipEvent_t e : evpool) (void)hipEventDestroy(e);
    if (img_pool) (void)hipMemPoolDestroy(img_pool);
    if (stream) (void)hipStreamDestroy(stream);
  }

  double now() { return now_s(); }

  int64_t tiles(const Payload& p) {
    return (int64_t)((p.view.width + tw - 1) / tw) * ((p.view.height + th - 1) / th);
  }

  // reserve in the budget first, as dev_alloc does, then allocate on the serving stream
  void* try_alloc(size_t bytes) {
    const uint64_t before = c->used.fetch_add(bytes);
    if (!c->budget || before + bytes <= c->budget) {
      void* p = nullptr;
      if (hipMallocFromPoolAsync(&p, bytes, img_pool, stream) == hipSuccess) return p;
    }
    c->used -= bytes;
    return nullptr;
  }

  void dealloc(void* p, size_t bytes) {
    (void)hipFreeAsync(p, stream);
    c->used -= bytes;
  }

  int launch(const Pieces& pieces, int64_t ntiles, Handle* h) {
    int st = sched::kEDEVICE;
    if (ntiles > 0 && dev_ok) st = enqueue(pieces, ntiles);
    if (evpool.empty()) {
      hipEvent_t ev = nullptr;
      if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        dev_ok = false;
        (void)hipStreamSynchronize(stream);  // no event: make the launch complete now
      }
      evpool.push_back(ev);
    }
    h->ev = evpool.back();
    evpool.pop_back();
    if (h->ev && hipEventRecord(h->ev, stream) != hipSuccess) {
      (void)hipStreamSynchronize(stream);
      (void)hipEventDestroy(h->ev);
      h->ev = nullptr;
    }
    slot = (slot + 1) % slots;
    return st;
  }

  int enqueue(const Pieces& pieces, int64_t ntiles) {
    std::vector<ViewDev> vds;
    std::vector<TileRun> runs;
    int64_t start = 0;
    for (const auto& pc : pieces) {
      ViewDev vd;
      if (make_view(&pc.r->payload.view, pc.r->out, nullptr, &vd) != BH_OK) return sched::kEINVAL;
      const int tx = (pc.r->payload.view.width + tw - 1) / tw;
      runs.push_back(TileRun{(int)vds.size(), (int)pc.first, (int)start, tx});
      vds.push_back(vd);
      start += pc.count;
    }
    // this slot's device records (its previous launch has finished: fewer than `slots`
    // launches are in flight, and the upload also waits for its slot_free event)
    if (rcap[slot] < vds.size()) {
      if (dviews[slot]) (void)hipFree(dviews[slot]);
      if (druns[slot]) (void)hipFree(druns[slot]);
      dviews[slot] = nullptr;
      druns[slot] = nullptr;
      rcap[slot] = 0;
      const size_t cap = std::max<size_t>(vds.size(), 256);
      if (hipMalloc(&dviews[slot], sizeof(ViewDev) * cap) != hipSuccess ||
          hipMalloc(&druns[slot], sizeof(TileRun) * cap) != hipSuccess) {
        dev_ok = false;
        return sched::kEDEVICE;
      }
      rcap[slot] = cap;
    }
    bh_status st = enqueue_batch(c, cfg, pers, tables_dev(pieces.front().r->payload.tables), vds,
                                 runs, (int)ntiles, dviews[slot], druns[slot], dcounter[slot],
                                 stg[slot], stream, false, copy_stream, slot_free[slot],
                                 copied[slot]);
    if (st == BH_OK && hipEventRecord(slot_free[slot], stream) != hipSuccess) st = BH_EDEVICE;
    return st;
  }

  bool done(Handle& h) { return !h.ev || hipEventQuery(h.ev) == hipSuccess; }
  void wait(Handle& h) {
    if (h.ev) (void)hipEventSynchronize(h.ev);
  }
  void release(Handle& h) {
    if (h.ev) evpool.push_back(h.ev);
    h.ev = nullptr;
  }
};

static_assert((int)sched::kEAGAIN == (int)BH_EAGAIN && (int)sched::kENOMEM == (int)BH_ENOMEM &&
                  (int)sched::kECANCELED == (int)BH_ECANCELED &&
                  (int)sched::kENOTFOUND == (int)BH_ENOTFOUND &&
                  (int)sched::kEDEVICE == (int)BH_EDEVICE,
              "scheduler status codes are those of bh_status");

// Most tiles one serving launch may hold: the one-workgroup-per-tile launch runs
// tiles x (tile pixels / pixels per thread) work-items, at most 1024 per tile (every tile
// configuration), which must stay below 2^32; tile indices are ints.
constexpr int64_t kMaxServeTiles = ((int64_t)1 << 32) / 1024 - 1;

extern "C" bh_status bh_serve_start(bh_ctx* c, const bh_serve_params* p) {
  if (p && p->max_tiles_per_launch > kMaxServeTiles)
    return fail(BH_EINVAL, "max_tiles_per_launch above " + std::to_string(kMaxServeTiles) +
                               " (one launch covers fewer than 2^32 work-items)");
  if (!c) return fail(BH_EINVAL, "NULL context");
  std::lock_guard<std::mutex> lk(c->smu);
  if (c->sched) return fail(BH_EINVAL, "serving already started");
  sched::Params sp;
  sp.max_queue = p && p->max_queue > 0 ? p->max_queue : 1 << 20;
  sp.max_inflight = p && p->max_inflight_launches > 0 ? p->max_inflight_launches : 6;
  sp.max_tiles = p && p->max_tiles_per_launch > 0 ? p->max_tiles_per_launch : 262144;
  HIPCHK(hipSetDevice(c->device));
  std::unique_ptr<ServeBackend> be;
  {
    std::lock_guard<std::mutex> g(c->mu);  // tile configuration and launch form
    be.reset(new ServeBackend(c, sp.max_inflight));
  }
  hipError_t e = be->init();
  if (e != hipSuccess) return fail(BH_EDEVICE, std::string("serving set-up: ") + hipGetErrorString(e));
  c->serve_backend = std::move(be);
  c->sched.reset(new sched::Scheduler<ServeBackend>(*c->serve_backend, sp));
  c->serve_thread = std::thread([c] {
    (void)hipSetDevice(c->device);
    c->sched->run();
  });
  return BH_OK;
}

// Queued requests are cancelled, admitted ones finish; then every serving resource goes.
static void serve_stop(bh_ctx* c) {
  std::lock_guard<std::mutex> lk(c->smu);
  if (!c->sched) return;
  c->sched->stop();
  c->serve_thread.join();
  c->sched.reset();          // returns the requests' and the pool's images
  c->serve_backend.reset();  // then the streams, slots and pool
}

static sched::Scheduler<ServeBackend>* serving(bh_ctx* c) {
  std::lock_guard<std::mutex> lk(c->smu);
  return c->sched.get();
}

extern "C" bh_status bh_submit(bh_ctx* c, const bh_tables* t, const bh_view* v, float* out,
                               uint64_t* ticket) {
  if (!c || !t || !v || !ticket) return fail(BH_EINVAL, "NULL argument");
  ViewDev tmp;
  float dummy = 0;
  bh_status st = make_view(v, out ? out : &dummy, nullptr, &tmp);
  if (st) return st;
  auto* s = serving(c);
  if (!s) return fail(BH_EINVAL, "serving not started");
  const size_t bytes = sizeof(float4) * (size_t)v->width * v->height;
  if (!out && c->budget && bytes > c->budget) return fail(BH_ENOMEM, "image larger than the HBM budget");
  const int rc = s->submit(ServePayload{*v, t}, t, out, bytes, ticket);
  if (rc == sched::kEAGAIN) return fail(BH_EAGAIN, "serving queue full");
  if (rc != sched::kOK) return fail((bh_status)rc, "serving stopped");
  return BH_OK;
}

extern "C" bh_status bh_poll(bh_ctx* c, uint64_t ticket, int32_t* done, double* latency) {
  if (!c || !done) return fail(BH_EINVAL, "NULL argument");
  auto* s = serving(c);
  if (!s) return fail(BH_ENOTFOUND, "serving not started");
  int d = 0;
  const int rc = s->poll(ticket, &d, latency);
  if (rc == sched::kENOTFOUND) return fail(BH_ENOTFOUND, "unknown ticket");
  *done = d;
  return (bh_status)rc;
}

extern "C" bh_status bh_ticket_image(bh_ctx* c, uint64_t ticket, float** img) {
  if (!c || !img) return fail(BH_EINVAL, "NULL argument");
  auto* s = serving(c);
  if (!s) return fail(BH_ENOTFOUND, "serving not started");
  const int rc = s->image(ticket, img);
  if (rc == sched::kENOTFOUND) return fail(BH_ENOTFOUND, "unknown ticket");
  if (rc == sched::kEAGAIN) return fail(BH_EAGAIN, "not finished");
  return BH_OK;
}

extern "C" bh_status bh_ticket_free(bh_ctx* c, uint64_t ticket) {
  if (!c) return fail(BH_EINVAL, "NULL context");
  auto* s = serving(c);
  if (!s) return fail(BH_ENOTFOUND, "serving not started");
  const int rc = s->release(ticket);
  if (rc == sched::kENOTFOUND) return fail(BH_ENOTFOUND, "unknown ticket");
  if (rc == sched::kEAGAIN) return fail(BH_EAGAIN, "not finished");
  return BH_OK;
}

extern "C" bh_status bh_serve_drain(bh_ctx* c) {
  if (!c) return fail(BH_EINVAL, "NULL context");
  auto* s = serving(c);
  if (s) s->drain();
  return BH_OK;
}
