// C ABI of the MARS library: context and scene management, the per-iteration
// wavefront schedule, the update step, read-back, checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mars.h"
#include "bvh_build.h"
#include "mars_internal.h"

using namespace mars;

namespace {

struct Status : std::exception {
  mars_status code;
  std::string msg;
  Status(mars_status c, std::string m) : code(c), msg(std::move(m)) {}
};

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess)                                                              \
      throw Status(MARS_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_));        \
  } while (0)

struct Ctx;

struct Scene {
  Ctx* ctx = nullptr;
  std::vector<void*> owned;
  uint64_t uid = 0;    // unique per context: keys captured graphs
  uint64_t epoch = 0;  // bumped whenever a device buffer captured by a graph moves
  // configuration
  int W = 0, H = 0, mode = 0, max_depth = 0, max_cells = 0, max_tree_depth = 8, split_visits = 32;
  int nee = 1;
  uint64_t seed = 1;
  size_t cap = 0;
  int tile_roots = 0;
  int n_tris = 0, n_mats = 0;
  // host copies kept for checkpoints and re-validation
  std::vector<float> mats;
  // device views
  SceneDev sd{};
  CacheDev cd{};
  QueuesDev qd{};
  ImageDev img{};
  LightDev lt{};
  Counters* cnt = nullptr;
  DebugRec* dbg = nullptr;
  uint32_t dbg_cap = 0;
  int32_t* n_cells_dev = nullptr;  // [2]: cells, nodes
  uint32_t* scratch = nullptr;     // [max_cells + 1]
  float* fixed = nullptr;
  int n_fixed = 0;
  size_t roots_cap = 0;            // Ls / beta1 capacity in roots
  // host mirrors
  int n_cells = 1, n_nodes = 1;
  double total_spp = 0.0;
  int spp_last = 0;
  uint64_t rays_last = 0;
  int bvh_depth = 0;
  int n_bvh_nodes = 0;
  uint32_t dbg_last = 0;
  // learned cache
  bool mlp_on = false;
  MlpDev mlp{};
  uint32_t mlp_n_train = 0;
  int mlp_step = 0;
  uint64_t vertices_last = 0;
  // largest queue level per camera sample over the tiles of the last eager
  // iteration: of the ray queues, of the shadow queues, and the larger
  double peak_ray = 0.0, peak_shadow = 0.0, peak_per_root = 0.0;
  size_t scap = 0;  // shadow-queue entries per level (cap: ray-queue entries)
};

// per-kernel HIP-event timing on the context's stream
// (fixed_point: the per-cell update with the guided distribution and the
// inverse-variance weighted image)
enum KernelId {
  KID_RAYGEN, KID_TRACE, KID_SHADE, KID_BACKPROP, KID_PIXEL_SUMS, KID_UPDATE_IMAGE,
  KID_FIXED_POINT, KID_REFINE, KID_LIGHT, KID_MLP, KID_MLP_TRAIN, KID_BATCH, KID_CONNECT, KID_COUNT
};
const char* kKernelNames[KID_COUNT] = {
    "raygen", "trace", "shade", "backprop", "pixel_sums", "update_image",
    "fixed_point", "refine", "light", "mlp_infer", "mlp_train", "batch", "connect"};

struct Profiler {
  uint64_t mask = 0;  // bit k: kernel k is timed
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  std::vector<hipEvent_t> pool;
  double ms[KID_COUNT] = {0};
  uint64_t n[KID_COUNT] = {0};
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    // timing events only: every host read waits on the stream after a copy,
    // so the events need no system-scope fence (one costs a few
    // microseconds between the launches an event brackets)
    hipEvent_t e;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    return e;
  }
  // call only after the stream has been synchronised
  void flush() {
    for (auto& p : pending) {
      float t = 0.0f;
      HIPCHK(hipEventElapsedTime(&t, p.second.first, p.second.second));
      ms[p.first] += t;
      n[p.first] += 1;
      pool.push_back(p.second.first);
      pool.push_back(p.second.second);
    }
    pending.clear();
  }
  void reset() {
    for (int k = 0; k < KID_COUNT; ++k) { ms[k] = 0.0; n[k] = 0; }
  }
  ~Profiler() {
    for (auto& p : pending) { (void)hipEventDestroy(p.second.first); (void)hipEventDestroy(p.second.second); }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// a captured batch: the key lists everything the launches bake in
struct BatchGraph {
  std::vector<uint64_t> key;
  std::vector<hipGraphExec_t> exec;  // one single-chain graph per scene (batch order)
  int32_t* iter = nullptr;    // device: iteration index read by the kernels
  double* summary = nullptr;  // device: [n][kSumWords]
};

constexpr size_t kPinnedBytes = 4096;
static_assert(sizeof(Counters) <= kPinnedBytes && 8 * 8 + 4 * 4 + 4 <= kPinnedBytes,
              "the pinned readback buffer holds the counters and the update's scalars");

struct Ctx {
  int device = 0;
  float* noalloc_scratch = nullptr;  // device address of the fixed gradient array
  std::string noalloc_error;
  uint64_t next_uid = 1;
  // batched iterations: a pool of default-priority streams and the graph cache
  std::vector<hipStream_t> pool;
  std::vector<hipEvent_t> pool_ev;
  std::vector<BatchGraph> graphs;
  int batch_streams = 4;
  Profiler prof;
  unsigned long long* tcount = nullptr;  // traversal counters (instrumented runs)
  bool counting = false;
  hipStream_t stream = nullptr;
  // pinned host memory for the readbacks of every tile and update (a copy
  // into pageable memory is staged through a host buffer by the runtime)
  unsigned char* pinned = nullptr;
  mars_alloc_fn alloc = nullptr;
  mars_free_fn free_ = nullptr;
  void* user = nullptr;
  int cu = 256;
  std::string err;
  std::vector<std::unique_ptr<Scene>> scenes;

  void* dalloc(size_t bytes) {
    if (bytes == 0) bytes = 16;
    void* p = nullptr;
    if (alloc) {
      p = alloc(bytes, (void*)stream, user);
      if (!p) throw Status(MARS_E_OOM, "allocator callback returned NULL");
    } else {
      if (hipMalloc(&p, bytes) != hipSuccess) throw Status(MARS_E_OOM, "hipMalloc failed");
    }
    return p;
  }
  void dfree(void* p) {
    if (!p) return;
    if (free_) free_(p, (void*)stream, user);
    else (void)hipFree(p);
  }
  void drop_graph(BatchGraph& g) {
    for (auto e : g.exec) (void)hipGraphExecDestroy(e);
    dfree(g.iter);
    dfree(g.summary);
    g = BatchGraph{};
  }
  Scene* scene(int id) {
    if (id < 0 || id >= (int)scenes.size() || !scenes[id])
      throw Status(MARS_E_ARG, "invalid scene id");
    return scenes[id].get();
  }
};

template <typename F>
void timed(Ctx* c, int kid, F&& launch) {
  if (!((c->prof.mask >> kid) & 1u)) {
    launch();
    return;
  }
  hipEvent_t a = c->prof.get(), b = c->prof.get();
  HIPCHK(hipEventRecord(a, c->stream));
  launch();
  HIPCHK(hipEventRecord(b, c->stream));
  c->prof.pending.push_back({kid, {a, b}});
}

// the same for a launch that stamps the two events itself (at its kernel's
// start and end): launch(a, b), with null events when the kernel is not timed
template <typename F>
void timed_ext(Ctx* c, int kid, F&& launch) {
  if (!((c->prof.mask >> kid) & 1u)) {
    launch(nullptr, nullptr);
    return;
  }
  hipEvent_t a = c->prof.get(), b = c->prof.get();
  launch(a, b);
  c->prof.pending.push_back({kid, {a, b}});
}

template <typename T>
T* salloc(Scene* s, size_t n) {
  void* p = s->ctx->dalloc(n * sizeof(T));
  s->owned.push_back(p);
  return (T*)p;
}

void release_scene(Scene* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->ctx->stream);
  for (void* p : s->owned) s->ctx->dfree(p);
  s->owned.clear();
  s->epoch++;
}

// frees one buffer of the scene (the context's stream must be idle)
void sfree(Scene* s, void* p) {
  if (!p) return;
  auto it = std::find(s->owned.begin(), s->owned.end(), p);
  if (it != s->owned.end()) s->owned.erase(it);
  s->ctx->dfree(p);
}

template <typename F>
mars_status guard(Ctx* c, F&& f) {
  try {
    if (c) c->err.clear();
    f();
    return MARS_OK;
  } catch (const Status& st) {
    if (c) c->err = st.msg;
    return st.code;
  } catch (const std::bad_alloc&) {
    if (c) c->err = "host allocation failed";
    return MARS_E_OOM;
  } catch (...) {
    if (c) c->err = "unknown error";
    return MARS_E_STATE;
  }
}

void h2d(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes) HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
}
void d2h(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes) HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
}

IterDev to_dev(const mars_iter_params* p) {
  IterDev it{};  // iter_dev null: the iteration index is the field
  it.iteration = p->iteration;
  it.spp = p->spp;
  it.alloc = p->alloc;
  it.aware = p->budget_aware;
  it.rr_start = p->rr_start;
  it.fixed_scale = p->fixed_scale;
  it.clamp_lo = p->clamp_lo;
  it.clamp_hi = p->clamp_hi;
  it.stat_clamp = p->stat_clamp;
  it.center_jitter = p->center_jitter;
  it.debug_depth = p->debug_depth;
  it.lp_stride = p->lp_stride;
  it.rounding = p->rounding;
  return it;
}

void check_params(Scene* s, const mars_iter_params* p) {
  if (!p) throw Status(MARS_E_ARG, "null params");
  if (p->spp <= 0 || p->spp > 4096) throw Status(MARS_E_ARG, "spp out of range");
  if (p->alloc < 0 || p->alloc > 4) throw Status(MARS_E_ARG, "bad alloc mode");
  if (p->alloc == MARS_ALLOC_FIXED && !s->fixed) throw Status(MARS_E_STATE, "no fixed counts set");
  if (p->alloc == MARS_ALLOC_MLP && !s->mlp_on)
    throw Status(MARS_E_ARG, "learned cache not enabled for scene");
  if (s->sd.lp_classes == 3 && (p->alloc == MARS_ALLOC_EARS || p->rounding))
    throw Status(MARS_E_ARG, "per-length light-path budgets: no EARS iterations, Alg. 1 rounding only");
  if (!(p->clamp_lo > 0.0f) || !(p->clamp_hi >= p->clamp_lo) || !(p->clamp_hi <= 64.0f))
    throw Status(MARS_E_ARG, "count clamp must satisfy 0 < lo <= hi <= 64");
  if (!(p->stat_clamp >= 0.0f)) throw Status(MARS_E_ARG, "stat_clamp must be >= 0");
}

void ensure_roots(Scene* s, size_t roots) {
  if (roots <= s->roots_cap) return;
  if (s->roots_cap) {
    HIPCHK(hipStreamSynchronize(s->ctx->stream));
    for (void* p : {(void*)s->img.Ls, (void*)s->img.beta1, (void*)s->lt.V0, (void*)s->lt.V1,
                    (void*)s->lt.V2, (void*)s->lt.V3, (void*)s->lt.Y0, (void*)s->lt.len,
                    (void*)s->lt.y})
      sfree(s, p);
  }
  s->img.Ls = salloc<float>(s, roots * 3);
  s->img.beta1 = salloc<float>(s, roots * 3);
  if (s->mode == MARS_MODE_BDPT) {
    const size_t lm = (size_t)std::max(1, s->lt.lmax);
    s->lt.V0 = salloc<float4>(s, roots * lm);
    s->lt.V1 = salloc<float4>(s, roots * lm);
    s->lt.V2 = salloc<float4>(s, roots * lm);
    s->lt.V3 = salloc<float4>(s, roots * lm);
    s->lt.Y0 = salloc<float4>(s, roots);
    s->lt.len = salloc<uint2>(s, roots);
    // learned cache: network outputs at the light vertices (MIS weights)
    s->lt.y = s->mlp_on ? salloc<float>(s, roots * lm * 4) : nullptr;
  }
  s->roots_cap = roots;
  s->epoch++;
}

// per-depth path queues (levels 0 .. max_depth + 1): `cap` entries per level
// of the ray queues, `scap` of the shadow queues (NEE samples and light-path
// connections, which can far outnumber the rays)
void alloc_queues(Scene* s, size_t cap, size_t scap) {
  if (cap == 0 || cap > 0xFFFF0000ull || scap == 0 || scap > 0xFFFF0000ull)
    throw Status(MARS_E_ARG, "queue capacity out of range");
  QueuesDev& q = s->qd;
  if (q.R0) {
    HIPCHK(hipStreamSynchronize(s->ctx->stream));
    for (void* p : {(void*)q.R0, (void*)q.R1, (void*)q.S0, (void*)q.S1, (void*)q.S2, (void*)q.S3,
                    (void*)q.H, (void*)q.V0, (void*)q.V1, (void*)q.V2, (void*)q.RO, (void*)q.SH0,
                    (void*)q.SH1, (void*)q.SH2, (void*)q.W0, (void*)q.W1, (void*)q.W2, (void*)q.V3,
                    (void*)s->mlp.y})
      sfree(s, p);
    q = QueuesDev{};
    s->mlp.y = nullptr;
  }
  const size_t lv = (size_t)(s->max_depth + 2) * cap;
  q.R0 = salloc<float4>(s, lv); q.R1 = salloc<float4>(s, lv);
  q.S0 = salloc<float4>(s, lv); q.S1 = salloc<float4>(s, lv);
  q.S2 = salloc<float4>(s, lv); q.S3 = salloc<uint4>(s, lv);
  q.H = salloc<uint2>(s, lv);
  q.V0 = salloc<float4>(s, lv); q.V1 = salloc<float4>(s, lv);
  q.V2 = salloc<uint4>(s, lv); q.RO = salloc<float4>(s, lv);
  // shadow rays (SH0, SH1) live from the vertex kernel of their depth to the
  // traversal of that depth: one level serves every depth; the values (SH2)
  // stay until back-propagation
  const size_t lvs = (size_t)(s->max_depth + 2) * scap;
  q.SH0 = salloc<float4>(s, scap); q.SH1 = salloc<float4>(s, scap); q.SH2 = salloc<float4>(s, lvs);
  if (s->mode == MARS_MODE_BDPT) {
    q.W0 = salloc<float4>(s, lv);
    q.W1 = salloc<float4>(s, lv);
  }
  if (s->sd.lp_classes == 3) {
    q.W2 = salloc<float4>(s, lv);
    q.V3 = salloc<float4>(s, lv);
  }
  q.cap = cap;
  q.scap = scap;
  if (s->mlp_on) s->mlp.y = salloc<float>(s, lv * 4);
  s->cap = cap;
  s->scap = scap;
  s->epoch++;
}

// bytes of queue memory per entry: ray queues (per level), shadow values (per
// level) and shadow rays (one level for all depths)
constexpr size_t kRayEntryBytes = 10 * 16 + 8, kShadowValueBytes = 16, kShadowRayBytes = 32;

// BDPT: one light subpath per camera sample of the iteration, before any
// camera tile (connections may use any sample's subpath)
uint64_t trace_light_paths(Scene* s, const IterDev& it, size_t roots) {
  hipStream_t st = s->ctx->stream;
  Ctx* c = s->ctx;
  const int grid_trace = c->cu * kTraceBlocksPerCU;
  unsigned long long* tc = c->counting ? c->tcount : nullptr;
  k_fill_u32((uint32_t*)s->cnt, 0u, sizeof(Counters) / 4, st);
  for (size_t r0 = 0; r0 < roots; r0 += s->cap) {
    const uint32_t n = (uint32_t)std::min<size_t>(s->cap, roots - r0);
    timed(c, KID_LIGHT, [&] { k_light_start(s->sd, s->qd, s->lt, s->cnt, it, (uint32_t)r0, n, st); });
    for (int i = 1; i <= s->lt.lmax; ++i) {
      timed_ext(c, KID_TRACE, [&](hipEvent_t a, hipEvent_t b) {
        k_trace_pair(s->sd, s->qd, s->cnt, 0, 0, grid_trace, st, tc, a, b);
      });
      // learned-cache iterations: the network's counts at the new light
      // vertices, which the connections' MIS weights evaluate as if on the
      // camera side
      if (it.alloc == MARS_ALLOC_MLP && s->lt.y)
        timed(c, KID_MLP, [&] {
          k_mlp_infer_light(s->sd, s->qd, s->mlp, s->lt, s->cnt, i, c->cu * 32, st);
        });
      timed(c, KID_LIGHT, [&] { k_light_shade(s->sd, s->cd, s->qd, s->lt, s->cnt, it, i, st); });
    }
  }
  timed(c, KID_LIGHT, [&] { k_light_walk(s->sd, s->lt, (uint32_t)roots, st); });
  Counters* pc = (Counters*)c->pinned;
  d2h(pc, s->cnt, sizeof(Counters), st);
  HIPCHK(hipStreamSynchronize(st));
  return pc->rays_light;
}

// One wavefront tile: returns false on queue overflow.  The bottom-up pass is
// enqueued before the counters are read back (its kernels do nothing after an
// overflow), and so are the per-pixel sums after the last tile (a re-rendered
// tile enqueues them again), so that the host waits once per tile.
bool run_tile(Scene* s, const IterDev& it, uint32_t root0, uint32_t n, uint32_t dbg0,
              uint32_t npool, bool last, int spp, Counters* hc) {
  const bool bdpt = s->mode == MARS_MODE_BDPT;
  hipStream_t st = s->ctx->stream;
  // traversal: 128-thread groups, kTraceBlocksPerCU resident per CU; others 256-thread groups
  const int grid_trace = s->ctx->cu * kTraceBlocksPerCU, grid = s->ctx->cu * 8;
  Ctx* c = s->ctx;
  unsigned long long* tc = c->counting ? c->tcount : nullptr;
  k_fill_u32((uint32_t*)s->cnt, 0u, sizeof(Counters) / 4, st);
  if (dbg0) h2d(&s->cnt->n_debug, &dbg0, 4, st);  // debug records accumulate across tiles
  timed(c, KID_RAYGEN, [&] { k_raygen(s->sd, s->qd, s->cnt, it, root0, n, st); });
  timed_ext(c, KID_TRACE, [&](hipEvent_t a, hipEvent_t b) {
    k_trace_pair(s->sd, s->qd, s->cnt, 1, 0, grid_trace, st, tc, a, b);
  });
  for (int d = 1; d <= s->max_depth; ++d) {
    if (it.alloc == MARS_ALLOC_MLP && d < s->max_depth)
      timed(c, KID_MLP, [&] { k_mlp_infer_queue(s->sd, s->qd, s->mlp, s->cnt, d, grid * 4, st); });
    timed(c, KID_SHADE, [&] {
      if (bdpt)
        k_shade_bdpt(s->sd, s->cd, s->qd, s->lt, s->cnt, it, s->img, s->dbg, s->dbg_cap, d, npool,
                     st);
      else
        k_shade_pt(s->sd, s->cd, s->qd, s->cnt, it, s->img, s->dbg, s->dbg_cap, d, grid, st);
    });
    if (bdpt)
      timed(c, KID_CONNECT, [&] {
        k_connect_bdpt(s->sd, s->cd, s->qd, s->lt, s->cnt, it, s->img, d, st);
      });
    // shadow rays of depth d with the continuation rays of depth d + 1
    const int dc = d < s->max_depth ? d + 1 : -1;
    timed_ext(c, KID_TRACE, [&](hipEvent_t a, hipEvent_t b) {
      k_trace_pair(s->sd, s->qd, s->cnt, dc, d, grid_trace, st, tc, a, b);
    });
  }
  for (int d = s->max_depth; d >= 1; --d)
    timed(c, KID_BACKPROP, [&] {
      if (bdpt)
        k_backprop_bdpt(s->sd, s->cd, s->qd, s->lt, s->cnt, it, s->img, d, npool, st);
      else
        k_backprop_pt(s->sd, s->cd, s->qd, s->cnt, it, s->img, d, st);
    });
  if (last) timed(c, KID_PIXEL_SUMS, [&] { k_pixel_sums(s->img, s->W * s->H, spp, st); });
  Counters* pc = (Counters*)c->pinned;
  d2h(pc, s->cnt, sizeof(Counters), st);
  HIPCHK(hipStreamSynchronize(st));
  *hc = *pc;
  return hc->overflow == 0;
}

void render_iteration(Scene* s, const mars_iter_params* p, mars_iter_stats* out) {
  check_params(s, p);
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = s->ctx->stream;
  const size_t roots = (size_t)s->W * s->H * p->spp;
  if (roots > 0x7FFFFFFFull) throw Status(MARS_E_ARG, "too many camera samples");
  ensure_roots(s, roots);
  IterDev it = to_dev(p);
  // per-iteration statistics start at zero (Sec. 4.1: estimates per iteration)
  k_clear_iteration(s->cd, s->n_cells_dev, s->mode == MARS_MODE_PT_GUIDED, s->img.beta1, roots * 3,
                    st);
  if (p->debug_depth > 0) {
    // room for every vertex up to debug_depth with splitting headroom
    const size_t want = std::min<size_t>(roots * (size_t)p->debug_depth * 4 + 1024, 1u << 25);
    if (want > s->dbg_cap) {
      s->dbg = salloc<DebugRec>(s, want);
      s->dbg_cap = (uint32_t)want;
    }
  }
  // learned cache: outputs for MLP iterations, training vertices always
  s->cd.mlp_y = nullptr;
  s->cd.mlp_rec = nullptr;
  if (s->mlp_on) {
    if (p->alloc == MARS_ALLOC_MLP) s->cd.mlp_y = s->mlp.y;
    const double expect = (double)std::max<uint64_t>(s->vertices_last, 1);
    s->mlp.keep = (uint32_t)std::min(16777216.0, 16777216.0 * (double)s->mlp.rec_cap / expect);
    if (s->mlp.keep == 0) s->mlp.keep = 1;
    s->cd.mlp_rec = s->mlp.rec;
    s->cd.mlp_n_rec = s->mlp.n_rec;
    s->cd.mlp_rec_cap = s->mlp.rec_cap;
    s->cd.mlp_keep = s->mlp.keep;
    k_fill_u32(s->mlp.n_rec, 0u, 4, st);
  }
  mars_iter_stats S{};
  S.rays_camera = roots;
  if (s->mode == MARS_MODE_BDPT) S.rays_light = trace_light_paths(s, it, roots);
  const uint32_t tile = (uint32_t)std::max<size_t>(1, std::min<size_t>(s->tile_roots, s->cap));
  std::vector<std::pair<uint32_t, uint32_t>> work;
  for (size_t r = roots; r > 0;) {
    const uint32_t n = (uint32_t)std::min<size_t>(tile, r);
    r -= n;
    work.emplace_back((uint32_t)r, n);  // processed back to front: ascending roots
  }
  uint32_t dbg_total = 0;
  double peak_r = 0.0, peak_s = 0.0;
  uint32_t ok_tile = 0;  // largest tile that fit after an overflow
  bool overflowed = false;
  while (!work.empty()) {
    auto [r0, n] = work.back();
    work.pop_back();
    Counters hc;
    const bool ok = run_tile(s, it, r0, n, dbg_total, (uint32_t)roots, work.empty(), p->spp, &hc);
    S.tiles++;
    for (int d = 1; d <= s->max_depth + 1; ++d) {
      peak_r = std::max(peak_r, (double)hc.n_ray[d] / (double)n);
      peak_s = std::max(peak_s, (double)hc.n_shadow[d] / (double)n);
    }
    if (!ok) {
      if (n == 1) throw Status(MARS_E_OVERFLOW, "a single path tree exceeds the queue capacity");
      S.overflow_retries++;
      overflowed = true;
      const uint32_t h = n / 2;
      work.emplace_back(r0 + h, n - h);
      work.emplace_back(r0, h);
      continue;
    }
    dbg_total = hc.n_debug;
    ok_tile = std::max(ok_tile, n);
    S.rays_ext += hc.rays_ext;
    S.rays_shadow += hc.rays_shadow;
    S.vertices += hc.vertices;
    S.samples += hc.samples;
    S.rays_conn += hc.rays_conn;
  }
  HIPCHK(hipGetLastError());
  s->ctx->prof.flush();
  s->spp_last = p->spp;
  s->vertices_last = S.vertices;
  s->rays_last = S.rays_camera + S.rays_ext + S.rays_shadow + S.rays_light + S.rays_conn;
  s->dbg_last = dbg_total;
  s->peak_ray = peak_r;
  s->peak_shadow = peak_s;
  s->peak_per_root = std::max(peak_r, peak_s);
  // later iterations start from a tile that fitted (tiles do not change results)
  if (overflowed && ok_tile > 0 && (int)ok_tile < s->tile_roots) s->tile_roots = (int)ok_tile;
  S.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (out) *out = S;
}


// learned cache initial weights: He-uniform, zero biases, output layer scaled
// by 0.1, output padding zero (deterministic in the seed)
void mlp_write_master(Scene* s, const float* params) {
  hipStream_t st = s->ctx->stream;
  h2d(s->mlp.master, params, 4 * (size_t)kMlpParams, st);
  k_fill_f32(s->mlp.m, 0.0f, kMlpParams, st);
  k_fill_f32(s->mlp.v, 0.0f, kMlpParams, st);
  k_mlp_quantize(s->mlp, st);
  HIPCHK(hipStreamSynchronize(st));
  s->mlp_step = 0;
}
void mlp_init(Scene* s, uint64_t seed) {
  std::vector<float> p(kMlpParams, 0.0f);
  uint64_t x = seed ^ 0x9E3779B97F4A7C15ull;
  auto next = [&]() {  // splitmix64 -> uniform in [0, 1)
    x += 0x9E3779B97F4A7C15ull;
    uint64_t z = x;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
  };
  struct L { int w, rows, cols; double scale; };
  const L layers[4] = {{kMlpW1, 64, 80, 1.0}, {kMlpW2, 64, 64, 1.0}, {kMlpW3, 64, 64, 1.0},
                       {kMlpW4, 16, 64, 0.1}};
  for (const L& l : layers) {
    const double bound = std::sqrt(6.0 / l.cols) * l.scale;
    for (int r = 0; r < l.rows; ++r)
      for (int c = 0; c < l.cols; ++c)
        p[l.w + r * l.cols + c] = (l.w == kMlpW4 && r >= 3) ? 0.0f : (float)((2.0 * next() - 1.0) * bound);
  }
  mlp_write_master(s, p.data());
}

// ---------------------------------------------------------------------------
// scene upload: validation, derived quantities in binary64 stored as binary32
// (normals, emitter selection by area x luminance, octree root cube, camera
// basis), BVH, device buffers
// ---------------------------------------------------------------------------
int upload_scene(Ctx* c, const mars_scene_desc* d) {
  if (!d || !d->V || !d->tri_mat || !d->mats || !d->camera) throw Status(MARS_E_ARG, "null scene array");
  if (d->n_tris <= 0 || d->n_mats <= 0 || d->width <= 0 || d->height <= 0)
    throw Status(MARS_E_ARG, "bad scene sizes");
  if (d->mode < 0 || d->mode > 2) throw Status(MARS_E_ARG, "bad mode");
  if (d->max_depth < 1 || d->max_depth > kMaxDepth) throw Status(MARS_E_ARG, "max_depth out of range");
  if (d->max_cells < 8 || d->max_cells > (1 << 24)) throw Status(MARS_E_ARG, "max_cells out of range");
  if (d->max_tree_depth < 0 || d->max_tree_depth > 20) throw Status(MARS_E_ARG, "bad max_tree_depth");
  if ((int64_t)d->width * d->height > (1 << 26)) throw Status(MARS_E_ARG, "image too large");
  if (d->flags & ~(MARS_SCENE_MLP | MARS_SCENE_LP_LENGTHS)) throw Status(MARS_E_ARG, "unknown scene flags");
  if ((d->flags & MARS_SCENE_LP_LENGTHS) &&
      (d->mode != MARS_MODE_BDPT || (d->flags & MARS_SCENE_MLP)))
    throw Status(MARS_E_ARG, "per-length light-path budgets need a BDPT scene without the learned cache");
  const int nt = d->n_tris, nm = d->n_mats;
  for (size_t i = 0; i < (size_t)nt * 9; ++i)
    if (!std::isfinite(d->V[i])) throw Status(MARS_E_NONFINITE, "non-finite vertex");
  for (size_t i = 0; i < (size_t)nm * 8; ++i)
    if (!std::isfinite(d->mats[i])) throw Status(MARS_E_NONFINITE, "non-finite material");
  for (int i = 0; i < 10; ++i)
    if (!std::isfinite(d->camera[i])) throw Status(MARS_E_NONFINITE, "non-finite camera");
  for (int i = 0; i < nt; ++i)
    if (d->tri_mat[i] >= (uint32_t)nm) throw Status(MARS_E_ARG, "material index out of range");
  for (int i = 0; i < nm; ++i) {
    const float* m = d->mats + 8 * i;
    if (m[0] != 0.0f && m[0] != 1.0f) throw Status(MARS_E_ARG, "unknown material kind");
    if (m[0] == 1.0f && !(m[4] > 0.0f)) throw Status(MARS_E_ARG, "GGX alpha must be positive");
    for (int k = 5; k < 8; ++k)
      if (m[k] < 0.0f) throw Status(MARS_E_ARG, "negative emission");
  }

  auto sp = std::make_unique<Scene>();
  Scene* s = sp.get();
  s->ctx = c;
  s->W = d->width;
  s->H = d->height;
  s->mode = d->mode;
  s->max_depth = d->max_depth;
  s->max_cells = d->max_cells;
  s->max_tree_depth = d->max_tree_depth;
  s->split_visits = d->split_visits;
  s->nee = d->nee_enabled;
  s->seed = d->seed;
  s->n_tris = nt;
  s->n_mats = nm;
  s->mats.assign(d->mats, d->mats + 8 * (size_t)nm);
  hipStream_t st = c->stream;
  try {
    // per-triangle normals, areas; bounding box
    std::vector<float> ng(4 * (size_t)nt), geo(12 * (size_t)nt);
    std::vector<double> area(nt);
    float bmin[3] = {INFINITY, INFINITY, INFINITY}, bmax[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = 0; i < nt; ++i) {
      const float* p = d->V + 9 * (size_t)i;
      for (int k = 0; k < 9; ++k) {
        bmin[k % 3] = std::min(bmin[k % 3], p[k]);
        bmax[k % 3] = std::max(bmax[k % 3], p[k]);
      }
      const float e1[3] = {p[3] - p[0], p[4] - p[1], p[5] - p[2]};
      const float e2[3] = {p[6] - p[0], p[7] - p[1], p[8] - p[2]};
      float* g = &geo[12 * (size_t)i];
      g[0] = p[0]; g[1] = p[1]; g[2] = p[2]; g[3] = 0.0f;
      g[4] = e1[0]; g[5] = e1[1]; g[6] = e1[2]; g[7] = 0.0f;
      g[8] = e2[0]; g[9] = e2[1]; g[10] = e2[2]; g[11] = 0.0f;
      const double a[3] = {e1[0], e1[1], e1[2]}, b[3] = {e2[0], e2[1], e2[2]};
      const double cr[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2],
                            a[0] * b[1] - a[1] * b[0]};
      const double l = std::sqrt((cr[0] * cr[0] + cr[1] * cr[1]) + cr[2] * cr[2]);
      area[i] = 0.5 * l;
      float* n = &ng[4 * (size_t)i];
      if (l > 0.0) {
        n[0] = (float)(cr[0] / l); n[1] = (float)(cr[1] / l); n[2] = (float)(cr[2] / l);
      } else {
        n[0] = 0.0f; n[1] = 0.0f; n[2] = 1.0f;
      }
      n[3] = 0.0f;
    }
    // emitters, selected proportionally to area x luminance
    std::vector<int32_t> ltri;
    std::vector<double> lw;
    for (int i = 0; i < nt; ++i) {
      const float* m = d->mats + 8 * (size_t)d->tri_mat[i];
      if (std::max(std::max(m[5], m[6]), m[7]) > 0.0f && area[i] > 0.0) {
        const double L = (0.2126 * (double)m[5] + 0.7152 * (double)m[6]) + 0.0722 * (double)m[7];
        lw.push_back(area[i] * L);
        ltri.push_back(i);
      }
    }
    double wsum = 0.0;
    for (double w : lw) wsum += w;
    std::vector<float> lcdf(ltri.size());
    double run = 0.0;
    for (size_t k = 0; k < ltri.size(); ++k) {
      run += lw[k];
      lcdf[k] = (k + 1 == ltri.size()) ? 1.0f : (float)(run / wsum);
      ng[4 * (size_t)ltri[k] + 3] = (float)((lw[k] / wsum) / area[ltri[k]]);
    }
    const double ext = std::max(std::max((double)bmax[0] - bmin[0], (double)bmax[1] - bmin[1]),
                                (double)bmax[2] - bmin[2]);
    SceneDev& sd = s->sd;
    sd.eps = (float)(1e-4 * ext);
    const double side = ext * (1.0 + 2e-4);
    for (int k = 0; k < 3; ++k) {
      const double ctr = 0.5 * ((double)bmin[k] + (double)bmax[k]);
      sd.oct_lo[k] = (float)(ctr - 0.5 * side);
    }
    sd.oct_inv = (float)(1.0 / side);
    {
      const float* cam = d->camera;
      const double P[3] = {cam[0], cam[1], cam[2]}, Tg[3] = {cam[3], cam[4], cam[5]},
                   U[3] = {cam[6], cam[7], cam[8]};
      double f[3] = {Tg[0] - P[0], Tg[1] - P[1], Tg[2] - P[2]};
      const double fl = std::sqrt((f[0] * f[0] + f[1] * f[1]) + f[2] * f[2]);
      if (!(fl > 0.0)) throw Status(MARS_E_ARG, "camera target equals position");
      for (int k = 0; k < 3; ++k) f[k] /= fl;
      double r[3] = {f[1] * U[2] - f[2] * U[1], f[2] * U[0] - f[0] * U[2], f[0] * U[1] - f[1] * U[0]};
      const double rl = std::sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]);
      if (!(rl > 0.0)) throw Status(MARS_E_ARG, "camera up parallel to view direction");
      for (int k = 0; k < 3; ++k) r[k] /= rl;
      const double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2],
                           r[0] * f[1] - r[1] * f[0]};
      const double th = std::tan(0.5 * (double)cam[9] * 3.14159265358979323846 / 180.0);
      const double asp = (double)d->width / (double)d->height;
      for (int k = 0; k < 3; ++k) {
        sd.cam_o[k] = cam[k];
        sd.cam_f[k] = (float)f[k];
        sd.cam_r[k] = (float)(r[k] * th * asp);
        sd.cam_u[k] = (float)(u[k] * th);
      }
    }
    // BVH
    BvhResult bvh = build_bvh(d->V, nt, (float)(1e-5 * ext) + 1e-7f);
    s->bvh_depth = bvh.max_depth;
    s->n_bvh_nodes = (int)(bvh.nodes.size() / 32);
    static_assert(kBvhEmpty == kBvhNoChild, "empty child reference");
    float4* dbvh = salloc<float4>(s, bvh.nodes.size() / 4);
    sd.stack_spill = nullptr;
    sd.spill_threads = 0;
    if (bvh.max_stack > kStackDepth) {
      // the rest of the stack bound in device memory, one column per thread
      sd.spill_threads = (uint32_t)c->cu * (uint32_t)kTraceBlocksPerCU * (uint32_t)kTraceBlock;
      sd.stack_spill = salloc<int32_t>(s, (size_t)(bvh.max_stack - kStackDepth) * sd.spill_threads);
    }
    float4* dtri = salloc<float4>(s, bvh.tris.size() / 4);
    float4* dgeo = salloc<float4>(s, geo.size() / 4);
    float4* dng = salloc<float4>(s, ng.size() / 4);
    uint32_t* dmat = salloc<uint32_t>(s, nt);
    float* dmats = salloc<float>(s, 8 * (size_t)nm);
    int32_t* dlt = salloc<int32_t>(s, std::max<size_t>(1, ltri.size()));
    float* dlc = salloc<float>(s, std::max<size_t>(1, lcdf.size()));
    h2d(dbvh, bvh.nodes.data(), bvh.nodes.size() * 4, st);
    h2d(dtri, bvh.tris.data(), bvh.tris.size() * 4, st);
    h2d(dgeo, geo.data(), geo.size() * 4, st);
    h2d(dng, ng.data(), ng.size() * 4, st);
    h2d(dmat, d->tri_mat, (size_t)nt * 4, st);
    h2d(dmats, d->mats, (size_t)nm * 32, st);
    h2d(dlt, ltri.data(), ltri.size() * 4, st);
    h2d(dlc, lcdf.data(), lcdf.size() * 4, st);
    sd.bvh = dbvh;
    sd.tri_bvh = dtri;
    sd.tri_geo = dgeo;
    sd.tri_ng = dng;
    sd.tri_mat = dmat;
    sd.mats = dmats;
    sd.light_tri = dlt;
    sd.light_cdf = dlc;
    sd.n_lights = (int)ltri.size();
    sd.n_tris = nt;
    sd.W = d->width;
    sd.H = d->height;
    sd.mode = d->mode;
    sd.max_depth = d->max_depth;
    sd.nee = d->nee_enabled;
    sd.lp_classes = (d->flags & MARS_SCENE_LP_LENGTHS) ? 3 : 1;
    sd.key0 = (uint32_t)d->seed;
    sd.key1 = (uint32_t)(d->seed >> 32);
    // cache: one root leaf, no data (classic counts), uniform distribution
    const size_t mc = (size_t)d->max_cells;
    CacheDev& cd = s->cd;
    cd.nodes = salloc<uint32_t>(s, 1 + 8 * mc);
    cd.leaf_node = salloc<uint32_t>(s, mc);
    cd.leaf_depth = salloc<uint32_t>(s, mc);
    cd.visits = salloc<uint32_t>(s, mc);
    cd.fac = salloc<float>(s, mc * 18);
    cd.acc = salloc<double>(s, mc * 24);
    cd.pm = salloc<float>(s, mc * 64);
    cd.cdf = salloc<float>(s, mc * 64);
    cd.hacc = salloc<double>(s, mc * 64);
    if (sd.lp_classes == 3) {
      cd.fac_x = salloc<float>(s, mc * 12);
      cd.acc_x = salloc<double>(s, mc * 16);
    }
    cd.fixed = nullptr;
    cd.n_fixed = 0;
    cd.max_cells = d->max_cells;
    s->n_cells_dev = salloc<int32_t>(s, 4);
    s->scratch = salloc<uint32_t>(s, mc + 4);
    {
      const uint32_t root = kLeafBit;
      const int32_t nc[4] = {1, 1, 0, 0};
      std::vector<float> f0(18, -1.0f), pm0(64), cdf0(64);
      for (int b = 0; b < 64; ++b) {
        pm0[b] = (float)(1.0 / 64.0);
        cdf0[b] = (float)((double)(b + 1) / 64.0);
      }
      cdf0[63] = 1.0f;
      const uint32_t z = 0;
      h2d(cd.nodes, &root, 4, st);
      h2d(cd.leaf_node, &z, 4, st);
      h2d(cd.leaf_depth, &z, 4, st);
      h2d(cd.fac, f0.data(), 18 * 4, st);
      if (cd.fac_x) h2d(cd.fac_x, f0.data(), 12 * 4, st);
      h2d(cd.pm, pm0.data(), 256, st);
      h2d(cd.cdf, cdf0.data(), 256, st);
      h2d(s->n_cells_dev, nc, 16, st);
      HIPCHK(hipStreamSynchronize(st));
    }
    // queues
    const size_t px = (size_t)d->width * d->height;
    s->tile_roots = d->tile_roots > 0 ? d->tile_roots : (int)std::min<size_t>(px * 16, 1u << 20);
    size_t cap = d->queue_capacity > 0 ? (size_t)d->queue_capacity
                                       : std::max<size_t>(65536, 4 * (size_t)s->tile_roots);
    if (cap > 0xFFFF0000ull) cap = 0xFFFF0000ull;
    s->mlp_on = (d->flags & MARS_SCENE_MLP) != 0;
    alloc_queues(s, cap, cap);
    s->cnt = salloc<Counters>(s, 1);
    s->lt.lmax = d->max_depth - 2;
    s->dbg_cap = 0;  // allocated on the first iteration that asks for records
    s->dbg = nullptr;
    // images
    ImageDev& im = s->img;
    im.iter_sum = salloc<float>(s, px * 3);
    im.accum = salloc<float>(s, px * 3);
    im.mean = salloc<float>(s, px * 3);
    im.itilde = salloc<float>(s, px * 3);
    im.excl = salloc<uint8_t>(s, px);
    im.ivw_acc = salloc<double>(s, px * 3);
    im.count_map = salloc<float>(s, px * 3);
    im.red = salloc<double>(s, 8);
    const size_t nbright = (px + kBrightChunk - 1) / kBrightChunk * kBright;
    im.bright_l = salloc<float>(s, nbright);
    im.bright_i = salloc<int32_t>(s, nbright);
    im.part = salloc<double>(s, 8 * (size_t)kRedBlocks);
    k_fill_f32(im.iter_sum, 0.0f, px * 3, st);
    k_fill_f32(im.accum, 0.0f, px * 3, st);
    k_fill_f32(im.itilde, INFINITY, px * 3, st);
    k_fill_f64(im.ivw_acc, 0.0, px * 3, st);
    k_fill_f32(im.count_map, 0.0f, px * 3, st);
    k_fill_f64(im.red, 0.0, 8, st);
    ensure_roots(s, px);
    if (s->mlp_on) {
      MlpDev& m = s->mlp;
      m.master = salloc<float>(s, kMlpParams);
      m.wq = salloc<uint16_t>(s, kMlpParams);
      m.m = salloc<float>(s, kMlpParams);
      m.v = salloc<float>(s, kMlpParams);
      m.partial = salloc<float>(s, (size_t)kMlpMaxBlocks * (kMlpParams + 1));
      m.rec_cap = 1u << 18;
      m.rec = salloc<float4>(s, 3 * (size_t)m.rec_cap);
      m.n_rec = salloc<uint32_t>(s, 4);
      m.x6 = salloc<float>(s, 6 * (size_t)m.rec_cap);
      m.tgt = salloc<float>(s, 3 * (size_t)m.rec_cap);
      m.wt = salloc<float>(s, 3 * (size_t)m.rec_cap);
      m.keep = 1u << 24;
      mlp_init(s, d->seed);
      k_fill_u32(m.n_rec, 0u, 4, st);
    }
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipGetLastError());
  } catch (...) {
    release_scene(s);
    throw;
  }
  s->uid = c->next_uid++;
  c->scenes.push_back(std::move(sp));
  return (int)c->scenes.size() - 1;
}

void update_counts(Scene* s, const mars_iter_params* p, mars_update_stats* out) {
  if (s->spp_last <= 0) throw Status(MARS_E_STATE, "no iteration rendered");
  hipStream_t st = s->ctx->stream;
  const int npx = s->W * s->H, spp = s->spp_last;
  const float kc = p ? p->stat_clamp : 0.0f;
  Ctx* c = s->ctx;
  // the running sample count lives on the device (red[6]) so that captured
  // iterations can advance it
  timed(c, KID_UPDATE_IMAGE, [&] {
    k_update_image(s->img, s->W, s->H, spp, s->img.red + 6, s->mode == MARS_MODE_BDPT, kc,
                   nullptr, st);
  });
  const double C_I = (double)s->rays_last / ((double)npx * (double)spp);
  const int nb = s->n_cells;
  timed(c, KID_FIXED_POINT, [&] {
    k_fixed_point(s->cd, s->n_cells_dev, s->img.red, C_I, nullptr, 0.0, 1, 0.0,
                  s->mode == MARS_MODE_PT_GUIDED, s->max_cells, &s->img, npx, spp, nullptr, st,
                  p && p->alloc == MARS_ALLOC_EARS ? s->mode : -1);
  });
  if (s->mlp_on) {
    IterDev itd = p ? to_dev(p) : IterDev{};
    timed(c, KID_MLP, [&] {
      k_mlp_targets(s->sd, s->cd, s->mlp, s->img, itd, s->mlp.rec_cap, nullptr, st);
    });
  }
  timed(c, KID_REFINE, [&] {
    k_refine(s->cd, s->n_cells_dev, s->n_cells_dev + 1, s->scratch, s->split_visits,
             s->max_tree_depth, s->max_cells, nullptr, st);
  });
  double red[8];
  int32_t nc[4];
  uint32_t nrec = 0;
  unsigned char* pb = c->pinned;
  d2h(pb, s->img.red, sizeof(red), st);
  d2h(pb + sizeof(red), s->n_cells_dev, sizeof(nc), st);
  if (s->mlp_on) d2h(pb + sizeof(red) + sizeof(nc), s->mlp.n_rec, 4, st);
  HIPCHK(hipStreamSynchronize(st));
  std::memcpy(red, pb, sizeof(red));
  std::memcpy(nc, pb + sizeof(red), sizeof(nc));
  if (s->mlp_on) std::memcpy(&nrec, pb + sizeof(red) + sizeof(nc), 4);
  HIPCHK(hipGetLastError());
  c->prof.flush();
  s->n_cells = nc[0];
  s->n_nodes = nc[1];
  s->total_spp = red[6];
  if (s->mlp_on) s->mlp_n_train = std::min(nrec, s->mlp.rec_cap);
  if (out) {
    out->V_I = red[4] > 0.0 ? red[3] / red[4] : 0.0;
    out->C_I = C_I;
    out->n_cells_before = nb;
    out->n_cells_after = s->n_cells;
    out->n_excluded = npx - (int)red[4];
  }
}

// ---------------------------------------------------------------------------
// batched iterations: each scene's iteration enqueued with no host
// synchronisation on one stream of a pool; the batch captured once as a graph
// ---------------------------------------------------------------------------
// streams of the batch pool: the hardware queues a process gets by default;
// MARS_BATCH_STREAMS (1..16) overrides it at context creation
constexpr int kBatchStreams = 4;
constexpr int kGraphCache = 4;

size_t roots_of(const Scene* s, int spp) { return (size_t)s->W * s->H * (size_t)spp; }

// One scene's whole iteration: the tile plan of an eager iteration, queue
// counters of a tile reset on the device, iteration totals accumulated over
// the tiles; the update takes C_I and the cell count from device memory and
// becomes a no-op if any tile overflowed (the scene is then rendered again).
void enqueue_iteration(Scene* s, const IterDev& it, int spp, bool with_update, float stat_clamp,
                       hipStream_t st, double* summary) {
  Ctx* c = s->ctx;
  const bool bdpt = s->mode == MARS_MODE_BDPT;
  const size_t roots = roots_of(s, spp);
  const int grid_trace = c->cu * kTraceBlocksPerCU, grid = c->cu * 8;
  unsigned long long* tc = c->counting ? c->tcount : nullptr;
  k_fill_u32((uint32_t*)s->cnt, 0u, sizeof(Counters) / 4, st);
  k_clear_iteration(s->cd, s->n_cells_dev, s->mode == MARS_MODE_PT_GUIDED, s->img.beta1, roots * 3,
                    st);
  if (bdpt) {
    for (size_t r0 = 0; r0 < roots; r0 += s->cap) {
      const uint32_t n = (uint32_t)std::min<size_t>(s->cap, roots - r0);
      k_light_start(s->sd, s->qd, s->lt, s->cnt, it, (uint32_t)r0, n, st);
      for (int i = 1; i <= s->lt.lmax; ++i) {
        k_trace_pair(s->sd, s->qd, s->cnt, 0, 0, grid_trace, st, tc);
        k_light_shade(s->sd, s->cd, s->qd, s->lt, s->cnt, it, i, st);
      }
    }
    k_light_walk(s->sd, s->lt, (uint32_t)roots, st);
  }
  const size_t tile = std::max<size_t>(1, std::min<size_t>(s->tile_roots, s->cap));
  for (size_t r0 = 0; r0 < roots; r0 += tile) {
    const uint32_t n = (uint32_t)std::min(tile, roots - r0);
    k_fill_u32((uint32_t*)s->cnt, 0u, kTileWords, st);
    k_raygen(s->sd, s->qd, s->cnt, it, (uint32_t)r0, n, st);
      k_trace_pair(s->sd, s->qd, s->cnt, 1, 0, grid_trace, st, tc);
    for (int d = 1; d <= s->max_depth; ++d) {
      if (bdpt) {
        k_shade_bdpt(s->sd, s->cd, s->qd, s->lt, s->cnt, it, s->img, nullptr, 0, d, (uint32_t)roots,
                     st);
        k_connect_bdpt(s->sd, s->cd, s->qd, s->lt, s->cnt, it, s->img, d, st);
      } else {
        k_shade_pt(s->sd, s->cd, s->qd, s->cnt, it, s->img, nullptr, 0, d, grid, st);
      }
      k_trace_pair(s->sd, s->qd, s->cnt, d < s->max_depth ? d + 1 : -1, d, grid_trace, st, tc);
    }
    for (int d = s->max_depth; d >= 1; --d) {
      if (bdpt)
        k_backprop_bdpt(s->sd, s->cd, s->qd, s->lt, s->cnt, it, s->img, d, (uint32_t)roots, st);
      else
        k_backprop_pt(s->sd, s->cd, s->qd, s->cnt, it, s->img, d, st);
    }
  }
  k_pixel_sums(s->img, s->W * s->H, spp, st);
  if (with_update) {
    const uint32_t* skip = &s->cnt->overflow_any;
    k_update_image(s->img, s->W, s->H, spp, s->img.red + 6, bdpt, stat_clamp, skip, st);
    k_fixed_point(s->cd, s->n_cells_dev, s->img.red, 0.0, s->cnt, (double)roots, 1, 0.0,
                  s->mode == MARS_MODE_PT_GUIDED, s->max_cells, &s->img, s->W * s->H, spp, skip,
                  st, it.alloc == MARS_ALLOC_EARS ? s->mode : -1);
    k_refine(s->cd, s->n_cells_dev, s->n_cells_dev + 1, s->scratch, s->split_visits,
             s->max_tree_depth, s->max_cells, skip, st);
  }
  k_batch_summary(s->cnt, s->img.red, s->n_cells_dev, summary, st);
}

void ensure_pool(Ctx* c) {
  while ((int)c->pool.size() < c->batch_streams) {
    hipStream_t s;
    HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    c->pool.push_back(s);
  }
  while ((int)c->pool_ev.size() < c->batch_streams + 1) {
    hipEvent_t e;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    c->pool_ev.push_back(e);
  }
}

uint64_t fbits64(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return u;
}

void configure(Scene* s, size_t cap, size_t scap, int tile) {
  if ((cap && cap != s->cap) || (scap && scap != s->scap))
    alloc_queues(s, cap ? cap : s->cap, scap ? scap : s->scap);
  if (tile > 0) s->tile_roots = tile;  // part of the graph key, no new epoch needed
}

void batch_iterate(Ctx* c, const int32_t* ids, int n, const mars_iter_params* p, int flags,
                   mars_iter_stats* its, mars_update_stats* ups) {
  auto t0 = std::chrono::steady_clock::now();
  if (!ids || n <= 0 || !p) throw Status(MARS_E_ARG, "empty batch or null params");
  if (flags & ~(MARS_BATCH_UPDATE | MARS_BATCH_NO_GRAPH)) throw Status(MARS_E_ARG, "unknown batch flags");
  const bool with_update = (flags & MARS_BATCH_UPDATE) != 0;
  const bool use_graph = (flags & MARS_BATCH_NO_GRAPH) == 0;
  if (p->debug_depth > 0) throw Status(MARS_E_ARG, "debug records are not batched");
  std::vector<Scene*> sc(n);
  std::vector<double> work(n);
  for (int i = 0; i < n; ++i) {
    sc[i] = c->scene(ids[i]);
    for (int j = 0; j < i; ++j)
      if (sc[j] == sc[i]) throw Status(MARS_E_ARG, "a scene appears twice in the batch");
    check_params(sc[i], p);
    if (sc[i]->mlp_on) throw Status(MARS_E_ARG, "learned-cache scenes are not batched");
    if (roots_of(sc[i], p->spp) > 0x7FFFFFFFull) throw Status(MARS_E_ARG, "too many camera samples");
    work[i] = (double)roots_of(sc[i], p->spp) * sc[i]->max_depth *
              (sc[i]->mode == MARS_MODE_BDPT ? 2.0 : 1.0);
  }
  for (Scene* s : sc) ensure_roots(s, roots_of(s, p->spp));
  ensure_pool(c);
  // longest first onto the least loaded stream
  std::vector<int> order(n), lane(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
  const int K = std::min(n, c->batch_streams);
  std::vector<double> load(K, 0.0);
  for (int i : order) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    lane[i] = k;
    load[k] += work[i];
  }
  std::vector<uint64_t> key = {(uint64_t)n, (uint64_t)flags, (uint64_t)c->counting,
                               (uint64_t)p->spp, (uint64_t)p->alloc, (uint64_t)p->budget_aware,
                               (uint64_t)p->rr_start, (uint64_t)p->fixed_scale,
                               fbits64(p->clamp_lo), fbits64(p->clamp_hi), fbits64(p->stat_clamp),
                               (uint64_t)p->center_jitter, (uint64_t)p->lp_stride,
                               (uint64_t)p->rounding, (uint64_t)c->cu};
  for (int i = 0; i < n; ++i) {
    key.push_back(sc[i]->uid);
    key.push_back(sc[i]->epoch);
    key.push_back((uint64_t)lane[i]);
    key.push_back((uint64_t)sc[i]->tile_roots);
    key.push_back((uint64_t)sc[i]->cap);
    key.push_back((uint64_t)sc[i]->scap);
  }
  BatchGraph* g = nullptr;
  for (auto& e : c->graphs)
    if (e.key == key) g = &e;
  if (!g) {
    if ((int)c->graphs.size() >= kGraphCache) {
      HIPCHK(hipStreamSynchronize(c->stream));
      c->drop_graph(c->graphs.front());
      c->graphs.erase(c->graphs.begin());
    }
    BatchGraph ng;
    ng.key = key;
    try {
      ng.iter = (int32_t*)c->dalloc(sizeof(int32_t));
      ng.summary = (double*)c->dalloc((size_t)n * kSumWords * sizeof(double));
      if (use_graph) {
        // one chain per scene, captured on its stream of the pool; launched
        // in the batch order, so that every stream gets work at once (a graph
        // launch submits its kernels one by one on the host)
        IterDev it = to_dev(p);
        it.iter_dev = ng.iter;
        for (int i : order) {
          hipStream_t ls = c->pool[lane[i]];
          HIPCHK(hipStreamBeginCapture(ls, hipStreamCaptureModeThreadLocal));
          hipGraph_t graph = nullptr;
          try {
            enqueue_iteration(sc[i], it, p->spp, with_update, p->stat_clamp, ls,
                              ng.summary + (size_t)i * kSumWords);
          } catch (...) {
            (void)hipStreamEndCapture(ls, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            throw;
          }
          HIPCHK(hipStreamEndCapture(ls, &graph));
          hipGraphExec_t ex = nullptr;
          const hipError_t e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
          (void)hipGraphDestroy(graph);
          if (e != hipSuccess)
            throw Status(MARS_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
          ng.exec.push_back(ex);
        }
      }
    } catch (...) {
      c->drop_graph(ng);
      throw;
    }
    c->graphs.push_back(ng);
    g = &c->graphs.back();
  }
  hipStream_t st = c->stream;
  k_set_i32(g->iter, p->iteration, st);
  timed(c, KID_BATCH, [&] {
    HIPCHK(hipEventRecord(c->pool_ev[0], st));
    for (int k = 0; k < K; ++k) HIPCHK(hipStreamWaitEvent(c->pool[k], c->pool_ev[0], 0));
    if (use_graph) {
      for (size_t o = 0; o < order.size(); ++o)
        HIPCHK(hipGraphLaunch(g->exec[o], c->pool[lane[order[o]]]));
    } else {
      IterDev it = to_dev(p);
      it.iter_dev = g->iter;
      for (int i : order)
        enqueue_iteration(sc[i], it, p->spp, with_update, p->stat_clamp, c->pool[lane[i]],
                          g->summary + (size_t)i * kSumWords);
    }
    for (int k = 0; k < K; ++k) {
      HIPCHK(hipEventRecord(c->pool_ev[1 + k], c->pool[k]));
      HIPCHK(hipStreamWaitEvent(st, c->pool_ev[1 + k], 0));
    }
  });
  std::vector<double> hs((size_t)n * kSumWords);
  d2h(hs.data(), g->summary, hs.size() * sizeof(double), st);
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipGetLastError());
  c->prof.flush();
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  for (int i = 0; i < n; ++i) {
    Scene* s = sc[i];
    const double* h = &hs[(size_t)i * kSumWords];
    if (h[0] != 0.0) {
      // a queue overflowed: this scene again on its own, with tile halving;
      // later batches keep its tile (overflows are occasional, and smaller
      // tiles cost every iteration; tiles do not change results)
      const int tile0 = s->tile_roots;
      mars_iter_stats S{};
      render_iteration(s, p, &S);
      s->tile_roots = tile0;
      if (its) its[i] = S;
      if (with_update) {
        mars_update_stats U{};
        update_counts(s, p, &U);
        if (ups) ups[i] = U;
      }
      continue;
    }
    const size_t roots = roots_of(s, p->spp);
    const size_t tile = std::max<size_t>(1, std::min<size_t>(s->tile_roots, s->cap));
    mars_iter_stats S{};
    S.rays_camera = roots;
    S.rays_ext = (uint64_t)h[1];
    S.rays_shadow = (uint64_t)h[2];
    S.rays_light = (uint64_t)h[3];
    S.rays_conn = (uint64_t)h[4];
    S.vertices = (uint64_t)h[5];
    S.samples = (uint64_t)h[6];
    S.tiles = (int32_t)((roots + tile - 1) / tile);
    S.ms = ms;
    s->spp_last = p->spp;
    s->vertices_last = S.vertices;
    s->rays_last = S.rays_camera + S.rays_ext + S.rays_shadow + S.rays_light + S.rays_conn;
    s->dbg_last = 0;
    if (its) its[i] = S;
    if (with_update) {
      const double* red = h + 7;
      mars_update_stats U{};
      U.V_I = red[4] > 0.0 ? red[3] / red[4] : 0.0;
      U.C_I = (double)s->rays_last / (double)roots;
      U.n_cells_before = s->n_cells;
      s->n_cells = (int)h[15];
      s->n_nodes = (int)h[16];
      s->total_spp = red[6];
      U.n_cells_after = s->n_cells;
      U.n_excluded = s->W * s->H - (int)red[4];
      if (ups) ups[i] = U;
    }
  }
}

// ---------------------------------------------------------------------------
// queue / tile autotuner
// ---------------------------------------------------------------------------
// the probe's peak per camera sample with half again as much room: later
// iterations' peaks move with the counts, and an overflow re-runs a tile
size_t tuned_capacity(size_t tile, double e) {
  const double want = std::ceil((double)tile * std::max(1.0, e) * 1.5);
  size_t cap = (size_t)want;
  cap = (cap + 4095) / 4096 * 4096;
  return std::min<size_t>(std::max<size_t>(cap, 4096), 0xFFFF0000ull);
}

// smallest tile worth a launch sequence: about 2^18 queue entries at the
// peak level of either queue (enough rays to fill the chip), at least 4096
// camera samples
constexpr double kTuneMinEntries = 262144.0;
size_t min_tile(size_t roots, double e) {
  const size_t t = (size_t)std::ceil(kTuneMinEntries / std::max(1.0, e));
  return std::min(roots, (std::max<size_t>(t, 4096) + 63) / 64 * 64);
}

size_t queue_bytes(const Scene* s, size_t cap, size_t scap) {
  return (size_t)(s->max_depth + 2) *
             (cap * (kRayEntryBytes + (s->mlp_on ? 16 : 0) + (s->mode == MARS_MODE_BDPT ? 32 : 0) +
                     (s->sd.lp_classes == 3 ? 32 : 0)) +
              scap * kShadowValueBytes) +
         scap * kShadowRayBytes;
}

std::string scene_class(const Scene* s, const mars_iter_params* p) {
  char b[192];
  std::snprintf(b, sizeof(b), "%dx%d/spp%d/mode%d/depth%d/tris%d/alloc%d", s->W, s->H, p->spp,
                s->mode, s->max_depth, s->n_tris, p->alloc);
  return b;
}

struct TuneEntry {
  size_t cap = 0, scap = 0;  // ray-queue and shadow-queue entries per level
  int tile = 0;
  double e = 0.0, es = 0.0, ms = 0.0;  // peak ray / shadow entries per camera sample
};

void autotune(Ctx* c, const int32_t* ids, int n, const mars_iter_params* p, int64_t budget,
              const char* path, int64_t* ocap, int32_t* otile, double* opeak, int64_t* oscap,
              double* ospeak) {
  if (!ids || n <= 0 || !p) throw Status(MARS_E_ARG, "empty batch or null params");
  if (budget <= 0) {
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot));
    budget = (int64_t)(fr / 4);
  }
  std::vector<Scene*> sc(n);
  for (int i = 0; i < n; ++i) {
    sc[i] = c->scene(ids[i]);
    check_params(sc[i], p);
  }
  std::vector<std::pair<std::string, TuneEntry>> cache;
  if (path) {
    if (FILE* f = std::fopen(path, "r")) {
      char line[512], cls[192];
      unsigned long long cap, scap;
      int tile;
      double e, es, ms;
      while (std::fgets(line, sizeof(line), f))
        if (std::sscanf(line, "%191s %llu %llu %d %lf %lf %lf", cls, &cap, &scap, &tile, &e, &es,
                        &ms) == 7 &&
            cap > 0 && cap <= 0xFFFF0000ull && scap > 0 && scap <= 0xFFFF0000ull && tile > 0 &&
            (size_t)tile <= cap)
          cache.push_back({cls, TuneEntry{(size_t)cap, (size_t)scap, tile, e, es, ms}});
      std::fclose(f);
    }
  }
  auto find = [&](const std::string& k) -> TuneEntry* {
    for (auto& e : cache)
      if (e.first == k) return &e.second;
    return nullptr;
  };
  std::vector<TuneEntry> res(n);
  std::vector<int> todo;
  for (int i = 0; i < n; ++i) {
    if (TuneEntry* t = find(scene_class(sc[i], p))) {
      configure(sc[i], t->cap, t->scap, t->tile);
      res[i] = *t;
    } else {
      todo.push_back(i);
    }
  }
  // probe: peak queue levels per camera sample at the current sizes
  for (int i : todo) {
    render_iteration(sc[i], p, nullptr);
    res[i].e = std::max(1.0, sc[i]->peak_ray);
    res[i].es = std::max(1.0, sc[i]->peak_shadow);
  }
  auto bytes_at = [&](int i, size_t t) {
    return queue_bytes(sc[i], tuned_capacity(t, res[i].e), tuned_capacity(t, res[i].es));
  };
  auto floor_of = [&](int i) {
    return min_tile(roots_of(sc[i], p->spp), std::max(res[i].e, res[i].es));
  };
  // plan: whole-iteration tiles, the largest scenes halved until the queues fit
  std::vector<size_t> T(n);
  double used = 0.0;
  for (int i = 0; i < n; ++i) {
    const bool tuned = std::find(todo.begin(), todo.end(), i) != todo.end();
    T[i] = tuned ? roots_of(sc[i], p->spp) : (size_t)res[i].tile;
    used += (double)(tuned ? bytes_at(i, T[i]) : queue_bytes(sc[i], res[i].cap, res[i].scap));
  }
  while (used > (double)budget) {
    int best = -1;
    size_t bytes = 0;
    for (int i : todo) {
      const size_t b = bytes_at(i, T[i]);
      if (T[i] > floor_of(i) && b > bytes) { best = i; bytes = b; }
    }
    if (best < 0) throw Status(MARS_E_OOM, "queue memory budget too small for the batch");
    T[best] = std::max(floor_of(best), (T[best] + 1) / 2);
    used += (double)bytes_at(best, T[best]) - (double)bytes;
  }
  // measure: the planned tile and two smaller ones, one timed iteration each
  for (int i : todo) {
    Scene* s = sc[i];
    const size_t floor_t = floor_of(i);
    std::vector<size_t> cand;
    for (size_t t = T[i]; cand.size() < 3; t /= 2) {
      const size_t tt = std::max(floor_t, t);
      if (std::find(cand.begin(), cand.end(), tt) == cand.end()) cand.push_back(tt);
      if (tt == floor_t) break;
    }
    // each candidate's time is the better of two iterations; a smaller tile
    // replaces a larger one only when at least 3% faster (one iteration's
    // time varies by a few percent, and larger tiles fill the late bounces)
    double best_ms = INFINITY;
    size_t best_t = cand[0];
    for (size_t k = 0; k < cand.size(); ++k) {
      configure(s, tuned_capacity(cand[k], res[i].e), tuned_capacity(cand[k], res[i].es),
                (int)std::min<size_t>(cand[k], 0x7FFFFFFF));
      if (k == 0) render_iteration(s, p, nullptr);  // first use of the new buffers
      double ms = INFINITY;
      for (int r = 0; r < 2; ++r) {
        mars_iter_stats S{};
        render_iteration(s, p, &S);
        ms = std::min(ms, S.ms);
      }
      if (k == 0 || ms < 0.97 * best_ms) { best_ms = ms; best_t = cand[k]; }
    }
    res[i].tile = (int)std::min<size_t>(best_t, 0x7FFFFFFF);
    res[i].cap = tuned_capacity(best_t, res[i].e);
    res[i].scap = tuned_capacity(best_t, res[i].es);
    res[i].ms = best_ms;
    configure(s, res[i].cap, res[i].scap, res[i].tile);
    const std::string k = scene_class(s, p);
    if (TuneEntry* t = find(k)) *t = res[i];
    else cache.push_back({k, res[i]});
  }
  if (path && !todo.empty()) {
    FILE* f = std::fopen(path, "w");
    if (!f) throw Status(MARS_E_IO, "cannot write the autotuner cache");
    for (auto& e : cache)
      std::fprintf(f, "%s %llu %llu %d %.6g %.6g %.6g\n", e.first.c_str(),
                   (unsigned long long)e.second.cap, (unsigned long long)e.second.scap,
                   e.second.tile, e.second.e, e.second.es, e.second.ms);
    if (std::fclose(f) != 0) throw Status(MARS_E_IO, "cannot write the autotuner cache");
  }
  for (int i = 0; i < n; ++i) {
    if (ocap) ocap[i] = (int64_t)sc[i]->cap;
    if (otile) otile[i] = sc[i]->tile_roots;
    if (opeak) opeak[i] = res[i].e;
    if (oscap) oscap[i] = (int64_t)sc[i]->scap;
    if (ospeak) ospeak[i] = res[i].es;
  }
}

struct CkptHeader {
  char magic[8];
  int32_t version, W, H, max_cells, n_cells, n_nodes, mode, spp_last;
  double total_spp, ivw_w;
};

}  // namespace

namespace {
void out_copy(Ctx* c, float* dst, const float* host, size_t n, int dst_is_device) {
  if (dst_is_device) {
    HIPCHK(hipMemcpyAsync(dst, host, n * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  } else {
    std::memcpy(dst, host, n * 4);
  }
}
void dev_out(Ctx* c, float* dst, const float* src, size_t n, int dst_is_device) {
  HIPCHK(hipMemcpyAsync(dst, src, n * 4, dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
}
}  // namespace

namespace {
Scene* mlp_scene(Ctx* ctx, int32_t id) {
  Scene* s = ctx->scene(id);
  if (!s->mlp_on) throw Status(MARS_E_STATE, "learned cache not enabled for scene");
  return s;
}
// one Adam step over `batch` samples of (x6, tgt, wt) starting at offset
void mlp_step_once(Scene* s, const float* x6, const float* tgt, const float* wt, int n_set,
                   int offset, int batch, float lr, float* loss_dev) {
  hipStream_t st = s->ctx->stream;
  int nb = 0;
  k_mlp_train_pass(s->mlp, x6, tgt, wt, n_set, offset, batch, &nb, st);
  s->mlp_step += 1;
  const float bc1 = (float)(1.0 - std::pow(0.9, s->mlp_step));
  const float bc2 = (float)(1.0 - std::pow(0.99, s->mlp_step));
  k_mlp_adam(s->mlp, nb, nullptr, lr, bc1, bc2, loss_dev, st);
}
}  // namespace

namespace {
template <typename F>
void with_device_buffers(Ctx* c, std::initializer_list<size_t> sizes, F&& f) {
  std::vector<void*> bufs;
  try {
    for (size_t b : sizes) bufs.push_back(c->dalloc(b));
    f(bufs);
  } catch (...) {
    for (void* p : bufs) c->dfree(p);
    throw;
  }
  for (void* p : bufs) c->dfree(p);
}
}  // namespace

struct mars_ctx : Ctx {};

extern "C" {

const char* mars_version(void) { return "mars-mi355x 0.1"; }

const char* mars_last_error(const mars_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

mars_status mars_create(const mars_ctx_desc* desc, mars_ctx** out) {
  if (!desc || !out) return MARS_E_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return MARS_E_HIP;
  if (desc->device < 0 || desc->device >= n) return MARS_E_ARG;
  if (hipSetDevice(desc->device) != hipSuccess) return MARS_E_HIP;
  auto* c = new (std::nothrow) mars_ctx();
  if (!c) return MARS_E_OOM;
  c->device = desc->device;
  c->stream = (hipStream_t)desc->stream;
  c->alloc = desc->alloc;
  c->free_ = desc->free;
  c->user = desc->user;
  int cu = 0;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, desc->device) == hipSuccess &&
      cu > 0)
    c->cu = cu;
  if (hipHostMalloc((void**)&c->pinned, kPinnedBytes, hipHostMallocDefault) != hipSuccess) {
    delete c;
    return MARS_E_OOM;
  }
  {
    const hipError_t e = noalloc_scratch_address(desc->device, &c->noalloc_scratch);
    if (e != hipSuccess) {
      c->noalloc_scratch = nullptr;
      c->noalloc_error = std::string("address of the fixed gradient array: ") +
                         hipGetErrorString(e);
    }
  }
  // launch grids sized by occupancy, queried now rather than under a capture
  k_init_launch_grids();
  c->batch_streams = kBatchStreams;
  if (const char* e = std::getenv("MARS_BATCH_STREAMS")) {
    const int k = std::atoi(e);
    if (k >= 1 && k <= 16) c->batch_streams = k;
  }
  *out = c;
  return MARS_OK;
}

mars_status mars_destroy(mars_ctx* ctx) {
  if (!ctx) return MARS_E_ARG;
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& g : ctx->graphs) ctx->drop_graph(g);
  ctx->graphs.clear();
  for (auto s : ctx->pool) (void)hipStreamDestroy(s);
  for (auto e : ctx->pool_ev) (void)hipEventDestroy(e);
  for (auto& s : ctx->scenes) release_scene(s.get());
  if (ctx->tcount) ctx->dfree(ctx->tcount);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  delete ctx;
  return MARS_OK;
}

mars_status mars_profile_enable_mask(mars_ctx* ctx, uint64_t kernel_mask) {
  if (!ctx) return MARS_E_ARG;
  return guard(ctx, [&] {
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->prof.flush();
    ctx->prof.reset();
    ctx->prof.mask = kernel_mask & ((1ull << KID_COUNT) - 1);
  });
}

mars_status mars_profile_enable(mars_ctx* ctx, int32_t on) {
  return mars_profile_enable_mask(ctx, on ? ~0ull : 0ull);
}

mars_status mars_profile_read(mars_ctx* ctx, double* ms, uint64_t* launches, int32_t n,
                              int32_t* n_kernels) {
  if (!ctx) return MARS_E_ARG;
  return guard(ctx, [&] {
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->prof.flush();
    if (n_kernels) *n_kernels = KID_COUNT;
    for (int k = 0; k < n && k < KID_COUNT; ++k) {
      if (ms) ms[k] = ctx->prof.ms[k];
      if (launches) launches[k] = ctx->prof.n[k];
    }
  });
}

const char* mars_profile_kernel_name(int32_t id) {
  return (id >= 0 && id < KID_COUNT) ? kKernelNames[id] : "";
}

mars_status mars_trace_counting(mars_ctx* ctx, int32_t on) {
  if (!ctx) return MARS_E_ARG;
  return guard(ctx, [&] {
    if (!ctx->tcount) ctx->tcount = (unsigned long long*)ctx->dalloc(8 * 16);
    k_fill_u32((uint32_t*)ctx->tcount, 0u, 32, ctx->stream);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->counting = on != 0;
  });
}

mars_status mars_read_trace_counts(mars_ctx* ctx, uint64_t out[10]) {
  if (!ctx || !out) return MARS_E_ARG;
  return guard(ctx, [&] {
    if (!ctx->tcount) throw Status(MARS_E_STATE, "trace counting never enabled");
    d2h(out, ctx->tcount, 80, ctx->stream);
    HIPCHK(hipStreamSynchronize(ctx->stream));
  });
}

mars_status mars_scene_upload(mars_ctx* ctx, const mars_scene_desc* desc, int32_t* scene_id) {
  if (!ctx || !scene_id) return MARS_E_ARG;
  return guard(ctx, [&] {
    HIPCHK(hipSetDevice(ctx->device));
    *scene_id = upload_scene(ctx, desc);
  });
}

mars_status mars_scene_release(mars_ctx* ctx, int32_t scene_id) {
  if (!ctx) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = ctx->scene(scene_id);
    release_scene(s);
    ctx->scenes[scene_id].reset();
  });
}

mars_status mars_render_iteration(mars_ctx* ctx, int32_t scene_id, const mars_iter_params* p,
                                  mars_iter_stats* stats) {
  if (!ctx) return MARS_E_ARG;
  return guard(ctx, [&] { render_iteration(ctx->scene(scene_id), p, stats); });
}

mars_status mars_render_batch(mars_ctx* ctx, const int32_t* scene_ids, int32_t n,
                              const mars_iter_params* p, mars_iter_stats* stats) {
  if (!ctx || !scene_ids || n <= 0 || !p) return MARS_E_ARG;
  return guard(ctx, [&] {
    auto t0 = std::chrono::steady_clock::now();
    bool graph = p->debug_depth <= 0;
    for (int i = 0; i < n; ++i)
      if (ctx->scene(scene_ids[i])->mlp_on) graph = false;
    std::vector<mars_iter_stats> one(n);
    if (graph) {
      batch_iterate(ctx, scene_ids, n, p, 0, one.data(), nullptr);
    } else {
      for (int i = 0; i < n; ++i) {
        for (int j = 0; j < i; ++j)
          if (scene_ids[j] == scene_ids[i]) throw Status(MARS_E_ARG, "a scene appears twice in the batch");
        render_iteration(ctx->scene(scene_ids[i]), p, &one[i]);
      }
    }
    mars_iter_stats tot{};
    for (const auto& o : one) {
      tot.rays_camera += o.rays_camera; tot.rays_ext += o.rays_ext;
      tot.rays_shadow += o.rays_shadow; tot.rays_light += o.rays_light;
      tot.rays_conn += o.rays_conn; tot.vertices += o.vertices; tot.samples += o.samples;
      tot.tiles += o.tiles; tot.overflow_retries += o.overflow_retries;
    }
    tot.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = tot;
  });
}

mars_status mars_iterate_batch(mars_ctx* ctx, const int32_t* scene_ids, int32_t n,
                               const mars_iter_params* p, int32_t flags,
                               mars_iter_stats* iter_stats, mars_update_stats* upd_stats) {
  if (!ctx) return MARS_E_ARG;
  return guard(ctx, [&] { batch_iterate(ctx, scene_ids, n, p, flags, iter_stats, upd_stats); });
}

mars_status mars_scene_configure_queues(mars_ctx* ctx, int32_t scene_id, int64_t ray_capacity,
                                        int64_t shadow_capacity, int32_t tile_roots) {
  if (!ctx) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = ctx->scene(scene_id);
    if (ray_capacity < 0 || ray_capacity > (int64_t)0xFFFF0000ull || shadow_capacity < 0 ||
        shadow_capacity > (int64_t)0xFFFF0000ull || tile_roots < 0)
      throw Status(MARS_E_ARG, "bad queue capacity or tile size");
    const size_t cap = ray_capacity > 0 ? (size_t)ray_capacity : s->cap;
    const size_t scap = shadow_capacity > 0 ? (size_t)shadow_capacity : s->scap;
    const size_t tile = tile_roots > 0 ? (size_t)tile_roots : (size_t)s->tile_roots;
    if (tile > cap) throw Status(MARS_E_ARG, "tile larger than the queue capacity");
    configure(s, cap, scap, (int)tile);
  });
}

mars_status mars_scene_configure(mars_ctx* ctx, int32_t scene_id, int64_t queue_capacity,
                                 int32_t tile_roots) {
  return mars_scene_configure_queues(ctx, scene_id, queue_capacity, queue_capacity, tile_roots);
}

mars_status mars_scene_query(mars_ctx* ctx, int32_t scene_id, int64_t* queue_capacity,
                             int32_t* tile_roots, double* peak_per_root) {
  if (!ctx) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = ctx->scene(scene_id);
    if (queue_capacity) *queue_capacity = (int64_t)s->cap;
    if (tile_roots) *tile_roots = s->tile_roots;
    if (peak_per_root) *peak_per_root = s->peak_per_root;
  });
}

mars_status mars_scene_query_queues(mars_ctx* ctx, int32_t scene_id, int64_t* ray_capacity,
                                    int64_t* shadow_capacity, double* peak_ray,
                                    double* peak_shadow) {
  if (!ctx) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = ctx->scene(scene_id);
    if (ray_capacity) *ray_capacity = (int64_t)s->cap;
    if (shadow_capacity) *shadow_capacity = (int64_t)s->scap;
    if (peak_ray) *peak_ray = s->peak_ray;
    if (peak_shadow) *peak_shadow = s->peak_shadow;
  });
}

mars_status mars_autotune(mars_ctx* ctx, const int32_t* scene_ids, int32_t n,
                          const mars_iter_params* p, int64_t mem_budget, const char* cache_path,
                          int64_t* out_capacity, int32_t* out_tile, double* out_peak,
                          int64_t* out_shadow_capacity, double* out_shadow_peak) {
  if (!ctx) return MARS_E_ARG;
  return guard(ctx, [&] {
    autotune(ctx, scene_ids, n, p, mem_budget, cache_path, out_capacity, out_tile, out_peak,
             out_shadow_capacity, out_shadow_peak);
  });
}

mars_status mars_update_counts(mars_ctx* ctx, int32_t scene_id, const mars_iter_params* p,
                               mars_update_stats* stats) {
  if (!ctx) return MARS_E_ARG;
  return guard(ctx, [&] { update_counts(ctx->scene(scene_id), p, stats); });
}

mars_status mars_set_fixed_counts(mars_ctx* ctx, int32_t scene_id, const float* beta, int32_t n) {
  if (!ctx || !beta) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = ctx->scene(scene_id);
    if (n != 1 && n != s->n_cells) throw Status(MARS_E_ARG, "n must be 1 or the number of cells");
    for (int i = 0; i < 3 * n; ++i)
      if (!std::isfinite(beta[i]) || beta[i] < 0.0f) throw Status(MARS_E_ARG, "bad fixed count");
    if (!s->fixed) s->fixed = salloc<float>(s, 3 * (size_t)s->max_cells);
    h2d(s->fixed, beta, 12 * (size_t)n, ctx->stream);
    s->n_fixed = n;
    s->cd.fixed = s->fixed;
    s->cd.n_fixed = n;
    s->epoch++;  // the cache view is captured by value
    HIPCHK(hipStreamSynchronize(ctx->stream));
  });
}

mars_status mars_set_itilde(mars_ctx* ctx, int32_t scene_id, const float* itilde) {
  if (!ctx || !itilde) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = ctx->scene(scene_id);
    h2d(s->img.itilde, itilde, 12 * (size_t)s->W * s->H, ctx->stream);
    HIPCHK(hipStreamSynchronize(ctx->stream));
  });
}

mars_status mars_set_hist(mars_ctx* ctx, int32_t scene_id, int32_t n, const float* pm,
                          const float* cdf) {
  if (!ctx || !pm || !cdf) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = ctx->scene(scene_id);
    if (n <= 0 || n > s->n_cells) throw Status(MARS_E_ARG, "bad cell count");
    h2d(s->cd.pm, pm, 256 * (size_t)n, ctx->stream);
    h2d(s->cd.cdf, cdf, 256 * (size_t)n, ctx->stream);
    HIPCHK(hipStreamSynchronize(ctx->stream));
  });
}

mars_status mars_write_cells(mars_ctx* ctx, int32_t scene_id, int32_t n, const float* factors,
                             const double* acc, const uint32_t* visits) {
  if (!ctx) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = ctx->scene(scene_id);
    if (n != s->n_cells) throw Status(MARS_E_ARG, "n must equal the number of cells");
    if (factors) h2d(s->cd.fac, factors, 72 * (size_t)n, ctx->stream);
    if (acc) h2d(s->cd.acc, acc, 192 * (size_t)n, ctx->stream);
    if (visits) h2d(s->cd.visits, visits, 4 * (size_t)n, ctx->stream);
    HIPCHK(hipStreamSynchronize(ctx->stream));
  });
}

mars_status mars_update_cells_only(mars_ctx* ctx, int32_t scene_id, double V_I, double C_I) {
  if (!ctx) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = ctx->scene(scene_id);
    k_fixed_point(s->cd, s->n_cells_dev, s->img.red, C_I, nullptr, 0.0, 0, V_I, 0, s->max_cells,
                  nullptr, 0, 1, nullptr, ctx->stream);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipGetLastError());
  });
}

mars_status mars_refine_only(mars_ctx* ctx, int32_t scene_id, int32_t* n_split) {
  if (!ctx) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = ctx->scene(scene_id);
    const int before = s->n_cells;
    k_refine(s->cd, s->n_cells_dev, s->n_cells_dev + 1, s->scratch, s->split_visits,
             s->max_tree_depth, s->max_cells, nullptr, ctx->stream);
    int32_t nc[4];
    d2h(nc, s->n_cells_dev, sizeof(nc), ctx->stream);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    s->n_cells = nc[0];
    s->n_nodes = nc[1];
    if (n_split) *n_split = (s->n_cells - before) / 7;
  });
}


mars_status mars_read_image(mars_ctx* ctx, int32_t scene_id, int32_t which, float* dst,
                            int32_t dst_is_device) {
  if (!ctx || !dst) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = ctx->scene(scene_id);
    const size_t n = 3 * (size_t)s->W * s->H;
    std::vector<float> out(n, 0.0f);
    if (which == MARS_IMAGE_MEAN) {
      std::vector<float> a(n);
      d2h(a.data(), s->img.accum, n * 4, ctx->stream);
      HIPCHK(hipStreamSynchronize(ctx->stream));
      if (s->total_spp > 0)
        for (size_t i = 0; i < n; ++i) out[i] = a[i] / (float)s->total_spp;
    } else if (which == MARS_IMAGE_IVW) {
      std::vector<double> a(n), red(8);
      d2h(a.data(), s->img.ivw_acc, n * 8, ctx->stream);
      d2h(red.data(), s->img.red, 64, ctx->stream);
      HIPCHK(hipStreamSynchronize(ctx->stream));
      if (red[5] > 0)
        for (size_t i = 0; i < n; ++i) out[i] = (float)(a[i] / red[5]);
    } else if (which == MARS_IMAGE_LAST) {
      std::vector<float> a(n);
      d2h(a.data(), s->img.iter_sum, n * 4, ctx->stream);
      HIPCHK(hipStreamSynchronize(ctx->stream));
      if (s->spp_last > 0)
        for (size_t i = 0; i < n; ++i) out[i] = a[i] / (float)s->spp_last;
    } else {
      throw Status(MARS_E_ARG, "bad image kind");
    }
    out_copy(ctx, dst, out.data(), n, dst_is_device);
  });
}

mars_status mars_read_count_map(mars_ctx* ctx, int32_t scene_id, float* dst,
                                int32_t dst_is_device) {
  if (!ctx || !dst) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = ctx->scene(scene_id);
    dev_out(ctx, dst, s->img.count_map, 3 * (size_t)s->W * s->H, dst_is_device);
  });
}

mars_status mars_read_sample_radiance(mars_ctx* ctx, int32_t scene_id, float* dst,
                                      int32_t dst_is_device) {
  if (!ctx || !dst) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = ctx->scene(scene_id);
    if (s->spp_last <= 0) throw Status(MARS_E_STATE, "no iteration rendered");
    dev_out(ctx, dst, s->img.Ls, 3 * (size_t)s->W * s->H * s->spp_last, dst_is_device);
  });
}

mars_status mars_read_itilde(mars_ctx* ctx, int32_t scene_id, float* dst, int32_t dst_is_device) {
  if (!ctx || !dst) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = ctx->scene(scene_id);
    dev_out(ctx, dst, s->img.itilde, 3 * (size_t)s->W * s->H, dst_is_device);
  });
}

mars_status mars_num_cells(mars_ctx* ctx, int32_t scene_id, int32_t* n_cells, int32_t* n_nodes) {
  if (!ctx) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = ctx->scene(scene_id);
    if (n_cells) *n_cells = s->n_cells;
    if (n_nodes) *n_nodes = s->n_nodes;
  });
}

mars_status mars_read_cells(mars_ctx* ctx, int32_t scene_id, float* factors, double* acc,
                            uint32_t* visits, uint32_t* leaf_depth) {
  if (!ctx) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = ctx->scene(scene_id);
    const size_t n = (size_t)s->n_cells;
    if (factors) d2h(factors, s->cd.fac, 72 * n, ctx->stream);
    if (acc) d2h(acc, s->cd.acc, 192 * n, ctx->stream);
    if (visits) d2h(visits, s->cd.visits, 4 * n, ctx->stream);
    if (leaf_depth) d2h(leaf_depth, s->cd.leaf_depth, 4 * n, ctx->stream);
    HIPCHK(hipStreamSynchronize(ctx->stream));
  });
}

mars_status mars_read_cells_x(mars_ctx* ctx, int32_t scene_id, float* factors_x, double* acc_x) {
  if (!ctx) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = ctx->scene(scene_id);
    if (!s->cd.fac_x) throw Status(MARS_E_STATE, "scene has one light-path budget");
    const size_t n = (size_t)s->n_cells;
    if (factors_x) d2h(factors_x, s->cd.fac_x, 48 * n, ctx->stream);
    if (acc_x) d2h(acc_x, s->cd.acc_x, 128 * n, ctx->stream);
    HIPCHK(hipStreamSynchronize(ctx->stream));
  });
}

mars_status mars_write_cells_x(mars_ctx* ctx, int32_t scene_id, int32_t n, const float* factors_x,
                               const double* acc_x) {
  if (!ctx) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = ctx->scene(scene_id);
    if (!s->cd.fac_x) throw Status(MARS_E_STATE, "scene has one light-path budget");
    if (n != s->n_cells) throw Status(MARS_E_ARG, "n must equal the number of cells");
    if (factors_x) h2d(s->cd.fac_x, factors_x, 48 * (size_t)n, ctx->stream);
    if (acc_x) h2d(s->cd.acc_x, acc_x, 128 * (size_t)n, ctx->stream);
    HIPCHK(hipStreamSynchronize(ctx->stream));
  });
}

mars_status mars_read_nodes(mars_ctx* ctx, int32_t scene_id, uint32_t* nodes) {
  if (!ctx || !nodes) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = ctx->scene(scene_id);
    d2h(nodes, s->cd.nodes, 4 * (size_t)s->n_nodes, ctx->stream);
    HIPCHK(hipStreamSynchronize(ctx->stream));
  });
}

mars_status mars_read_hist(mars_ctx* ctx, int32_t scene_id, float* pm, float* cdf) {
  if (!ctx) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = ctx->scene(scene_id);
    if (pm) d2h(pm, s->cd.pm, 256 * (size_t)s->n_cells, ctx->stream);
    if (cdf) d2h(cdf, s->cd.cdf, 256 * (size_t)s->n_cells, ctx->stream);
    HIPCHK(hipStreamSynchronize(ctx->stream));
  });
}

mars_status mars_debug_vertices(mars_ctx* ctx, int32_t scene_id, mars_vertex_rec* dst, int32_t cap,
                                int32_t* n) {
  if (!ctx || !n) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = ctx->scene(scene_id);
    static_assert(sizeof(mars_vertex_rec) == sizeof(DebugRec), "record layout");
    const uint32_t total = std::min(s->dbg_last, s->dbg_cap);
    *n = (int32_t)total;
    const uint32_t m = std::min<uint32_t>(total, cap > 0 ? (uint32_t)cap : 0u);
    if (dst && m) {
      d2h(dst, s->dbg, sizeof(DebugRec) * m, ctx->stream);
      HIPCHK(hipStreamSynchronize(ctx->stream));
    }
  });
}

mars_status mars_checkpoint_save(mars_ctx* ctx, int32_t scene_id, const char* path) {
  if (!ctx || !path) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = ctx->scene(scene_id);
    hipStream_t st = ctx->stream;
    const size_t nc = (size_t)s->n_cells, nn = (size_t)s->n_nodes, px = (size_t)s->W * s->H;
    std::vector<uint32_t> nodes(nn), lnode(nc), ldep(nc);
    std::vector<float> fac(nc * 18), pm(nc * 64), cdf(nc * 64), accum(px * 3), it(px * 3);
    std::vector<double> ivw(px * 3), red(8);
    d2h(nodes.data(), s->cd.nodes, nn * 4, st);
    d2h(lnode.data(), s->cd.leaf_node, nc * 4, st);
    d2h(ldep.data(), s->cd.leaf_depth, nc * 4, st);
    d2h(fac.data(), s->cd.fac, nc * 72, st);
    d2h(pm.data(), s->cd.pm, nc * 256, st);
    d2h(cdf.data(), s->cd.cdf, nc * 256, st);
    d2h(accum.data(), s->img.accum, px * 12, st);
    d2h(it.data(), s->img.itilde, px * 12, st);
    d2h(ivw.data(), s->img.ivw_acc, px * 24, st);
    d2h(red.data(), s->img.red, 64, st);
    std::vector<float> facx(s->cd.fac_x ? nc * 12 : 0);
    if (s->cd.fac_x) d2h(facx.data(), s->cd.fac_x, nc * 48, st);
    HIPCHK(hipStreamSynchronize(st));
    CkptHeader h{};
    std::memcpy(h.magic, "MARSCKP1", 8);
    h.version = 1; h.W = s->W; h.H = s->H; h.max_cells = s->max_cells;
    h.n_cells = s->n_cells; h.n_nodes = s->n_nodes; h.mode = s->mode; h.spp_last = s->spp_last;
    h.total_spp = s->total_spp; h.ivw_w = red[5];
    FILE* f = std::fopen(path, "wb");
    if (!f) throw Status(MARS_E_IO, "cannot open checkpoint for writing");
    bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1;
    auto w = [&](const void* p, size_t b) { ok = ok && (b == 0 || std::fwrite(p, b, 1, f) == 1); };
    w(nodes.data(), nn * 4); w(lnode.data(), nc * 4); w(ldep.data(), nc * 4);
    w(fac.data(), nc * 72); w(pm.data(), nc * 256); w(cdf.data(), nc * 256);
    w(accum.data(), px * 12); w(it.data(), px * 12); w(ivw.data(), px * 24);
    w(facx.data(), facx.size() * 4);  // per-length light-path scenes only
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) throw Status(MARS_E_IO, "checkpoint write failed");
  });
}

mars_status mars_checkpoint_load(mars_ctx* ctx, int32_t scene_id, const char* path) {
  if (!ctx || !path) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = ctx->scene(scene_id);
    FILE* f = std::fopen(path, "rb");
    if (!f) throw Status(MARS_E_IO, "cannot open checkpoint");
    CkptHeader h{};
    bool ok = std::fread(&h, sizeof(h), 1, f) == 1;
    if (!ok || std::memcmp(h.magic, "MARSCKP1", 8) != 0 || h.version != 1) {
      std::fclose(f);
      throw Status(MARS_E_IO, "not a checkpoint");
    }
    if (h.W != s->W || h.H != s->H || h.max_cells != s->max_cells || h.mode != s->mode ||
        h.n_cells <= 0 || h.n_cells > s->max_cells || h.n_nodes <= 0 ||
        h.n_nodes > 1 + 8 * s->max_cells) {
      std::fclose(f);
      throw Status(MARS_E_ARG, "checkpoint does not match the scene");
    }
    const size_t nc = (size_t)h.n_cells, nn = (size_t)h.n_nodes, px = (size_t)s->W * s->H;
    std::vector<uint32_t> nodes(nn), lnode(nc), ldep(nc);
    std::vector<float> fac(nc * 18), pm(nc * 64), cdf(nc * 64), accum(px * 3), it(px * 3);
    std::vector<double> ivw(px * 3);
    auto r = [&](void* p, size_t b) { ok = ok && (b == 0 || std::fread(p, b, 1, f) == 1); };
    r(nodes.data(), nn * 4); r(lnode.data(), nc * 4); r(ldep.data(), nc * 4);
    r(fac.data(), nc * 72); r(pm.data(), nc * 256); r(cdf.data(), nc * 256);
    r(accum.data(), px * 12); r(it.data(), px * 12); r(ivw.data(), px * 24);
    std::vector<float> facx(s->cd.fac_x ? nc * 12 : 0);
    r(facx.data(), facx.size() * 4);  // per-length light-path scenes only
    std::fclose(f);
    if (!ok) throw Status(MARS_E_IO, "truncated checkpoint");
    // structural validation: every reference stays inside the arrays
    for (size_t i = 0; i < nn; ++i) {
      const uint32_t v = nodes[i];
      if (v & kLeafBit) {
        if ((v & ~kLeafBit) >= nc) throw Status(MARS_E_IO, "corrupt checkpoint (leaf id)");
      } else if ((size_t)v + 8 > nn || v == 0) {
        throw Status(MARS_E_IO, "corrupt checkpoint (child index)");
      }
    }
    for (size_t l = 0; l < nc; ++l)
      if (lnode[l] >= nn || ldep[l] > 30) throw Status(MARS_E_IO, "corrupt checkpoint (leaf)");
    hipStream_t st = ctx->stream;
    h2d(s->cd.nodes, nodes.data(), nn * 4, st);
    h2d(s->cd.leaf_node, lnode.data(), nc * 4, st);
    h2d(s->cd.leaf_depth, ldep.data(), nc * 4, st);
    h2d(s->cd.fac, fac.data(), nc * 72, st);
    if (s->cd.fac_x) h2d(s->cd.fac_x, facx.data(), nc * 48, st);
    h2d(s->cd.pm, pm.data(), nc * 256, st);
    h2d(s->cd.cdf, cdf.data(), nc * 256, st);
    h2d(s->img.accum, accum.data(), px * 12, st);
    h2d(s->img.itilde, it.data(), px * 12, st);
    h2d(s->img.ivw_acc, ivw.data(), px * 24, st);
    const int32_t ncv[4] = {h.n_cells, h.n_nodes, 0, 0};
    h2d(s->n_cells_dev, ncv, 16, st);
    std::vector<double> red(8, 0.0);
    red[5] = h.ivw_w;
    red[6] = h.total_spp;
    h2d(s->img.red, red.data(), 64, st);
    HIPCHK(hipStreamSynchronize(st));
    s->n_cells = h.n_cells;
    s->n_nodes = h.n_nodes;
    s->total_spp = h.total_spp;
    s->spp_last = 0;
  });
}

int32_t mars_mlp_num_params(void) { return kMlpParams; }


mars_status mars_mlp_train(mars_ctx* ctx, int32_t scene_id, int32_t steps, int32_t batch, float lr,
                           float* loss, int32_t* n_train) {
  if (!ctx || steps < 0 || batch <= 0 || !(lr > 0.0f)) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = mlp_scene(ctx, scene_id);
    const int n = (int)s->mlp_n_train;
    if (n_train) *n_train = n;
    if (n == 0 || steps == 0) {
      if (loss) *loss = 0.0f;
      return;
    }
    const int b = std::min(batch, std::min(n, kMlpMaxBlocks * 16 * 64));
    float* ld = (float*)ctx->dalloc(16);
    try {
      for (int k = 0; k < steps; ++k) {
        const int off = (int)(((int64_t)(s->mlp_step) * b) % n);
        timed(ctx, KID_MLP_TRAIN, [&] {
          mlp_step_once(s, s->mlp.x6, s->mlp.tgt, s->mlp.wt, n, off, b, lr, ld);
        });
      }
      float l = 0.0f;
      d2h(&l, ld, 4, ctx->stream);
      HIPCHK(hipStreamSynchronize(ctx->stream));
      ctx->prof.flush();
      if (loss) *loss = l;
    } catch (...) {
      ctx->dfree(ld);
      throw;
    }
    ctx->dfree(ld);
  });
}

mars_status mars_mlp_read_params(mars_ctx* ctx, int32_t scene_id, float* params) {
  if (!ctx || !params) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = mlp_scene(ctx, scene_id);
    d2h(params, s->mlp.master, 4 * (size_t)kMlpParams, ctx->stream);
    HIPCHK(hipStreamSynchronize(ctx->stream));
  });
}

mars_status mars_mlp_write_params(mars_ctx* ctx, int32_t scene_id, const float* params) {
  if (!ctx || !params) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = mlp_scene(ctx, scene_id);
    for (int i = 0; i < kMlpParams; ++i)
      if (!std::isfinite(params[i])) throw Status(MARS_E_NONFINITE, "non-finite parameter");
    mlp_write_master(s, params);
  });
}


mars_status mars_mlp_forward(mars_ctx* ctx, int32_t scene_id, const float* x6, int32_t n,
                             float* y3) {
  if (!ctx || !x6 || !y3 || n <= 0) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = mlp_scene(ctx, scene_id);
    with_device_buffers(ctx, {24 * (size_t)n, 12 * (size_t)n}, [&](std::vector<void*>& b) {
      h2d(b[0], x6, 24 * (size_t)n, ctx->stream);
      k_mlp_forward(s->mlp, (const float*)b[0], n, (float*)b[1], ctx->stream);
      d2h(y3, b[1], 12 * (size_t)n, ctx->stream);
      HIPCHK(hipStreamSynchronize(ctx->stream));
      HIPCHK(hipGetLastError());
    });
  });
}

mars_status mars_mlp_grad(mars_ctx* ctx, int32_t scene_id, const float* x6, const float* target,
                          const float* weight, int32_t n, float* grad, float* loss) {
  if (!ctx || !x6 || !target || !weight || !grad || n <= 0) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = mlp_scene(ctx, scene_id);
    if (n > kMlpMaxBlocks * 16 * 64) throw Status(MARS_E_ARG, "batch too large");
    with_device_buffers(ctx, {24 * (size_t)n, 12 * (size_t)n, 12 * (size_t)n, 4 * (size_t)kMlpParams + 4},
                        [&](std::vector<void*>& b) {
      h2d(b[0], x6, 24 * (size_t)n, ctx->stream);
      h2d(b[1], target, 12 * (size_t)n, ctx->stream);
      h2d(b[2], weight, 12 * (size_t)n, ctx->stream);
      int nb = 0;
      k_mlp_train_pass(s->mlp, (const float*)b[0], (const float*)b[1], (const float*)b[2], n, 0, n,
                       &nb, ctx->stream);
      float* g = (float*)b[3];
      k_mlp_sum_partials(s->mlp, nb, g, g + kMlpParams, ctx->stream);
      d2h(grad, g, 4 * (size_t)kMlpParams, ctx->stream);
      float l = 0.0f;
      d2h(&l, g + kMlpParams, 4, ctx->stream);
      HIPCHK(hipStreamSynchronize(ctx->stream));
      HIPCHK(hipGetLastError());
      if (loss) *loss = l;
    });
  });
}

mars_status mars_mlp_apply_grad(mars_ctx* ctx, int32_t scene_id, const float* grad, float lr) {
  if (!ctx || !grad || !(lr > 0.0f)) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = mlp_scene(ctx, scene_id);
    with_device_buffers(ctx, {4 * (size_t)kMlpParams}, [&](std::vector<void*>& b) {
      h2d(b[0], grad, 4 * (size_t)kMlpParams, ctx->stream);
      s->mlp_step += 1;
      const float bc1 = (float)(1.0 - std::pow(0.9, s->mlp_step));
      const float bc2 = (float)(1.0 - std::pow(0.99, s->mlp_step));
      k_mlp_adam(s->mlp, 0, (const float*)b[0], lr, bc1, bc2, nullptr, ctx->stream);
      HIPCHK(hipStreamSynchronize(ctx->stream));
      HIPCHK(hipGetLastError());
    });
  });
}

mars_status mars_mlp_grad_noalloc(mars_ctx* ctx, int32_t scene_id, const float* x6,
                                  const float* target, const float* weight, int32_t n,
                                  float* grad) {
  if (!ctx || !x6 || !target || !weight || !grad || n <= 0) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = mlp_scene(ctx, scene_id);
    if (n > kMlpMaxBlocks * 16 * 64)
      throw Status(MARS_E_ARG, "batch larger than the fixed gradient array allows (262144)");
    if (!ctx->noalloc_scratch) throw Status(MARS_E_STATE, ctx->noalloc_error);
    MlpDev m = s->mlp;
    m.partial = ctx->noalloc_scratch;
    int nb = 0;
    k_mlp_train_pass(m, x6, target, weight, n, 0, n, &nb, ctx->stream);
    if (nb > kMlpMaxBlocks) throw Status(MARS_E_STATE, "gradient pass wider than its array");
    k_mlp_sum_partials(m, nb, grad, grad + kMlpParams, ctx->stream);
    HIPCHK(hipGetLastError());
  });
}

mars_status mars_mlp_write_records(mars_ctx* ctx, int32_t scene_id, const float* pos,
                                   const float* nrm, const float* T, const uint32_t* pix,
                                   int32_t n) {
  if (!ctx || !pos || !nrm || !T || !pix || n < 0) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = mlp_scene(ctx, scene_id);
    if ((uint32_t)n > s->mlp.rec_cap) throw Status(MARS_E_ARG, "more records than the capacity");
    const uint32_t npx = (uint32_t)(s->W * s->H);
    std::vector<float> rec(12 * (size_t)n);
    for (int32_t r = 0; r < n; ++r) {
      if (pix[r] >= npx) throw Status(MARS_E_ARG, "pixel index out of range");
      for (int k = 0; k < 3; ++k) {
        if (!std::isfinite(pos[3 * r + k]) || !std::isfinite(nrm[3 * r + k]) ||
            !std::isfinite(T[3 * r + k]))
          throw Status(MARS_E_NONFINITE, "non-finite record");
        rec[12 * (size_t)r + k] = pos[3 * r + k];
        rec[12 * (size_t)r + 4 + k] = nrm[3 * r + k];
        rec[12 * (size_t)r + 8 + k] = T[3 * r + k];
      }
      std::memcpy(&rec[12 * (size_t)r + 3], &pix[r], 4);
      rec[12 * (size_t)r + 7] = 0.0f;
      rec[12 * (size_t)r + 11] = 0.0f;
    }
    const uint32_t nn = (uint32_t)n;
    if (n) h2d(s->mlp.rec, rec.data(), 48 * (size_t)n, ctx->stream);
    h2d(s->mlp.n_rec, &nn, 4, ctx->stream);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    s->mlp_n_train = nn;
  });
}

mars_status mars_mlp_targets_only(mars_ctx* ctx, int32_t scene_id) {
  if (!ctx) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = mlp_scene(ctx, scene_id);
    k_mlp_targets(s->sd, s->cd, s->mlp, s->img, IterDev{}, s->mlp.rec_cap, nullptr, ctx->stream);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipGetLastError());
  });
}

mars_status mars_mlp_read_train(mars_ctx* ctx, int32_t scene_id, float* x6, float* target,
                                float* weight, int32_t cap, int32_t* n) {
  if (!ctx || cap < 0) return MARS_E_ARG;
  return guard(ctx, [&] {
    Scene* s = mlp_scene(ctx, scene_id);
    const size_t m = std::min((size_t)s->mlp_n_train, (size_t)cap);
    if (n) *n = (int32_t)s->mlp_n_train;
    if (m) {
      if (x6) d2h(x6, s->mlp.x6, 24 * m, ctx->stream);
      if (target) d2h(target, s->mlp.tgt, 12 * m, ctx->stream);
      if (weight) d2h(weight, s->mlp.wt, 12 * m, ctx->stream);
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
  });
}

mars_status mars_probe(mars_ctx* ctx, int32_t kind, int32_t n, const void* in, void* out) {
  if (!ctx || !in || !out || n <= 0) return MARS_E_ARG;
  return guard(ctx, [&] {
    size_t ib, ob;
    if (kind == 3) {  // one 16x16x16 bfloat16 matrix-core product: in = A, B (u16), out = D
      if (n != 1) throw Status(MARS_E_ARG, "mfma probe takes n = 1");
      with_device_buffers(ctx, {1024, 1024}, [&](std::vector<void*>& b) {
        h2d(b[0], in, 1024, ctx->stream);
        k_mfma_probe((const uint16_t*)b[0], (const uint16_t*)b[0] + 256, (float*)b[1], ctx->stream);
        d2h(out, b[1], 1024, ctx->stream);
        HIPCHK(hipStreamSynchronize(ctx->stream));
        HIPCHK(hipGetLastError());
      });
      return;
    }
    if (kind == 0) { ib = 24; ob = 16; }
    else if (kind == 1) { ib = 4; ob = 8; }
    else if (kind == 2) { ib = 16; ob = 12; }
    else throw Status(MARS_E_ARG, "bad probe kind");
    void* din = ctx->dalloc(ib * n);
    void* dout = nullptr;
    try {
      dout = ctx->dalloc(ob * n);
      h2d(din, in, ib * n, ctx->stream);
      k_probe(kind, n, din, dout, ctx->stream);
      d2h(out, dout, ob * n, ctx->stream);
      HIPCHK(hipStreamSynchronize(ctx->stream));
      HIPCHK(hipGetLastError());
    } catch (...) {
      ctx->dfree(din);
      ctx->dfree(dout);
      throw;
    }
    ctx->dfree(din);
    ctx->dfree(dout);
  });
}

}  // extern "C"
