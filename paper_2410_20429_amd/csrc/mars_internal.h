// Internal layout shared by the host orchestration and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mars {

constexpr uint32_t kLeafBit = 0x80000000u;  // octree node word: leaf flag | leaf id
constexpr int kMaxDepth = 16;       // maximum path segments supported
constexpr int kTraceBlock = 128;    // threads per traversal workgroup
constexpr int kStackDepth = 16;     // per-lane LDS part of the traversal stack
// traversal launch: 128-thread groups with 8 KB of LDS stack each; at <= 64
// VGPRs 16 groups (32 waves) fit a CU
constexpr int kTraceBlocksPerCU = 16;
constexpr int32_t kBvhNoChild = 0x7FFFFFFF;  // unused slot of a 4-wide node

// scene on the device (read-only during an iteration)
struct SceneDev {
  const float4* bvh;       // [n_nodes][4][2]: per child (lo.xyz, reference), (hi.xyz, -)
  const float4* tri_bvh;   // [n_tris][3] leaf order: (v0, prim bits), (e1, 0), (e2, 0)
  const float4* tri_geo;   // [n_tris][3] primitive order: v0, e1, e2
  const float4* tri_ng;    // [n_tris] primitive order: (geometric normal, p_select / area)
  const uint32_t* tri_mat; // [n_tris]
  const float* mats;       // [n_mats][8]
  const int32_t* light_tri;
  const float* light_cdf;
  int32_t n_lights, n_tris;
  float cam_o[3], cam_f[3], cam_r[3], cam_u[3];
  int32_t W, H;
  float eps;
  float oct_lo[3];
  float oct_inv;
  int32_t mode, max_depth, nee;
  // BDPT light-path budgets per camera vertex: 1, or 3 (connections to the
  // light vertex y_1, y_2 and y_3+ each with its own count, techniques 2-4)
  int32_t lp_classes;
  uint32_t key0, key1;
  // traversal stack entries beyond the LDS part, [depth][spill_threads]
  // (null when the tree's stack bound fits in LDS)
  int32_t* stack_spill;
  uint32_t spill_threads;
};

// spatial cache (octree leaves = cells)
struct CacheDev {
  uint32_t* nodes;       // [1 + 8 max_cells]
  uint32_t* leaf_node;   // [max_cells]
  uint32_t* leaf_depth;  // [max_cells]
  uint32_t* visits;      // [max_cells]
  float* fac;            // [max_cells][2][3][3]  a^RR, a^S per technique and channel
  double* acc;           // [max_cells][3][8]     sum v (3), sum v^2 (3), n, cost
  float* fac_x;          // lp_classes 3: [max_cells][2][2][3] factors of techniques 3, 4
  double* acc_x;         // lp_classes 3: [max_cells][2][8]
  float* pm;             // [max_cells][64]       directional pmf (guided)
  float* cdf;            // [max_cells][64]
  double* hacc;          // [max_cells][64]       directional training sums
  const float* fixed;    // [n_fixed][3]
  int32_t n_fixed;
  int32_t max_cells;
  const float* mlp_y;    // learned-cache outputs per queue entry ([d * cap + j][4]), or null
  float4* mlp_rec;       // training vertex records, or null
  uint32_t* mlp_n_rec;
  uint32_t mlp_rec_cap, mlp_keep;
};

// per-depth SoA queues; entry (d, j) lives at d * cap + j
struct QueuesDev {
  float4* R0;   // origin, flags (1 = traced)
  float4* R1;   // direction, pixel (bits)
  float4* S0;   // prefix throughput T, parent index (bits)
  float4* S1;   // B|cos|/p_t (rgb), w_ind
  float4* S2;   // beta_t p_t, sum_{B,G} beta p, beta_N, beta_t   (parent's MIS data)
  uint4* S3;    // stream lo/hi, tech << 16 | k, root
  uint2* H;     // hit: t (bits), primitive
  float4* V0;   // weighted emission for the parent's direct term, cell (bits)
  float4* V1;   // beta_B, beta_N, beta_third, unused
  uint4* V2;    // NEE first, NEE count, continuation first, continuation count
  float4* RO;   // the entry's value as its parent's continuation sample, its cost (bits)
  // BDPT camera-vertex records for the full-path MIS weights (null otherwise):
  // W0 = (throughput of the camera prefix recomputed from positions, raw
  // BSDF count), W1 = (raw NEE count, raw LP count, pF here, pR two back)
  float4* W0;
  float4* W1;
  // lp_classes 3 only: W2 = (raw count of the y_2 class, of the y_3+ class,
  // -, -); V3 = (beta of those classes, their rounded counts (bits))
  float4* W2;
  float4* V3;
  float4* SH0;  // shadow origin, tmax (one level of scap entries, reused by every depth)
  float4* SH1;  // shadow direction, parent vertex (bits) (one level, as SH0)
  float4* SH2;  // unoccluded sample value, flags (1 = traced); one level per depth
  size_t cap;   // entries per depth level of the ray queues
  size_t scap;  // entries per depth level of the shadow queues (SH0..SH2)
};

// queue counters of a tile (the first kTileWords words, reset per tile) and
// totals of an iteration (reset per iteration)
struct Counters {
  uint32_t n_ray[kMaxDepth + 2];
  uint32_t n_shadow[kMaxDepth + 2];
  uint32_t overflow;
  uint32_t overflow_any;  // sticky over the iteration: the update then skips
  uint32_t n_debug;
  uint32_t pad;
  unsigned long long rays_ext, rays_shadow, vertices, samples, rays_light, rays_conn;
};
constexpr int kTileWords = 2 * (kMaxDepth + 2) + 1;

// BDPT light subpaths of an iteration, one per camera sample (root)
struct LightDev {
  float4* V0;     // [root][lmax]: position y_i, primitive (bits)
  float4* V1;     // [root][lmax]: direction towards y_{i-1}, alpha.r
  float4* V2;     // [root][lmax]: alpha.g, alpha.b, octree cell of y_i (bits), and the
                  // area density of reaching y_i from y_{i-1} (y_0: emission density)
  // [root][lmax]: the BSDF at y_i towards y_{i-1} when the path arrives from
  // y_{i+1}: f cos / p per channel (-1 where p = 0) and the area density at
  // y_{i-1}; set for i < the subpath's length
  float4* V3;
  float4* Y0;     // [root]: point on the emitter, emitter primitive (bits)
  uint2* len;     // [root]: vertices stored, rays traced
  float* y;       // [root][lmax][4]: learned-cache outputs at the light vertices (null if none)
  int32_t lmax;   // max_depth - 2
};

struct IterDev {
  int32_t iteration, spp, alloc, aware, rr_start, fixed_scale;
  float clamp_lo, clamp_hi, stat_clamp;
  int32_t center_jitter, debug_depth, lp_stride, rounding;
  const int32_t* iter_dev;  // if set, the iteration index is read here (graph replays)
};
__host__ __device__ inline int32_t iter_index(const IterDev& it) {
  return it.iter_dev ? *it.iter_dev : it.iteration;
}

struct DebugRec {
  uint32_t root, depth, stream_lo, stream_hi, cell;
  float beta[3];
  uint32_t gamma[3];
  float T[3];
  float beta_x[2];     // techniques 3, 4 (per-length light paths), else 0
  uint32_t gamma_x[2];
};

// per-iteration image buffers
struct ImageDev {
  float* Ls;        // [roots][3] camera-sample radiance of the iteration
  float* beta1;     // [roots][3] counts at the first hit
  float* iter_sum;  // [px][3]
  float* accum;     // [px][3]
  float* mean;      // [px][3] scratch
  float* itilde;    // [px][3]
  uint8_t* excl;    // [px]
  double* ivw_acc;  // [px][3]
  float* count_map; // [px][3]
  double* red;      // [8] reductions: image mean rgb, V_I sum, included count, ...
  float* bright_l;  // [ceil(px / kBrightChunk)][kBright] brightest-pixel candidates
  int32_t* bright_i;
  double* part;     // [kRedBlocks][8] per-workgroup partial sums of the image reductions
};
// image reductions: a fixed grid of workgroups, partial sums summed in order
// (deterministic, no contended atomics)
constexpr int kRedBlocks = 1024;
// brightest pixels dropped from V_I in BDPT, selected in chunks of pixels
constexpr int kBright = 10, kBrightChunk = 4096;

// learned cache: parameter layout (binary32 master) -- W1 [64][80], b1 [64],
// W2 [64][64], b2, W3 [64][64], b3, W4 [16][64] (rows 3..15 zero), b4 [16]
constexpr int kMlpW1 = 0, kMlpB1 = 5120, kMlpW2 = 5184, kMlpB2 = 9280, kMlpW3 = 9344,
              kMlpB3 = 13440, kMlpW4 = 13504, kMlpB4 = 14528, kMlpParams = 14544;
constexpr int kMlpMaxBlocks = 256;  // workgroups of one training pass
// fixed device array of the allocation-free gradient pass: one partial
// gradient (+ loss) per workgroup of a pass of at most kMlpMaxBlocks
constexpr size_t kNoAllocScratchFloats = (size_t)kMlpMaxBlocks * (kMlpParams + 1);
constexpr int kMaxDevices = 64;
// device address of that array on `device`, which must be the current device
hipError_t noalloc_scratch_address(int device, float** out);

struct MlpDev {
  float* master;    // [kMlpParams]
  uint16_t* wq;     // bfloat16 weights
  float* m;         // Adam first moments
  float* v;         // Adam second moments
  float* partial;   // [kMlpMaxBlocks][kMlpParams + 1] gradient partials + loss
  float* y;         // [levels * cap][4] outputs at the queue vertices
  float4* rec;      // [rec_cap][3] training vertices: (P, pixel), (n, -), (T, -)
  uint32_t* n_rec;  // number of records written
  uint32_t rec_cap;
  uint32_t keep;    // a vertex is recorded if (stream.lo >> 8) < keep
  float* x6;        // [rec_cap][6] training inputs
  float* tgt;       // [rec_cap][3] targets (log counts relative to |T / I~|)
  float* wt;        // [rec_cap][3] loss weights
};

// ---- launchers (kernels.hip) ----
void k_clear_iteration(const CacheDev& c, const int32_t* n_cells_dev, int guided, float* beta1,
                       size_t n_beta, hipStream_t s);
void k_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);
void k_fill_f64(double* p, double v, size_t n, hipStream_t s);
void k_fill_f32(float* p, float v, size_t n, hipStream_t s);
void k_raygen(const SceneDev& sc, const QueuesDev& q, Counters* cnt, const IterDev& it,
              uint32_t root0, uint32_t n_roots, hipStream_t s);
// traverses the closest-hit queue of depth dc (-1 = none; 0 is the light
// queue) and the shadow queue of depth ds (0 = none) in one launch.  tc (optional): traversal counters {rays,
// nodes, triangles} of closest-hit rays at tc[0..2], shadow rays at tc[3..5]
// stream: the streaming traversal (queues longer than the lanes resident).
// ev0, ev1 (optional, timing runs): events stamped by the dispatch itself at
// the kernel's start and end, with no marker packets around the launch
void k_trace_pair(const SceneDev& sc, const QueuesDev& q, const Counters* cnt, int dc, int ds,
                  int grid, hipStream_t s, unsigned long long* tc, hipEvent_t ev0 = nullptr,
                  hipEvent_t ev1 = nullptr);
void k_shade_pt(const SceneDev& sc, const CacheDev& c, const QueuesDev& q, Counters* cnt,
                const IterDev& it, const ImageDev& img, DebugRec* dbg, uint32_t dbg_cap, int d,
                int grid, hipStream_t s);
void k_backprop_pt(const SceneDev& sc, const CacheDev& c, const QueuesDev& q, const Counters* cnt,
                   const IterDev& it, const ImageDev& img, int d, hipStream_t s);
void k_light_start(const SceneDev& sc, const QueuesDev& q, const LightDev& lt, Counters* cnt,
                   const IterDev& it, uint32_t root0, uint32_t n, hipStream_t s);
void k_light_shade(const SceneDev& sc, const CacheDev& c, const QueuesDev& q, const LightDev& lt,
                   Counters* cnt, const IterDev& it, int bounce, hipStream_t s);
// resident-group grids of the kernels that loop over equal shares of their
// work, for the current device (cached; launches query them otherwise)
void k_init_launch_grids();
void k_light_walk(const SceneDev& sc, const LightDev& lt, uint32_t roots, hipStream_t s);
void k_shade_bdpt(const SceneDev& sc, const CacheDev& c, const QueuesDev& q, const LightDev& lt,
                  Counters* cnt, const IterDev& it, const ImageDev& img, DebugRec* dbg,
                  uint32_t dbg_cap, int d, uint32_t npool, hipStream_t s);
// the NEE samples' and light-path connections' weights and contributions of
// the camera vertices of depth d (after k_shade_bdpt)
void k_connect_bdpt(const SceneDev& sc, const CacheDev& c, const QueuesDev& q, const LightDev& lt,
                    Counters* cnt, const IterDev& it, const ImageDev& img, int d, hipStream_t s);
void k_backprop_bdpt(const SceneDev& sc, const CacheDev& c, const QueuesDev& q,
                     const LightDev& lt, const Counters* cnt, const IterDev& it,
                     const ImageDev& img, int d, uint32_t npool, hipStream_t s);
void k_mlp_targets(const SceneDev& sc, const CacheDev& c, const MlpDev& m, const ImageDev& img,
                   const IterDev& it, uint32_t n, const uint32_t* skip, hipStream_t s);
// ---- launchers (mlp.hip) ----
void k_mlp_forward(const MlpDev& m, const float* x6, int n, float* y3, hipStream_t s);
void k_mlp_infer_queue(const SceneDev& sc, const QueuesDev& q, const MlpDev& m, const Counters* cnt,
                       int d, int grid, hipStream_t s);
void k_mlp_infer_light(const SceneDev& sc, const QueuesDev& q, const MlpDev& m, const LightDev& lt,
                       const Counters* cnt, int i, int grid, hipStream_t s);
void k_mlp_train_pass(const MlpDev& m, const float* x6, const float* tgt, const float* wt, int n_set,
                      int offset, int batch, int* nblocks_out, hipStream_t s);
void k_mlp_adam(const MlpDev& m, int nblocks, const float* ext_grad, float lr, float bc1, float bc2,
                float* loss_out, hipStream_t s);
void k_mlp_sum_partials(const MlpDev& m, int nblocks, float* grad, float* loss, hipStream_t s);
void k_mlp_quantize(const MlpDev& m, hipStream_t s);
void k_mfma_probe(const uint16_t* A, const uint16_t* B, float* D, hipStream_t s);
void k_pixel_sums(const ImageDev& img, int npx, int spp, hipStream_t s);
// update kernels: `skip` (optional) points at a flag that makes them no-ops
// (an iteration whose queues overflowed is re-run before its update)
void k_update_image(const ImageDev& img, int W, int H, int spp, const double* total_spp, int bdpt,
                    float stat_clamp, const uint32_t* skip, hipStream_t s);
// C_I from rays / (pixels x spp): given on the host (cnt == null) or taken
// from the iteration totals in `cnt` plus the camera rays `roots`
// ears_mode: the scene mode when the update belongs to an EARS iteration
// (shared factors into technique slot 0), else -1
void k_fixed_point(const CacheDev& c, const int32_t* n_cells_dev, const double* red, double C_I,
                   const Counters* cnt, double roots, int use_device_vi, double V_I_host,
                   int guided, int max_cells, const ImageDev* img, int npx, int spp,
                   const uint32_t* skip, hipStream_t s, int ears_mode = -1);
void k_refine(const CacheDev& c, int32_t* n_cells_dev, int32_t* n_nodes_dev, uint32_t* scratch,
              int split_visits, int max_tree_depth, int max_cells, const uint32_t* skip,
              hipStream_t s);
constexpr int kSumWords = 17;
void k_batch_summary(const Counters* cnt, const double* red, const int32_t* n_cells_dev,
                     double* out, hipStream_t s);
void k_set_i32(int32_t* p, int32_t v, hipStream_t s);
// fills n_dev[0] * mult elements (n_dev read on the device)
void k_probe(int kind, int n, const void* in, void* out, hipStream_t s);

}  // namespace mars
