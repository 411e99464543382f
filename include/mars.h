/* mars.h -- C ABI of the MI355X implementation of MARS
 * (Meyer, Rath, Yazici, Slusallek: "MARS: Multi-sample Allocation through
 * Russian roulette and Splitting", SIGGRAPH Asia 2024).
 *
 * The iterative scheme the interface follows is the paper's (Sec. 4.1
 * "Fixed-point iteration", Sec. 5.1): render an iteration with the current
 * per-cell, per-technique sample counts, collect local and image estimates,
 * update the counts by the fixed-point rule, repeat.
 *
 * Conventions
 *  - Every function returns a mars_status; no exception crosses the ABI.
 *    mars_last_error() gives a message for the last failing call on a context.
 *  - Scene arrays are copied at upload; the caller may free them afterwards.
 *  - Device memory comes from the allocator callbacks given at creation (the
 *    Python binding passes PyTorch's caching allocator); NULL callbacks mean
 *    hipMalloc/hipFree.  The library frees everything it allocated at
 *    mars_scene_release / mars_destroy.
 *  - Work is ordered on the HIP stream given at creation.  Functions that
 *    fill host-side stats synchronise that stream before returning.
 *  - A context is not thread-safe; use one context per host thread.
 *  - Host pointers ("dst" with dst_is_device = 0) must hold the documented
 *    number of elements; device pointers must be on the context's device.
 */
#ifndef MARS_H
#define MARS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MARS_OK = 0,
  MARS_E_ARG = -1,        /* invalid argument (null pointer, bad size, bad id) */
  MARS_E_OOM = -2,        /* an allocation failed */
  MARS_E_HIP = -3,        /* a HIP runtime call failed (no device, launch error) */
  MARS_E_STATE = -4,      /* call not valid in the current state */
  MARS_E_OVERFLOW = -5,   /* a single path tree exceeds the queue capacity */
  MARS_E_NONFINITE = -6,  /* non-finite scene input */
  MARS_E_IO = -7          /* checkpoint file error */
} mars_status;

/* rendering modes: the paper's two applications (Sec. 4: path guiding with
 * BSDF/NEE/guided techniques; Sec. 5: bidirectional path tracing with
 * BSDF/NEE/light-path-connection techniques) and plain BSDF+NEE tracing */
enum { MARS_MODE_PT = 0, MARS_MODE_PT_GUIDED = 1, MARS_MODE_BDPT = 2 };
/* how per-vertex counts are chosen: classic throughput RR (the baseline and
 * warm-up of Sec. 4.1/5.2), the MARS fixed point (Sec. 3.1 "Optimization"),
 * fixed counts (tests of unbiasedness, supplement A.1), the learned cache, or
 * EARS (the comparison method of Sec. 5: one count shared by every technique
 * of a vertex, beta_t = r_t lambda with the classic ratios r, lambda from the
 * same fixed point restricted to that line; the update of an EARS iteration
 * keeps the shared factors in technique slot 0 of the cell factors) */
enum { MARS_ALLOC_CLASSIC = 0, MARS_ALLOC_MARS = 1, MARS_ALLOC_FIXED = 2, MARS_ALLOC_MLP = 3,
       MARS_ALLOC_EARS = 4 };
/* technique slots: 0 BSDF, 1 NEE, 2 guided (PT_GUIDED) or light path (BDPT) */
enum { MARS_TECH_BSDF = 0, MARS_TECH_NEE = 1, MARS_TECH_THIRD = 2 };
enum { MARS_IMAGE_MEAN = 0, MARS_IMAGE_IVW = 1, MARS_IMAGE_LAST = 2 };

typedef struct mars_ctx mars_ctx;

typedef void* (*mars_alloc_fn)(size_t bytes, void* stream, void* user);
typedef void (*mars_free_fn)(void* ptr, void* stream, void* user);

typedef struct {
  int32_t device;          /* HIP device ordinal */
  void* stream;            /* hipStream_t, NULL = default stream */
  mars_alloc_fn alloc;     /* optional */
  mars_free_fn free;       /* optional */
  void* user;              /* passed to alloc/free */
} mars_ctx_desc;

typedef struct {
  /* geometry, host pointers, copied at upload */
  const float* V;           /* [n_tris][9]: v0, v1, v2 */
  const uint32_t* tri_mat;  /* [n_tris] material index */
  const float* mats;        /* [n_mats][8]: kind (0 Lambert, 1 GGX), albedo rgb, GGX alpha,
                               emitted radiance rgb (one-sided, front = winding normal) */
  const float* camera;      /* [10]: position, target, up, vertical fov (degrees) */
  int32_t n_tris, n_mats, width, height;
  /* algorithm configuration */
  int32_t mode;             /* MARS_MODE_* */
  int32_t max_depth;        /* maximum number of path segments D */
  int32_t max_cells;        /* octree leaf budget (the paper caps the cache at 72 MB) */
  int32_t max_tree_depth;   /* 8 */
  int32_t split_visits;     /* a leaf splits after more than this many vertex visits (32) */
  int32_t nee_enabled;      /* NEE technique available */
  uint64_t seed;            /* Philox key */
  int64_t queue_capacity;   /* entries per path-depth queue; 0 = automatic */
  int32_t tile_roots;       /* camera samples per wavefront tile; 0 = automatic */
  int32_t flags;            /* MARS_SCENE_* bits */
} mars_scene_desc;

/* scene flags: MARS_SCENE_MLP allocates the learned cache (counts predicted
 * by a small network trained online on the octree's estimates).
 * MARS_SCENE_LP_LENGTHS (BDPT): separate light-path budgets per light-vertex
 * index, the variant Sec. 5 leaves to future work.  A camera vertex then has
 * five counts: BSDF, NEE, and connections to the light vertex y_1
 * (technique 2), y_2 (technique 3) and y_3 and beyond (technique 4), each
 * with its own moments, cost and fixed point; Alg. 1 rounds all five with
 * one uniform, and sample k of every class connects to the same light
 * subpath.  Not combined with MARS_SCENE_MLP, EARS iterations or
 * independent rounding (MARS_E_ARG). */
enum { MARS_SCENE_MLP = 1, MARS_SCENE_LP_LENGTHS = 2 };

typedef struct {
  int32_t iteration;        /* keys the random streams */
  int32_t spp;              /* camera samples per pixel in this iteration */
  int32_t alloc;            /* MARS_ALLOC_* */
  int32_t budget_aware;     /* 1: budget-aware balance heuristic (Sec. 3 "Proxy model") */
  int32_t rr_start;         /* classic RR from this depth on (5 in Sec. 4.2) */
  int32_t fixed_scale;      /* FIXED: multiply the counts by |T / I~| */
  float clamp_lo, clamp_hi; /* count clamp, [0.05, 20] in Sec. 4.1 */
  float stat_clamp;         /* outlier clamp of statistics (50 in Sec. 4.1; 0 = off) */
  int32_t center_jitter;    /* 1: pixel-centre camera rays */
  int32_t debug_depth;      /* record per-vertex decisions up to this depth */
  int32_t lp_stride;        /* BDPT: light-path sample j of a camera vertex connects to
                               light subpath (b + j lp_stride) mod N of the iteration's N
                               (one per camera sample), b a word of the vertex's random
                               stream (Sec. 5: connections with light paths) */
  int32_t rounding;         /* 0: the low-discrepancy rounding of supplement Alg. 1 (one
                               uniform for every technique of a vertex); 1: each count
                               rounded with its own uniform (the naive scheme it replaces) */
} mars_iter_params;

typedef struct {
  uint64_t rays_camera, rays_ext, rays_shadow, rays_light, rays_conn;
  uint64_t vertices, samples;
  int32_t tiles, overflow_retries;
  double ms;                /* wall time of the call */
} mars_iter_stats;

typedef struct {
  double V_I, C_I;          /* image relative variance and cost (Sec. 4.1 "Image estimates") */
  int32_t n_cells_before, n_cells_after, n_excluded;
  int32_t reserved;
} mars_update_stats;

/* per-vertex decision record (parity tests): the vertex's random stream
 * identifies its position in the path tree */
typedef struct {
  uint32_t root, depth, stream_lo, stream_hi, cell;
  float beta[3];
  uint32_t gamma[3];
  float T[3];
  float beta_x[2];          /* MARS_SCENE_LP_LENGTHS: counts of techniques 3, 4, else 0 */
  uint32_t gamma_x[2];
} mars_vertex_rec;

/* ---- lifetime ---------------------------------------------------------- */
/* Creates a context on desc->device.  MARS_E_HIP if no device is usable. */
mars_status mars_create(const mars_ctx_desc* desc, mars_ctx** out);
mars_status mars_destroy(mars_ctx* ctx);
const char* mars_last_error(const mars_ctx* ctx);
const char* mars_version(void);

/* ---- scenes ------------------------------------------------------------ */
/* Builds the BVH on the host, uploads geometry, emitter table and camera,
 * and initialises the cache (one root cell, classic counts until data, a
 * uniform directional distribution).  MARS_E_NONFINITE for non-finite
 * vertices/materials, MARS_E_ARG for bad sizes or indices. */
mars_status mars_scene_upload(mars_ctx* ctx, const mars_scene_desc* desc, int32_t* scene_id);
mars_status mars_scene_release(mars_ctx* ctx, int32_t scene_id);

/* ---- the iteration ----------------------------------------------------- */
/* Renders one iteration: camera rays, per-depth closest-hit traversal,
 * shading with per-vertex counts (Sec. 3.1 "Optimization"; colour rule of
 * Sec. 4.1), low-discrepancy rounding (supplement Alg. 1), multi-sample MIS
 * (Sec. 3 "The model"), shadow traversal, back-propagation of the secondary
 * estimates, per-cell moment/cost accumulation (Sec. 4.1 "Local
 * estimates") and the per-pixel sums.  stats is filled (host pointer). */
mars_status mars_render_iteration(mars_ctx* ctx, int32_t scene_id, const mars_iter_params* p,
                                  mars_iter_stats* stats);
/* Renders one iteration of n distinct scenes as one batch (the workload of
 * many independent requests of uneven size).  Equivalent to calling
 * mars_render_iteration on each scene; stats (optional) receives the totals.
 * Batches of scenes without the learned cache and without debug records run
 * as one captured launch graph (see mars_iterate_batch); others one scene
 * after another. */
mars_status mars_render_batch(mars_ctx* ctx, const int32_t* scene_ids, int32_t n,
                              const mars_iter_params* p, mars_iter_stats* stats);

/* Batched iteration: the render iteration of each of n distinct scenes and,
 * with MARS_BATCH_UPDATE, its update (as mars_update_counts), every scene's
 * work enqueued without host synchronisation on one stream of a pool
 * (scenes assigned longest-first to the least loaded stream), each scene's
 * iteration captured once as a HIP graph and the graphs replayed, in the
 * same order on the same streams, by later calls with the same scenes and
 * parameters apart from the iteration index.  The device
 * reads the iteration index, the image cost C_I and the number of cells
 * itself.  A scene whose queues overflowed skips its update inside the graph
 * and is rendered (and updated) again on its own with tile halving (its
 * tile for later batches unchanged), so the result always equals the
 * per-scene calls.  Scenes with the learned cache
 * and debug records (p->debug_depth > 0) are refused (MARS_E_ARG).
 * iter_stats / upd_stats: optional host arrays of n.  The graph keeps device
 * pointers of the scenes: mars_scene_configure, mars_set_fixed_counts,
 * releases and a change of parameters rebuild it on the next call.
 * MARS_BATCH_NO_GRAPH enqueues the same work on the stream pool directly. */
enum { MARS_BATCH_UPDATE = 1, MARS_BATCH_NO_GRAPH = 2 };
mars_status mars_iterate_batch(mars_ctx* ctx, const int32_t* scene_ids, int32_t n,
                               const mars_iter_params* p, int32_t flags,
                               mars_iter_stats* iter_stats, mars_update_stats* upd_stats);

/* Re-sizes a scene's path queues.  A scene holds per depth level (levels
 * 0 .. max_depth + 1) ray queues (camera, continuation and light rays with
 * their vertices) and shadow queues (NEE samples and light-path
 * connections, which splitting and connections can make far longer).
 * mars_scene_configure_queues: ray_capacity and shadow_capacity entries per
 * level, camera samples per wavefront tile (<= ray_capacity); 0 keeps a
 * value.  Queue memory is about (max_depth + 2) x (168 B x ray_capacity +
 * 16 B x shadow_capacity) + 32 B x shadow_capacity (the shadow rays hold one
 * level, reused by every depth; their values stay per level), plus per ray
 * entry and level 32 B for BDPT, 32 B more with per-length light-path
 * budgets and 16 B with the learned cache.
 * mars_scene_configure: both capacities queue_capacity. */
mars_status mars_scene_configure_queues(mars_ctx* ctx, int32_t scene_id, int64_t ray_capacity,
                                        int64_t shadow_capacity, int32_t tile_roots);
mars_status mars_scene_configure(mars_ctx* ctx, int32_t scene_id, int64_t queue_capacity,
                                 int32_t tile_roots);
/* ray-queue capacity and tile size of a scene, the peak queue occupancy
 * per camera sample (the larger of the two queues) seen by the last eager
 * render iteration */
mars_status mars_scene_query(mars_ctx* ctx, int32_t scene_id, int64_t* queue_capacity,
                             int32_t* tile_roots, double* peak_per_root);
/* both capacities and both peaks (entries per camera sample at the fullest
 * level) of the last eager render iteration; any pointer may be null */
mars_status mars_scene_query_queues(mars_ctx* ctx, int32_t scene_id, int64_t* ray_capacity,
                                    int64_t* shadow_capacity, double* peak_ray,
                                    double* peak_shadow);

/* Autotuner of queue and tile sizes.  For each scene: one probe render
 * iteration with p (no update; the last-iteration image and sample radiance
 * then hold the probe's) measures the peak occupancy per camera sample of
 * the ray queues e and of the shadow queues e_s (each at least 1); tiles of
 * up to all camera samples are planned under mem_budget bytes of queue
 * memory for the n scenes together (capacities tile x e x 1.5 and
 * tile x e_s x 1.5, rounded up to 4096; largest scenes halved first, no
 * tile below min(all samples, max(4096, 2^18 / max(e, e_s))) rounded up to
 * 64); then up to three tile sizes (plan, plan/2, plan/4, same floor) are
 * timed (the better of two render iterations each) and the fastest kept, a
 * smaller tile only when at least 3% faster than the best larger one.  cache_path
 * (optional): a text file of lines
 * "<class> <capacity> <shadow capacity> <tile> <e> <e_s> <ms>" keyed by the
 * scene class (resolution, spp, mode, depth, triangles, allocation mode);
 * classes found there are applied without probing and new ones appended
 * (lines of another form are ignored).  out (optional, n entries each):
 * chosen ray capacity, tile, e, shadow capacity, e_s. */
mars_status mars_autotune(mars_ctx* ctx, const int32_t* scene_ids, int32_t n,
                          const mars_iter_params* p, int64_t mem_budget, const char* cache_path,
                          int64_t* out_capacity, int32_t* out_tile, double* out_peak,
                          int64_t* out_shadow_capacity, double* out_shadow_peak);
/* Image estimates (I~, V_I, C_I), the fixed-point update of every cell's
 * factors, the directional distribution of the guided technique, octree
 * refinement and the inverse-variance weighted image (Sec. 4.1, 5.1). */
mars_status mars_update_counts(mars_ctx* ctx, int32_t scene_id, const mars_iter_params* p,
                               mars_update_stats* stats);

/* ---- inputs for tests and fixed allocations ---------------------------- */
/* beta: host [n][3]; n = 1 (global) or the current number of cells. */
mars_status mars_set_fixed_counts(mars_ctx* ctx, int32_t scene_id, const float* beta, int32_t n);
/* Itilde: host [H*W][3] pixel estimates used by the next iteration. */
mars_status mars_set_itilde(mars_ctx* ctx, int32_t scene_id, const float* itilde);
/* pm, cdf: host [n][64] directional distributions of the first n cells. */
mars_status mars_set_hist(mars_ctx* ctx, int32_t scene_id, int32_t n, const float* pm,
                          const float* cdf);
/* factors [n][2][3][3] (float), acc [n][3][8] (double), visits [n]; any may
 * be NULL.  n must equal the current number of cells. */
mars_status mars_write_cells(mars_ctx* ctx, int32_t scene_id, int32_t n, const float* factors,
                             const double* acc, const uint32_t* visits);
/* Runs only the fixed-point update of the cells with the given V_I, C_I. */
mars_status mars_update_cells_only(mars_ctx* ctx, int32_t scene_id, double V_I, double C_I);
/* Runs only the octree refinement from the current visit counts. */
mars_status mars_refine_only(mars_ctx* ctx, int32_t scene_id, int32_t* n_split);

/* ---- outputs ----------------------------------------------------------- */
/* which = MARS_IMAGE_*; dst [H*W][3].  MEAN is the plain average of all
 * iterations, IVW the inverse-variance weighted combination of Sec. 5.1
 * (iteration i weighted by spp_i / V_I,i), LAST the last iteration alone. */
mars_status mars_read_image(mars_ctx* ctx, int32_t scene_id, int32_t which, float* dst,
                            int32_t dst_is_device);
/* dst [H*W][3]: mean count per technique at the first hit of the last
 * iteration -- the allocation maps the paper shows beside its results
 * (Sec. 4.2, Sec. 5.2: BSDF, NEE and the third technique per pixel) */
mars_status mars_read_count_map(mars_ctx* ctx, int32_t scene_id, float* dst,
                                int32_t dst_is_device);
/* dst [H*W*spp][3]: radiance of every camera sample of the last iteration,
 * sample s of pixel i at i*spp+s */
mars_status mars_read_sample_radiance(mars_ctx* ctx, int32_t scene_id, float* dst,
                                      int32_t dst_is_device);
mars_status mars_read_itilde(mars_ctx* ctx, int32_t scene_id, float* dst, int32_t dst_is_device);
mars_status mars_num_cells(mars_ctx* ctx, int32_t scene_id, int32_t* n_cells, int32_t* n_nodes);
/* host arrays sized by mars_num_cells; any may be NULL */
mars_status mars_read_cells(mars_ctx* ctx, int32_t scene_id, float* factors, double* acc,
                            uint32_t* visits, uint32_t* leaf_depth);
mars_status mars_read_nodes(mars_ctx* ctx, int32_t scene_id, uint32_t* nodes);
/* MARS_SCENE_LP_LENGTHS scenes: factors [n][2][2][3] (RR/S, technique 3 or 4,
 * channel) and acc [n][2][8] of the two extra light-path classes, host arrays
 * sized by mars_num_cells (either may be NULL; Sec. 3.1 "Optimization" per
 * technique).  MARS_E_STATE for scenes without them. */
mars_status mars_read_cells_x(mars_ctx* ctx, int32_t scene_id, float* factors_x, double* acc_x);
/* the same arrays written in; n must equal the current number of cells */
mars_status mars_write_cells_x(mars_ctx* ctx, int32_t scene_id, int32_t n, const float* factors_x,
                               const double* acc_x);
mars_status mars_read_hist(mars_ctx* ctx, int32_t scene_id, float* pm, float* cdf);
/* per-vertex decisions of the last iteration up to params.debug_depth;
 * writes at most cap records, returns the total in *n */
mars_status mars_debug_vertices(mars_ctx* ctx, int32_t scene_id, mars_vertex_rec* dst,
                                int32_t cap, int32_t* n);

/* ---- checkpoint --------------------------------------------------------- */
/* Cache (nodes, cells, distributions), images and iteration state. */
mars_status mars_checkpoint_save(mars_ctx* ctx, int32_t scene_id, const char* path);
mars_status mars_checkpoint_load(mars_ctx* ctx, int32_t scene_id, const char* path);

/* ---- learned cache (scenes uploaded with MARS_SCENE_MLP) -----------------
 * Not in the paper: its Sec. 6 ("Discontinuity artefacts") asks for sample
 * counts that vary smoothly in space; a small network fitted online to the
 * octree's estimates gives them.  The network maps a vertex (its position
 * normalised to the octree's cube, and its geometric normal as stored, not
 * turned toward the incoming ray, so that the same value can be evaluated at
 * a light vertex) to one log count per technique relative to |T / I~| =
 * sqrt((1/3) sum_ch (T_ch / I~_ch)^2).
 * Render iterations with alloc = MARS_ALLOC_MLP pool the network's count
 * |T / I~| exp(y_t) with the octree's count beta_t as their geometric mean
 * sqrt(beta_t |T / I~| exp(y_t)), clamped like the octree's counts; where
 * that is not finite the octree's count is used, and a technique the octree
 * disables stays off.  Every MIS weight evaluates these pooled counts: the
 * unidirectional records keep the counts each vertex drew with, and in
 * bidirectional paths the camera-side records hold them and light vertices
 * get network outputs too, so the weights of a path still sum to one.
 * Training data: a random subset of the iteration's camera vertices,
 * recorded while shading; mars_update_counts turns them into targets from
 * the cells' updated factors: y*_t = log(beta^_t) - log|T / I~| with beta^_t
 * the octree's resolved, unclamped count (Sec. 3.1, colour rule of
 * Sec. 4.1), weight min(n_t, 64)/64 for cells with at least 4 samples of
 * technique t in the iteration, else 0.
 * The network: sin/cos(2^k pi x), k < 6, of the 6 inputs (72 features,
 * padded to 80), 3 hidden layers of 64 ReLU units, 3 outputs; bfloat16
 * matrix-core products with binary32 accumulation; Adam (0.9, 0.99, 1e-8)
 * on binary32 master weights.  Parameter layout (binary32): W1 [64][80],
 * b1 [64], W2 [64][64], b2, W3 [64][64], b3, W4 [16][64] (rows 3..15 zero),
 * b4 [16]. */
int32_t mars_mlp_num_params(void);
/* steps Adam steps over the current training set, batch samples each;
 * *loss (host, optional) receives the loss of the last step */
mars_status mars_mlp_train(mars_ctx* ctx, int32_t scene_id, int32_t steps, int32_t batch, float lr,
                           float* loss, int32_t* n_train);
mars_status mars_mlp_read_params(mars_ctx* ctx, int32_t scene_id, float* params);
/* sets the master weights, re-quantises, resets the Adam state */
mars_status mars_mlp_write_params(mars_ctx* ctx, int32_t scene_id, const float* params);
/* host buffers: x6 [n][6] (q.xyz, n.xyz) -> y3 [n][3] */
mars_status mars_mlp_forward(mars_ctx* ctx, int32_t scene_id, const float* x6, int32_t n,
                             float* y3);
/* gradient of the weighted squared loss over one batch (no update):
 * x6 [n][6], target [n][3], weight [n][3] -> grad [num_params], *loss */
mars_status mars_mlp_grad(mars_ctx* ctx, int32_t scene_id, const float* x6, const float* target,
                          const float* weight, int32_t n, float* grad, float* loss);
/* one Adam step with the given gradient (host [num_params]) */
mars_status mars_mlp_apply_grad(mars_ctx* ctx, int32_t scene_id, const float* grad, float lr);

/* Allocation-free variant of mars_mlp_grad, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops): it calls no hipMalloc, hipFree or allocating routine.  x6 [n][6],
 * target [n][3], weight [n][3] and grad [num_params + 1] (the gradient, then
 * the loss) are DEVICE pointers on the context's device, owned by the
 * caller.  The work is enqueued on the context's stream and not waited
 * for; grad is complete when the stream reaches that point.  The
 * per-workgroup partial gradients go to a fixed device array of 256 x
 * (num_params + 1) binary32 words (14.9 MB), one per device, held until the
 * process ends: n is limited to 262144 (MARS_E_ARG beyond), and calls that
 * overlap on one device (on different streams or contexts) race on that
 * array.  The result equals mars_mlp_grad's bit for bit. */
mars_status mars_mlp_grad_noalloc(mars_ctx* ctx, int32_t scene_id, const float* x6,
                                  const float* target, const float* weight, int32_t n,
                                  float* grad);
/* The training set (tests).  mars_mlp_write_records replaces the recorded
 * vertices: host pos, nrm, T [n][3] (binary32, finite) and pix [n] (< W*H);
 * n at most the record capacity (2^18), else MARS_E_ARG.
 * mars_mlp_targets_only recomputes inputs, targets and weights of the
 * recorded vertices from the cells and I~ as they are (the step
 * mars_update_counts runs after the fixed point, before refinement).
 * mars_mlp_read_train copies up to cap entries (host x6 [n][6], target
 * [n][3], weight [n][3]; any may be NULL) and the set's size into *n. */
mars_status mars_mlp_write_records(mars_ctx* ctx, int32_t scene_id, const float* pos,
                                   const float* nrm, const float* T, const uint32_t* pix,
                                   int32_t n);
mars_status mars_mlp_targets_only(mars_ctx* ctx, int32_t scene_id);
mars_status mars_mlp_read_train(mars_ctx* ctx, int32_t scene_id, float* x6, float* target,
                                float* weight, int32_t cap, int32_t* n);

/* ---- measurement ------------------------------------------------------- */
/* Per-kernel timing with HIP events recorded on the context's stream around
 * every launch.  Enabling resets the totals. */
mars_status mars_profile_enable(mars_ctx* ctx, int32_t on);
/* The same for a subset: bit k of kernel_mask times kernel k (names from
 * mars_profile_kernel_name); the others launch without events, so a timed
 * run carries the events of the kernels it reports only.  0 turns it off. */
mars_status mars_profile_enable_mask(mars_ctx* ctx, uint64_t kernel_mask);
/* ms[k], launches[k] for kernel k < n; *n_kernels receives the kernel count */
mars_status mars_profile_read(mars_ctx* ctx, double* ms, uint64_t* launches, int32_t n,
                              int32_t* n_kernels);
const char* mars_profile_kernel_name(int32_t id);
/* Instrumented traversal (slower; for the algorithmic byte count per ray):
 * out[0..2] = closest-hit rays, BVH nodes visited, triangles tested;
 * out[3..5] = the same for shadow rays; out[6], out[7] = most nodes visited
 * by one closest-hit / shadow ray; out[8], out[9] = closest-hit / shadow
 * rays that visited more than 64 nodes.  Enabling resets the counters. */
mars_status mars_trace_counting(mars_ctx* ctx, int32_t on);
mars_status mars_read_trace_counts(mars_ctx* ctx, uint64_t out[10]);

/* ---- device probes (tests): evaluates a building block on the GPU ------ */
/* kind 0: Philox4x32-10, in [n][6] u32 (key0, key1, ctr0..3), out [n][4] u32
 * kind 1: sin/cos of 2 pi u, in [n] f32, out [n][2] f32
 * kind 2: Alg. 1 rounding, in [n][4] f32 (beta x3, u), out [n][3] u32
 * host buffers */
mars_status mars_probe(mars_ctx* ctx, int32_t kind, int32_t n, const void* in, void* out);

#ifdef __cplusplus
}
#endif
#endif
