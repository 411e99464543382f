/* CPU oracle for the MARS hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests, the smoke check and the benchmark's CPU-baseline leg may load
 * this library.  The product path (the HIP library) shares no code with it.
 *
 * It implements, plainly and recursively, what the method computes:
 *   - multi-sample MIS with real-valued per-technique counts (Sec. 3, Eq. 1),
 *   - stochastic rounding by Alg. 1 (supplement, "Low discrepancy rounding"),
 *   - the budget-aware / budget-unaware balance heuristic (Sec. 3 "Proxy
 *     model", supplement A.1),
 *   - the path-tracing recursion with prefix throughput T (Sec. 3.1),
 *   - per-cell moment and cost estimates (Sec. 4.1 "Local estimates"),
 *   - image variance / cost estimates (Sec. 4.1 "Image estimates"),
 *   - the fixed-point update with the image-relative extension (Sec. 3.1
 *     "Optimization", supplement A.3).
 * Path arithmetic is IEEE binary32 with a fixed operation order (compiled with
 * -ffp-contract=off) so that integer decisions (cells, rounded counts) can be
 * compared bit-exactly; statistics are accumulated in binary64.
 */
#ifndef MARS_ORACLE_H
#define MARS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_MODE_PT = 0, ORC_MODE_PT_GUIDED = 1, ORC_MODE_BDPT = 2 };
/* EARS: one shared count per vertex for every technique, scaled by the
 * classic per-technique ratios (value 3 is the GPU library's learned cache) */
enum { ORC_ALLOC_CLASSIC = 0, ORC_ALLOC_MARS = 1, ORC_ALLOC_FIXED = 2, ORC_ALLOC_EARS = 4 };
enum { ORC_TECH_B = 0, ORC_TECH_N = 1, ORC_TECH_G = 2 }; /* third = guided or light path */
/* BDPT with separate light-path budgets per light-vertex index (Sec. 5,
 * the variant left to future work there): technique 2 connects to y_1,
 * technique 3 to y_2 and technique 4 to y_3 and beyond */
enum { ORC_TECH_L2 = 3, ORC_TECH_L3 = 4 };

typedef struct {
  int32_t mode;          /* ORC_MODE_* */
  int32_t max_depth;     /* D: maximum number of path segments */
  int32_t max_cells;     /* octree leaf budget */
  int32_t max_tree_depth;/* 8 */
  int32_t split_visits;  /* split a leaf after more than this many visits (32) */
  int32_t nee_enabled;   /* 1: NEE technique on (requires emitters) */
  uint64_t seed;
  int32_t lp_classes;    /* BDPT: 3 = separate light-path budgets for y_1, y_2, y_3+;
                            anything else = one budget for every light vertex */
} orc_config;

typedef struct {
  int32_t iteration;     /* keys the RNG */
  int32_t spp;
  int32_t alloc;         /* ORC_ALLOC_* */
  int32_t budget_aware;  /* 1: budget-aware balance heuristic */
  int32_t rr_start;      /* classic RR from this depth on */
  int32_t fixed_scale;   /* FIXED mode: multiply by |T/I~| */
  float clamp_lo, clamp_hi;
  float stat_clamp;      /* >0: clamp local samples to stat_clamp * I~/T */
  int32_t center_jitter; /* 1: pixel-centre rays */
  int32_t debug_depth;   /* record per-vertex decisions up to this depth */
  int32_t lp_stride;     /* BDPT: pool stride P for extra light paths */
  int32_t rounding;      /* 0: Alg. 1; 1: each count rounded with its own uniform */
} orc_iter_params;

typedef struct {
  uint64_t rays_camera, rays_ext, rays_shadow, rays_light, rays_conn;
  uint64_t vertices, samples;
} orc_iter_stats;

typedef struct {
  double V_I, C_I;
  int32_t n_cells_before, n_cells_after, n_excluded;
} orc_update_stats;

typedef struct {
  uint32_t root, depth, stream_lo, stream_hi, cell;
  float beta[3];
  uint32_t gamma[3];
  float T[3];
  float beta_x[2];       /* counts of techniques 3 and 4 (per-length light paths) */
  uint32_t gamma_x[2];
} orc_vertex_rec;

typedef struct oracle oracle;

oracle* orc_create(const float* V, const uint32_t* tri_mat, int32_t ntri, const float* mats,
                   int32_t nmat, const float* cam, int32_t width, int32_t height,
                   const orc_config* cfg);
void orc_destroy(oracle* o);
int32_t orc_set_threads(int32_t n);
int32_t orc_render_iteration(oracle* o, const orc_iter_params* p, orc_iter_stats* st);
int32_t orc_update(oracle* o, const orc_iter_params* p, orc_update_stats* st);

/* read-back */
int32_t orc_num_cells(const oracle* o);
int32_t orc_num_nodes(const oracle* o);
void orc_read_nodes(const oracle* o, uint32_t* dst);
void orc_read_sample_radiance(const oracle* o, float* dst);     /* [n_roots][3] last iteration */
void orc_read_image(const oracle* o, int32_t which, float* dst);/* 0 mean, 1 ivw, 2 last */
void orc_read_Itilde(const oracle* o, float* dst);              /* [H*W][3] */
void orc_read_count_map(const oracle* o, float* dst);           /* [H*W][3] */
/* cells: factors [n][2][3][3] (RR/S, tech, ch); acc [n][3][8] (sum3, sum2_3, n, cost) ; visits [n] */
void orc_read_cells(const oracle* o, float* factors, double* acc, uint32_t* visits,
                    uint32_t* leaf_depth);
void orc_read_hist(const oracle* o, float* pm, float* cdf);      /* [n][64] each */
int32_t orc_read_debug(const oracle* o, orc_vertex_rec* dst, int32_t cap);
/* write-in for parity tests */
void orc_write_cells(oracle* o, int32_t n, const float* factors, const double* acc,
                     const uint32_t* visits);
/* per-length light-path budgets (lp_classes = 3): the factors [n][2][2][3]
 * (RR/S, technique 3 or 4, ch) and accumulators [n][2][8] of techniques 3, 4;
 * orc_lp_classes returns 3 when the scene has them, else 1 */
int32_t orc_lp_classes(const oracle* o);
void orc_read_cells_x(const oracle* o, float* factors_x, double* acc_x);
void orc_write_cells_x(oracle* o, int32_t n, const float* factors_x, const double* acc_x);
void orc_set_Itilde(oracle* o, const float* src);
/* render only the listed pixels (NULL / 0: all); others get zero radiance */
void orc_set_pixel_subset(oracle* o, const int32_t* pix, int32_t n);
void orc_set_fixed_beta(oracle* o, const float* beta, int32_t n);
/* tests: log sample statistics only for vertices up to `depth` (0: all) */
void orc_set_record_depth(oracle* o, int32_t depth);
void orc_set_hist(oracle* o, int32_t n, const float* pm, const float* cdf);
int32_t orc_update_cells_only(oracle* o, double V_I, double C_I);
/* the same update as an EARS iteration's: shared factors into slot 0 */
int32_t orc_update_cells_ears(oracle* o, double V_I, double C_I);
int32_t orc_refine_only(oracle* o);

/* building blocks exported for the pin tests */
void orc_philox(uint32_t k0, uint32_t k1, const uint32_t ctr[4], uint32_t out[4]);
void orc_sincos2pi(float u, float* s, float* c);
void orc_alg1(const float beta[3], float u, uint32_t gamma[3]);
void orc_alg1_enumerate(const float beta[3], uint32_t n, double mean[3], uint32_t tot_minmax[2],
                        float r_minmax[2]);
void orc_cell_beta(const oracle* o, const orc_iter_params* p, uint32_t cell, const float T[3],
                   const float It[3], int32_t depth, float beta[3]);
int32_t orc_bsdf_sample(const float* mat, const float n[3], const float wo[3], float u0, float u1,
                        float wi[3]);
void orc_bsdf_eval(const float* mat, const float n[3], const float wo[3], const float wi[3],
                   float fcos[3], float* pdf);
void orc_guided_sample(const float* pm, const float* cdf, float u0, float u1, float u2,
                       float wi[3]);
float orc_guided_pdf(const float* pm, const float wi[3]);
void orc_mis(int32_t aware, const float beta[3], const float p[3], float wdir[3], float wind[3]);
uint32_t orc_octree_lookup(const oracle* o, const float p[3], uint32_t* depth);
int32_t orc_intersect(const oracle* o, const float orig[3], const float dir[3], float tmax,
                      float* t, uint32_t* prim);
void orc_bdpt_weights(const oracle* o, const orc_iter_params* p, const float* P,
                      const uint32_t* prims, int32_t k, const float* It, float* out);
void orc_camera_ray(const oracle* o, int32_t px, int32_t py, float jx, float jy, float orig[3],
                    float dir[3]);

#ifdef __cplusplus
}
#endif
#endif
