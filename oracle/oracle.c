/* CPU oracle for the MARS hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Loaded only by the tests, the smoke check and the benchmark's CPU-baseline
 * leg.  Plain, slow and recursive on purpose: every function states the
 * passage of the paper it follows.  It shares no code with the HIP library.
 *
 * Numerics: path arithmetic in binary32 with the operation order written out
 * below (build with -ffp-contract=off, no fast-math); statistics in binary64.
 * Parity status of each part is listed at the function.
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* small float3 helpers, fixed evaluation order                             */
/* ------------------------------------------------------------------------ */
typedef struct { float x, y, z; } v3;
static inline v3 mk(float x, float y, float z) { v3 r = {x, y, z}; return r; }
static inline v3 vsub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static inline v3 vadd(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static inline v3 vscale(v3 a, float s) { return mk(a.x * s, a.y * s, a.z * s); }
static inline float vdot(v3 a, v3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
static inline v3 vcross(v3 a, v3 b) {
  return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static inline v3 vnorm(v3 a) {
  float il = 1.0f / sqrtf(vdot(a, a));
  return vscale(a, il);
}
static inline float lum3(v3 c) { return (0.2126f * c.x + 0.7152f * c.y) + 0.0722f * c.z; }
static inline float maxc3(v3 c) { return fmaxf(fmaxf(c.x, c.y), c.z); }

#define PI_F 3.14159265358979323846f
#define INV_PI_F 0.318309886183790671538f
#define ONE_MINUS_EPS 0.99999994f /* 1 - 2^-24 */

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11).  Written from the round function definition:  */
/* two 32x32->64 multiplications per round, Weyl-sequence key schedule.     */
/* Absolute known-answer parity: unpinned (no vectors available here);      */
/* pinned statistically and GPU-vs-CPU bit-exactly.                         */
/* ------------------------------------------------------------------------ */
void orc_philox(uint32_t k0, uint32_t k1, const uint32_t ctr[4], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Stream tags (high byte of the fourth counter word). */
#define TAG_CAM 0x43000000u
#define TAG_CHILD 0x4B000000u
#define TAG_DRAW 0x44000000u
#define TAG_LIGHT 0x4C000000u

typedef struct { uint32_t lo, hi; } stream_t;
typedef struct { uint32_t k0, k1; } key_t2;

static stream_t root_stream(key_t2 k, uint32_t px, uint32_t s, uint32_t iter, uint32_t tag) {
  uint32_t c[4] = {px, s, iter, tag}, o[4];
  orc_philox(k.k0, k.k1, c, o);
  stream_t r = {o[0], o[1]};
  return r;
}
/* child stream: a pure function of the parent stream and the tree address */
static stream_t child_stream(key_t2 k, stream_t p, uint32_t tech, uint32_t idx, uint32_t depth) {
  uint32_t c[4] = {p.lo, p.hi, (tech << 16) | (idx & 0xFFFFu), TAG_CHILD | (depth & 0xFFFFu)}, o[4];
  orc_philox(k.k0, k.k1, c, o);
  stream_t r = {o[0], o[1]};
  return r;
}
static inline float u01(uint32_t x) { return (float)(x >> 8) * 5.9604644775390625e-8f; }
static void draw4(key_t2 k, stream_t s, uint32_t j, float u[4]) {
  uint32_t c[4] = {s.lo, s.hi, j, TAG_DRAW}, o[4];
  orc_philox(k.k0, k.k1, c, o);
  for (int i = 0; i < 4; ++i) u[i] = u01(o[i]);
}

/* ------------------------------------------------------------------------ */
/* sin/cos of 2*pi*u for u in [0,1): reduction to a quarter turn, then      */
/* Taylor polynomials in theta^2 (coefficients (-1)^k/(2k+1)!, (-1)^k/(2k)!)*/
/* ------------------------------------------------------------------------ */
void orc_sincos2pi(float u, float* s_out, float* c_out) {
  float k = floorf(u * 4.0f + 0.5f);
  float r = u - k * 0.25f;
  int q = ((int)k) & 3;
  float th = r * 6.28318530717958647692f;
  float x2 = th * th;
  float ps = (float)(-1.0 / 39916800.0);
  ps = ps * x2 + (float)(1.0 / 362880.0);
  ps = ps * x2 + (float)(-1.0 / 5040.0);
  ps = ps * x2 + (float)(1.0 / 120.0);
  ps = ps * x2 + (float)(-1.0 / 6.0);
  float sn = th + (th * x2) * ps;
  float pc = (float)(1.0 / 479001600.0);
  pc = pc * x2 + (float)(-1.0 / 3628800.0);
  pc = pc * x2 + (float)(1.0 / 40320.0);
  pc = pc * x2 + (float)(-1.0 / 720.0);
  pc = pc * x2 + (float)(1.0 / 24.0);
  pc = pc * x2 + (float)(-1.0 / 2.0);
  float cs = 1.0f + x2 * pc;
  float S, C;
  switch (q) {
    case 0: S = sn; C = cs; break;
    case 1: S = cs; C = -sn; break;
    case 2: S = -sn; C = -cs; break;
    default: S = -cs; C = sn; break;
  }
  *s_out = S;
  *c_out = C;
}

/* ------------------------------------------------------------------------ */
/* Alg. 1 (supplement B.1): one uniform decides the rounding of all counts. */
/* gamma_t = floor(beta_t + r);  r <- r + beta_t - gamma_t                   */
/* Pinned by exhaustive enumeration (E[gamma_t] = beta_t).                  */
/* ------------------------------------------------------------------------ */
static void alg1n(const float* beta, int n, float u, uint32_t* gamma) {
  float r = u;
  for (int t = 0; t < n; ++t) {
    float s = r + beta[t];
    float g = floorf(s);
    gamma[t] = (uint32_t)g;
    r = s - g;
  }
}
static void alg1(const float beta[3], float u, uint32_t gamma[3]) { alg1n(beta, 3, u, gamma); }
void orc_alg1(const float beta[3], float u, uint32_t gamma[3]) { alg1(beta, u, gamma); }
/* the rounding of a vertex's counts: Alg. 1 with the first uniform of its
 * draw block 0, or (the naive scheme Alg. 1 replaces) each count rounded
 * with its own uniform, gamma_t = floor(beta_t + u_t), u_t the t-th uniform
 * of that block */
static void round_vertex(const orc_iter_params* p, const float* beta, const float u[4],
                         uint32_t* gamma, int n) {
  if (p->rounding) {  /* three counts only (rejected with per-length light paths) */
    for (int t = 0; t < 3; ++t) gamma[t] = (uint32_t)floorf(beta[t] + u[t]);
    return;
  }
  alg1n(beta, n, u[0], gamma);
}
/* enumerate u = k / n for k = 0..n-1: mean counts, range of the total and of r */
void orc_alg1_enumerate(const float beta[3], uint32_t n, double mean[3], uint32_t tot_minmax[2],
                        float r_minmax[2]) {
  double acc[3] = {0, 0, 0};
  uint32_t tmin = 0xFFFFFFFFu, tmax = 0;
  float rmin = INFINITY, rmax = -INFINITY;
  for (uint32_t k = 0; k < n; ++k) {
    float u = (float)((double)k / (double)n);
    float r = u;
    uint32_t tot = 0;
    for (int t = 0; t < 3; ++t) {
      float s = r + beta[t];
      float g = floorf(s);
      r = s - g;
      acc[t] += g;
      tot += (uint32_t)g;
      if (r < rmin) rmin = r;
      if (r > rmax) rmax = r;
    }
    if (tot < tmin) tmin = tot;
    if (tot > tmax) tmax = tot;
  }
  for (int t = 0; t < 3; ++t) mean[t] = acc[t] / (double)n;
  tot_minmax[0] = tmin; tot_minmax[1] = tmax;
  r_minmax[0] = rmin; r_minmax[1] = rmax;
}

/* ------------------------------------------------------------------------ */
/* Balance heuristic (supplement A.1 w_it = 1_it p_t / sum_k 1_ik p_k; the   */
/* budget-aware form multiplies every p_k by beta_k, Sec. 3 "Proxy model"). */
/* direct light: techniques {B, N, G}; indirect: {B, G} (Sec. 3 "The model")*/
/* denominators: (b_B p_B + b_G p_G) + b_N p_N  and  b_B p_B + b_G p_G.     */
/* Pinned: sum_t w = 1 (supplement A.1, "Unbiasedness").                    */
/* ------------------------------------------------------------------------ */
void orc_mis(int32_t aware, const float beta[3], const float p[3], float wdir[3], float wind[3]) {
  float b[3];
  for (int t = 0; t < 3; ++t) b[t] = aware ? beta[t] : (beta[t] > 0.0f ? 1.0f : 0.0f);
  float nb = b[0] * p[0], nn = b[1] * p[1], ng = b[2] * p[2];
  float dind = nb + ng;
  float ddir = dind + nn;
  wdir[0] = ddir > 0.0f ? nb / ddir : 0.0f;
  wdir[1] = ddir > 0.0f ? nn / ddir : 0.0f;
  wdir[2] = ddir > 0.0f ? ng / ddir : 0.0f;
  wind[0] = dind > 0.0f ? nb / dind : 0.0f;
  wind[1] = 0.0f;
  wind[2] = dind > 0.0f ? ng / dind : 0.0f;
}

/* ------------------------------------------------------------------------ */
/* scene                                                                    */
/* ------------------------------------------------------------------------ */
typedef struct {
  float lo[3], hi[3];
  int32_t left, right; /* -1 for leaves */
  int32_t first, count;
} obvh_node;

struct oracle {
  orc_config cfg;
  int32_t ntri, nmat, W, H;
  v3 *v0, *e1, *e2, *ng;
  uint32_t* tmat;
  float* mats; /* [nmat][8] */
  float* lpdf; /* per triangle: p_select / area, 0 if not emissive */
  int32_t nlights;
  int32_t* light_tri;
  float* light_cdf;
  float eps;
  v3 oct_lo;
  float oct_inv;
  v3 cam_o, cam_f, cam_r, cam_u;
  /* acceleration (median split BVH, independent of the GPU builder) */
  obvh_node* bvh;
  int32_t nbvh;
  int32_t* bvh_idx;
  /* octree */
  uint32_t* nodes;
  int32_t nnodes, ncells, maxc;
  uint32_t *leaf_node, *leaf_depth, *visits;
  float* fac;     /* [maxc][2][3][3] */
  double* acc;    /* [maxc][3][8] */
  int32_t nlp;    /* light-path budgets per vertex: 1, or 3 (y_1, y_2, y_3+) */
  float* fac_x;   /* nlp = 3: [maxc][2][2][3], techniques 3 and 4 */
  double* acc_x;  /* nlp = 3: [maxc][2][8] */
  float *pm, *cdf;/* [maxc][64] */
  double* hacc;   /* [maxc][64] */
  float* fixed_beta; int32_t nfixed;
  int32_t rec_depth; /* tests: > 0 logs only the samples of vertices up to this depth */
  int32_t ears_update; /* the running update belongs to an EARS iteration */
  /* image */
  int32_t spp_last;
  float* Ls;      /* per root radiance [W*H*spp][3] */
  float* iter_sum;/* [W*H][3] */
  float* accum;   /* [W*H][3] */
  double total_spp;
  float* Itilde;  /* [W*H][3] */
  double* ivw_acc; double ivw_w;
  float* count_map; /* [W*H][3] */
  float* beta1;   /* per root beta at x1 [W*H*spp][3] */
  uint64_t rays_last;
  /* debug */
  orc_vertex_rec* dbg; int32_t ndbg;
  unsigned char* pix_mask; /* optional: render only these pixels */
  /* BDPT light subpaths of the current iteration (one per camera sample) */
  struct lightpath* lpaths; size_t nlpaths;
};

/* ---- median-split BVH over triangle indices (oracle's own, simple) ---- */
static const float* g_cent;
static int g_axis;
static int cmp_cent(const void* a, const void* b) {
  int32_t i = *(const int32_t*)a, j = *(const int32_t*)b;
  float ci = g_cent[3 * i + g_axis], cj = g_cent[3 * j + g_axis];
  if (ci < cj) return -1;
  if (ci > cj) return 1;
  return (i > j) - (i < j);
}
static int32_t obvh_build(oracle* o, float* cent, int32_t first, int32_t count, float pad) {
  int32_t id = o->nbvh++;
  obvh_node* n = &o->bvh[id];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  float clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int32_t k = first; k < first + count; ++k) {
    int32_t t = o->bvh_idx[k];
    v3 a = o->v0[t], b = vadd(o->v0[t], o->e1[t]), c = vadd(o->v0[t], o->e2[t]);
    float xs[3][3] = {{a.x, a.y, a.z}, {b.x, b.y, b.z}, {c.x, c.y, c.z}};
    for (int v = 0; v < 3; ++v)
      for (int d = 0; d < 3; ++d) {
        lo[d] = fminf(lo[d], xs[v][d]);
        hi[d] = fmaxf(hi[d], xs[v][d]);
      }
    for (int d = 0; d < 3; ++d) {
      clo[d] = fminf(clo[d], cent[3 * t + d]);
      chi[d] = fmaxf(chi[d], cent[3 * t + d]);
    }
  }
  for (int d = 0; d < 3; ++d) {
    n->lo[d] = lo[d] - pad;
    n->hi[d] = hi[d] + pad;
  }
  if (count <= 4) {
    n->left = n->right = -1;
    n->first = first;
    n->count = count;
    return id;
  }
  int axis = 0;
  float ext = chi[0] - clo[0];
  if (chi[1] - clo[1] > ext) { axis = 1; ext = chi[1] - clo[1]; }
  if (chi[2] - clo[2] > ext) { axis = 2; }
  g_cent = cent;
  g_axis = axis;
  qsort(o->bvh_idx + first, (size_t)count, sizeof(int32_t), cmp_cent);
  int32_t half = count / 2;
  int32_t l = obvh_build(o, cent, first, half, pad);
  int32_t r = obvh_build(o, cent, first + half, count - half, pad);
  n = &o->bvh[id];
  n->left = l;
  n->right = r;
  n->first = n->count = 0;
  return id;
}

/* Moller-Trumbore ray/triangle test, two-sided, fixed operation order.
 * Returns 1 with t/u/v if the ray meets the triangle plane inside the
 * triangle; the caller applies the t-range. */
static int isect_tri(const oracle* o, int32_t i, v3 org, v3 dir, float* t_out) {
  v3 e1 = o->e1[i], e2 = o->e2[i];
  v3 p = vcross(dir, e2);
  float det = vdot(e1, p);
  if (det == 0.0f) return 0;
  float inv = 1.0f / det;
  v3 s = vsub(org, o->v0[i]);
  float u = vdot(s, p) * inv;
  if (u < 0.0f || u > 1.0f) return 0;
  v3 q = vcross(s, e1);
  float v = vdot(dir, q) * inv;
  if (v < 0.0f || u + v > 1.0f) return 0;
  *t_out = vdot(e2, q) * inv;
  return 1;
}

static int box_hit(const obvh_node* n, v3 org, v3 dir, float tmax) {
  float tn = -INFINITY, tf = INFINITY;
  float o3[3] = {org.x, org.y, org.z}, d3[3] = {dir.x, dir.y, dir.z};
  for (int a = 0; a < 3; ++a) {
    if (d3[a] == 0.0f) {
      if (o3[a] < n->lo[a] || o3[a] > n->hi[a]) return 0;
      continue;
    }
    float inv = 1.0f / d3[a];
    float t1 = (n->lo[a] - o3[a]) * inv, t2 = (n->hi[a] - o3[a]) * inv;
    float a1 = fminf(t1, t2), a2 = fmaxf(t1, t2);
    if (a1 > tn) tn = a1;
    if (a2 < tf) tf = a2;
  }
  return tn <= tf && tf >= 0.0f && tn <= tmax;
}

/* Closest hit: the smallest t in (0, tmax); equal t resolved to the smaller
 * primitive index, so the answer does not depend on traversal order. */
static int closest_hit(const oracle* o, v3 org, v3 dir, float tmax, float* t_out, uint32_t* prim) {
  int32_t stack[128];
  int sp = 0;
  stack[sp++] = 0;
  float bt = tmax;
  uint32_t bp = 0xFFFFFFFFu;
  while (sp) {
    const obvh_node* n = &o->bvh[stack[--sp]];
    if (!box_hit(n, org, dir, bt)) continue;
    if (n->left < 0) {
      for (int32_t k = n->first; k < n->first + n->count; ++k) {
        int32_t i = o->bvh_idx[k];
        float t;
        if (!isect_tri(o, i, org, dir, &t)) continue;
        if (!(t > 0.0f && t < tmax)) continue;
        if (t < bt || (t == bt && (uint32_t)i < bp)) {
          bt = t;
          bp = (uint32_t)i;
        }
      }
    } else {
      stack[sp++] = n->left;
      stack[sp++] = n->right;
    }
  }
  if (bp == 0xFFFFFFFFu) return 0;
  *t_out = bt;
  *prim = bp;
  return 1;
}

static int occluded(const oracle* o, v3 org, v3 dir, float tmax) {
  int32_t stack[128];
  int sp = 0;
  stack[sp++] = 0;
  while (sp) {
    const obvh_node* n = &o->bvh[stack[--sp]];
    if (!box_hit(n, org, dir, tmax)) continue;
    if (n->left < 0) {
      for (int32_t k = n->first; k < n->first + n->count; ++k) {
        float t;
        if (isect_tri(o, o->bvh_idx[k], org, dir, &t) && t > 0.0f && t < tmax) return 1;
      }
    } else {
      stack[sp++] = n->left;
      stack[sp++] = n->right;
    }
  }
  return 0;
}

int32_t orc_intersect(const oracle* o, const float orig[3], const float dir[3], float tmax,
                      float* t, uint32_t* prim) {
  return closest_hit(o, mk(orig[0], orig[1], orig[2]), mk(dir[0], dir[1], dir[2]), tmax, t, prim);
}

/* ------------------------------------------------------------------------ */
/* octree (the EARS-style spatial cache of Sec. 5.1; max depth 8, split     */
/* after more than 32 visits).  Lookup: per level, one bit per axis from    */
/* q >= 0.5, then q <- 2q - bit (exact in binary32).                         */
/* Pinned against floor(q * 2^depth) computed independently in the tests.  */
/* ------------------------------------------------------------------------ */
#define LEAF_BIT 0x80000000u
static uint32_t octree_lookup(const oracle* o, v3 p, uint32_t* depth_out) {
  float qx = (p.x - o->oct_lo.x) * o->oct_inv;
  float qy = (p.y - o->oct_lo.y) * o->oct_inv;
  float qz = (p.z - o->oct_lo.z) * o->oct_inv;
  qx = fminf(fmaxf(qx, 0.0f), ONE_MINUS_EPS);
  qy = fminf(fmaxf(qy, 0.0f), ONE_MINUS_EPS);
  qz = fminf(fmaxf(qz, 0.0f), ONE_MINUS_EPS);
  uint32_t node = 0, d = 0;
  while (!(o->nodes[node] & LEAF_BIT)) {
    uint32_t bx = qx >= 0.5f, by = qy >= 0.5f, bz = qz >= 0.5f;
    qx = qx * 2.0f - (float)bx;
    qy = qy * 2.0f - (float)by;
    qz = qz * 2.0f - (float)bz;
    node = o->nodes[node] + (bx | (by << 1) | (bz << 2));
    ++d;
  }
  if (depth_out) *depth_out = d;
  return o->nodes[node] & ~LEAF_BIT;
}
uint32_t orc_octree_lookup(const oracle* o, const float p[3], uint32_t* depth) {
  return octree_lookup(o, mk(p[0], p[1], p[2]), depth);
}

/* ------------------------------------------------------------------------ */
/* BSDFs.  Lambert: cosine sampling.  GGX (Walter et al. 2007): D cos(th_h) */
/* half-vector sampling, Smith G, Schlick F with F0 = albedo.  Two-sided:   */
/* n is the geometric normal flipped towards wo.                            */
/* Pinned: pdf normalisation and E[f cos / p] against quadrature (tests).  */
/* ------------------------------------------------------------------------ */
static void onb(v3 n, v3* t, v3* b) {
  float sgn = n.z >= 0.0f ? 1.0f : -1.0f;
  float a = -1.0f / (sgn + n.z);
  float bb = (n.x * n.y) * a;
  *t = mk(1.0f + (sgn * (n.x * n.x)) * a, sgn * bb, -(sgn * n.x));
  *b = mk(bb, sgn + (n.y * n.y) * a, -n.y);
}
static inline v3 to_world(v3 l, v3 t, v3 b, v3 n) {
  return mk((l.x * t.x + l.y * b.x) + l.z * n.x, (l.x * t.y + l.y * b.y) + l.z * n.y,
            (l.x * t.z + l.y * b.z) + l.z * n.z);
}

/* returns 1 and a direction if the sample is above the surface */
static int bsdf_sample(const float* m, v3 n, v3 wo, float u0, float u1, v3* wi) {
  v3 t, b;
  onb(n, &t, &b);
  float sn, cs;
  if (m[0] == 0.0f) {
    float r = sqrtf(u0);
    orc_sincos2pi(u1, &sn, &cs);
    v3 l = mk(r * cs, r * sn, sqrtf(fmaxf(0.0f, 1.0f - u0)));
    *wi = to_world(l, t, b, n);
  } else {
    float a2 = m[4] * m[4];
    float t2 = (a2 * u0) / (1.0f - u0);
    float ch = 1.0f / sqrtf(1.0f + t2);
    float sh = sqrtf(fmaxf(0.0f, 1.0f - ch * ch));
    orc_sincos2pi(u1, &sn, &cs);
    v3 h = to_world(mk(sh * cs, sh * sn, ch), t, b, n);
    float d = vdot(wo, h);
    *wi = mk((2.0f * d) * h.x - wo.x, (2.0f * d) * h.y - wo.y, (2.0f * d) * h.z - wo.z);
  }
  return vdot(n, *wi) > 0.0f;
}

/* f(wo,wi)|cos theta_i| per channel, and the BSDF-sampling solid-angle pdf */
static void bsdf_eval(const float* m, v3 n, v3 wo, v3 wi, v3* fcos, float* pdf) {
  float ci = vdot(n, wi), co = vdot(n, wo);
  if (ci <= 0.0f || co <= 0.0f) {
    *fcos = mk(0, 0, 0);
    *pdf = 0.0f;
    return;
  }
  if (m[0] == 0.0f) {
    *fcos = mk((m[1] * INV_PI_F) * ci, (m[2] * INV_PI_F) * ci, (m[3] * INV_PI_F) * ci);
    *pdf = ci * INV_PI_F;
    return;
  }
  float a2 = m[4] * m[4];
  v3 h = vnorm(vadd(wo, wi));
  float ch = vdot(n, h), oh = vdot(wo, h);
  if (ch <= 0.0f || oh <= 0.0f) {
    *fcos = mk(0, 0, 0);
    *pdf = 0.0f;
    return;
  }
  float k = (ch * ch) * (a2 - 1.0f) + 1.0f;
  float D = a2 / ((PI_F * k) * k);
  float g1o = (2.0f * co) / (co + sqrtf(a2 + (1.0f - a2) * (co * co)));
  float g1i = (2.0f * ci) / (ci + sqrtf(a2 + (1.0f - a2) * (ci * ci)));
  float G = g1o * g1i;
  float mm = fmaxf(0.0f, 1.0f - vdot(wi, h));
  float m5 = ((mm * mm) * (mm * mm)) * mm;
  float F[3];
  for (int c = 0; c < 3; ++c) F[c] = m[1 + c] + (1.0f - m[1 + c]) * m5;
  float den = 4.0f * co;
  *fcos = mk(((D * G) * F[0]) / den, ((D * G) * F[1]) / den, ((D * G) * F[2]) / den);
  *pdf = (D * ch) / (4.0f * oh);
}

int32_t orc_bsdf_sample(const float* mat, const float n[3], const float wo[3], float u0, float u1,
                        float wi[3]) {
  v3 w;
  int ok = bsdf_sample(mat, mk(n[0], n[1], n[2]), mk(wo[0], wo[1], wo[2]), u0, u1, &w);
  wi[0] = w.x; wi[1] = w.y; wi[2] = w.z;
  return ok;
}
void orc_bsdf_eval(const float* mat, const float n[3], const float wo[3], const float wi[3],
                   float fcos[3], float* pdf) {
  v3 f;
  bsdf_eval(mat, mk(n[0], n[1], n[2]), mk(wo[0], wo[1], wo[2]), mk(wi[0], wi[1], wi[2]), &f, pdf);
  fcos[0] = f.x; fcos[1] = f.y; fcos[2] = f.z;
}

/* ------------------------------------------------------------------------ */
/* Guided technique: per-cell 8x8 equal-area directional histogram (z =    */
/* cos(theta) in 8 bins of [-1,1], phi in 8 bins of [0,2pi), world frame).  */
/* pm[b] is the mixed pmf (0.9 learned + 0.1 uniform); pdf = pm * 64/(4pi). */
/* Pinned: pdf integrates to 1; sample histogram matches pm (tests).       */
/* ------------------------------------------------------------------------ */
static int phi_octant(float x, float y) {
  if (y >= 0.0f) {
    if (x > 0.0f) return (y < x) ? 0 : 1;
    return (y > -x) ? 2 : 3;
  }
  if (x < 0.0f) return (-y < -x) ? 4 : 5;
  return (-y > x) ? 6 : 7;
}
static int guided_bin(v3 w) {
  int bz = (int)floorf((w.z + 1.0f) * 4.0f);
  bz = bz < 0 ? 0 : (bz > 7 ? 7 : bz);
  return bz * 8 + phi_octant(w.x, w.y);
}
static float guided_pdf(const float* pm, v3 w) {
  return pm[guided_bin(w)] * (float)(16.0 / 3.14159265358979323846);
}
static v3 guided_sample(const float* cdf, float u0, float u1, float u2) {
  int b = 0;
  while (b < 63 && !(u0 < cdf[b])) ++b;
  int bz = b >> 3, bp = b & 7;
  float z = -1.0f + 0.25f * ((float)bz + u1);
  float sn, cs;
  orc_sincos2pi(((float)bp + u2) * 0.125f, &sn, &cs);
  float s = sqrtf(fmaxf(0.0f, 1.0f - z * z));
  return mk(s * cs, s * sn, z);
}
void orc_guided_sample(const float* pm, const float* cdf, float u0, float u1, float u2,
                       float wi[3]) {
  (void)pm;
  v3 w = guided_sample(cdf, u0, u1, u2);
  wi[0] = w.x; wi[1] = w.y; wi[2] = w.z;
}
float orc_guided_pdf(const float* pm, const float wi[3]) {
  return guided_pdf(pm, mk(wi[0], wi[1], wi[2]));
}

/* ------------------------------------------------------------------------ */
/* camera: pinhole, W/p = 1, uniform jitter inside the pixel               */
/* ------------------------------------------------------------------------ */
static void camera_ray(const oracle* o, int32_t px, int32_t py, float jx, float jy, v3* org,
                       v3* dir) {
  float sx = (((float)px + jx) / (float)o->W) * 2.0f - 1.0f;
  float sy = 1.0f - (((float)py + jy) / (float)o->H) * 2.0f;
  v3 d = mk((o->cam_f.x + sx * o->cam_r.x) + sy * o->cam_u.x,
            (o->cam_f.y + sx * o->cam_r.y) + sy * o->cam_u.y,
            (o->cam_f.z + sx * o->cam_r.z) + sy * o->cam_u.z);
  *org = o->cam_o;
  *dir = vnorm(d);
}
void orc_camera_ray(const oracle* o, int32_t px, int32_t py, float jx, float jy, float orig[3],
                    float dir[3]) {
  v3 a, b;
  camera_ray(o, px, py, jx, jy, &a, &b);
  orig[0] = a.x; orig[1] = a.y; orig[2] = a.z;
  dir[0] = b.x; dir[1] = b.y; dir[2] = b.z;
}

/* ------------------------------------------------------------------------ */
/* creation                                                                 */
/* ------------------------------------------------------------------------ */
static void octree_reset(oracle* o) {
  o->nodes[0] = LEAF_BIT | 0u;
  o->nnodes = 1;
  o->ncells = 1;
  o->leaf_node[0] = 0;
  o->leaf_depth[0] = 0;
  for (int t = 0; t < 3; ++t)
    for (int k = 0; k < 2; ++k)
      for (int c = 0; c < 3; ++c) o->fac[((0 * 2 + k) * 3 + t) * 3 + c] = -1.0f;
  if (o->fac_x)
    for (int k = 0; k < 12; ++k) o->fac_x[k] = -1.0f;
  for (int b = 0; b < 64; ++b) {
    o->pm[b] = (float)(1.0 / 64.0);
    o->cdf[b] = (float)((double)(b + 1) / 64.0);
  }
  o->cdf[63] = 1.0f;
}

oracle* orc_create(const float* V, const uint32_t* tri_mat, int32_t ntri, const float* mats,
                   int32_t nmat, const float* cam, int32_t width, int32_t height,
                   const orc_config* cfg) {
  if (ntri <= 0 || width <= 0 || height <= 0) return NULL;
  oracle* o = (oracle*)calloc(1, sizeof(oracle));
  o->cfg = *cfg;
  o->ntri = ntri;
  o->nmat = nmat;
  o->W = width;
  o->H = height;
  o->v0 = malloc(sizeof(v3) * ntri);
  o->e1 = malloc(sizeof(v3) * ntri);
  o->e2 = malloc(sizeof(v3) * ntri);
  o->ng = malloc(sizeof(v3) * ntri);
  o->tmat = malloc(sizeof(uint32_t) * ntri);
  o->lpdf = calloc(ntri, sizeof(float));
  o->mats = malloc(sizeof(float) * 8 * nmat);
  memcpy(o->mats, mats, sizeof(float) * 8 * nmat);
  memcpy(o->tmat, tri_mat, sizeof(uint32_t) * ntri);
  double* area = malloc(sizeof(double) * ntri);
  float bmin[3] = {INFINITY, INFINITY, INFINITY}, bmax[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int32_t i = 0; i < ntri; ++i) {
    const float* p = V + 9 * i;
    for (int k = 0; k < 9; ++k) {
      bmin[k % 3] = fminf(bmin[k % 3], p[k]);
      bmax[k % 3] = fmaxf(bmax[k % 3], p[k]);
    }
    o->v0[i] = mk(p[0], p[1], p[2]);
    o->e1[i] = mk(p[3] - p[0], p[4] - p[1], p[5] - p[2]);
    o->e2[i] = mk(p[6] - p[0], p[7] - p[1], p[8] - p[2]);
    double a[3] = {o->e1[i].x, o->e1[i].y, o->e1[i].z}, b[3] = {o->e2[i].x, o->e2[i].y, o->e2[i].z};
    double c[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    double l = sqrt((c[0] * c[0] + c[1] * c[1]) + c[2] * c[2]);
    area[i] = 0.5 * l;
    if (l > 0.0)
      o->ng[i] = mk((float)(c[0] / l), (float)(c[1] / l), (float)(c[2] / l));
    else
      o->ng[i] = mk(0.0f, 0.0f, 1.0f);
  }
  /* emitters: selection proportional to area * luminance(Le) */
  double wsum = 0.0;
  int32_t nl = 0;
  for (int32_t i = 0; i < ntri; ++i) {
    const float* m = o->mats + 8 * o->tmat[i];
    if (fmaxf(fmaxf(m[5], m[6]), m[7]) > 0.0f && area[i] > 0.0) ++nl;
  }
  o->nlights = nl;
  o->light_tri = malloc(sizeof(int32_t) * (nl ? nl : 1));
  o->light_cdf = malloc(sizeof(float) * (nl ? nl : 1));
  double* lw = malloc(sizeof(double) * (nl ? nl : 1));
  nl = 0;
  for (int32_t i = 0; i < ntri; ++i) {
    const float* m = o->mats + 8 * o->tmat[i];
    if (fmaxf(fmaxf(m[5], m[6]), m[7]) > 0.0f && area[i] > 0.0) {
      double L = (0.2126 * (double)m[5] + 0.7152 * (double)m[6]) + 0.0722 * (double)m[7];
      lw[nl] = area[i] * L;
      o->light_tri[nl] = i;
      ++nl;
    }
  }
  for (int32_t k = 0; k < nl; ++k) wsum += lw[k];
  double run = 0.0;
  for (int32_t k = 0; k < nl; ++k) {
    run += lw[k];
    o->light_cdf[k] = (k == nl - 1) ? 1.0f : (float)(run / wsum);
    o->lpdf[o->light_tri[k]] = (float)((lw[k] / wsum) / area[o->light_tri[k]]);
  }
  free(lw);
  free(area);
  double ext = fmax(fmax((double)bmax[0] - bmin[0], (double)bmax[1] - bmin[1]),
                    (double)bmax[2] - bmin[2]);
  o->eps = (float)(1e-4 * ext);
  double side = ext * (1.0 + 2e-4);
  double ctr[3];
  for (int k = 0; k < 3; ++k) ctr[k] = 0.5 * ((double)bmin[k] + (double)bmax[k]);
  o->oct_lo = mk((float)(ctr[0] - 0.5 * side), (float)(ctr[1] - 0.5 * side),
                 (float)(ctr[2] - 0.5 * side));
  o->oct_inv = (float)(1.0 / side);
  /* camera basis in binary64 */
  {
    double P[3] = {cam[0], cam[1], cam[2]}, Tg[3] = {cam[3], cam[4], cam[5]},
           U[3] = {cam[6], cam[7], cam[8]};
    double f[3] = {Tg[0] - P[0], Tg[1] - P[1], Tg[2] - P[2]};
    double fl = sqrt((f[0] * f[0] + f[1] * f[1]) + f[2] * f[2]);
    for (int k = 0; k < 3; ++k) f[k] /= fl;
    double r[3] = {f[1] * U[2] - f[2] * U[1], f[2] * U[0] - f[0] * U[2], f[0] * U[1] - f[1] * U[0]};
    double rl = sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]);
    for (int k = 0; k < 3; ++k) r[k] /= rl;
    double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
    double th = tan(0.5 * (double)cam[9] * 3.14159265358979323846 / 180.0);
    double asp = (double)width / (double)height;
    o->cam_o = mk(cam[0], cam[1], cam[2]);
    o->cam_f = mk((float)f[0], (float)f[1], (float)f[2]);
    o->cam_r = mk((float)(r[0] * th * asp), (float)(r[1] * th * asp), (float)(r[2] * th * asp));
    o->cam_u = mk((float)(u[0] * th), (float)(u[1] * th), (float)(u[2] * th));
  }
  /* BVH */
  {
    float* cent = malloc(sizeof(float) * 3 * ntri);
    for (int32_t i = 0; i < ntri; ++i) {
      v3 a = o->v0[i], b = vadd(o->v0[i], o->e1[i]), c = vadd(o->v0[i], o->e2[i]);
      cent[3 * i + 0] = (a.x + b.x + c.x) / 3.0f;
      cent[3 * i + 1] = (a.y + b.y + c.y) / 3.0f;
      cent[3 * i + 2] = (a.z + b.z + c.z) / 3.0f;
    }
    o->bvh_idx = malloc(sizeof(int32_t) * ntri);
    for (int32_t i = 0; i < ntri; ++i) o->bvh_idx[i] = i;
    o->bvh = malloc(sizeof(obvh_node) * 2 * (size_t)ntri);
    o->nbvh = 0;
    obvh_build(o, cent, 0, ntri, (float)(1e-5 * ext) + 1e-7f);
    free(cent);
  }
  /* octree + caches */
  int32_t mc = cfg->max_cells > 8 ? cfg->max_cells : 8;
  o->maxc = mc;
  o->nodes = malloc(sizeof(uint32_t) * (1 + 8 * (size_t)mc));
  o->leaf_node = calloc(mc, sizeof(uint32_t));
  o->leaf_depth = calloc(mc, sizeof(uint32_t));
  o->visits = calloc(mc, sizeof(uint32_t));
  o->fac = calloc((size_t)mc * 18, sizeof(float));
  o->acc = calloc((size_t)mc * 24, sizeof(double));
  o->pm = calloc((size_t)mc * 64, sizeof(float));
  o->cdf = calloc((size_t)mc * 64, sizeof(float));
  o->hacc = calloc((size_t)mc * 64, sizeof(double));
  o->nlp = (cfg->mode == ORC_MODE_BDPT && cfg->lp_classes == 3) ? 3 : 1;
  if (o->nlp == 3) {
    o->fac_x = calloc((size_t)mc * 12, sizeof(float));
    o->acc_x = calloc((size_t)mc * 16, sizeof(double));
  }
  octree_reset(o);
  size_t npx = (size_t)width * height;
  o->iter_sum = calloc(npx * 3, sizeof(float));
  o->accum = calloc(npx * 3, sizeof(float));
  o->Itilde = malloc(npx * 3 * sizeof(float));
  for (size_t i = 0; i < npx * 3; ++i) o->Itilde[i] = INFINITY;
  o->ivw_acc = calloc(npx * 3, sizeof(double));
  o->count_map = calloc(npx * 3, sizeof(float));
  return o;
}

void orc_destroy(oracle* o) {
  if (!o) return;
  free(o->v0); free(o->e1); free(o->e2); free(o->ng); free(o->tmat); free(o->lpdf);
  free(o->mats); free(o->light_tri); free(o->light_cdf); free(o->bvh); free(o->bvh_idx);
  free(o->nodes); free(o->leaf_node); free(o->leaf_depth); free(o->visits); free(o->fac);
  free(o->acc); free(o->pm); free(o->cdf); free(o->hacc); free(o->fixed_beta); free(o->Ls);
  free(o->iter_sum); free(o->accum); free(o->Itilde); free(o->ivw_acc); free(o->count_map);
  free(o->beta1); free(o->dbg); free(o->pix_mask); free(o->lpaths);
  free(o->fac_x); free(o->acc_x);
  free(o);
}

int32_t orc_set_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* per-row logs: every statistic is logged and merged in row order, so the */
/* result does not depend on the thread count                              */
/* ------------------------------------------------------------------------ */
enum { REC_SAMPLE = 0, REC_VISIT = 1, REC_HIST = 2 };
typedef struct {
  uint32_t kind, cell, tech, bin;
  float v[3];
  uint32_t cost;
  float w;
} stat_rec;
typedef struct {
  stat_rec* r; size_t n, cap;
  orc_vertex_rec* d; size_t nd, capd;
  uint64_t rays_ext, rays_shadow, rays_light, rays_conn, vertices, samples;
} rowlog;
static void log_push(rowlog* L, stat_rec s) {
  if (L->n == L->cap) {
    L->cap = L->cap ? 2 * L->cap : 256;
    L->r = realloc(L->r, L->cap * sizeof(stat_rec));
  }
  L->r[L->n++] = s;
}
static void dbg_push(rowlog* L, orc_vertex_rec s) {
  if (L->nd == L->capd) {
    L->capd = L->capd ? 2 * L->capd : 64;
    L->d = realloc(L->d, L->capd * sizeof(orc_vertex_rec));
  }
  L->d[L->nd++] = s;
}

typedef struct {
  const oracle* o;
  const orc_iter_params* p;
  key_t2 key;
  rowlog* L;
  uint32_t pix, root;
  float It[3];   /* I~ of the pixel */
} tctx;

/* ------------------------------------------------------------------------ */
/* per-vertex sample counts                                                 */
/*  MARS (Sec. 3.1 "Optimization" with the colour rule of Sec. 4.1):        */
/*   beta^X_t = sqrt( (1/3) sum_ch (T_ch / I~_ch)^2 a^X_{t,ch} ),            */
/*   a^RR = C_I/(C_t V_I) E[<L_t>^2],  a^S = C_I/(C_t V_I) V[<L_t>]          */
/*   beta = beta^RR if < 1, else beta^S if > 1, else 1; clamped [lo, hi].   */
/*  classic RR (Sec. 4.2 baseline): q = min(1, max_ch T) from rr_start on.  */
/* ------------------------------------------------------------------------ */
static void classic_beta(const tctx* c, v3 T, int depth, float beta[3]) {
  float q = (depth >= c->p->rr_start) ? fminf(1.0f, maxc3(T)) : 1.0f;
  int mode = c->o->cfg.mode;
  if (mode == ORC_MODE_PT_GUIDED) {
    beta[0] = q * 0.5f; beta[1] = 1.0f; beta[2] = q * 0.5f;
  } else if (mode == ORC_MODE_BDPT) {
    beta[0] = q; beta[1] = 1.0f; beta[2] = 1.0f;
  } else {
    beta[0] = q; beta[1] = 1.0f; beta[2] = 0.0f;
  }
}

/* ------------------------------------------------------------------------ */
/* EARS (the baseline of Sec. 5; Fig. 1: the same number of samples for    */
/* every technique).  Counts beta_t = r_t lambda with the per-technique    */
/* ratios r of the classic scheme at q = 1.  On that line the efficiency   */
/* model of Sec. 3.1 (variance sum_t V_t / beta_t, cost sum_t beta_t C_t)  */
/* is optimal at lambda^2 = (C_I / V_I) sum_t (M_t / r_t) / sum_t r_t C_t, */
/* with M the per-sample second moment (RR) or variance (splitting) of     */
/* technique t: the fixed point of Sec. 3.1 restricted to that line, which */
/* the supplemental derivation notes reduces to the EARS scheme.  The      */
/* shared factors are kept in technique slot 0 of the cell factors.        */
/* ------------------------------------------------------------------------ */
static void ears_ratios(int mode, double r[3]) {
  if (mode == ORC_MODE_PT_GUIDED) { r[0] = 0.5; r[1] = 1.0; r[2] = 0.5; }
  else if (mode == ORC_MODE_BDPT) { r[0] = 1.0; r[1] = 1.0; r[2] = 1.0; }
  else { r[0] = 1.0; r[1] = 1.0; r[2] = 0.0; }
}

/* resolve one technique's count from its cell factors (Sec. 3.1 fixed
 * point, three cases; "Handling colors": L2 norm over the channels of the
 * image-relative throughput z); classic count cb when the cell has no data */
static float resolve_beta(const float* aRR, const float* aS, const float z[3], float cb) {
  if (aRR[0] < 0.0f) return cb;
  float sr = ((z[0] * z[0]) * aRR[0] + (z[1] * z[1]) * aRR[1]) + (z[2] * z[2]) * aRR[2];
  float ss = ((z[0] * z[0]) * aS[0] + (z[1] * z[1]) * aS[1]) + (z[2] * z[2]) * aS[2];
  float bRR = sqrtf(sr * (1.0f / 3.0f));
  float bS = sqrtf(ss * (1.0f / 3.0f));
  if (bRR < 1.0f) return bRR;
  if (bS > 1.0f) return bS;
  return 1.0f;
}

/* counts of a vertex: beta[0..2] (BSDF, NEE, guided or light path); with
 * per-length light-path budgets also beta[3], beta[4] (light vertex y_2,
 * y_3+; beta[2] then belongs to y_1).  beta has room for five. */
static void vertex_beta(const tctx* c, uint32_t cell, v3 T, int depth, float beta[5]) {
  const oracle* o = c->o;
  const orc_iter_params* p = c->p;
  float cb[3];
  classic_beta(c, T, depth, cb);
  int enabled[3] = {1, o->cfg.nee_enabled && o->nlights > 0, o->cfg.mode != ORC_MODE_PT};
  float z[3] = {T.x / c->It[0], T.y / c->It[1], T.z / c->It[2]};
  beta[3] = 0.0f;
  beta[4] = 0.0f;
  if (p->alloc == ORC_ALLOC_EARS) {
    const float* aRR = o->fac + ((cell * 2 + 0) * 3 + 0) * 3;
    const float* aS = o->fac + ((cell * 2 + 1) * 3 + 0) * 3;
    double r[3];
    ears_ratios(o->cfg.mode, r);
    float lam = 0.0f;
    if (!(aRR[0] < 0.0f)) {
      float sr = ((z[0] * z[0]) * aRR[0] + (z[1] * z[1]) * aRR[1]) + (z[2] * z[2]) * aRR[2];
      float ss = ((z[0] * z[0]) * aS[0] + (z[1] * z[1]) * aS[1]) + (z[2] * z[2]) * aS[2];
      float bRR = sqrtf(sr * (1.0f / 3.0f));
      float bS = sqrtf(ss * (1.0f / 3.0f));
      if (bRR < 1.0f) lam = bRR;
      else if (bS > 1.0f) lam = bS;
      else lam = 1.0f;
      lam = fminf(fmaxf(lam, p->clamp_lo), p->clamp_hi);
    }
    for (int t = 0; t < 3; ++t) {
      if (!enabled[t]) beta[t] = 0.0f;
      else if (aRR[0] < 0.0f) beta[t] = cb[t]; /* no data yet: classic */
      else beta[t] = (float)r[t] * lam;
    }
    return;
  }
  int ntech = o->nlp == 3 ? 5 : 3;
  for (int t = 0; t < ntech; ++t) {
    float b;
    int tc = t < 3 ? t : 2;   /* the light-path classes share the light-path rules */
    if (!enabled[tc]) { beta[t] = 0.0f; continue; }
    if (p->alloc == ORC_ALLOC_CLASSIC) {
      b = cb[tc];
      beta[t] = b;
      continue;
    }
    if (p->alloc == ORC_ALLOC_FIXED) {
      int32_t idx = o->nfixed > 1 ? (int32_t)cell : 0;
      b = o->fixed_beta[idx * 3 + tc];
      if (p->fixed_scale) {
        float s = ((z[0] * z[0] + z[1] * z[1]) + z[2] * z[2]) * (1.0f / 3.0f);
        b = b * sqrtf(s);
      }
    } else if (t < 3) {
      b = resolve_beta(o->fac + ((cell * 2 + 0) * 3 + t) * 3, o->fac + ((cell * 2 + 1) * 3 + t) * 3,
                       z, cb[t]);
    } else {
      b = resolve_beta(o->fac_x + ((cell * 2 + 0) * 2 + (t - 3)) * 3,
                       o->fac_x + ((cell * 2 + 1) * 2 + (t - 3)) * 3, z, cb[2]);
    }
    beta[t] = fminf(fmaxf(b, p->clamp_lo), p->clamp_hi);
  }
}

/* counts a vertex in `cell` with prefix throughput T and pixel estimate It
 * would draw (exported for the fixed-point pin tests) */
void orc_cell_beta(const oracle* o, const orc_iter_params* p, uint32_t cell, const float T[3],
                   const float It[3], int32_t depth, float beta[3]) {
  tctx c;
  memset(&c, 0, sizeof(c));
  c.o = o; c.p = p;
  c.It[0] = It[0]; c.It[1] = It[1]; c.It[2] = It[2];
  float b5[5];
  vertex_beta(&c, cell, mk(T[0], T[1], T[2]), depth, b5);
  beta[0] = b5[0]; beta[1] = b5[1]; beta[2] = b5[2];
}

/* ------------------------------------------------------------------------ */
/* the unidirectional recursion (Sec. 3.1 "Random walks", "Secondary       */
/* estimator"): <L_r> = sum_t (1/beta_t) sum_s <L_r,t>, each primary sample */
/* <L_r,t> = L_i B |cos| / p_t * w_t with L_i split into the direct part   */
/* (emission, MIS over {B,N,G}) and the indirect part (MIS over {B,G}).    */
/* ------------------------------------------------------------------------ */
typedef struct { float bt_pt, dsum, betaN; int camera; } parent_mis;
typedef struct { v3 E, Ew, R; uint32_t cost; int hit; } trace_out;

static v3 stat_clamp_v(const tctx* c, v3 v, v3 T) {
  if (!(c->p->stat_clamp > 0.0f)) return v;
  float k = c->p->stat_clamp;
  return mk(fminf(v.x, (k * c->It[0]) / T.x), fminf(v.y, (k * c->It[1]) / T.y),
            fminf(v.z, (k * c->It[2]) / T.z));
}

/* sample records of a vertex at `depth` are logged unless a test limits
 * them to shallower vertices */
static void log_sample(const tctx* c, int depth, stat_rec s) {
  if (c->o->rec_depth > 0 && depth > c->o->rec_depth) return;
  log_push(c->L, s);
}

static trace_out trace_pt(tctx* c, v3 org, v3 dir, v3 T, int depth, stream_t strm, parent_mis pm) {
  const oracle* o = c->o;
  const orc_iter_params* p = c->p;
  trace_out out;
  memset(&out, 0, sizeof(out));
  float t;
  uint32_t prim;
  if (!closest_hit(o, org, dir, INFINITY, &t, &prim)) return out;
  out.hit = 1;
  const float* m = o->mats + 8 * o->tmat[prim];
  v3 ngeo = o->ng[prim];
  v3 x = mk(org.x + t * dir.x, org.y + t * dir.y, org.z + t * dir.z);
  /* emission (one-sided) and its direct-light MIS weight */
  float cosl = -vdot(dir, ngeo);
  if (cosl > 0.0f && (m[5] > 0.0f || m[6] > 0.0f || m[7] > 0.0f)) {
    out.E = mk(m[5], m[6], m[7]);
    if (pm.camera) {
      out.Ew = out.E;
    } else {
      float pN = (o->lpdf[prim] * (t * t)) / cosl;
      float w = pm.bt_pt / (pm.dsum + pm.betaN * pN);
      out.Ew = mk(w * out.E.x, w * out.E.y, w * out.E.z);
    }
  }
  if (depth >= o->cfg.max_depth) return out;
  /* vertex */
  v3 n = vdot(ngeo, dir) < 0.0f ? ngeo : mk(-ngeo.x, -ngeo.y, -ngeo.z);
  v3 wo = mk(-dir.x, -dir.y, -dir.z);
  v3 ov = mk(x.x + n.x * o->eps, x.y + n.y * o->eps, x.z + n.z * o->eps);
  uint32_t cdepth;
  uint32_t cell = octree_lookup(o, x, &cdepth);
  float beta[5];
  vertex_beta(c, cell, T, depth, beta);
  float ur[4];
  draw4(c->key, strm, 0, ur);
  uint32_t gam[3];
  round_vertex(p, beta, ur, gam, 3);
  c->L->vertices++;
  { stat_rec s = {REC_VISIT, cell, 0, 0, {0, 0, 0}, 0, 0}; log_push(c->L, s); }
  if (depth == 1) {
    float* b1 = o->beta1 + 3 * (size_t)c->root;
    b1[0] = beta[0]; b1[1] = beta[1]; b1[2] = beta[2];
  }
  if (depth <= p->debug_depth) {
    orc_vertex_rec d;
    d.root = c->root; d.depth = depth; d.stream_lo = strm.lo; d.stream_hi = strm.hi; d.cell = cell;
    for (int k = 0; k < 3; ++k) { d.beta[k] = beta[k]; d.gamma[k] = gam[k]; }
    d.beta_x[0] = d.beta_x[1] = 0.0f; d.gamma_x[0] = d.gamma_x[1] = 0u;
    d.T[0] = T.x; d.T[1] = T.y; d.T[2] = T.z;
    dbg_push(c->L, d);
  }
  const float* pmf = o->pm + 64 * (size_t)cell;
  const float* cdf = o->cdf + 64 * (size_t)cell;
  int guided = o->cfg.mode == ORC_MODE_PT_GUIDED;
  v3 R = mk(0, 0, 0);
  uint32_t cost = 0;
  /* NEE samples (technique N) */
  for (uint32_t k = 0; k < gam[1]; ++k) {
    stream_t ss = child_stream(c->key, strm, ORC_TECH_N, k, depth);
    float u[4];
    draw4(c->key, ss, 1, u);
    c->L->samples++;
    int li = 0;
    while (li < o->nlights - 1 && !(u[0] < o->light_cdf[li])) ++li;
    int32_t lt = o->light_tri[li];
    float su = sqrtf(u[1]);
    float a = su * (1.0f - u[2]), b = su * u[2];
    v3 y = mk((o->v0[lt].x + a * o->e1[lt].x) + b * o->e2[lt].x,
              (o->v0[lt].y + a * o->e1[lt].y) + b * o->e2[lt].y,
              (o->v0[lt].z + a * o->e1[lt].z) + b * o->e2[lt].z);
    v3 dv = vsub(y, ov);
    float d2 = vdot(dv, dv);
    float dist = sqrtf(d2);
    v3 w = vscale(dv, 1.0f / dist);
    float cl = -vdot(w, o->ng[lt]);
    v3 fc;
    float pB;
    bsdf_eval(m, n, wo, w, &fc, &pB);
    v3 v = mk(0, 0, 0);
    if (cl > 0.0f && (fc.x > 0.0f || fc.y > 0.0f || fc.z > 0.0f)) {
      float pN = (o->lpdf[lt] * d2) / cl;
      float pG = guided ? guided_pdf(pmf, w) : 0.0f;
      float pr[3] = {pB, pN, pG}, wd[3], wi[3];
      orc_mis(p->budget_aware, beta, pr, wd, wi);
      c->L->rays_shadow++;
      if (!occluded(o, ov, w, dist * (1.0f - 1e-3f))) {
        const float* Le = o->mats + 8 * o->tmat[lt] + 5;
        v = mk((fc.x / pN) * (wd[1] * Le[0]), (fc.y / pN) * (wd[1] * Le[1]),
               (fc.z / pN) * (wd[1] * Le[2]));
      }
    }
    R = mk(R.x + v.x / beta[1], R.y + v.y / beta[1], R.z + v.z / beta[1]);
    cost += 1;
    v3 vs = stat_clamp_v(c, v, T);
    stat_rec s = {REC_SAMPLE, cell, ORC_TECH_N, 0, {vs.x, vs.y, vs.z}, 1, 0};
    log_sample(c, depth, s);
  }
  /* continuation samples: BSDF (technique B) then guided (technique G) */
  for (int tech = 0; tech < 3; tech += 2) {
    for (uint32_t k = 0; k < gam[tech]; ++k) {
      stream_t ss = child_stream(c->key, strm, (uint32_t)tech, k, depth);
      float u[4];
      draw4(c->key, ss, 1, u);
      c->L->samples++;
      v3 w;
      int ok;
      if (tech == 0) ok = bsdf_sample(m, n, wo, u[0], u[1], &w);
      else {
        w = guided_sample(cdf, u[0], u[1], u[2]);
        ok = vdot(n, w) > 0.0f;
      }
      v3 fc = mk(0, 0, 0);
      float pB = 0.0f, pG = 0.0f;
      if (ok) {
        bsdf_eval(m, n, wo, w, &fc, &pB);
        pG = guided ? guided_pdf(pmf, w) : 0.0f;
        float pt = tech == 0 ? pB : pG;
        ok = (fc.x > 0.0f || fc.y > 0.0f || fc.z > 0.0f) && pt > 0.0f;
      }
      v3 v = mk(0, 0, 0);
      uint32_t scost = 1;
      if (ok) {
        float pr[3] = {pB, 0.0f, pG}, wd[3], wi[3];
        (void)wd;
        orc_mis(p->budget_aware, beta, pr, wd, wi);
        float bB = p->budget_aware ? beta[0] : (beta[0] > 0.0f ? 1.0f : 0.0f);
        float bG = p->budget_aware ? beta[2] : (beta[2] > 0.0f ? 1.0f : 0.0f);
        float bN = p->budget_aware ? beta[1] : (beta[1] > 0.0f ? 1.0f : 0.0f);
        float dsum = bB * pB + bG * pG;
        float pt = tech == 0 ? pB : pG;
        /* throughput of the child prefix: T B|cos| / p_t * w_ind,t / beta_t (Sec. 3.1) */
        float wind = wi[tech];
        float g0 = ((fc.x / pt) * wind) / beta[tech];
        float g1 = ((fc.y / pt) * wind) / beta[tech];
        float g2 = ((fc.z / pt) * wind) / beta[tech];
        v3 Tc = mk(T.x * g0, T.y * g1, T.z * g2);
        parent_mis cm = {(tech == 0 ? bB : bG) * pt, dsum, bN, 0};
        c->L->rays_ext++;
        trace_out ch = trace_pt(c, ov, w, Tc, depth + 1, ss, cm);
        v = mk((fc.x / pt) * (ch.Ew.x + wind * ch.R.x), (fc.y / pt) * (ch.Ew.y + wind * ch.R.y),
               (fc.z / pt) * (ch.Ew.z + wind * ch.R.z));
        scost = 1 + ch.cost;
        if (guided && dsum > 0.0f) {
          v3 Li = vadd(ch.E, ch.R);
          stat_rec hs = {REC_HIST, cell, 0, (uint32_t)guided_bin(w), {0, 0, 0}, 0,
                         lum3(Li) / dsum};
          log_push(c->L, hs);
        }
      }
      R = mk(R.x + v.x / beta[tech], R.y + v.y / beta[tech], R.z + v.z / beta[tech]);
      cost += scost;
      v3 vs = stat_clamp_v(c, v, T);
      stat_rec s = {REC_SAMPLE, cell, (uint32_t)tech, 0, {vs.x, vs.y, vs.z}, scost, 0};
      log_sample(c, depth, s);
    }
  }
  out.R = R;
  out.cost = cost;
  return out;
}

/* bidirectional variant (Sec. 5): defined further below */
typedef struct lightpath lightpath;
static void bdpt_root(tctx* c, v3* I);
static void build_light_paths(oracle* o, const orc_iter_params* p, key_t2 key, rowlog* logs);

/* ------------------------------------------------------------------------ */
/* one rendering iteration over all pixels (Sec. 4.1 "Fixed-point          */
/* iteration": each iteration renders with the current counts and collects */
/* the estimates for the next update)                                       */
/* ------------------------------------------------------------------------ */
int32_t orc_render_iteration(oracle* o, const orc_iter_params* p, orc_iter_stats* st) {
  if (!o || !p || p->spp <= 0) return -1;
  if (p->alloc == ORC_ALLOC_FIXED && !o->fixed_beta) return -2;
  /* per-length light-path budgets: Alg. 1 rounding over the five counts and
   * per-technique fixed points only (no EARS line, no per-count uniforms) */
  if (o->nlp == 3 && (p->alloc == ORC_ALLOC_EARS || p->rounding)) return -3;
  int32_t W = o->W, H = o->H, spp = p->spp;
  size_t nroots = (size_t)W * H * spp;
  if (o->spp_last != spp) {
    free(o->Ls);
    free(o->beta1);
    o->Ls = calloc(nroots * 3, sizeof(float));
    o->beta1 = calloc(nroots * 3, sizeof(float));
    o->spp_last = spp;
  }
  memset(o->beta1, 0, nroots * 3 * sizeof(float));
  memset(o->Ls, 0, nroots * 3 * sizeof(float));
  memset(o->visits, 0, sizeof(uint32_t) * o->ncells);
  memset(o->acc, 0, sizeof(double) * 24 * o->ncells);
  if (o->acc_x) memset(o->acc_x, 0, sizeof(double) * 16 * o->ncells);
  memset(o->hacc, 0, sizeof(double) * 64 * o->ncells);
  rowlog* logs = calloc(H, sizeof(rowlog));
  key_t2 key = {(uint32_t)o->cfg.seed, (uint32_t)(o->cfg.seed >> 32)};
  int bdpt = o->cfg.mode == ORC_MODE_BDPT;
  if (bdpt) build_light_paths(o, p, key, logs);
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t py = 0; py < H; ++py) {
    tctx c;
    c.o = o; c.p = p; c.key = key; c.L = &logs[py];
    for (int32_t px = 0; px < W; ++px) {
      uint32_t pix = (uint32_t)(py * W + px);
      if (o->pix_mask && !o->pix_mask[pix]) continue;
      c.pix = pix;
      c.It[0] = o->Itilde[3 * pix]; c.It[1] = o->Itilde[3 * pix + 1]; c.It[2] = o->Itilde[3 * pix + 2];
      for (int32_t s = 0; s < spp; ++s) {
        uint32_t root = pix * (uint32_t)spp + (uint32_t)s;
        c.root = root;
        v3 I;
        if (bdpt) {
          bdpt_root(&c, &I);
        } else {
          stream_t rs = root_stream(key, pix, (uint32_t)s, (uint32_t)p->iteration, TAG_CAM);
          float u[4];
          draw4(key, rs, 1, u);
          float jx = p->center_jitter ? 0.5f : u[0], jy = p->center_jitter ? 0.5f : u[1];
          v3 org, dir;
          camera_ray(o, px, py, jx, jy, &org, &dir);
          parent_mis cm = {0, 0, 0, 1};
          trace_out r = trace_pt(&c, org, dir, mk(1.0f, 1.0f, 1.0f), 1, rs, cm);
          I = mk(r.Ew.x + r.R.x, r.Ew.y + r.R.y, r.Ew.z + r.R.z);
        }
        float* dst = o->Ls + 3 * (size_t)root;
        dst[0] = I.x; dst[1] = I.y; dst[2] = I.z;
      }
    }
  }
  /* merge logs in row order */
  orc_iter_stats S;
  memset(&S, 0, sizeof(S));
  S.rays_camera = nroots;
  free(o->dbg);
  o->dbg = NULL;
  o->ndbg = 0;
  size_t ndbg = 0;
  for (int32_t y = 0; y < H; ++y) ndbg += logs[y].nd;
  if (ndbg) o->dbg = malloc(ndbg * sizeof(orc_vertex_rec));
  for (int32_t y = 0; y < H; ++y) {
    rowlog* L = &logs[y];
    for (size_t i = 0; i < L->n; ++i) {
      const stat_rec* r = &L->r[i];
      if (r->kind == REC_VISIT) {
        o->visits[r->cell]++;
      } else if (r->kind == REC_SAMPLE) {
        double* a = r->tech < 3 ? o->acc + ((size_t)r->cell * 3 + r->tech) * 8
                                : o->acc_x + ((size_t)r->cell * 2 + (r->tech - 3)) * 8;
        for (int ch = 0; ch < 3; ++ch) {
          a[ch] += (double)r->v[ch];
          a[3 + ch] += (double)r->v[ch] * (double)r->v[ch];
        }
        a[6] += 1.0;
        a[7] += (double)r->cost;
      } else {
        o->hacc[(size_t)r->cell * 64 + r->bin] += (double)r->w;
      }
    }
    if (L->nd) memcpy(o->dbg + o->ndbg, L->d, L->nd * sizeof(orc_vertex_rec));
    o->ndbg += (int32_t)L->nd;
    S.rays_ext += L->rays_ext; S.rays_shadow += L->rays_shadow; S.rays_light += L->rays_light;
    S.rays_conn += L->rays_conn; S.vertices += L->vertices; S.samples += L->samples;
    free(L->r);
    free(L->d);
  }
  free(logs);
  /* per-pixel sum over the iteration's samples, in sample order */
  for (int32_t i = 0; i < W * H; ++i) {
    float sr = 0, sg = 0, sb = 0;
    float br = 0, bg = 0, bb = 0;
    for (int32_t s = 0; s < spp; ++s) {
      const float* l = o->Ls + 3 * ((size_t)i * spp + s);
      sr += l[0]; sg += l[1]; sb += l[2];
      const float* b = o->beta1 + 3 * ((size_t)i * spp + s);
      br += b[0]; bg += b[1]; bb += b[2];
    }
    o->iter_sum[3 * i] = sr; o->iter_sum[3 * i + 1] = sg; o->iter_sum[3 * i + 2] = sb;
    o->count_map[3 * i] = br / (float)spp;
    o->count_map[3 * i + 1] = bg / (float)spp;
    o->count_map[3 * i + 2] = bb / (float)spp;
  }
  o->rays_last = S.rays_camera + S.rays_ext + S.rays_shadow + S.rays_light + S.rays_conn;
  if (st) *st = S;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* fixed-point update per cell and technique (Sec. 3.1 "Optimization";      */
/* supplement A.3).  Moments are those of the primary estimator <L_r,t>     */
/* (Sec. 4.1 "Local estimates"); cost = mean rays per sample.  Cells whose */
/* technique has no sample keep their previous factors.                    */
/* ------------------------------------------------------------------------ */
int32_t orc_update_cells_only(oracle* o, double V_I, double C_I) {
  if (!(V_I > 0.0) || !(C_I > 0.0)) return 0;
  for (int32_t cidx = 0; cidx < o->ncells; ++cidx) {
    for (int t = 0; t < 3; ++t) {
      const double* a = o->acc + ((size_t)cidx * 3 + t) * 8;
      double n = a[6];
      if (!(n > 0.0)) continue;
      double Ct = a[7] / n;
      if (!(Ct > 0.0)) continue;
      double k = C_I / (Ct * V_I);
      for (int ch = 0; ch < 3; ++ch) {
        double E1 = a[ch] / n, E2 = a[3 + ch] / n;
        double var = E2 - E1 * E1;
        if (var < 0.0) var = 0.0;
        o->fac[((cidx * 2 + 0) * 3 + t) * 3 + ch] = (float)(k * E2);
        o->fac[((cidx * 2 + 1) * 3 + t) * 3 + ch] = (float)(k * var);
      }
    }
    /* per-length light paths: techniques 3 and 4, the same update */
    for (int x = 0; o->nlp == 3 && x < 2; ++x) {
      const double* a = o->acc_x + ((size_t)cidx * 2 + x) * 8;
      double n = a[6];
      if (!(n > 0.0)) continue;
      double Ct = a[7] / n;
      if (!(Ct > 0.0)) continue;
      double k = C_I / (Ct * V_I);
      for (int ch = 0; ch < 3; ++ch) {
        double E1 = a[ch] / n, E2 = a[3 + ch] / n;
        double var = E2 - E1 * E1;
        if (var < 0.0) var = 0.0;
        o->fac_x[((cidx * 2 + 0) * 2 + x) * 3 + ch] = (float)(k * E2);
        o->fac_x[((cidx * 2 + 1) * 2 + x) * 3 + ch] = (float)(k * var);
      }
    }
    if (o->ears_update) {
      /* the shared EARS factors of the cell, into technique slot 0 */
      double r[3], num[2][3] = {{0, 0, 0}, {0, 0, 0}}, den = 0.0;
      int any = 0;
      ears_ratios(o->cfg.mode, r);
      for (int t = 0; t < 3; ++t) {
        const double* a = o->acc + ((size_t)cidx * 3 + t) * 8;
        double n = a[6];
        if (!(r[t] > 0.0) || !(n > 0.0)) continue;
        double Ct = a[7] / n;
        if (!(Ct > 0.0)) continue;
        any = 1;
        den = den + r[t] * Ct;
        for (int ch = 0; ch < 3; ++ch) {
          double E1 = a[ch] / n, E2 = a[3 + ch] / n;
          double var = E2 - E1 * E1;
          if (var < 0.0) var = 0.0;
          num[0][ch] = num[0][ch] + E2 / r[t];
          num[1][ch] = num[1][ch] + var / r[t];
        }
      }
      if (any) {
        double k = C_I / V_I;
        for (int ch = 0; ch < 3; ++ch) {
          o->fac[((cidx * 2 + 0) * 3 + 0) * 3 + ch] = (float)(k * (num[0][ch] / den));
          o->fac[((cidx * 2 + 1) * 3 + 0) * 3 + ch] = (float)(k * (num[1][ch] / den));
        }
      }
    }
  }
  return 1;
}

int32_t orc_update_cells_ears(oracle* o, double V_I, double C_I) {
  o->ears_update = 1;
  int32_t r = orc_update_cells_only(o, V_I, C_I);
  o->ears_update = 0;
  return r;
}

/* learned directional distribution of the next iteration: 0.9 learned +  */
/* 0.1 uniform; cells without training data keep their distribution        */
static void hist_normalize(oracle* o) {
  for (int32_t cidx = 0; cidx < o->ncells; ++cidx) {
    const double* h = o->hacc + 64 * (size_t)cidx;
    double tot = 0.0;
    for (int b = 0; b < 64; ++b) tot += h[b];
    if (!(tot > 0.0)) continue;
    double run = 0.0;
    for (int b = 0; b < 64; ++b) {
      double pmb = 0.9 * (h[b] / tot) + 0.1 / 64.0;
      run += pmb;
      o->pm[64 * (size_t)cidx + b] = (float)pmb;
      o->cdf[64 * (size_t)cidx + b] = (b == 63) ? 1.0f : (float)run;
    }
  }
}

/* refinement: leaves with more than split_visits visits and depth below   */
/* the maximum are split, in increasing leaf order, while the leaf budget  */
/* allows; child 0 keeps the leaf id, children 1..7 get new ids; children  */
/* inherit factors and the directional distribution.                       */
int32_t orc_refine_only(oracle* o) {
  int32_t n0 = o->ncells, nn0 = o->nnodes, r = 0;
  for (int32_t l = 0; l < n0; ++l) {
    if (!(o->visits[l] > (uint32_t)o->cfg.split_visits)) continue;
    if (!(o->leaf_depth[l] < (uint32_t)o->cfg.max_tree_depth)) continue;
    if (n0 + 7 * (r + 1) > o->maxc) continue;
    uint32_t node = o->leaf_node[l];
    uint32_t base = (uint32_t)(nn0 + 8 * r);
    uint32_t child_depth = o->leaf_depth[l] + 1; /* all eight children sit one level below */
    o->nodes[node] = base;
    for (int ch = 0; ch < 8; ++ch) {
      uint32_t id = ch == 0 ? (uint32_t)l : (uint32_t)(n0 + 7 * r + (ch - 1));
      o->nodes[base + ch] = LEAF_BIT | id;
      o->leaf_node[id] = base + ch;
      o->leaf_depth[id] = child_depth;
      if (ch) {
        memcpy(o->fac + 18 * (size_t)id, o->fac + 18 * (size_t)l, 18 * sizeof(float));
        if (o->fac_x)
          memcpy(o->fac_x + 12 * (size_t)id, o->fac_x + 12 * (size_t)l, 12 * sizeof(float));
        memcpy(o->pm + 64 * (size_t)id, o->pm + 64 * (size_t)l, 64 * sizeof(float));
        memcpy(o->cdf + 64 * (size_t)id, o->cdf + 64 * (size_t)l, 64 * sizeof(float));
      }
    }
    ++r;
  }
  o->ncells = n0 + 7 * r;
  o->nnodes = nn0 + 8 * r;
  return r;
}

/* ------------------------------------------------------------------------ */
/* image estimates (Sec. 4.1 "Image estimates"; Sec. 5.1 for BDPT)          */
/*  I~: 3x3 box filter (edge clamped) of the running mean image, floored at */
/*      1e-3 x the image-mean channel value (stand-in for the denoiser);    */
/*  V_I: mean over pixels of (1/spp) sum_s (1/3) sum_ch ((I_s - I~)/I~)^2,   */
/*      samples clamped to stat_clamp x I~ (guiding); BDPT drops the 10     */
/*      brightest pixels of the iteration; floored pixels are excluded;     */
/*  C_I: rays traced / (pixels x spp).                                       */
/* ------------------------------------------------------------------------ */
int32_t orc_update(oracle* o, const orc_iter_params* p, orc_update_stats* st) {
  int32_t W = o->W, H = o->H, npx = W * H, spp = o->spp_last;
  if (spp <= 0) return -1;
  for (int32_t i = 0; i < 3 * npx; ++i) o->accum[i] = o->accum[i] + o->iter_sum[i];
  o->total_spp += (double)spp;
  float* mean = malloc(sizeof(float) * 3 * npx);
  float tsp = (float)o->total_spp;
  double im[3] = {0, 0, 0};
  for (int32_t i = 0; i < npx; ++i)
    for (int ch = 0; ch < 3; ++ch) {
      mean[3 * i + ch] = o->accum[3 * i + ch] / tsp;
      im[ch] += (double)mean[3 * i + ch];
    }
  float flo[3];
  for (int ch = 0; ch < 3; ++ch) flo[ch] = fmaxf(1e-3f * (float)(im[ch] / (double)npx), 1e-6f);
  unsigned char* excl = calloc(npx, 1);
  for (int32_t y = 0; y < H; ++y)
    for (int32_t x = 0; x < W; ++x)
      for (int ch = 0; ch < 3; ++ch) {
        float s = 0.0f;
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            int yy = y + dy < 0 ? 0 : (y + dy >= H ? H - 1 : y + dy);
            int xx = x + dx < 0 ? 0 : (x + dx >= W ? W - 1 : x + dx);
            s += mean[3 * (yy * W + xx) + ch];
          }
        s = s / 9.0f;
        if (!(s > flo[ch])) {
          s = flo[ch];
          excl[y * W + x] = 1;
        }
        o->Itilde[3 * (y * W + x) + ch] = s;
      }
  if (o->cfg.mode == ORC_MODE_BDPT) {
    /* drop the 10 brightest pixels (iteration mean luminance), ties -> lower index */
    for (int k = 0; k < 10 && k < npx; ++k) {
      int32_t best = -1;
      float bl = -1.0f;
      for (int32_t i = 0; i < npx; ++i) {
        if (excl[i] == 2) continue;
        float l = lum3(mk(o->iter_sum[3 * i], o->iter_sum[3 * i + 1], o->iter_sum[3 * i + 2]));
        if (l > bl) { bl = l; best = i; }
      }
      if (best >= 0) excl[best] = 2;
    }
  }
  double vsum = 0.0;
  int32_t nin = 0;
  float kc = p ? p->stat_clamp : 0.0f;
  for (int32_t i = 0; i < npx; ++i) {
    if (excl[i]) continue;
    const float* It = o->Itilde + 3 * i;
    double e = 0.0;
    for (int32_t s = 0; s < spp; ++s) {
      const float* l = o->Ls + 3 * ((size_t)i * spp + s);
      float d[3];
      for (int ch = 0; ch < 3; ++ch) {
        float xv = kc > 0.0f ? fminf(l[ch], kc * It[ch]) : l[ch];
        d[ch] = (xv - It[ch]) / It[ch];
      }
      e += (double)((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
    }
    vsum += e / (3.0 * (double)spp);
    ++nin;
  }
  double V_I = nin ? vsum / (double)nin : 0.0;
  double C_I = (double)o->rays_last / ((double)npx * (double)spp);
  int32_t nb = o->ncells;
  o->ears_update = p && p->alloc == ORC_ALLOC_EARS;
  orc_update_cells_only(o, V_I, C_I);
  o->ears_update = 0;
  if (o->cfg.mode == ORC_MODE_PT_GUIDED) hist_normalize(o);
  orc_refine_only(o);
  /* inverse-variance weighted combination of iterations (Sec. 5.1) */
  if (V_I > 0.0) {
    double w = (double)spp / V_I;
    for (int32_t i = 0; i < 3 * npx; ++i) o->ivw_acc[i] += w * (double)(o->iter_sum[i] / (float)spp);
    o->ivw_w += w;
  }
  if (st) {
    st->V_I = V_I;
    st->C_I = C_I;
    st->n_cells_before = nb;
    st->n_cells_after = o->ncells;
    st->n_excluded = npx - nin;
  }
  free(excl);
  free(mean);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* read-back / write-in                                                     */
/* ------------------------------------------------------------------------ */
int32_t orc_num_cells(const oracle* o) { return o->ncells; }
int32_t orc_num_nodes(const oracle* o) { return o->nnodes; }
void orc_read_nodes(const oracle* o, uint32_t* dst) {
  memcpy(dst, o->nodes, sizeof(uint32_t) * o->nnodes);
}
void orc_read_sample_radiance(const oracle* o, float* dst) {
  memcpy(dst, o->Ls, sizeof(float) * 3 * (size_t)o->W * o->H * o->spp_last);
}
void orc_read_image(const oracle* o, int32_t which, float* dst) {
  int32_t n = 3 * o->W * o->H;
  for (int32_t i = 0; i < n; ++i) {
    if (which == 0) dst[i] = o->total_spp > 0 ? o->accum[i] / (float)o->total_spp : 0.0f;
    else if (which == 1) dst[i] = o->ivw_w > 0 ? (float)(o->ivw_acc[i] / o->ivw_w) : 0.0f;
    else dst[i] = o->spp_last > 0 ? o->iter_sum[i] / (float)o->spp_last : 0.0f;
  }
}
void orc_read_Itilde(const oracle* o, float* dst) {
  memcpy(dst, o->Itilde, sizeof(float) * 3 * o->W * o->H);
}
void orc_read_count_map(const oracle* o, float* dst) {
  memcpy(dst, o->count_map, sizeof(float) * 3 * o->W * o->H);
}
void orc_read_cells(const oracle* o, float* factors, double* acc, uint32_t* visits,
                    uint32_t* leaf_depth) {
  if (factors) memcpy(factors, o->fac, sizeof(float) * 18 * o->ncells);
  if (acc) memcpy(acc, o->acc, sizeof(double) * 24 * o->ncells);
  if (visits) memcpy(visits, o->visits, sizeof(uint32_t) * o->ncells);
  if (leaf_depth) memcpy(leaf_depth, o->leaf_depth, sizeof(uint32_t) * o->ncells);
}
void orc_read_hist(const oracle* o, float* pm, float* cdf) {
  if (pm) memcpy(pm, o->pm, sizeof(float) * 64 * o->ncells);
  if (cdf) memcpy(cdf, o->cdf, sizeof(float) * 64 * o->ncells);
}
int32_t orc_read_debug(const oracle* o, orc_vertex_rec* dst, int32_t cap) {
  int32_t n = o->ndbg < cap ? o->ndbg : cap;
  if (dst && n) memcpy(dst, o->dbg, sizeof(orc_vertex_rec) * n);
  return o->ndbg;
}
void orc_write_cells(oracle* o, int32_t n, const float* factors, const double* acc,
                     const uint32_t* visits) {
  if (n > o->ncells) n = o->ncells;
  if (factors) memcpy(o->fac, factors, sizeof(float) * 18 * n);
  if (acc) memcpy(o->acc, acc, sizeof(double) * 24 * n);
  if (visits) memcpy(o->visits, visits, sizeof(uint32_t) * n);
}
void orc_set_pixel_subset(oracle* o, const int32_t* pix, int32_t n) {
  free(o->pix_mask);
  o->pix_mask = NULL;
  if (!pix || n <= 0) return;
  o->pix_mask = calloc((size_t)o->W * o->H, 1);
  for (int32_t i = 0; i < n; ++i)
    if (pix[i] >= 0 && pix[i] < o->W * o->H) o->pix_mask[pix[i]] = 1;
}
int32_t orc_lp_classes(const oracle* o) { return o->nlp; }
void orc_read_cells_x(const oracle* o, float* factors_x, double* acc_x) {
  if (!o->fac_x) return;
  if (factors_x) memcpy(factors_x, o->fac_x, sizeof(float) * 12 * o->ncells);
  if (acc_x) memcpy(acc_x, o->acc_x, sizeof(double) * 16 * o->ncells);
}
void orc_write_cells_x(oracle* o, int32_t n, const float* factors_x, const double* acc_x) {
  if (!o->fac_x) return;
  if (n > o->ncells) n = o->ncells;
  if (factors_x) memcpy(o->fac_x, factors_x, sizeof(float) * 12 * n);
  if (acc_x) memcpy(o->acc_x, acc_x, sizeof(double) * 16 * n);
}
void orc_set_Itilde(oracle* o, const float* src) {
  memcpy(o->Itilde, src, sizeof(float) * 3 * o->W * o->H);
}
void orc_set_record_depth(oracle* o, int32_t depth) { o->rec_depth = depth; }
void orc_set_fixed_beta(oracle* o, const float* beta, int32_t n) {
  free(o->fixed_beta);
  o->fixed_beta = malloc(sizeof(float) * 3 * (n > 0 ? n : 1));
  memcpy(o->fixed_beta, beta, sizeof(float) * 3 * n);
  o->nfixed = n;
}
void orc_set_hist(oracle* o, int32_t n, const float* pm, const float* cdf) {
  if (n > o->ncells) n = o->ncells;
  memcpy(o->pm, pm, sizeof(float) * 64 * n);
  memcpy(o->cdf, cdf, sizeof(float) * 64 * n);
}

/* ------------------------------------------------------------------------ */
/* Bidirectional path tracing (Sec. 5).  Techniques at every camera vertex: */
/* BSDF continuation, NEE, and light-path connections (LP), each with its   */
/* own count.  One light subpath per camera sample, throughput RR only     */
/* (Sec. 5: no splitting on the light side).  LP sample j connects to the  */
/* light subpath (root + j * stride) mod N and to every light vertex y_i,  */
/* i >= 1, with total path length <= D.  MIS: balance heuristic over the   */
/* strategies (s, t), t >= 2, of the full path; the budget-aware form     */
/* weights strategy (s, t) by the expected number of its samples,          */
/* n = prod_{j<=t-2} beta_B(z_j) * beta_tech(s)(z_{t-1}).  The weight is a  */
/* function of the path's vertices only: every vertex's counts (also those */
/* on the light side) come from the same formula with the throughput of    */
/* the camera prefix computed from vertex positions.                       */
/* ------------------------------------------------------------------------ */
#define BD_MAXK 34
typedef struct {
  v3 P, ng;
  const float* m;
  float lpdf;
} pvert;

struct lightpath {
  int len;            /* number of vertices y_1..y_len stored (y_0 separately) */
  int rays;           /* rays traced for this light subpath */
  pvert y0;
  pvert y[BD_MAXK];
  v3 wo[BD_MAXK];     /* direction from y_i towards y_{i-1} */
  v3 alpha[BD_MAXK];  /* light-subpath throughput arriving at y_i */
};

static inline v3 dir_between(v3 a, v3 b, float* d2) {
  v3 dv = vsub(b, a);
  *d2 = vdot(dv, dv);
  float dist = sqrtf(*d2);
  return vscale(dv, 1.0f / dist);
}

/* BSDF value and sampling density with the shading normal facing wo */
static void eval_facing(const float* m, v3 ng, v3 wo, v3 wi, v3* fc, float* pdf) {
  v3 n = vdot(ng, wo) > 0.0f ? ng : mk(-ng.x, -ng.y, -ng.z);
  bsdf_eval(m, n, wo, wi, fc, pdf);
}

/* counts of a vertex at depth `depth` used as camera vertex (room for five) */
static void counts_for(const tctx* c, v3 P, v3 T, int depth, float beta[5]) {
  uint32_t cell = octree_lookup(c->o, P, NULL);
  vertex_beta(c, cell, T, depth, beta);
}

/* Balance-heuristic weight of strategy t (t camera vertices z_0..z_{t-1})
 * for the path z[0] (camera), z[1..k] (z[k] on an emitter). */
static float bdpt_weight(const tctx* c, const pvert* z, int k, int t) {
  if (k <= 1) return 1.0f;
  float pF[BD_MAXK + 2], pR[BD_MAXK + 2], nB[BD_MAXK + 2], nN[BD_MAXK + 2];
  float nL[3][BD_MAXK + 2]; /* light-path counts; [1], [2] with per-length budgets */
  float d2;
  /* area densities of z_i sampled from the camera side (i >= 2) */
  for (int i = 2; i <= k; ++i) {
    v3 wo = dir_between(z[i - 1].P, z[i - 2].P, &d2);
    v3 wi = dir_between(z[i - 1].P, z[i].P, &d2);
    v3 fc;
    float p;
    eval_facing(z[i - 1].m, z[i - 1].ng, wo, wi, &fc, &p);
    pF[i] = (p * fabsf(vdot(z[i].ng, wi))) / d2;
  }
  /* area densities of z_i sampled from the light side */
  pR[k] = z[k].lpdf;
  {
    v3 w = dir_between(z[k].P, z[k - 1].P, &d2);
    float cl = vdot(z[k].ng, w);
    float pe = cl > 0.0f ? cl * INV_PI_F : 0.0f;
    pR[k - 1] = (pe * fabsf(vdot(z[k - 1].ng, w))) / d2;
  }
  for (int i = k - 2; i >= 1; --i) {
    v3 wo = dir_between(z[i + 1].P, z[i + 2].P, &d2);
    v3 wi = dir_between(z[i + 1].P, z[i].P, &d2);
    v3 fc;
    float p;
    eval_facing(z[i + 1].m, z[i + 1].ng, wo, wi, &fc, &p);
    pR[i] = (p * fabsf(vdot(z[i].ng, wi))) / d2;
  }
  /* counts of z_1..z_{k-1} as camera vertices, throughput from positions */
  v3 T = mk(1.0f, 1.0f, 1.0f);
  int aware = c->p->budget_aware;
  for (int i = 1; i <= k - 1; ++i) {
    float b[5];
    counts_for(c, z[i].P, T, i, b);
    nB[i] = aware ? b[0] : (b[0] > 0.0f ? 1.0f : 0.0f);
    nN[i] = aware ? b[1] : (b[1] > 0.0f ? 1.0f : 0.0f);
    for (int x = 0; x < 3; ++x) {
      float bl = b[x == 0 ? 2 : 2 + x];
      nL[x][i] = aware ? bl : (bl > 0.0f ? 1.0f : 0.0f);
    }
    if (i < k - 1) {
      v3 wo = dir_between(z[i].P, z[i - 1].P, &d2);
      v3 wi = dir_between(z[i].P, z[i + 1].P, &d2);
      v3 fc;
      float p;
      eval_facing(z[i].m, z[i].ng, wo, wi, &fc, &p);
      if (p > 0.0f && b[0] > 0.0f)
        T = mk(T.x * (((fc.x / p) * 1.0f) / b[0]), T.y * (((fc.y / p) * 1.0f) / b[0]),
               T.z * (((fc.z / p) * 1.0f) / b[0]));
      else
        T = mk(0.0f, 0.0f, 0.0f);
    }
  }
  /* strategy tt connects z_{tt-1} to z_tt = y_{k-tt}: the count of its
   * light-vertex class (one class unless per-length budgets) */
  const int nlp = c->o->nlp;
#define LCLS(i) (nlp == 3 ? ((i) < 3 ? (i) - 1 : 2) : 0)
#define TF(tt) ((tt) == k + 1 ? 1.0f : ((tt) == k ? nN[k - 1] : nL[LCLS(k - (tt))][(tt) - 1]))
  float tft = TF(t);
  if (!(tft > 0.0f)) return 0.0f;
  float sum = 1.0f, rp = 1.0f, rb = 1.0f;
  for (int tt = t + 1; tt <= k + 1; ++tt) {
    rp = rp * (pF[tt - 1] / pR[tt - 1]);
    rb = rb * nB[tt - 2];
    sum = sum + (rp * rb) * (TF(tt) / tft);
  }
  rp = 1.0f;
  rb = 1.0f;
  for (int tt = t - 1; tt >= 2; --tt) {
    rp = rp * (pR[tt] / pF[tt]);
    rb = rb * nB[tt - 1];
    sum = sum + rp * (TF(tt) / (rb * tft));
  }
#undef TF
#undef LCLS
  if (!(sum < INFINITY)) return 0.0f; /* also NaN */
  return 1.0f / sum;
}

/* light subpath of a camera sample: emission point by power, cosine
 * direction, then BSDF sampling with throughput RR q = min(1, max_ch prod
 * B|cos|/p); vertices y_1.. up to max_depth - 2 */
static void trace_light(const tctx* c, uint32_t pix, uint32_t s, lightpath* lp) {
  const oracle* o = c->o;
  lp->len = 0;
  lp->rays = 0;
  if (o->nlights == 0) return;
  stream_t st = root_stream(c->key, pix, s, (uint32_t)c->p->iteration, TAG_LIGHT);
  float u[4], u2[4];
  draw4(c->key, st, 0, u);
  draw4(c->key, st, 1, u2);
  int li = 0;
  while (li < o->nlights - 1 && !(u[0] < o->light_cdf[li])) ++li;
  int32_t lt = o->light_tri[li];
  float su = sqrtf(u[1]);
  float a = su * (1.0f - u[2]), b = su * u[2];
  v3 y0 = mk((o->v0[lt].x + a * o->e1[lt].x) + b * o->e2[lt].x,
             (o->v0[lt].y + a * o->e1[lt].y) + b * o->e2[lt].y,
             (o->v0[lt].z + a * o->e1[lt].z) + b * o->e2[lt].z);
  v3 nl = o->ng[lt];
  const float* ml = o->mats + 8 * o->tmat[lt];
  lp->y0.P = y0; lp->y0.ng = nl; lp->y0.m = ml; lp->y0.lpdf = o->lpdf[lt];
  int maxv = o->cfg.max_depth - 2;
  if (maxv <= 0) return;
  /* cosine-weighted emission direction about the emitting side */
  v3 tt, bb;
  onb(nl, &tt, &bb);
  float sn, cs;
  float r = sqrtf(u2[0]);
  orc_sincos2pi(u2[1], &sn, &cs);
  v3 w = to_world(mk(r * cs, r * sn, sqrtf(fmaxf(0.0f, 1.0f - u2[0]))), tt, bb, nl);
  v3 alpha = mk((ml[5] * PI_F) / lp->y0.lpdf, (ml[6] * PI_F) / lp->y0.lpdf,
                (ml[7] * PI_F) / lp->y0.lpdf);
  v3 org = mk(y0.x + nl.x * o->eps, y0.y + nl.y * o->eps, y0.z + nl.z * o->eps);
  v3 rr = mk(1.0f, 1.0f, 1.0f);
  for (int i = 1; i <= maxv; ++i) {
    float t;
    uint32_t prim;
    lp->rays++;
    if (!closest_hit(o, org, w, INFINITY, &t, &prim)) return;
    v3 x = mk(org.x + t * w.x, org.y + t * w.y, org.z + t * w.z);
    pvert* y = &lp->y[i - 1];
    y->P = x; y->ng = o->ng[prim]; y->m = o->mats + 8 * o->tmat[prim]; y->lpdf = o->lpdf[prim];
    v3 wo = mk(-w.x, -w.y, -w.z);
    lp->wo[i - 1] = wo;
    lp->alpha[i - 1] = alpha;
    lp->len = i;
    if (i == maxv) return;
    float uu[4];
    draw4(c->key, st, (uint32_t)(1 + i), uu);
    float q = fminf(1.0f, maxc3(rr));
    if (!(uu[0] < q)) return;
    v3 n = vdot(y->ng, wo) > 0.0f ? y->ng : mk(-y->ng.x, -y->ng.y, -y->ng.z);
    v3 wn;
    if (!bsdf_sample(y->m, n, wo, uu[1], uu[2], &wn)) return;
    v3 fc;
    float p;
    bsdf_eval(y->m, n, wo, wn, &fc, &p);
    if (!(p > 0.0f) || !(fc.x > 0.0f || fc.y > 0.0f || fc.z > 0.0f)) return;
    alpha = mk(alpha.x * ((fc.x / p) / q), alpha.y * ((fc.y / p) / q), alpha.z * ((fc.z / p) / q));
    rr = mk(rr.x * (fc.x / p), rr.y * (fc.y / p), rr.z * (fc.z / p));
    org = mk(x.x + n.x * o->eps, x.y + n.y * o->eps, x.z + n.z * o->eps);
    w = wn;
  }
}

/* camera-side recursion of BDPT: z[1..depth-1] is the prefix, z[0] the camera */
static trace_out trace_bdpt(tctx* c, v3 org, v3 dir, v3 T, int depth, stream_t strm, pvert* z) {
  const oracle* o = c->o;
  const orc_iter_params* p = c->p;
  trace_out out;
  memset(&out, 0, sizeof(out));
  float t;
  uint32_t prim;
  if (!closest_hit(o, org, dir, INFINITY, &t, &prim)) return out;
  out.hit = 1;
  const float* m = o->mats + 8 * o->tmat[prim];
  v3 ngeo = o->ng[prim];
  v3 x = mk(org.x + t * dir.x, org.y + t * dir.y, org.z + t * dir.z);
  z[depth].P = x; z[depth].ng = ngeo; z[depth].m = m; z[depth].lpdf = o->lpdf[prim];
  float cosl = -vdot(dir, ngeo);
  if (cosl > 0.0f && (m[5] > 0.0f || m[6] > 0.0f || m[7] > 0.0f)) {
    out.E = mk(m[5], m[6], m[7]);
    float w = depth == 1 ? 1.0f : bdpt_weight(c, z, depth, depth + 1);
    out.Ew = mk(w * out.E.x, w * out.E.y, w * out.E.z);
  }
  if (depth >= o->cfg.max_depth) return out;
  v3 n = vdot(ngeo, dir) < 0.0f ? ngeo : mk(-ngeo.x, -ngeo.y, -ngeo.z);
  v3 wo = mk(-dir.x, -dir.y, -dir.z);
  v3 ov = mk(x.x + n.x * o->eps, x.y + n.y * o->eps, x.z + n.z * o->eps);
  uint32_t cell = octree_lookup(o, x, NULL);
  float beta[5];
  vertex_beta(c, cell, T, depth, beta);
  float ur[4];
  draw4(c->key, strm, 0, ur);
  uint32_t gam[5] = {0, 0, 0, 0, 0};
  round_vertex(p, beta, ur, gam, 2 + o->nlp);
  c->L->vertices++;
  { stat_rec s = {REC_VISIT, cell, 0, 0, {0, 0, 0}, 0, 0}; log_push(c->L, s); }
  if (depth == 1) {
    float* b1 = o->beta1 + 3 * (size_t)c->root;
    /* per-length light paths: the light-path count is the sum over lengths */
    b1[0] = beta[0]; b1[1] = beta[1]; b1[2] = o->nlp == 3 ? (beta[2] + beta[3]) + beta[4] : beta[2];
  }
  if (depth <= p->debug_depth) {
    orc_vertex_rec d;
    d.root = c->root; d.depth = depth; d.stream_lo = strm.lo; d.stream_hi = strm.hi; d.cell = cell;
    for (int k = 0; k < 3; ++k) { d.beta[k] = beta[k]; d.gamma[k] = gam[k]; }
    d.beta_x[0] = beta[3]; d.beta_x[1] = beta[4]; d.gamma_x[0] = gam[3]; d.gamma_x[1] = gam[4];
    d.T[0] = T.x; d.T[1] = T.y; d.T[2] = T.z;
    dbg_push(c->L, d);
  }
  v3 R = mk(0, 0, 0);
  uint32_t cost = 0;
  /* NEE */
  for (uint32_t k = 0; k < gam[1]; ++k) {
    stream_t ss = child_stream(c->key, strm, ORC_TECH_N, k, depth);
    float u[4];
    draw4(c->key, ss, 1, u);
    c->L->samples++;
    int li = 0;
    while (li < o->nlights - 1 && !(u[0] < o->light_cdf[li])) ++li;
    int32_t lt = o->light_tri[li];
    float su = sqrtf(u[1]);
    float a = su * (1.0f - u[2]), b = su * u[2];
    v3 y = mk((o->v0[lt].x + a * o->e1[lt].x) + b * o->e2[lt].x,
              (o->v0[lt].y + a * o->e1[lt].y) + b * o->e2[lt].y,
              (o->v0[lt].z + a * o->e1[lt].z) + b * o->e2[lt].z);
    v3 dv = vsub(y, ov);
    float d2 = vdot(dv, dv);
    float dist = sqrtf(d2);
    v3 w = vscale(dv, 1.0f / dist);
    float cl = -vdot(w, o->ng[lt]);
    v3 fc;
    float pB;
    bsdf_eval(m, n, wo, w, &fc, &pB);
    v3 v = mk(0, 0, 0);
    if (cl > 0.0f && (fc.x > 0.0f || fc.y > 0.0f || fc.z > 0.0f)) {
      float pN = (o->lpdf[lt] * d2) / cl;
      z[depth + 1].P = y; z[depth + 1].ng = o->ng[lt]; z[depth + 1].m = o->mats + 8 * o->tmat[lt];
      z[depth + 1].lpdf = o->lpdf[lt];
      float wN = bdpt_weight(c, z, depth + 1, depth + 1);
      c->L->rays_shadow++;
      if (!occluded(o, ov, w, dist * (1.0f - 1e-3f))) {
        const float* Le = o->mats + 8 * o->tmat[lt] + 5;
        v = mk((fc.x / pN) * (wN * Le[0]), (fc.y / pN) * (wN * Le[1]), (fc.z / pN) * (wN * Le[2]));
      }
    }
    R = mk(R.x + v.x / beta[1], R.y + v.y / beta[1], R.z + v.z / beta[1]);
    cost += 1;
    stat_rec s = {REC_SAMPLE, cell, ORC_TECH_N, 0, {v.x, v.y, v.z}, 1, 0};
    log_sample(c, depth, s);
  }
  /* BSDF continuation */
  for (uint32_t k = 0; k < gam[0]; ++k) {
    stream_t ss = child_stream(c->key, strm, ORC_TECH_B, k, depth);
    float u[4];
    draw4(c->key, ss, 1, u);
    c->L->samples++;
    v3 w;
    int ok = bsdf_sample(m, n, wo, u[0], u[1], &w);
    v3 fc = mk(0, 0, 0);
    float pB = 0.0f;
    if (ok) {
      bsdf_eval(m, n, wo, w, &fc, &pB);
      ok = (fc.x > 0.0f || fc.y > 0.0f || fc.z > 0.0f) && pB > 0.0f;
    }
    v3 v = mk(0, 0, 0);
    uint32_t scost = 1;
    if (ok) {
      float c0 = fc.x / pB, c1 = fc.y / pB, c2 = fc.z / pB;
      v3 Tc = mk(T.x * ((c0 * 1.0f) / beta[0]), T.y * ((c1 * 1.0f) / beta[0]),
                 T.z * ((c2 * 1.0f) / beta[0]));
      c->L->rays_ext++;
      trace_out ch = trace_bdpt(c, ov, w, Tc, depth + 1, ss, z);
      v = mk(c0 * (ch.Ew.x + 1.0f * ch.R.x), c1 * (ch.Ew.y + 1.0f * ch.R.y),
             c2 * (ch.Ew.z + 1.0f * ch.R.z));
      scost = 1 + ch.cost;
    }
    R = mk(R.x + v.x / beta[0], R.y + v.y / beta[0], R.z + v.z / beta[0]);
    cost += scost;
    stat_rec s = {REC_SAMPLE, cell, ORC_TECH_B, 0, {v.x, v.y, v.z}, scost, 0};
    log_sample(c, depth, s);
  }
  /* light-path connections: one budget for every light vertex, or with
   * per-length budgets (Sec. 5, the variant named there as future work) a
   * class per light-vertex index: technique 2 connects to y_1, 3 to y_2,
   * 4 to y_3 and beyond.  Sample k of every class uses the same pool entry
   * sequence, so with all class counts 1 the connections are those of one
   * light-path sample. */
  uint32_t npool = (uint32_t)(o->W * o->H * p->spp);
  for (int cls = 0; cls < o->nlp; ++cls) {
    const int tech = cls == 0 ? ORC_TECH_G : 2 + cls;
    const int ilo = o->nlp == 1 ? 1 : cls + 1;
    const int icap = (o->nlp == 1 || cls == 2) ? BD_MAXK : cls + 1;
    for (uint32_t k = 0; k < gam[tech]; ++k) {
      c->L->samples++;
      /* light subpath: pool entry (b + k stride) mod npool with b the first
       * word of this vertex's stream, so the vertices of one path tree use
       * unrelated light subpaths (their samples stay independent) */
      uint32_t lpi = (uint32_t)(((uint64_t)strm.lo + (uint64_t)k * (uint32_t)p->lp_stride) % npool);
      const lightpath* lp = &o->lpaths[lpi];
      v3 v = mk(0, 0, 0);
      /* cost of an LP sample: its connection rays (at least 1); the light
       * subpath is traced once per camera sample whatever the counts */
      uint32_t scost = 0;
      int imax = o->cfg.max_depth - depth - 1;
      if (imax > lp->len) imax = lp->len;
      if (imax > icap) imax = icap;
      for (int i = ilo; i <= imax; ++i) {
        const pvert* y = &lp->y[i - 1];
        float d2;
        v3 w = dir_between(x, y->P, &d2);
        v3 fcC, fcL;
        float pc, pl;
        bsdf_eval(m, n, wo, w, &fcC, &pc);
        eval_facing(y->m, y->ng, lp->wo[i - 1], mk(-w.x, -w.y, -w.z), &fcL, &pl);
        if (!(fcC.x > 0.0f || fcC.y > 0.0f || fcC.z > 0.0f)) continue;
        if (!(fcL.x > 0.0f || fcL.y > 0.0f || fcL.z > 0.0f)) continue;
        /* the full path: z_1..z_depth, y_i, .., y_1, y_0 */
        for (int j = 1; j <= i; ++j) z[depth + j] = lp->y[i - j];
        z[depth + i + 1] = lp->y0;
        float wc = bdpt_weight(c, z, depth + 1 + i, depth + 1);
        v3 a = lp->alpha[i - 1];
        v3 ny = vdot(y->ng, lp->wo[i - 1]) > 0.0f ? y->ng : mk(-y->ng.x, -y->ng.y, -y->ng.z);
        v3 yo = mk(y->P.x + ny.x * o->eps, y->P.y + ny.y * o->eps, y->P.z + ny.z * o->eps);
        float sd2;
        v3 sw = dir_between(ov, yo, &sd2);
        c->L->rays_conn++;
        scost += 1;
        if (!occluded(o, ov, sw, sqrtf(sd2) * (1.0f - 1e-3f))) {
          v = mk(v.x + wc * (((a.x * fcL.x) * fcC.x) / d2), v.y + wc * (((a.y * fcL.y) * fcC.y) / d2),
                 v.z + wc * (((a.z * fcL.z) * fcC.z) / d2));
        }
      }
      if (scost == 0) scost = 1;
      R = mk(R.x + v.x / beta[tech], R.y + v.y / beta[tech], R.z + v.z / beta[tech]);
      cost += scost;
      stat_rec s = {REC_SAMPLE, cell, (uint32_t)tech, 0, {v.x, v.y, v.z}, scost, 0};
      log_sample(c, depth, s);
    }
  }
  out.R = R;
  out.cost = cost;
  return out;
}

static void bdpt_root(tctx* c, v3* I) {
  const oracle* o = c->o;
  uint32_t pix = c->pix, s = c->root % (uint32_t)c->p->spp;
  stream_t rs = root_stream(c->key, pix, s, (uint32_t)c->p->iteration, TAG_CAM);
  float u[4];
  draw4(c->key, rs, 1, u);
  float jx = c->p->center_jitter ? 0.5f : u[0], jy = c->p->center_jitter ? 0.5f : u[1];
  v3 org, dir;
  camera_ray(o, (int32_t)(pix % (uint32_t)o->W), (int32_t)(pix / (uint32_t)o->W), jx, jy, &org, &dir);
  pvert z[2 * BD_MAXK + 4];
  memset(z, 0, sizeof(z));
  z[0].P = o->cam_o;
  z[0].ng = dir;
  trace_out r = trace_bdpt(c, org, dir, mk(1.0f, 1.0f, 1.0f), 1, rs, z);
  *I = mk(r.Ew.x + r.R.x, r.Ew.y + r.R.y, r.Ew.z + r.R.z);
}

static void build_light_paths(oracle* o, const orc_iter_params* p, key_t2 key, rowlog* logs) {
  size_t n = (size_t)o->W * o->H * p->spp;
  if (o->nlpaths < n) {
    free(o->lpaths);
    o->lpaths = calloc(n, sizeof(lightpath));
    o->nlpaths = n;
  }
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t r = 0; r < (int64_t)n; ++r) {
    tctx c;
    memset(&c, 0, sizeof(c));
    c.o = o; c.p = p; c.key = key;
    trace_light(&c, (uint32_t)(r / p->spp), (uint32_t)(r % p->spp), &o->lpaths[r]);
  }
  uint64_t rays = 0;
  for (size_t r = 0; r < n; ++r) rays += (uint64_t)o->lpaths[r].rays;
  logs[0].rays_light += rays;
}

/* weights of every strategy t = 2..k+1 of an explicit path (tests):
 * P [k+1][3] (camera position first), prims [k+1] (prims[0] unused),
 * It [3] pixel estimate; out [k] */
void orc_bdpt_weights(const oracle* o, const orc_iter_params* p, const float* P,
                      const uint32_t* prims, int32_t k, const float* It, float* out) {
  tctx c;
  memset(&c, 0, sizeof(c));
  c.o = o; c.p = p;
  c.It[0] = It[0]; c.It[1] = It[1]; c.It[2] = It[2];
  pvert z[BD_MAXK + 2];
  memset(z, 0, sizeof(z));
  for (int i = 0; i <= k; ++i) {
    z[i].P = mk(P[3 * i], P[3 * i + 1], P[3 * i + 2]);
    if (i > 0) {
      z[i].ng = o->ng[prims[i]];
      z[i].m = o->mats + 8 * o->tmat[prims[i]];
      z[i].lpdf = o->lpdf[prims[i]];
    }
  }
  for (int t = 2; t <= k + 1; ++t) out[t - 2] = bdpt_weight(&c, z, k, t);
}
