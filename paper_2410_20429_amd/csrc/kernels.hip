// Wavefront kernels of the MARS hot path for gfx950 (CDNA4).
//
// One iteration (Sec. 4.1 "Fixed-point iteration") is a sequence of
// per-depth stages over SoA queues:
//   raygen -> [trace_closest -> shade -> trace_any] x D -> backprop (D..1)
//   -> pixel sums
// and the update between iterations:
//   image estimates (I~, V_I) -> fixed-point factors -> guided distribution
//   -> octree refinement -> inverse-variance image.
// Splitting turns a camera path into a tree; every child sample is written
// to the next depth's queue at an offset from a wave-level prefix sum (one
// global atomic per wave), and the tree is reduced bottom-up afterwards by a
// pull over each vertex's contiguous child range, so per-pixel radiance does
// not depend on queue order.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <utility>

#include "device_math.hpp"
#include "mars_internal.h"

namespace mars {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(v, off, 64);
    if (lane >= off) v += o;
  }
  return v;
}
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// bidirectional vertex and connection kernels: 256-thread groups (one queue
// allocation per group; a connection group sorts one tile by walk length).
// A group's barriers wait for its slowest wave, so small groups keep the
// SIMDs busy: at four waves per SIMD a 1024-thread group held a whole CU.
constexpr int kShadeBlock = 256, kConnectBlock = 256;

// Launch grid of a kernel whose workgroups loop over equal shares of the
// work: exactly the groups the device holds at once (CUs x resident groups
// per CU at the kernel's register and LDS use), so that no group starts
// after the first ones finish and leaves the CUs half empty for its share.
template <class K>
int resident_grid(K* kernel, int block) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  const std::pair<const void*, int> key{(const void*)kernel, dev};
  std::lock_guard<std::mutex> lk(mu);
  auto f = cache.find(key);
  if (f != cache.end()) return f->second;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  return cache[key] = per_cu * cus;
}
// unidirectional shading: 256-thread groups held to 80 VGPRs (6 waves per
// SIMD) to hide its dependent loads (octree walk, distribution search)
constexpr int kShadePtBlock = 256;

// the overflow flag read once per workgroup, so that every thread of the
// group takes the same exit (the kernels below use workgroup barriers)
__device__ __forceinline__ bool group_overflowed(const Counters* cnt) {
  __shared__ uint32_t flag;
  if (threadIdx.x == 0) flag = cnt->overflow;
  __syncthreads();
  return flag != 0u;
}

// Workgroup-wide allocation in two queues: lane counts (a, b) -> the lane's
// first slot in each.  One atomic per queue per workgroup: device-scope
// atomics on one address serialise across the chip, so the fewer the better.
// lds: 2 * kThreads / 64 + 2 words.  Every thread of the group must call it.
template <int kThreads>
__device__ __forceinline__ void group_alloc(uint32_t a, uint32_t b, uint32_t* ca, uint32_t* cb,
                                            uint32_t* fa, uint32_t* fb, uint32_t* lds) {
  constexpr int kW = kThreads / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t ia = wave_scan_incl(a), ib = wave_scan_incl(b);
  if (lane == 63) {
    lds[wid] = ia;
    lds[kW + wid] = ib;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t sa = 0, sb = 0;
    for (int w = 0; w < kW; ++w) {
      const uint32_t x = lds[w], y = lds[kW + w];
      lds[w] = sa;
      lds[kW + w] = sb;
      sa += x;
      sb += y;
    }
    lds[2 * kW] = sa ? atomicAdd(ca, sa) : 0u;
    lds[2 * kW + 1] = sb ? atomicAdd(cb, sb) : 0u;
  }
  __syncthreads();
  *fa = lds[2 * kW] + lds[wid] + (ia - a);
  *fb = lds[2 * kW + 1] + lds[kW + wid] + (ib - b);
  __syncthreads();
}

// adds per-thread counts into N 64-bit counters, one atomic per counter per
// workgroup; lds: N * kThreads / 64 words.  Every thread must call it.
template <int kThreads, int N>
__device__ __forceinline__ void group_add(const uint32_t (&v)[N], unsigned long long* const (&dst)[N],
                                          uint32_t* lds) {
  constexpr int kW = kThreads / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const uint32_t s = wave_sum(v[i]);
    if (lane == 0) lds[i * kW + wid] = s;
  }
  __syncthreads();
  if ((int)threadIdx.x < N) {
    unsigned long long s = 0;
    for (int w = 0; w < kW; ++w) s += lds[threadIdx.x * kW + w];
    if (s) atomicAdd(dst[threadIdx.x], s);
  }
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ float fbits(uint32_t u) { return __uint_as_float(u); }
__device__ __forceinline__ uint32_t ubits(float f) { return __float_as_uint(f); }
__device__ __forceinline__ Mat load_mat(const float* m) {
  return Mat{m[0], m[1], m[2], m[3], m[4], m[5], m[6], m[7]};
}

template <typename T>
__global__ void fill_kernel(T* p, T v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}
void k_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s) {
  if (n) fill_kernel<uint32_t><<<(unsigned)std::min<size_t>((n + 255) / 256, 4096), 256, 0, s>>>(p, v, n);
}
void k_fill_f64(double* p, double v, size_t n, hipStream_t s) {
  if (n) fill_kernel<double><<<(unsigned)std::min<size_t>((n + 255) / 256, 4096), 256, 0, s>>>(p, v, n);
}
// Per-iteration clear in one launch: the moment and cost accumulators and
// visit counts of the cells in use (count read on the device), the guided
// training histograms when used, and the first-hit counts.
__global__ void clear_iteration_kernel(CacheDev c, const int32_t* n_cells_dev, int guided,
                                       float* beta1, size_t n_beta) {
  const size_t n = (size_t)*n_cells_dev;
  const size_t na = n * 24, nx = c.acc_x ? n * 16 : 0, nh = guided ? n * 64 : 0, nv = n;
  const size_t total = na + nx + nh + nv + n_beta;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    size_t k = i;
    if (k < na) { c.acc[k] = 0.0; continue; }
    k -= na;
    if (k < nx) { c.acc_x[k] = 0.0; continue; }
    k -= nx;
    if (k < nh) { c.hacc[k] = 0.0; continue; }
    k -= nh;
    if (k < nv) { c.visits[k] = 0u; continue; }
    k -= nv;
    beta1[k] = 0.0f;
  }
}
void k_clear_iteration(const CacheDev& c, const int32_t* n_cells_dev, int guided, float* beta1,
                       size_t n_beta, hipStream_t s) {
  clear_iteration_kernel<<<2048, 256, 0, s>>>(c, n_cells_dev, guided, beta1, n_beta);
}

// update kernels become no-ops while a skip flag is set (an overflowed
// iteration that is rendered again before its update)
#define SKIP_IF(flag) \
  if ((flag) && *(flag)) return

void k_fill_f32(float* p, float v, size_t n, hipStream_t s) {
  if (n) fill_kernel<float><<<(unsigned)std::min<size_t>((n + 255) / 256, 4096), 256, 0, s>>>(p, v, n);
}

// ---------------------------------------------------------------------------
// camera rays: pinhole, W/p = 1, jitter from block 1 of the root stream
// ---------------------------------------------------------------------------
__global__ void raygen_kernel(SceneDev sc, QueuesDev q, Counters* cnt, IterDev it, uint32_t root0,
                              uint32_t n) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0) cnt->n_ray[1] = n;
  if (j >= n) return;
  const Key key{sc.key0, sc.key1};
  const uint32_t root = root0 + j;
  const uint32_t pix = root / (uint32_t)it.spp, s = root % (uint32_t)it.spp;
  const int px = (int)(pix % (uint32_t)sc.W), py = (int)(pix / (uint32_t)sc.W);
  const uint2 st = stream_root(key, pix, s, (uint32_t)iter_index(it), kTagCam);
  const float4 u = draw4(key, st, 1);
  const float jx = it.center_jitter ? 0.5f : u.x, jy = it.center_jitter ? 0.5f : u.y;
  const float sx = (((float)px + jx) / (float)sc.W) * 2.0f - 1.0f;
  const float sy = 1.0f - (((float)py + jy) / (float)sc.H) * 2.0f;
  const f3 d = norm3(mk3((sc.cam_f[0] + sx * sc.cam_r[0]) + sy * sc.cam_u[0],
                         (sc.cam_f[1] + sx * sc.cam_r[1]) + sy * sc.cam_u[1],
                         (sc.cam_f[2] + sx * sc.cam_r[2]) + sy * sc.cam_u[2]));
  const size_t e = q.cap + j;  // depth 1
  q.R0[e] = make_float4(sc.cam_o[0], sc.cam_o[1], sc.cam_o[2], 1.0f);
  q.R1[e] = make_float4(d.x, d.y, d.z, fbits(pix));
  q.S0[e] = make_float4(1.0f, 1.0f, 1.0f, fbits(0xFFFFFFFFu));
  q.S1[e] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  q.S2[e] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  q.S3[e] = make_uint4(st.x, st.y, 0u, root);
}
void k_raygen(const SceneDev& sc, const QueuesDev& q, Counters* cnt, const IterDev& it,
              uint32_t root0, uint32_t n_roots, hipStream_t s) {
  raygen_kernel<<<(n_roots + 255) / 256, 256, 0, s>>>(sc, q, cnt, it, root0, n_roots);
}

// ---------------------------------------------------------------------------
// BVH traversal.  Node (128 B): four 32-byte child records, each a float4
// (lo.x, lo.y, lo.z, reference bits) and a float4 (hi.x, hi.y, hi.z, -);
// reference >= 0 inner node, < 0 leaf = -1 - (first << 4 | count),
// kBvhNoChild unused.  Leaf children are intersected as soon as their box
// is hit; the nearest inner child is visited next and the others are pushed.
// traverse() is the one-lane form (instrumented runs count node visits with
// it); traverse_quad() is the four-lane form every other launch uses.
// ---------------------------------------------------------------------------
struct RayInv {
  float ix, iy, iz, ox, oy, oz;
};
__device__ __forceinline__ RayInv ray_inv(f3 o, f3 d) {
  const float dx = fabsf(d.x) > 1e-30f ? d.x : copysignf(1e-30f, d.x);
  const float dy = fabsf(d.y) > 1e-30f ? d.y : copysignf(1e-30f, d.y);
  const float dz = fabsf(d.z) > 1e-30f ? d.z : copysignf(1e-30f, d.z);
  RayInv r;
  r.ix = 1.0f / dx; r.iy = 1.0f / dy; r.iz = 1.0f / dz;
  r.ox = o.x * r.ix; r.oy = o.y * r.iy; r.oz = o.z * r.iz;
  return r;
}
__device__ __forceinline__ float box_near(const RayInv& r, float lx, float ly, float lz, float hx,
                                          float hy, float hz, float tmax) {
  const float ax = __builtin_fmaf(lx, r.ix, -r.ox), bx = __builtin_fmaf(hx, r.ix, -r.ox);
  const float ay = __builtin_fmaf(ly, r.iy, -r.oy), by = __builtin_fmaf(hy, r.iy, -r.oy);
  const float az = __builtin_fmaf(lz, r.iz, -r.oz), bz = __builtin_fmaf(hz, r.iz, -r.oz);
  const float tn = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fminf(az, bz));
  const float tf = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fmaxf(az, bz));
  return (tn <= tf && tf >= 0.0f && tn <= tmax) ? tn : INFINITY;
}

// Moller-Trumbore, two-sided, fixed operation order.  Evaluated without
// early exits (a wave's lanes rarely all leave at the same test, and the
// three loads then go out together); the hit conditions are the rejections
// det == 0, u < 0, u > 1, v < 0, u + v > 1 negated, so a NaN u or v is
// rejected only by the caller's test of t.  *t is written in every case and
// is meaningful only when the result is true.
__device__ __forceinline__ bool tri_hit(f3 o, f3 d, float4 A, float4 B, float4 Cc, float* t) {
  const f3 v0 = xyz(A), e1 = xyz(B), e2 = xyz(Cc);
  const f3 p = cross3(d, e2);
  const float det = dot3(e1, p);
  const float inv = 1.0f / det;
  const f3 s = sub3(o, v0);
  const float u = dot3(s, p) * inv;
  const f3 qv = cross3(s, e1);
  const float v = dot3(d, qv) * inv;
  *t = dot3(e2, qv) * inv;
  return (det != 0.0f) & !(u < 0.0f) & !(u > 1.0f) & !(v < 0.0f) & !(u + v > 1.0f);
}

// Visit order of the inner children of a node: by entry distance clamped at
// 0 (every box holding the ray origin is entered at 0), children within 4
// ulps of each other by slot.  The key is the distance's bit pattern with its
// two low bits replaced by the slot, compared as an unsigned integer, so the
// keys of a node are distinct; a culled child has key >= kKeyCulled.  Any
// visit order gives the same closest hit (ties go to the smaller primitive
// index), so the order only decides how much is visited.
constexpr uint32_t kKeyCulled = 0x7F800000u;  // bits of +infinity
__device__ __forceinline__ uint32_t visit_key(float t, int slot) {
  return ((uint32_t)max(__float_as_int(t), 0) & ~3u) | (uint32_t)slot;
}

// ordered swap of two (key, reference) pairs, by selects
__device__ __forceinline__ void kswap(uint32_t& ka, int& ra, uint32_t& kb, int& rb) {
  const bool sw = kb < ka;
  const uint32_t lo = sw ? kb : ka, hi = sw ? ka : kb;
  const int rlo = sw ? rb : ra, rhi = sw ? ra : rb;
  ka = lo; kb = hi; ra = rlo; rb = rhi;
}

// 4-wide BVH traversal.  Leaf children are intersected when their box is
// hit; the hit inner children are sorted by entry distance, the nearest
// visited next and the others pushed (far first).  The stack's first
// kStackDepth entries per lane live in LDS, deeper ones (rare; bounded by
// the builder) in the scene's spill area.  Closest hit: smallest t, ties by
// smaller primitive index (independent of the traversal order).
template <bool kAny, bool kCount>
__device__ __forceinline__ bool traverse(const SceneDev& sc, f3 o, f3 d, float tmax, int* stk,
                                         float* bt_out, uint32_t* bp_out, uint32_t* n_nodes,
                                         uint32_t* n_tris) {
  const RayInv ri = ray_inv(o, d);
  float bt = tmax;
  uint32_t bp = kMiss;
  int sp = 0;
  int node = 0;
  const int lane = threadIdx.x;
  const size_t gtid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  auto push = [&](int v) {
    if (sp < kStackDepth) stk[sp * kTraceBlock + lane] = v;
    else sc.stack_spill[(size_t)(sp - kStackDepth) * sc.spill_threads + gtid] = v;
    ++sp;
  };
  while (true) {
    const float4* N = sc.bvh + (size_t)node * 8;
    if (kCount) ++*n_nodes;
    const float4 a0 = N[0], b0 = N[1], a1 = N[2], b1 = N[3];
    const float4 a2 = N[4], b2 = N[5], a3 = N[6], b3 = N[7];
    int r0 = (int)ubits(a0.w), r1 = (int)ubits(a1.w), r2 = (int)ubits(a2.w), r3 = (int)ubits(a3.w);
    // all four boxes tested unconditionally (branch-free, on the loaded
    // registers), unused slots masked afterwards
    float t0 = box_near(ri, a0.x, a0.y, a0.z, b0.x, b0.y, b0.z, bt);
    float t1 = box_near(ri, a1.x, a1.y, a1.z, b1.x, b1.y, b1.z, bt);
    float t2 = box_near(ri, a2.x, a2.y, a2.z, b2.x, b2.y, b2.z, bt);
    float t3 = box_near(ri, a3.x, a3.y, a3.z, b3.x, b3.y, b3.z, bt);
    t0 = r0 == kBvhNoChild ? INFINITY : t0;
    t1 = r1 == kBvhNoChild ? INFINITY : t1;
    t2 = r2 == kBvhNoChild ? INFINITY : t2;
    t3 = r3 == kBvhNoChild ? INFINITY : t3;
#pragma unroll
    for (int side = 0; side < 4; ++side) {
      const int ch = side == 0 ? r0 : side == 1 ? r1 : side == 2 ? r2 : r3;
      const float tn = side == 0 ? t0 : side == 1 ? t1 : side == 2 ? t2 : t3;
      if (ch < 0 && tn != INFINITY) {
        const uint32_t code = (uint32_t)(-1 - ch);
        const uint32_t first = code >> 4, count = code & 15u;
        for (uint32_t k = first; k < first + count; ++k) {
          const float4* T = sc.tri_bvh + (size_t)k * 3;
          if (kCount) ++*n_tris;
          const float4 A = T[0];
          float t;
          if (!tri_hit(o, d, A, T[1], T[2], &t)) continue;
          if (!(t > 0.0f && t < tmax)) continue;
          const uint32_t prim = ubits(A.w);
          if (kAny) {
            *bt_out = t;
            *bp_out = prim;
            return true;
          }
          if (t < bt || (t == bt && prim < bp)) {
            bt = t;
            bp = prim;
          }
        }
      }
    }
    // inner children still in front of the closest hit (a box entered at
    // exactly bt may hold an equal-t hit of smaller index), sorted by key
    uint32_t k0 = visit_key((r0 >= 0 && t0 <= bt) ? t0 : INFINITY, 0);
    uint32_t k1 = visit_key((r1 >= 0 && t1 <= bt) ? t1 : INFINITY, 1);
    uint32_t k2 = visit_key((r2 >= 0 && t2 <= bt) ? t2 : INFINITY, 2);
    uint32_t k3 = visit_key((r3 >= 0 && t3 <= bt) ? t3 : INFINITY, 3);
    kswap(k0, r0, k1, r1);
    kswap(k2, r2, k3, r3);
    kswap(k0, r0, k2, r2);
    kswap(k1, r1, k3, r3);
    kswap(k1, r1, k2, r2);
    if (k0 < kKeyCulled) {
      if (k3 < kKeyCulled) push(r3);
      if (k2 < kKeyCulled) push(r2);
      if (k1 < kKeyCulled) push(r1);
      node = r0;
    } else {
      if (sp == 0) break;
      --sp;
      node = sp < kStackDepth ? stk[sp * kTraceBlock + lane]
                              : sc.stack_spill[(size_t)(sp - kStackDepth) * sc.spill_threads + gtid];
    }
  }
  *bt_out = bt;
  *bp_out = bp;
  return bp != kMiss;
}

__device__ __forceinline__ void add_counts(unsigned long long* tc, uint32_t rays, uint32_t nodes,
                                           uint32_t tris) {
  const uint32_t a = wave_sum(rays), b = wave_sum(nodes), c = wave_sum(tris);
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(tc + 0, (unsigned long long)a);
    atomicAdd(tc + 1, (unsigned long long)b);
    atomicAdd(tc + 2, (unsigned long long)c);
  }
}

// Shadow rays of depth d and continuation rays of depth d+1 both come out of
// shade(d) and are independent, so one launch traverses both queues (closest
// hits first, then any hits); this halves the number of tail-bound launches.
template <bool kCount>
__global__ __launch_bounds__(kTraceBlock) void trace_pair_kernel(SceneDev sc, QueuesDev q,
                                                                 const Counters* cnt, int dc,
                                                                 int ds, unsigned long long* tc) {
  __shared__ int stk[kStackDepth * kTraceBlock];
  if (cnt->overflow) return;
  const uint32_t nc = dc >= 0 ? min(cnt->n_ray[dc], (uint32_t)q.cap) : 0u;
  const uint32_t ns = ds > 0 ? min(cnt->n_shadow[ds], (uint32_t)q.scap) : 0u;
  const size_t Lc = (size_t)(dc >= 0 ? dc : 0) * q.cap, Ls = (size_t)ds * q.scap;
  uint32_t cr = 0, cn = 0, ct = 0, sr = 0, sn = 0, st = 0;
  uint32_t cmax = 0, smax = 0, clong = 0, slong = 0;  // per-ray node visits: max, rays > 64
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < nc + ns;
       j += gridDim.x * blockDim.x) {
    float t;
    uint32_t p;
    if (j < nc) {
      const float4 r0 = q.R0[Lc + j];
      uint2 h = make_uint2(ubits(INFINITY), kMiss);
      if (r0.w != 0.0f) {
        const float4 r1 = q.R1[Lc + j];
        if (kCount) ++cr;
        const uint32_t cn0 = cn;
        if (traverse<false, kCount>(sc, xyz(r0), xyz(r1), INFINITY, stk, &t, &p, &cn, &ct))
          h = make_uint2(ubits(t), p);
        if (kCount) {
          cmax = max(cmax, cn - cn0);
          clong += (cn - cn0) > 64u ? 1u : 0u;
        }
      }
      q.H[Lc + j] = h;
    } else {
      const uint32_t k = j - nc;
      const float4 v = q.SH2[Ls + k];
      if (v.w == 0.0f) continue;
      const float4 a = q.SH0[k], b = q.SH1[k];
      if (kCount) ++sr;
      const uint32_t sn0 = sn;
      if (traverse<true, kCount>(sc, xyz(a), xyz(b), a.w, stk, &t, &p, &sn, &st))
        q.SH2[Ls + k] = make_float4(0.0f, 0.0f, 0.0f, v.w);
      if (kCount) {
        smax = max(smax, sn - sn0);
        slong += (sn - sn0) > 64u ? 1u : 0u;
      }
    }
  }
  if (kCount) {
    add_counts(tc, cr, cn, ct);
    add_counts(tc + 3, sr, sn, st);
    const uint32_t cl = wave_sum(clong), sl = wave_sum(slong);
    if ((threadIdx.x & 63) == 0) {
      if (cl) atomicAdd(tc + 8, (unsigned long long)cl);
      if (sl) atomicAdd(tc + 9, (unsigned long long)sl);
    }
    if (cmax) atomicMax(tc + 6, (unsigned long long)cmax);
    if (smax) atomicMax(tc + 7, (unsigned long long)smax);
  }
}
// ---------------------------------------------------------------------------
// Quad traversal: four lanes per ray.  Lane s of a quad loads and tests
// child s of the node.  The hit leaf children are broadcast to the quad as
// (first << 4 | count) words, their triangles numbered in child order and
// dealt round-robin to the four lanes; the quad's closest hit is reduced in
// the (t, primitive index) order, which is the order traverse() keeps.  Each
// lane then ranks its own inner child among the quad's four visit keys (read
// with quad rotations), and two quad reductions give every lane the number of
// children to visit and the nearest one; lane s pushes its child by rank, far
// first.  The quad thus takes the decisions of traverse(): the same visit
// order, the same stack and the same result.  Every branch below is taken
// alike by the four lanes of a quad (their inputs are quad-uniform), except
// the per-lane triangle loop, which closes before the reductions, so the
// permutes never read a lane of the quad that is off.
// ---------------------------------------------------------------------------
constexpr int kQuadsPerBlock = kTraceBlock / 4;
constexpr int kQuadStack = 4 * kStackDepth;      // LDS entries per ray
constexpr int kQuadStride = kQuadsPerBlock + 1;  // padded: a quad's pushes hit distinct banks

template <int k>
__device__ __forceinline__ int quad_bcast(int v) {
  return __builtin_amdgcn_mov_dpp(v, k * 0x55, 0xF, 0xF, false);
}
template <int k>
__device__ __forceinline__ uint32_t quad_bcast(uint32_t v) {
  return (uint32_t)quad_bcast<k>((int)v);
}
// value of lane (s ^ m) of the quad
template <int m>
__device__ __forceinline__ int quad_xor(int v) {
  return __builtin_amdgcn_mov_dpp(v, m == 1 ? 0xB1 : 0x4E, 0xF, 0xF, false);
}
// value of lane (s + m) & 3 of the quad
template <int m>
__device__ __forceinline__ uint32_t quad_rot(uint32_t v) {
  constexpr int ctrl = (m & 3) | (((1 + m) & 3) << 2) | (((2 + m) & 3) << 4) | (((3 + m) & 3) << 6);
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, ctrl, 0xF, 0xF, false);
}
// (t, primitive) minimum over the quad: smaller t, ties by smaller index
__device__ __forceinline__ void quad_min_hit(float& t, uint32_t& p) {
  // non-short-circuit conditions and selects keep the reduction branch-free
  float t2 = __int_as_float(quad_xor<1>(__float_as_int(t)));
  uint32_t p2 = (uint32_t)quad_xor<1>((int)p);
  bool take = (t2 < t) | ((t2 == t) & (p2 < p));
  t = take ? t2 : t;
  p = take ? p2 : p;
  t2 = __int_as_float(quad_xor<2>(__float_as_int(t)));
  p2 = (uint32_t)quad_xor<2>((int)p);
  take = (t2 < t) | ((t2 == t) & (p2 < p));
  t = take ? t2 : t;
  p = take ? p2 : p;
}
__device__ __forceinline__ bool quad_any(bool b) {
  int v = b ? 1 : 0;
  v |= quad_xor<1>(v);
  v |= quad_xor<2>(v);
  return v != 0;
}

// Each ray is traced by 4^kSplit quads (kSplit = 0, 1, 2).  With kSplit > 0
// the quads split the top kSplit levels of the tree: quad g follows child
// (g >> 2l) & 3 at level l, a leaf met on that descent is intersected by the
// one quad whose remaining digits are 0, and below the split each quad
// traverses its subtree as usual.  Every leaf is reached by exactly one quad.
// The quads of a ray share *sh (LDS): the bits of the smallest hit distance
// found so far, which every quad culls with, or for any-hit rays a found
// flag, on which the others stop.  Each quad returns its own closest hit; the
// caller reduces them in the (t, primitive) order.
typedef __attribute__((address_space(3))) uint32_t lds_u32;
enum { kStepGo = 0, kStepEnd = 1, kStepFound = 2 };
// One node of a quad's traversal.  State: bt, bp (the quad's closest hit so
// far), sp and node (stack depth and the node to visit), split (while
// splitting: levels still to split in bits 4.. and the digits of the path
// below this level in bits 0..3, the next digit in bits 0..1).  Returns
// kStepGo to go on, kStepEnd when the ray's traversal is over, kStepFound when
// an any-hit ray found a hit (bt, bp then hold this lane's hit).
template <bool kAny, int kSplit>
__device__ __forceinline__ int quad_step(const SceneDev& sc, const RayInv& ri, f3 o, f3 d, float tmax,
                                         int* stk, int sub, int qcol, uint32_t qid, lds_u32* sh,
                                         float& bt, uint32_t& bp, int& sp, int& node, uint32_t& split) {
  {
    float cut = bt;
    if (kSplit > 0) {
      const uint32_t v = *(volatile lds_u32*)sh;
      if (kAny) {
        if (v != 0u) return kStepEnd;
      } else {
        cut = fminf(bt, __uint_as_float(v));
      }
    }
    // child `sub` of the node: its record's two 16-byte words
    const float4* N = sc.bvh + (size_t)node * 8 + 2 * sub;
    const float4 ca = N[0], cb = N[1];
    const int rs = __float_as_int(ca.w);
    float ts = box_near(ri, ca.x, ca.y, ca.z, cb.x, cb.y, cb.z, cut);
    ts = rs == kBvhNoChild ? INFINITY : ts;
    // while splitting, only the child on this quad's path counts, and a leaf
    // there only for the quad whose remaining digits are 0
    bool mine = true, leaf_mine = true;
    if (kSplit > 0 && split >= 16u) {
      mine = (uint32_t)sub == (split & 3u);
      leaf_mine = mine && (split & 12u) == 0u;
    }
    // the quad's hit leaf children and their triangle counts (at most 4 each)
    const uint32_t lw = (rs < 0 && ts != INFINITY && leaf_mine) ? (uint32_t)(-1 - rs) : 0u;
    const uint32_t w0 = quad_bcast<0>(lw), w1 = quad_bcast<1>(lw), w2 = quad_bcast<2>(lw),
                   w3 = quad_bcast<3>(lw);
    const uint32_t p1 = w0 & 15u, p2 = p1 + (w1 & 15u), p3 = p2 + (w2 & 15u),
                   ntri = p3 + (w3 & 15u);
    if (ntri != 0u) {
      float ht = INFINITY;
      uint32_t hp = kMiss;
      bool hit = false;
      for (uint32_t m = (uint32_t)sub; m < ntri; m += 4) {
        // the leaf holding triangle m and m's offset in it, by selects
        const bool b1 = m >= p1, b2 = m >= p2, b3 = m >= p3;
        const uint32_t w = b3 ? w3 : b2 ? w2 : b1 ? w1 : w0;
        const uint32_t base = b3 ? p3 : b2 ? p2 : b1 ? p1 : 0u;
        const uint32_t k = (w >> 4) + (m - base);
        const float4* T = sc.tri_bvh + (size_t)k * 3;
        const float4 A = T[0];
        float t;
        const bool h = tri_hit(o, d, A, T[1], T[2], &t) & (t > 0.0f) & (t < tmax);
        const uint32_t prim = ubits(A.w);
        if (kAny) {
          if (h) {
            hit = true;
            ht = t;
            hp = prim;
            break;
          }
        } else {
          const bool take = h & ((t < ht) | ((t == ht) & (prim < hp)));
          ht = take ? t : ht;
          hp = take ? prim : hp;
        }
      }
      if (kAny) {
        if (quad_any(hit)) {
          if (kSplit > 0 && sub == 0) *(volatile lds_u32*)sh = 1u;
          bt = ht;
          bp = hp;
          return kStepFound;
        }
      } else {
        quad_min_hit(ht, hp);
        const bool take = (ht < bt) | ((ht == bt) & (hp < bp));
        bt = take ? ht : bt;
        bp = take ? hp : bp;
        // hit distances are positive, so their bits order as the distances
        if (kSplit > 0 && take && sub == 0)
          __hip_atomic_fetch_min(sh, __float_as_uint(bt), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        cut = fminf(cut, bt);
      }
    }
    // this lane's inner child, if still in front of the closest hit (a box
    // entered at exactly the cut may hold an equal-t hit of smaller index):
    // its key, its rank among the quad's keys, the number of children to
    // visit and the nearest child
    const uint32_t key = visit_key((rs >= 0 && ts <= cut && mine) ? ts : INFINITY, sub);
    const uint32_t q1 = quad_rot<1>(key), q2 = quad_rot<2>(key), q3 = quad_rot<3>(key);
    const int rank = (q1 < key ? 1 : 0) + (q2 < key ? 1 : 0) + (q3 < key ? 1 : 0);
    const bool live = key < kKeyCulled;
    int nlive = live ? 1 : 0;
    nlive += quad_xor<1>(nlive);
    nlive += quad_xor<2>(nlive);
    int nearest = (live && rank == 0) ? rs : -1;
    nearest = max(nearest, quad_xor<1>(nearest));
    nearest = max(nearest, quad_xor<2>(nearest));
    if (nlive != 0) {
      // the live children other than the nearest, far first: rank j goes to
      // sp + nlive - 1 - j
      if (live && rank != 0) {
        const int pos = sp + nlive - 1 - rank;
        if (pos < kQuadStack) stk[pos * kQuadStride + qcol] = rs;
        else sc.stack_spill[(size_t)(pos - kQuadStack) * sc.spill_threads + qid] = rs;
      }
      sp += nlive - 1;
      node = nearest;
      if (kSplit > 0 && split >= 16u) split = ((split - 16u) & ~15u) | ((split & 15u) >> 2);
    } else {
      if (sp == 0) return kStepEnd;
      --sp;
      // (the LDS read through an LDS-qualified pointer, so that it is not
      // merged with the spill read into one generic-address load)
      node = sp < kQuadStack
                 ? ((__attribute__((address_space(3))) int*)stk)[sp * kQuadStride + qcol]
                 : sc.stack_spill[(size_t)(sp - kQuadStack) * sc.spill_threads + qid];
    }
  }
  return kStepGo;
}

template <bool kAny, int kSplit>
__device__ __forceinline__ bool traverse_quad(const SceneDev& sc, f3 o, f3 d, float tmax, int* stk,
                                              int sub, int qcol, uint32_t qid, int g, lds_u32* sh,
                                              float* bt_out, uint32_t* bp_out) {
  const RayInv ri = ray_inv(o, d);
  float bt = tmax;
  uint32_t bp = kMiss;
  int sp = 0, node = 0;
  uint32_t split = ((uint32_t)kSplit << 4) | (uint32_t)g;
  int r;
  do {
    r = quad_step<kAny, kSplit>(sc, ri, o, d, tmax, stk, sub, qcol, qid, sh, bt, bp, sp, node, split);
  } while (r == kStepGo);
  *bt_out = bt;
  *bp_out = bp;
  return r == kStepFound || bp != kMiss;
}

// One quad per ray, each quad taking the rays j, j + R, j + 2R, .. of one
// kind below n and starting its next ray as soon as its current one is done,
// so that a wave's quads do not wait for the wave's slowest ray after every
// ray (only once, at the end of the stream).  Per ray the node order and the
// result are those of traverse_quad.
template <bool kAny>
__device__ __forceinline__ void trace_stream(const SceneDev& sc, const QueuesDev& q, uint32_t j,
                                             uint32_t n, uint32_t R, size_t L, int* stk, int sub,
                                             int qcol, uint32_t qid) {
  RayInv ri;
  f3 o, d;
  float tmax = INFINITY, bt = INFINITY;
  uint32_t bp = kMiss, split = 0u;
  int sp = 0, node = 0;
  bool busy = false;
  while (true) {
    if (!busy) {
      // the quad's next ray with work
      float4 a, b;
      for (; j < n; j += R) {
        if (kAny) {
          if (q.SH2[L + j].w != 0.0f) break;
        } else {
          a = q.R0[L + j];
          if (a.w != 0.0f) break;
          if (sub == 0) q.H[L + j] = make_uint2(ubits(INFINITY), kMiss);
        }
      }
      if (j >= n) break;
      if (kAny) {
        a = q.SH0[j];
        b = q.SH1[j];
        tmax = a.w;
      } else {
        b = q.R1[L + j];
      }
      o = xyz(a);
      d = xyz(b);
      ri = ray_inv(o, d);
      bt = tmax;
      bp = kMiss;
      sp = 0;
      node = 0;
      busy = true;
    }
    const int r = quad_step<kAny, 0>(sc, ri, o, d, tmax, stk, sub, qcol, qid, nullptr, bt, bp, sp, node, split);
    if (r != kStepGo) {
      if (sub == 0) {
        if (kAny) {
          if (r == kStepFound) {
            // occluded: the contribution's colour cleared, its last word kept
            float* c = (float*)&q.SH2[L + j];
            c[0] = 0.0f;
            c[1] = 0.0f;
            c[2] = 0.0f;
          }
        } else {
          // the quad's reduced closest hit (a miss leaves bt = inf, bp = kMiss)
          q.H[L + j] = make_uint2(ubits(bt), bp);
        }
      }
      busy = false;
      j += R;
    }
  }
}

// LDS writes of some lanes of a wave made visible to reads by other lanes of
// the same wave: the writes complete (workgroup-scope release), no code moves
// across (wave barrier), then the reads (acquire)
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// The rays of one launch with 4^kSplit quads per ray: ray j is traced by the
// quads of group j mod R (R groups), quad g of its group taking its share of
// the tree; the group's first lane writes the result.
template <int kSplit>
__device__ __forceinline__ void trace_rays(const SceneDev& sc, const QueuesDev& q, uint32_t nc,
                                           uint32_t ns, size_t Lc, size_t Ls, int* stk,
                                           uint32_t* shared_t, uint2* res) {
  constexpr int kLog = 2 * kSplit;
  const int sub = threadIdx.x & 3, qcol = threadIdx.x >> 2;
  const uint32_t qid = (blockIdx.x * blockDim.x + threadIdx.x) >> 2;
  const int g = (int)(qid & ((1u << kLog) - 1u));
  const uint32_t R = (gridDim.x * (blockDim.x >> 2)) >> kLog;
  lds_u32* sh = (lds_u32*)shared_t + (qcol >> kLog);
  const bool lead = g == 0 && sub == 0;
  for (uint32_t j = (uint32_t)(qid >> kLog); j < nc + ns; j += R) {
    float t;
    uint32_t p;
    if (j < nc) {
      const float4 r0 = q.R0[Lc + j];
      if (r0.w == 0.0f) {
        if (lead) q.H[Lc + j] = make_uint2(ubits(INFINITY), kMiss);
        continue;
      }
      const float4 r1 = q.R1[Lc + j];
      if (kSplit > 0) {
        if (lead) *sh = ubits(INFINITY);
        wave_lds_fence();
      }
      const bool hit =
          traverse_quad<false, kSplit>(sc, xyz(r0), xyz(r1), INFINITY, stk, sub, qcol, qid, g, sh, &t, &p);
      uint2 h = hit ? make_uint2(ubits(t), p) : make_uint2(ubits(INFINITY), kMiss);
      if (kSplit > 0) {
        // the group's closest hit: smallest t, ties by smaller primitive
        if (sub == 0) res[qcol] = h;
        wave_lds_fence();
        if (lead) {
          for (int k = 1; k < (1 << kLog); ++k) {
            const uint2 o = res[qcol + k];
            const float to = fbits(o.x), th = fbits(h.x);
            if (to < th || (to == th && o.y < h.y)) h = o;
          }
        }
        wave_lds_fence();
      }
      if (lead) q.H[Lc + j] = h;
    } else {
      const uint32_t k = j - nc;
      const float4 v = q.SH2[Ls + k];
      if (v.w == 0.0f) continue;
      const float4 a = q.SH0[k], b = q.SH1[k];
      if (kSplit > 0) {
        if (lead) *sh = 0u;
        wave_lds_fence();
      }
      bool hit = traverse_quad<true, kSplit>(sc, xyz(a), xyz(b), a.w, stk, sub, qcol, qid, g, sh, &t, &p);
      if (kSplit > 0) {
        wave_lds_fence();
        hit = *(volatile lds_u32*)sh != 0u;
        wave_lds_fence();
      }
      if (hit && lead) q.SH2[Ls + k] = make_float4(0.0f, 0.0f, 0.0f, v.w);
    }
  }
}

// The rays of trace_pair_kernel: one quad per ray, or when the launch has at
// most a quarter (a sixteenth) as many rays as resident quads, 4 (16) quads
// per ray, so that the few rays of the deep bounces finish sooner.
constexpr uint64_t kSplitDiv16 = 16, kSplitDiv4 = 4;
__global__ __launch_bounds__(kTraceBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void trace_quad_kernel(SceneDev sc, QueuesDev q,
                                                                 const Counters* cnt, int dc,
                                                                 int ds) {
  __shared__ int stk[kQuadStack * kQuadStride];
  __shared__ uint32_t shared_t[kQuadsPerBlock];
  __shared__ uint2 res[kQuadsPerBlock];
  if (cnt->overflow) return;
  const uint32_t nc = dc >= 0 ? min(cnt->n_ray[dc], (uint32_t)q.cap) : 0u;
  const uint32_t ns = ds > 0 ? min(cnt->n_shadow[ds], (uint32_t)q.scap) : 0u;
  const size_t Lc = (size_t)(dc >= 0 ? dc : 0) * q.cap, Ls = (size_t)ds * q.scap;
  const uint32_t Q = gridDim.x * (blockDim.x >> 2);
  const uint32_t n = nc + ns;
  if ((uint64_t)n * kSplitDiv16 <= Q) trace_rays<2>(sc, q, nc, ns, Lc, Ls, stk, shared_t, res);
  else if ((uint64_t)n * kSplitDiv4 <= Q) trace_rays<1>(sc, q, nc, ns, Lc, Ls, stk, shared_t, res);
  else {
    // one quad per ray, the closest rays first; quad i takes ray j of the
    // combined numbering (closest, then shadow) when j = i mod Q
    const uint32_t qid = (blockIdx.x * blockDim.x + threadIdx.x) >> 2;
    const int sub = threadIdx.x & 3, qcol = threadIdx.x >> 2;
    trace_stream<false>(sc, q, qid, nc, Q, Lc, stk, sub, qcol, qid);
    const uint32_t k0 = (qid + Q - nc % Q) % Q;
    trace_stream<true>(sc, q, k0, ns, Q, Ls, stk, sub, qcol, qid);
  }
}

void k_trace_pair(const SceneDev& sc, const QueuesDev& q, const Counters* cnt, int dc, int ds,
                  int grid, hipStream_t s, unsigned long long* tc, hipEvent_t ev0, hipEvent_t ev1) {
  // the spill area has one column per thread of the launch
  if (sc.stack_spill) grid = std::min(grid, (int)(sc.spill_threads / kTraceBlock));
  // instrumented runs count node visits per ray with the one-lane loop
  if (tc) {
    if (ev0) (void)hipEventRecord(ev0, s);
    trace_pair_kernel<true><<<grid, kTraceBlock, 0, s>>>(sc, q, cnt, dc, ds, tc);
    if (ev1) (void)hipEventRecord(ev1, s);
  } else if (ev0)
    hipExtLaunchKernelGGL(trace_quad_kernel, dim3(grid), dim3(kTraceBlock), 0, s, ev0, ev1, 0u, sc, q,
                          cnt, dc, ds);
  else trace_quad_kernel<<<grid, kTraceBlock, 0, s>>>(sc, q, cnt, dc, ds);
}

// ---------------------------------------------------------------------------
// per-vertex sample counts (Sec. 3.1 "Optimization", colour rule Sec. 4.1):
//   beta^X_t = sqrt((1/3) sum_ch (T_ch / I~_ch)^2 a^X_{t,ch}),
//   beta = beta^RR if < 1, else beta^S if > 1, else 1; clamped.
// classic throughput RR: q = min(1, max T) from rr_start on (baseline and
// warm-up of Sec. 4.1 / 5.2).
// ---------------------------------------------------------------------------
// EARS (the baseline the paper compares against, Sec. 5: the same number of
// samples for every technique): beta_t = r_t lambda, with the classic
// per-technique ratios r at q = 1.  Along that line the efficiency model of
// Sec. 3.1 is optimal at lambda^2 = (C_I / V_I) sum_t (M_t / r_t) /
// sum_t r_t C_t (M: per-sample second moment for RR, variance for
// splitting), the fixed point restricted to the line; the update keeps these
// shared factors in technique slot 0.
__host__ __device__ inline void ears_ratios(int mode, double r[3]) {
  if (mode == 1) { r[0] = 0.5; r[1] = 1.0; r[2] = 0.5; }
  else if (mode == 2) { r[0] = 1.0; r[1] = 1.0; r[2] = 1.0; }
  else { r[0] = 1.0; r[1] = 1.0; r[2] = 0.0; }
}
// (mask: the techniques whose counts are wanted; the others are left as they are)
__device__ __forceinline__ void counts_at(const SceneDev& sc, const CacheDev& c, const IterDev& it,
                                          uint32_t cell, f3 T, const float* It, int depth,
                                          float beta[3], uint32_t mask = 7u) {
  const float q = (depth >= it.rr_start) ? fminf(1.0f, fmaxf(fmaxf(T.x, T.y), T.z)) : 1.0f;
  float cb[3];
  if (sc.mode == 1) { cb[0] = q * 0.5f; cb[1] = 1.0f; cb[2] = q * 0.5f; }
  else if (sc.mode == 2) { cb[0] = q; cb[1] = 1.0f; cb[2] = 1.0f; }
  else { cb[0] = q; cb[1] = 1.0f; cb[2] = 0.0f; }
  const bool en[3] = {true, sc.nee != 0 && sc.n_lights > 0, sc.mode != 0};
  const float z0 = T.x / It[0], z1 = T.y / It[1], z2 = T.z / It[2];
  if (it.alloc == 4) {
    // EARS: one shared count lambda from technique slot 0, beta_t = r_t lambda
    const float* aRR = c.fac + (size_t)cell * 18;
    const float* aS = c.fac + (size_t)cell * 18 + 9;
    double r[3];
    ears_ratios(sc.mode, r);
    float lam = 0.0f;
    if (!(aRR[0] < 0.0f)) {
      const float sr = ((z0 * z0) * aRR[0] + (z1 * z1) * aRR[1]) + (z2 * z2) * aRR[2];
      const float ss = ((z0 * z0) * aS[0] + (z1 * z1) * aS[1]) + (z2 * z2) * aS[2];
      const float bRR = sqrtf(sr * (1.0f / 3.0f));
      const float bS = sqrtf(ss * (1.0f / 3.0f));
      lam = bRR < 1.0f ? bRR : (bS > 1.0f ? bS : 1.0f);
      lam = fminf(fmaxf(lam, it.clamp_lo), it.clamp_hi);
    }
#pragma unroll
    for (int t = 0; t < 3; ++t)
      if ((mask >> t) & 1u) beta[t] = !en[t] ? 0.0f : (aRR[0] < 0.0f ? cb[t] : (float)r[t] * lam);
    return;
  }
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    if (!((mask >> t) & 1u)) continue;
    if (!en[t]) { beta[t] = 0.0f; continue; }
    if (it.alloc == 0) { beta[t] = cb[t]; continue; }
    float b;
    if (it.alloc == 2) {
      const int idx = c.n_fixed > 1 ? (int)cell : 0;
      b = c.fixed[idx * 3 + t];
      if (it.fixed_scale) {
        const float s = ((z0 * z0 + z1 * z1) + z2 * z2) * (1.0f / 3.0f);
        b = b * sqrtf(s);
      }
    } else {
      const float* aRR = c.fac + (size_t)cell * 18 + (0 * 3 + t) * 3;
      const float* aS = c.fac + (size_t)cell * 18 + (1 * 3 + t) * 3;
      if (aRR[0] < 0.0f) {
        b = cb[t];
      } else {
        const float sr = ((z0 * z0) * aRR[0] + (z1 * z1) * aRR[1]) + (z2 * z2) * aRR[2];
        const float ss = ((z0 * z0) * aS[0] + (z1 * z1) * aS[1]) + (z2 * z2) * aS[2];
        const float bRR = sqrtf(sr * (1.0f / 3.0f));
        const float bS = sqrtf(ss * (1.0f / 3.0f));
        b = bRR < 1.0f ? bRR : (bS > 1.0f ? bS : 1.0f);
      }
    }
    beta[t] = fminf(fmaxf(b, it.clamp_lo), it.clamp_hi);
  }
}

// counts of the light-path classes y_2 and y_3+ (techniques 3 and 4) of a
// bidirectional scene with per-length budgets: the light-path rules of
// counts_at (classic count 1, the fixed count of the light-path slot, the
// fixed point of Sec. 3.1 with the class's own factors and the same colour
// rule and clamp)
__device__ __forceinline__ void counts_at_x(const CacheDev& c, const IterDev& it, uint32_t cell,
                                            f3 T, const float* It, float bx[2],
                                            uint32_t mask = 3u) {
  const float z0 = T.x / It[0], z1 = T.y / It[1], z2 = T.z / It[2];
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    if (!((mask >> x) & 1u)) continue;
    if (it.alloc == 0) { bx[x] = 1.0f; continue; }
    float b;
    if (it.alloc == 2) {
      const int idx = c.n_fixed > 1 ? (int)cell : 0;
      b = c.fixed[idx * 3 + 2];
      if (it.fixed_scale) {
        const float s = ((z0 * z0 + z1 * z1) + z2 * z2) * (1.0f / 3.0f);
        b = b * sqrtf(s);
      }
    } else {
      const float* aRR = c.fac_x + (size_t)cell * 12 + (0 * 2 + x) * 3;
      const float* aS = c.fac_x + (size_t)cell * 12 + (1 * 2 + x) * 3;
      if (aRR[0] < 0.0f) {
        b = 1.0f;
      } else {
        const float sr = ((z0 * z0) * aRR[0] + (z1 * z1) * aRR[1]) + (z2 * z2) * aRR[2];
        const float ss = ((z0 * z0) * aS[0] + (z1 * z1) * aS[1]) + (z2 * z2) * aS[2];
        const float bRR = sqrtf(sr * (1.0f / 3.0f));
        const float bS = sqrtf(ss * (1.0f / 3.0f));
        b = bRR < 1.0f ? bRR : (bS > 1.0f ? bS : 1.0f);
      }
    }
    bx[x] = fminf(fmaxf(b, it.clamp_lo), it.clamp_hi);
  }
}

// the count of the light-path class of light vertex y_i (i >= 1): one class
// unless per-length budgets, then b2 for y_1, b3 for y_2, b4 for y_3+
__device__ __forceinline__ float lp_class_count(const SceneDev& sc, float b2, float b3, float b4,
                                                int i) {
  return sc.lp_classes == 3 ? (i == 1 ? b2 : (i == 2 ? b3 : b4)) : b2;
}

// learned cache (alloc mode 3): from the network's outputs y at a vertex,
// its count |T / I~| exp(y_t) (colour rule's norm) is pooled with the
// octree's count beta_t as their geometric mean, then clamped; the octree
// count stays where the result is not finite, and techniques it disables
// stay off.  The network's input normal is the geometric normal as stored
// (not turned toward the incoming ray), so that the same counts can be
// evaluated at a light vertex for the MIS weights of bidirectional paths.
__device__ __forceinline__ void mlp_apply(const IterDev& it, f3 T, const float* It, const float* y,
                                          float beta[3], uint32_t mask = 7u) {
  const float z0 = T.x / It[0], z1 = T.y / It[1], z2 = T.z / It[2];
  const float sm = sqrtf(((z0 * z0 + z1 * z1) + z2 * z2) * (1.0f / 3.0f));
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    if (!((mask >> t) & 1u) || !(beta[t] > 0.0f)) continue;
    const float b = sqrtf(beta[t] * (sm * expf(y[t])));
    if (isfinite(b)) beta[t] = fminf(fmaxf(b, it.clamp_lo), it.clamp_hi);
  }
}
// in learned-cache iterations, the counts of queue entry e from the network
__device__ __forceinline__ bool mlp_active(const CacheDev& c, const IterDev& it) {
  return it.alloc == 3 && c.mlp_y != nullptr;
}
__device__ __forceinline__ void mlp_counts(const CacheDev& c, const IterDev& it, size_t e, f3 T,
                                           const float* It, float beta[3]) {
  if (!mlp_active(c, it)) return;
  mlp_apply(it, T, It, c.mlp_y + e * 4, beta);
}

// training vertices for the learned cache: a seeded random subset.  The
// wave's recording lanes take their slots with one atomic: the first adds
// their number, each lane counts the recording lanes below it.
__device__ __forceinline__ void mlp_record(const CacheDev& c, uint2 strm, f3 x, uint32_t pix, f3 n,
                                           f3 T) {
  if (!c.mlp_rec || (strm.x >> 8) >= c.mlp_keep) return;
  const uint64_t m = __ballot(1);
  const uint32_t first = (uint32_t)__builtin_ctzll(m);
  uint32_t base = 0u;
  if (__lane_id() == first) base = atomicAdd(c.mlp_n_rec, (uint32_t)__popcll(m));
  base = (uint32_t)__builtin_amdgcn_readlane((int)base, (int)first);
  const uint32_t k =
      base + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
  if (k >= c.mlp_rec_cap) return;
  c.mlp_rec[3 * (size_t)k] = make_float4(x.x, x.y, x.z, __uint_as_float(pix));
  c.mlp_rec[3 * (size_t)k + 1] = make_float4(n.x, n.y, n.z, 0.0f);
  c.mlp_rec[3 * (size_t)k + 2] = make_float4(T.x, T.y, T.z, 0.0f);
}

// ---------------------------------------------------------------------------
// shading of unidirectional paths (Sec. 3.1, Sec. 4): emission with its
// direct-light MIS weight, cell lookup, counts, Alg. 1 rounding, and the
// samples of every technique: NEE (shadow queue), BSDF and guided
// (continuation queue).  Balance heuristic over {B,N,G} for direct light and
// {B,G} for indirect light; budget-aware multiplies every density by beta.
// Child throughput T' = T B|cos| / p_t * w_ind,t / beta_t (Sec. 3.1).
// ---------------------------------------------------------------------------
// Vertex state shared with the sample phase of shade_pt_kernel (SoA, one
// column per thread of the group) and the group's inclusive prefix sums of
// its NEE, BSDF and guided sample counts.
struct ShadeVerts {
  float ov[3][kShadePtBlock], ns[3][kShadePtBlock], wo[3][kShadePtBlock], T[3][kShadePtBlock],
      beta[3][kShadePtBlock];
  uint32_t s0[kShadePtBlock], s1[kShadePtBlock], cell[kShadePtBlock], mat[kShadePtBlock],
      j[kShadePtBlock], root[kShadePtBlock], sfirst[kShadePtBlock], cfirst[kShadePtBlock];
  uint32_t pre[3][kShadePtBlock];
};

// inclusive prefix sums over the group of three per-thread counts, into
// pre[0..2][thread]; lds: 3 * kThreads / 64 words.  Every thread must call it.
template <int kThreads>
__device__ __forceinline__ void group_scan3(uint32_t a, uint32_t b, uint32_t c,
                                            uint32_t (&pre)[3][kThreads], uint32_t* lds) {
  constexpr int kW = kThreads / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t ia = wave_scan_incl(a), ib = wave_scan_incl(b), ic = wave_scan_incl(c);
  if (lane == 63) {
    lds[wid] = ia;
    lds[kW + wid] = ib;
    lds[2 * kW + wid] = ic;
  }
  __syncthreads();
  uint32_t oa = 0, ob = 0, oc = 0;
  for (int w = 0; w < wid; ++w) {
    oa += lds[w];
    ob += lds[kW + w];
    oc += lds[2 * kW + w];
  }
  pre[0][threadIdx.x] = oa + ia;
  pre[1][threadIdx.x] = ob + ib;
  pre[2][threadIdx.x] = oc + ic;
  __syncthreads();
}

// the thread (vertex) that owns sample i of the group: the first v with
// pre[v] > i, and the sample's index among that vertex's samples
template <int kThreads>
__device__ __forceinline__ uint32_t owner_of(const uint32_t* pre, uint32_t i, uint32_t* k) {
  int lo = 0, hi = kThreads - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (i < pre[mid]) hi = mid; else lo = mid + 1;
  }
  *k = i - (lo > 0 ? pre[lo - 1] : 0u);
  return (uint32_t)lo;
}

// Unidirectional shading of depth d.  Vertex phase, one thread per queue
// entry: emission, cell, counts, rounding, queue allocation.  Sample phase:
// the group's NEE, BSDF and guided samples are dealt to its threads, one
// sample per thread at a time, so that a vertex that splits into many samples
// does not hold its wave; each sample computes exactly what it would on its
// vertex's thread and writes the same queue slot.
__global__ __launch_bounds__(kShadePtBlock) __attribute__((amdgpu_waves_per_eu(6, 8))) void shade_pt_kernel(SceneDev sc, CacheDev c, QueuesDev q,
                                                       Counters* cnt, IterDev it, ImageDev img,
                                                       DebugRec* dbg, uint32_t dbg_cap, int d) {
  __shared__ ShadeVerts sv;
  __shared__ uint32_t alloc_lds[4 * kShadePtBlock / 64 + 2];
  if (group_overflowed(cnt)) return;
  const Key key{sc.key0, sc.key1};
  const uint32_t n = min(cnt->n_ray[d], (uint32_t)q.cap);
  const int lane = threadIdx.x & 63;
  const size_t L = (size_t)d * q.cap, Ln = (size_t)(d + 1) * q.cap;
  const bool guided = sc.mode == 1;
  uint32_t my_vert = 0, my_samp = 0, my_ext = 0, my_sh = 0;
  for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
    const uint32_t j = base + threadIdx.x;
    const bool active = j < n;
    bool vert = false;
    f3 Ew = mk3(0.0f, 0.0f, 0.0f);
    uint32_t cell = kNoCell;
    float beta[3] = {0.0f, 0.0f, 0.0f};
    uint32_t gam[3] = {0u, 0u, 0u};
    f3 x = mk3(0, 0, 0), n_s = mk3(0, 0, 0), wo = mk3(0, 0, 0), T = mk3(0, 0, 0), ov = mk3(0, 0, 0);
    uint32_t prim = kMiss, pix = 0, root = 0;
    uint2 strm = make_uint2(0, 0);
    float It[3] = {1.0f, 1.0f, 1.0f};
    if (active) {
      const uint2 h = q.H[L + j];
      prim = h.y;
      const float4 r1 = q.R1[L + j];
      pix = ubits(r1.w);
      const uint4 s3 = q.S3[L + j];
      root = s3.w;
      if (prim != kMiss) {
        const float t = fbits(h.x);
        const float4 r0 = q.R0[L + j];
        const f3 dir = xyz(r1);
        const float4 ngl = sc.tri_ng[prim];
        const f3 ng = xyz(ngl);
        const float* m = sc.mats + 8 * (size_t)sc.tri_mat[prim];
        x = mk3(r0.x + t * dir.x, r0.y + t * dir.y, r0.z + t * dir.z);
        const float cosl = -dot3(dir, ng);
        if (cosl > 0.0f && (m[5] > 0.0f || m[6] > 0.0f || m[7] > 0.0f)) {
          if (d == 1) {
            Ew = mk3(m[5], m[6], m[7]);
          } else {
            const float4 s2 = q.S2[L + j];
            const float pN = (ngl.w * (t * t)) / cosl;
            const float w = s2.x / (s2.y + s2.z * pN);
            Ew = mk3(w * m[5], w * m[6], w * m[7]);
          }
        }
        if (d < sc.max_depth) {
          vert = true;
          n_s = dot3(ng, dir) < 0.0f ? ng : mk3(-ng.x, -ng.y, -ng.z);
          wo = mk3(-dir.x, -dir.y, -dir.z);
          ov = mk3(x.x + n_s.x * sc.eps, x.y + n_s.y * sc.eps, x.z + n_s.z * sc.eps);
          cell = cell_of(c.nodes, mk3(sc.oct_lo[0], sc.oct_lo[1], sc.oct_lo[2]), sc.oct_inv, x);
          const float4 s0 = q.S0[L + j];
          T = xyz(s0);
          It[0] = img.itilde[3 * (size_t)pix];
          It[1] = img.itilde[3 * (size_t)pix + 1];
          It[2] = img.itilde[3 * (size_t)pix + 2];
          counts_at(sc, c, it, cell, T, It, d, beta);
          mlp_counts(c, it, L + j, T, It, beta);
          strm = make_uint2(s3.x, s3.y);
          const float4 u = draw4(key, strm, 0);
          if (it.rounding) round_counts_independent(beta, u, gam);
          else round_counts(beta, u.x, gam);
          mlp_record(c, strm, x, pix, ng, T);
        }
      }
    }
    const uint32_t ncont = vert ? gam[0] + gam[2] : 0u, nnee = vert ? gam[1] : 0u;
    // workgroup-level allocation in the next-depth and shadow queues
    uint32_t cfirst, sfirst;
    group_alloc<kShadePtBlock>(ncont, nnee, &cnt->n_ray[d + 1], &cnt->n_shadow[d], &cfirst, &sfirst,
                             alloc_lds);
    bool ovf = false;
    if (vert && ((size_t)cfirst + ncont > q.cap || (size_t)sfirst + nnee > q.scap)) {
      ovf = true;
      atomicMax(&cnt->overflow, 1u);
      atomicMax(&cnt->overflow_any, 1u);
    }
    const bool live = active && vert && !ovf;
    if (active) {
      q.V0[L + j] = make_float4(Ew.x, Ew.y, Ew.z, fbits(cell));
      q.V1[L + j] = make_float4(beta[0], beta[1], beta[2], 0.0f);
      q.V2[L + j] = ovf ? make_uint4(0, 0, 0, 0) : make_uint4(sfirst, nnee, cfirst, ncont);
      if (d == 1) {
        img.beta1[3 * (size_t)root] = beta[0];
        img.beta1[3 * (size_t)root + 1] = beta[1];
        img.beta1[3 * (size_t)root + 2] = beta[2];
      }
    }
    if (live) {
      ++my_vert;
      my_samp += gam[0] + gam[1] + gam[2];
      if (d <= it.debug_depth && dbg) {
        const uint32_t k = atomicAdd(&cnt->n_debug, 1u);
        if (k < dbg_cap) {
          DebugRec r;
          r.root = root; r.depth = (uint32_t)d; r.stream_lo = strm.x; r.stream_hi = strm.y;
          r.cell = cell;
          for (int t = 0; t < 3; ++t) { r.beta[t] = beta[t]; r.gamma[t] = gam[t]; }
          r.T[0] = T.x; r.T[1] = T.y; r.T[2] = T.z;
          dbg[k] = r;
        }
      }
      const int t = threadIdx.x;
      sv.ov[0][t] = ov.x; sv.ov[1][t] = ov.y; sv.ov[2][t] = ov.z;
      sv.ns[0][t] = n_s.x; sv.ns[1][t] = n_s.y; sv.ns[2][t] = n_s.z;
      sv.wo[0][t] = wo.x; sv.wo[1][t] = wo.y; sv.wo[2][t] = wo.z;
      sv.T[0][t] = T.x; sv.T[1][t] = T.y; sv.T[2][t] = T.z;
      sv.beta[0][t] = beta[0]; sv.beta[1][t] = beta[1]; sv.beta[2][t] = beta[2];
      sv.s0[t] = strm.x; sv.s1[t] = strm.y;
      sv.cell[t] = cell;
      sv.mat[t] = sc.tri_mat[prim];
      sv.j[t] = j;
      sv.root[t] = root;
      sv.sfirst[t] = sfirst;
      sv.cfirst[t] = cfirst;
    }
    group_scan3<kShadePtBlock>(live ? gam[1] : 0u, live ? gam[0] : 0u, live ? gam[2] : 0u, sv.pre,
                               alloc_lds);
    const uint32_t nN = sv.pre[0][kShadePtBlock - 1], nB = sv.pre[1][kShadePtBlock - 1],
                   nG = sv.pre[2][kShadePtBlock - 1];
    // NEE: light by power, uniform point on the triangle
    for (uint32_t i = threadIdx.x; i < nN; i += kShadePtBlock) {
      uint32_t k;
      const uint32_t v = owner_of<kShadePtBlock>(sv.pre[0], i, &k);
      const uint2 ss = stream_child(key, make_uint2(sv.s0[v], sv.s1[v]), 1u, k, (uint32_t)d);
      const float4 u = draw4(key, ss, 1);
      int lo = 0, hi = sc.n_lights - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (u.x < sc.light_cdf[mid]) hi = mid; else lo = mid + 1;
      }
      const int lt = sc.light_tri[lo];
      const float4* G = sc.tri_geo + (size_t)lt * 3;
      const f3 v0 = xyz(G[0]), e1 = xyz(G[1]), e2 = xyz(G[2]);
      const float su = sqrtf(u.y);
      const float a = su * (1.0f - u.z), b = su * u.z;
      const f3 y = mk3((v0.x + a * e1.x) + b * e2.x, (v0.y + a * e1.y) + b * e2.y,
                       (v0.z + a * e1.z) + b * e2.z);
      const f3 vo = mk3(sv.ov[0][v], sv.ov[1][v], sv.ov[2][v]);
      const f3 dv = sub3(y, vo);
      const float d2 = dot3(dv, dv);
      const float dist = sqrtf(d2);
      const f3 w = scl3(dv, 1.0f / dist);
      const float4 lng = sc.tri_ng[lt];
      const float cl = -dot3(w, xyz(lng));
      const Mat mat = load_mat(sc.mats + 8 * (size_t)sv.mat[v]);
      f3 fc;
      float pB;
      eval_bsdf(mat, mk3(sv.ns[0][v], sv.ns[1][v], sv.ns[2][v]),
                mk3(sv.wo[0][v], sv.wo[1][v], sv.wo[2][v]), w, &fc, &pB);
      float4 sh2 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (cl > 0.0f && (fc.x > 0.0f || fc.y > 0.0f || fc.z > 0.0f)) {
        const float b0 = sv.beta[0][v], b1 = sv.beta[1][v], b2 = sv.beta[2][v];
        const float bB = it.aware ? b0 : (b0 > 0.0f ? 1.0f : 0.0f);
        const float bN = it.aware ? b1 : (b1 > 0.0f ? 1.0f : 0.0f);
        const float bG = it.aware ? b2 : (b2 > 0.0f ? 1.0f : 0.0f);
        const float pN = (lng.w * d2) / cl;
        const float pG = guided ? guided_density(c.pm + 64 * (size_t)sv.cell[v], w) : 0.0f;
        const float nb = bB * pB, nn = bN * pN, ngd = bG * pG;
        const float ddir = (nb + ngd) + nn;
        const float wN = ddir > 0.0f ? nn / ddir : 0.0f;
        const float* Le = sc.mats + 8 * (size_t)sc.tri_mat[lt] + 5;
        sh2 = make_float4((fc.x / pN) * (wN * Le[0]), (fc.y / pN) * (wN * Le[1]),
                          (fc.z / pN) * (wN * Le[2]), 1.0f);
        ++my_sh;
      }
      const size_t e = sv.sfirst[v] + k;
      q.SH0[e] = make_float4(vo.x, vo.y, vo.z, dist * (1.0f - 1e-3f));
      q.SH1[e] = make_float4(w.x, w.y, w.z, fbits(sv.j[v]));
      q.SH2[(size_t)d * q.scap + e] = sh2;
    }
    // continuation: BSDF samples (slots 0..) then guided samples (after the
    // vertex's BSDF samples)
    for (int tech = 0; tech < 3; tech += 2) {
      const uint32_t* pre = sv.pre[tech == 0 ? 1 : 2];
      const uint32_t nt = tech == 0 ? nB : nG;
      for (uint32_t i = threadIdx.x; i < nt; i += kShadePtBlock) {
        uint32_t k;
        const uint32_t v = owner_of<kShadePtBlock>(pre, i, &k);
        const uint2 ss = stream_child(key, make_uint2(sv.s0[v], sv.s1[v]), (uint32_t)tech, k,
                                      (uint32_t)d);
        const float4 u = draw4(key, ss, 1);
        const Mat mat = load_mat(sc.mats + 8 * (size_t)sv.mat[v]);
        const f3 ns = mk3(sv.ns[0][v], sv.ns[1][v], sv.ns[2][v]);
        const f3 wo = mk3(sv.wo[0][v], sv.wo[1][v], sv.wo[2][v]);
        const uint32_t cl = sv.cell[v];
        f3 w;
        bool ok;
        if (tech == 0) {
          ok = sample_bsdf(mat, ns, wo, u.x, u.y, &w);
        } else {
          w = guided_direction(c.cdf + 64 * (size_t)cl, u.x, u.y, u.z);
          ok = dot3(ns, w) > 0.0f;
        }
        f3 fc = mk3(0.0f, 0.0f, 0.0f);
        float pB = 0.0f, pG = 0.0f, pt = 0.0f;
        if (ok) {
          eval_bsdf(mat, ns, wo, w, &fc, &pB);
          pG = guided ? guided_density(c.pm + 64 * (size_t)cl, w) : 0.0f;
          pt = tech == 0 ? pB : pG;
          ok = (fc.x > 0.0f || fc.y > 0.0f || fc.z > 0.0f) && pt > 0.0f;
        }
        // guided samples follow the vertex's BSDF samples
        const uint32_t nb0 = sv.pre[1][v] - (v > 0 ? sv.pre[1][v - 1] : 0u);
        const uint32_t slot = tech == 0 ? k : nb0 + k;
        const size_t e = Ln + sv.cfirst[v] + slot;
        const f3 vo = mk3(sv.ov[0][v], sv.ov[1][v], sv.ov[2][v]);
        const uint32_t vj = sv.j[v], vroot = sv.root[v];
        const uint32_t pix = vroot / (uint32_t)it.spp;
        const float bt = sv.beta[tech][v];
        if (ok) {
          const float b0 = sv.beta[0][v], b1 = sv.beta[1][v], b2 = sv.beta[2][v];
          const float bB = it.aware ? b0 : (b0 > 0.0f ? 1.0f : 0.0f);
          const float bN = it.aware ? b1 : (b1 > 0.0f ? 1.0f : 0.0f);
          const float bG = it.aware ? b2 : (b2 > 0.0f ? 1.0f : 0.0f);
          const float nb = bB * pB, ngd = bG * pG;
          const float dind = nb + ngd;
          const float wind = dind > 0.0f ? (tech == 0 ? nb : ngd) / dind : 0.0f;
          const float dsum = bB * pB + bG * pG;
          const float c0 = fc.x / pt, c1 = fc.y / pt, c2 = fc.z / pt;
          const f3 Tc = mk3(sv.T[0][v] * ((c0 * wind) / bt), sv.T[1][v] * ((c1 * wind) / bt),
                            sv.T[2][v] * ((c2 * wind) / bt));
          q.R0[e] = make_float4(vo.x, vo.y, vo.z, 1.0f);
          q.R1[e] = make_float4(w.x, w.y, w.z, fbits(pix));
          q.S0[e] = make_float4(Tc.x, Tc.y, Tc.z, fbits(vj));
          q.S1[e] = make_float4(c0, c1, c2, wind);
          q.S2[e] = make_float4((tech == 0 ? bB : bG) * pt, dsum, bN, bt);
          ++my_ext;
        } else {
          q.R0[e] = make_float4(vo.x, vo.y, vo.z, 0.0f);
          q.R1[e] = make_float4(w.x, w.y, w.z, fbits(pix));
          q.S0[e] = make_float4(0.0f, 0.0f, 0.0f, fbits(vj));
          q.S1[e] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
          q.S2[e] = make_float4(0.0f, 0.0f, 0.0f, bt);
        }
        q.S3[e] = make_uint4(ss.x, ss.y, ((uint32_t)tech << 16) | k, vroot);
      }
    }
    // the next round of the loop overwrites the shared vertex state
    __syncthreads();
  }
  // one atomic per wave for the iteration counters
  group_add<kShadePtBlock, 4>({my_vert, my_samp, my_ext, my_sh},
                            {&cnt->vertices, &cnt->samples, &cnt->rays_ext, &cnt->rays_shadow},
                            alloc_lds);
}
void k_shade_pt(const SceneDev& sc, const CacheDev& c, const QueuesDev& q, Counters* cnt,
                const IterDev& it, const ImageDev& img, DebugRec* dbg, uint32_t dbg_cap, int d,
                int grid, hipStream_t s) {
  shade_pt_kernel<<<grid * 256 / kShadePtBlock * 6 / 8, kShadePtBlock, 0, s>>>(sc, c, q, cnt, it, img,
                                                                              dbg, dbg_cap, d);
}

// ---------------------------------------------------------------------------
// back-propagation over the path tree (Sec. 3.1 "Secondary estimator"):
//   R(vertex) = sum_t (1/beta_t) sum_s v_s,
//   v_s = B|cos|/p_t (w_dir,t E' + w_ind,t R')   (continuation samples),
//   v_s = B|cos|/p_N w_dir,N Le                   (NEE samples, 0 if occluded)
// summed in the order NEE, BSDF, guided.  Every sample also feeds the cell's
// moment and cost accumulators (Sec. 4.1 "Local estimates"); continuation
// samples train the directional histogram of the guided technique.  The
// launches run from the deepest depth up; the launch of depth d computes the
// value, cost and histogram training of each of its entries as a sample of
// its parent, so that the parent's fold over its samples (in their order)
// reads one record per sample.
// ---------------------------------------------------------------------------
// Cell statistics are first summed per vertex (all samples of a vertex fall
// in its cell), then merged per workgroup in an LDS hash table keyed by
// (cell, technique), and flushed with one set of global binary64 atomics per
// table slot.  A workgroup walks a contiguous range of the queue, so
// neighbouring vertices (often in the same cell) share slots; keys that find
// no slot within a few probes go straight to global memory.
constexpr int kAggSlots = 256;
constexpr int kAggVals = 9;  // sum v (3), sum v^2 (3), n, cost, visits
constexpr uint32_t kAggEmpty = 0xFFFFFFFFu;

struct AggTable {
  uint32_t key[kAggSlots];
  double val[kAggSlots][kAggVals];
};

// key = cell << 3 | technique; techniques 3 and 4 (per-length light paths)
// live in acc_x
__device__ __forceinline__ void global_add_stats(const CacheDev& c, uint32_t key, const double* v) {
  const uint32_t cell = key >> 3, t = key & 7u;
  double* a = t < 3u ? c.acc + ((size_t)cell * 3 + t) * 8 : c.acc_x + ((size_t)cell * 2 + (t - 3u)) * 8;
#pragma unroll
  for (int i = 0; i < 8; ++i)
    if (v[i] != 0.0) atomicAdd(a + i, v[i]);
  if (v[8] != 0.0) atomicAdd(c.visits + cell, (uint32_t)v[8]);
}

__device__ __forceinline__ void agg_add(AggTable& A, const CacheDev& c, uint32_t key,
                                        const double* v) {
  uint32_t h = (key * 2654435761u) >> 24;  // 8 bits
#pragma unroll 1
  for (int probe = 0; probe < 8; ++probe) {
    const uint32_t prev = atomicCAS(&A.key[h], kAggEmpty, key);
    if (prev == kAggEmpty || prev == key) {
#pragma unroll
      for (int i = 0; i < kAggVals; ++i)
        if (v[i] != 0.0) atomicAdd(&A.val[h][i], v[i]);
      return;
    }
    h = (h + 1) & (kAggSlots - 1);
  }
  global_add_stats(c, key, v);
}

__global__ __launch_bounds__(256) void backprop_pt_kernel(SceneDev sc, CacheDev c, QueuesDev q,
                                                          const Counters* cnt, IterDev it,
                                                          ImageDev img, int d) {
  __shared__ AggTable A;
  // an overflowed tile left child ranges unwritten: it is rendered again
  if (cnt->overflow) return;
  for (int k = threadIdx.x; k < kAggSlots; k += blockDim.x) {
    A.key[k] = kAggEmpty;
    for (int i = 0; i < kAggVals; ++i) A.val[k][i] = 0.0;
  }
  __syncthreads();
  const uint32_t n = min(cnt->n_ray[d], (uint32_t)q.cap);
  const size_t L = (size_t)d * q.cap, Ln = (size_t)(d + 1) * q.cap;
  const bool guided = sc.mode == 1;
  const uint32_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const uint32_t j0 = blockIdx.x * chunk, j1 = min(n, j0 + chunk);
  for (uint32_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
    const float4 v0 = q.V0[L + j];
    const uint32_t cell = ubits(v0.w);
    f3 R = mk3(0.0f, 0.0f, 0.0f);
    uint32_t cost = 0;
    if (cell != kNoCell) {
      double st[3][8];
#pragma unroll
      for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int i = 0; i < 8; ++i) st[t][i] = 0.0;
      const uint4 v2 = q.V2[L + j];
      const float4 b = q.V1[L + j];
      const f3 T = xyz(q.S0[L + j]);
      const uint32_t pix = ubits(q.R1[L + j].w);
      float lim[3] = {INFINITY, INFINITY, INFINITY};
      if (it.stat_clamp > 0.0f) {
        const float k = it.stat_clamp;
        lim[0] = (k * img.itilde[3 * (size_t)pix]) / T.x;
        lim[1] = (k * img.itilde[3 * (size_t)pix + 1]) / T.y;
        lim[2] = (k * img.itilde[3 * (size_t)pix + 2]) / T.z;
      }
      auto record = [&](int t, f3 v, uint32_t cst) {
        const double x0 = (double)fminf(v.x, lim[0]), x1 = (double)fminf(v.y, lim[1]),
                     x2 = (double)fminf(v.z, lim[2]);
        st[t][0] += x0; st[t][1] += x1; st[t][2] += x2;
        st[t][3] += x0 * x0; st[t][4] += x1 * x1; st[t][5] += x2 * x2;
        st[t][6] += 1.0; st[t][7] += (double)cst;
      };
      for (uint32_t k = 0; k < v2.y; ++k) {
        const f3 v = xyz(q.SH2[(size_t)d * q.scap + v2.x + k]);
        R = mk3(R.x + v.x / b.y, R.y + v.y / b.y, R.z + v.z / b.y);
        cost += 1;
        record(1, v, 1u);
      }
      for (uint32_t k = 0; k < v2.w; ++k) {
        // the sample's value and cost, left by the launch of the next depth
        const size_t e = Ln + v2.z + k;
        const float4 sv = q.RO[e];
        const float bt = q.S2[e].w;
        const uint32_t tech = q.S3[e].z >> 16;
        const f3 v = xyz(sv);
        const uint32_t sc_ = ubits(sv.w);
        R = mk3(R.x + v.x / bt, R.y + v.y / bt, R.z + v.z / bt);
        cost += sc_;
        record(tech == 0 ? 0 : 2, v, sc_);
      }
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        if (t != 0 && st[t][6] == 0.0) continue;
        double vals[kAggVals];
#pragma unroll
        for (int i = 0; i < 8; ++i) vals[i] = st[t][i];
        vals[8] = t == 0 ? 1.0 : 0.0;
        agg_add(A, c, (cell << 3) | (uint32_t)t, vals);
      }
    }
    if (d >= 2) {
      // this entry as a continuation sample of its parent vertex (depth
      // d - 1): v = B|cos|/p_t (w_dir,t E' + w_ind,t R') with the factors
      // the parent stored, and its cost 1 + the cost of this subtree (1 for
      // a sample whose direction was rejected).  The parent's pass reads
      // the pair with one load.  A guided parent's directional histogram is
      // trained here, with the incident radiance E + R' over the density of
      // its continuation samples.
      f3 v = mk3(0.0f, 0.0f, 0.0f);
      uint32_t sc_ = 1u;
      if (q.R0[L + j].w != 0.0f) {
        const float4 s1 = q.S1[L + j];
        v = mk3(s1.x * (v0.x + s1.w * R.x), s1.y * (v0.y + s1.w * R.y), s1.z * (v0.z + s1.w * R.z));
        sc_ = 1u + cost;
        if (guided) {
          const float dsum = q.S2[L + j].y;
          if (dsum > 0.0f) {
            f3 E = mk3(0.0f, 0.0f, 0.0f);
            const uint2 h = q.H[L + j];
            const f3 dir = xyz(q.R1[L + j]);
            if (h.y != kMiss) {
              const float* m = sc.mats + 8 * (size_t)sc.tri_mat[h.y];
              const float cosl = -dot3(dir, xyz(sc.tri_ng[h.y]));
              if (cosl > 0.0f && (m[5] > 0.0f || m[6] > 0.0f || m[7] > 0.0f))
                E = mk3(m[5], m[6], m[7]);
            }
            const f3 Li = add3(E, R);
            const uint32_t pcell =
                ubits(q.V0[(size_t)(d - 1) * q.cap + ubits(q.S0[L + j].w)].w);
            atomicAdd(c.hacc + (size_t)pcell * 64 + dir_bin(dir), (double)(lum(Li) / dsum));
          }
        }
      }
      q.RO[L + j] = make_float4(v.x, v.y, v.z, fbits(sc_));
    }
    if (d == 1) {
      const uint32_t root = q.S3[L + j].w;
      img.Ls[3 * (size_t)root] = v0.x + R.x;
      img.Ls[3 * (size_t)root + 1] = v0.y + R.y;
      img.Ls[3 * (size_t)root + 2] = v0.z + R.z;
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kAggSlots; k += blockDim.x) {
    if (A.key[k] == kAggEmpty) continue;
    double vals[kAggVals];
    for (int i = 0; i < kAggVals; ++i) vals[i] = A.val[k][i];
    global_add_stats(c, A.key[k], vals);
  }
}
void k_backprop_pt(const SceneDev& sc, const CacheDev& c, const QueuesDev& q, const Counters* cnt,
                   const IterDev& it, const ImageDev& img, int d, hipStream_t s) {
  backprop_pt_kernel<<<resident_grid(backprop_pt_kernel, 256), 256, 0, s>>>(sc, c, q, cnt, it, img, d);
}

// ---------------------------------------------------------------------------
// Bidirectional path tracing (Sec. 5).  Techniques per camera vertex: BSDF
// continuation, NEE, light-path connections (LP), each with its own count.
// One light subpath per camera sample with throughput RR only (no splitting
// on the light side).  LP sample j connects to light subpath
// (root + j * stride) mod N, to every vertex y_i (i >= 1) that keeps the path
// length within D.  MIS is the full-path balance heuristic over strategies
// (s, t), t >= 2; the budget-aware form weights strategy (s, t) by
// prod_{j <= t-2} beta_B(z_j) * beta_tech(s)(z_{t-1}).  The weight is a
// function of the path vertices only: counts of every vertex, also of those
// on the light side, come from the camera-prefix throughput computed from
// vertex positions.
// ---------------------------------------------------------------------------
struct PV {
  f3 P, ng;
  uint32_t mat;
  float lpdf;
};

__device__ __forceinline__ f3 dir_between(f3 a, f3 b, float* d2) {
  const f3 dv = sub3(b, a);
  *d2 = dot3(dv, dv);
  const float dist = sqrtf(*d2);
  return scl3(dv, 1.0f / dist);
}

__device__ __forceinline__ void eval_facing(const Mat& m, f3 ng, f3 wo, f3 wi, f3* fc, float* pdf) {
  const f3 n = dot3(ng, wo) > 0.0f ? ng : mk3(-ng.x, -ng.y, -ng.z);
  eval_bsdf(m, n, wo, wi, fc, pdf);
}

__device__ __forceinline__ PV prim_vertex(const SceneDev& sc, f3 P, uint32_t prim) {
  const float4 ng = sc.tri_ng[prim];
  return PV{P, xyz(ng), sc.tri_mat[prim], ng.w};
}

// per-vertex record of a camera vertex (see bdpt_record): the camera-prefix
// throughput recomputed from positions, the counts there, pF and pR terms
struct VRec {
  f3 T;
  float b0, b1, b2, pF, pRg;
  float b3, b4;  // per-length light paths: the y_2 and y_3+ classes (else unused)
};
__device__ __forceinline__ VRec load_rec(const QueuesDev& q, int l, uint32_t e) {
  const size_t a = (size_t)l * q.cap + e;
  const float4 w0 = q.W0[a], w1 = q.W1[a];
  const float4 w2 = q.W2 ? q.W2[a] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  return VRec{xyz(w0), w0.w, w1.x, w1.y, w1.z, w1.w, w2.x, w2.y};
}
__device__ __forceinline__ float mis_count(const IterDev& it, float b) {
  return it.aware ? b : (b > 0.0f ? 1.0f : 0.0f);
}

// light subpaths: emission point by power, cosine direction; the light
// queue lives at depth 0 of the queues: R0 origin/flag, R1 direction/root,
// S0 alpha, S1 RR throughput
__global__ void light_start_kernel(SceneDev sc, QueuesDev q, LightDev lt, Counters* cnt,
                                   IterDev it, uint32_t root0, uint32_t n) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0) cnt->n_ray[0] = n;
  if (j >= n) return;
  const Key key{sc.key0, sc.key1};
  const uint32_t root = root0 + j;
  lt.len[root] = make_uint2(0u, 0u);
  q.R0[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  q.R1[j] = make_float4(0.0f, 0.0f, 0.0f, fbits(root));
  if (sc.n_lights == 0) return;
  const uint32_t pix = root / (uint32_t)it.spp, s = root % (uint32_t)it.spp;
  const uint2 st = stream_root(key, pix, s, (uint32_t)iter_index(it), kTagLight);
  const float4 u = draw4(key, st, 0), u2 = draw4(key, st, 1);
  int lo = 0, hi = sc.n_lights - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (u.x < sc.light_cdf[mid]) hi = mid; else lo = mid + 1;
  }
  const int li = sc.light_tri[lo];
  const float4* G = sc.tri_geo + (size_t)li * 3;
  const f3 v0 = xyz(G[0]), e1 = xyz(G[1]), e2 = xyz(G[2]);
  const float su = sqrtf(u.y);
  const float a = su * (1.0f - u.z), b = su * u.z;
  const f3 y0 = mk3((v0.x + a * e1.x) + b * e2.x, (v0.y + a * e1.y) + b * e2.y,
                    (v0.z + a * e1.z) + b * e2.z);
  lt.Y0[root] = make_float4(y0.x, y0.y, y0.z, fbits((uint32_t)li));
  if (lt.lmax <= 0) return;
  const float4 ngl = sc.tri_ng[li];
  const f3 nl = xyz(ngl);
  const float* ml = sc.mats + 8 * (size_t)sc.tri_mat[li];
  f3 tt, bb;
  frame(nl, &tt, &bb);
  float sn, cs;
  const float r = sqrtf(u2.x);
  sincos_turns(u2.y, &sn, &cs);
  const f3 w = local_to_world(mk3(r * cs, r * sn, sqrtf(fmaxf(0.0f, 1.0f - u2.x))), tt, bb, nl);
  q.R0[j] = make_float4(y0.x + nl.x * sc.eps, y0.y + nl.y * sc.eps, y0.z + nl.z * sc.eps, 1.0f);
  q.R1[j] = make_float4(w.x, w.y, w.z, fbits(root));
  q.S0[j] = make_float4((ml[5] * kPi) / ngl.w, (ml[6] * kPi) / ngl.w, (ml[7] * kPi) / ngl.w, 0.0f);
  q.S1[j] = make_float4(1.0f, 1.0f, 1.0f, 0.0f);
}
void k_light_start(const SceneDev& sc, const QueuesDev& q, const LightDev& lt, Counters* cnt,
                   const IterDev& it, uint32_t root0, uint32_t n, hipStream_t s) {
  light_start_kernel<<<(n + 255) / 256, 256, 0, s>>>(sc, q, lt, cnt, it, root0, n);
}

// stores light vertex y_i and continues with throughput RR and BSDF sampling
__global__ void light_shade_kernel(SceneDev sc, const uint32_t* __restrict__ oct_nodes, QueuesDev q,
                                   LightDev lt, Counters* cnt, IterDev it, int i) {
  const uint32_t n = min(cnt->n_ray[0], (uint32_t)q.cap);
  const Key key{sc.key0, sc.key1};
  uint32_t my_rays = 0;
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const float4 r0 = q.R0[j];
    if (r0.w == 0.0f) continue;
    ++my_rays;
    const float4 r1 = q.R1[j];
    const uint32_t root = ubits(r1.w);
    const uint2 h = q.H[j];
    if (h.y == kMiss) {
      q.R0[j] = make_float4(r0.x, r0.y, r0.z, 0.0f);
      lt.len[root] = make_uint2(lt.len[root].x, lt.len[root].y + 1u);
      continue;
    }
    const float t = fbits(h.x);
    const f3 w = xyz(r1);
    const f3 x = mk3(r0.x + t * w.x, r0.y + t * w.y, r0.z + t * w.z);
    const f3 wo = mk3(-w.x, -w.y, -w.z);
    const float4 al = q.S0[j];
    const size_t e = (size_t)root * lt.lmax + (i - 1);
    lt.V0[e] = make_float4(x.x, x.y, x.z, fbits(h.y));
    lt.V1[e] = make_float4(wo.x, wo.y, wo.z, al.x);
    // the octree cell of y_i, which every connection to it evaluates counts
    // in (the octree is fixed until the iteration's update)
    const uint32_t ycell =
        cell_of(oct_nodes, mk3(sc.oct_lo[0], sc.oct_lo[1], sc.oct_lo[2]), sc.oct_inv, x);
    lt.V2[e] = make_float4(al.y, al.z, fbits(ycell), 0.0f);
    lt.len[root] = make_uint2((uint32_t)i, lt.len[root].y + 1u);
    bool alive = false;
    if (i < lt.lmax) {
      const uint32_t pix = root / (uint32_t)it.spp, s = root % (uint32_t)it.spp;
      const uint2 st = stream_root(key, pix, s, (uint32_t)iter_index(it), kTagLight);
      const float4 u = draw4(key, st, (uint32_t)(1 + i));
      const float4 rr = q.S1[j];
      const float qv = fminf(1.0f, fmaxf(fmaxf(rr.x, rr.y), rr.z));
      if (u.x < qv) {
        const float4 ngl = sc.tri_ng[h.y];
        const f3 ng = xyz(ngl);
        const f3 nn = dot3(ng, wo) > 0.0f ? ng : mk3(-ng.x, -ng.y, -ng.z);
        const Mat mat = load_mat(sc.mats + 8 * (size_t)sc.tri_mat[h.y]);
        f3 wn;
        if (sample_bsdf(mat, nn, wo, u.y, u.z, &wn)) {
          f3 fc;
          float p;
          eval_bsdf(mat, nn, wo, wn, &fc, &p);
          if (p > 0.0f && (fc.x > 0.0f || fc.y > 0.0f || fc.z > 0.0f)) {
            alive = true;
            q.S0[j] = make_float4(al.x * ((fc.x / p) / qv), al.y * ((fc.y / p) / qv),
                                  al.z * ((fc.z / p) / qv), 0.0f);
            q.S1[j] = make_float4(rr.x * (fc.x / p), rr.y * (fc.y / p), rr.z * (fc.z / p), 0.0f);
            q.R0[j] = make_float4(x.x + nn.x * sc.eps, x.y + nn.y * sc.eps, x.z + nn.z * sc.eps, 1.0f);
            q.R1[j] = make_float4(wn.x, wn.y, wn.z, r1.w);
          }
        }
      }
    }
    if (!alive) q.R0[j] = make_float4(r0.x, r0.y, r0.z, 0.0f);
  }
  const uint32_t sr = wave_sum(my_rays);
  if ((threadIdx.x & 63) == 0 && sr) atomicAdd(&cnt->rays_light, (unsigned long long)sr);
}
void k_light_shade(const SceneDev& sc, const CacheDev& c, const QueuesDev& q, const LightDev& lt,
                   Counters* cnt, const IterDev& it, int bounce, hipStream_t s) {
  light_shade_kernel<<<resident_grid(light_shade_kernel, 256), 256, 0, s>>>(sc, c.nodes, q, lt, cnt,
                                                                            it, bounce);
}

// ---------------------------------------------------------------------------
// Full-path MIS weights (Sec. 5) from per-vertex records.  The weight of
// strategy t of a path z_0..z_k is 1 / sum_s (beta_s p_s) / (beta_t p_t),
// summed as ratios in a fixed order: 1 for s = t, then s = t + 1 .. k + 1
// outward along the light side (each step multiplying pF / pR and the BSDF
// count of the vertex passed), then s = t - 1 .. 2 up the camera side.
// Every term that depends on camera vertices only (pF, pR, counts along the
// position-derived throughput) is computed once, when the vertex is shaded,
// and stored with it; terms that depend on light vertices only once per
// light vertex (light_walk_kernel); a NEE sample or connection evaluates
// only the terms that involve both sides.  Each term is computed by the same
// operations wherever it is evaluated, so the weight does not depend on
// where its terms come from.
// ---------------------------------------------------------------------------
// the hit vertex of queue entry e at level l
__device__ __forceinline__ PV hit_vertex(const SceneDev& sc, const QueuesDev& q, int l, uint32_t e) {
  const size_t a = (size_t)l * q.cap + e;
  const float4 a0 = q.R0[a], a1 = q.R1[a];
  const uint2 ah = q.H[a];
  const float at = fbits(ah.x);
  return prim_vertex(sc, mk3(a0.x + at * a1.x, a0.y + at * a1.y, a0.z + at * a1.z), ah.y);
}

// record of the camera vertex j at depth d (hit x with geometric normal ng,
// octree cell `cell`): pF[d] and pR[d-2] of any full path through it, the
// camera-prefix throughput recomputed from positions and the counts there
// (in learned-cache iterations the network's, as the vertex's samples use)
__device__ __forceinline__ void bdpt_record(const SceneDev& sc, const CacheDev& c,
                                            const QueuesDev& q, const IterDev& it, int d,
                                            uint32_t j, f3 x, f3 ng, uint32_t cell,
                                            const float* It) {
  f3 T = mk3(1.0f, 1.0f, 1.0f);
  float pF = 0.0f, pRg = 0.0f;
  if (d >= 2) {
    const uint32_t e1 = ubits(q.S0[(size_t)d * q.cap + j].w);
    const PV zp = hit_vertex(sc, q, d - 1, e1);
    f3 zpp;
    PV zg{};
    if (d == 2) {
      zpp = mk3(sc.cam_o[0], sc.cam_o[1], sc.cam_o[2]);
    } else {
      zg = hit_vertex(sc, q, d - 2, ubits(q.S0[(size_t)(d - 1) * q.cap + e1].w));
      zpp = zg.P;
    }
    const VRec rp = load_rec(q, d - 1, e1);
    const Mat mp = load_mat(sc.mats + 8 * (size_t)zp.mat);
    float d2;
    const f3 wo = dir_between(zp.P, zpp, &d2);
    const f3 wi = dir_between(zp.P, x, &d2);
    f3 fc;
    float p;
    eval_facing(mp, zp.ng, wo, wi, &fc, &p);
    pF = (p * fabsf(dot3(ng, wi))) / d2;
    if (p > 0.0f && rp.b0 > 0.0f)
      T = mk3(rp.T.x * (((fc.x / p) * 1.0f) / rp.b0), rp.T.y * (((fc.y / p) * 1.0f) / rp.b0),
              rp.T.z * (((fc.z / p) * 1.0f) / rp.b0));
    else
      T = mk3(0.0f, 0.0f, 0.0f);
    if (d >= 3) {
      const f3 wo2 = dir_between(zp.P, x, &d2);
      const f3 wi2 = dir_between(zp.P, zpp, &d2);
      f3 fc2;
      float p2;
      eval_facing(mp, zp.ng, wo2, wi2, &fc2, &p2);
      pRg = (p2 * fabsf(dot3(zg.ng, wi2))) / d2;
    }
  }
  float b[3];
  counts_at(sc, c, it, cell, T, It, d, b);
  const size_t a = (size_t)d * q.cap + j;
  if (mlp_active(c, it)) mlp_apply(it, T, It, c.mlp_y + a * 4, b);
  q.W0[a] = make_float4(T.x, T.y, T.z, b[0]);
  q.W1[a] = make_float4(b[1], b[2], pF, pRg);
  if (q.W2) {
    float bx[2];
    counts_at_x(c, it, cell, T, It, bx);
    q.W2[a] = make_float4(bx[0], bx[1], 0.0f, 0.0f);
  }
}

// a light vertex (or emitter point) as stored: position, primitive (bits)
__device__ __forceinline__ PV light_vertex(const SceneDev& sc, float4 v) {
  const uint32_t prim = ubits(v.w);
  const float4 ng = sc.tri_ng[prim];
  return PV{xyz(v), xyz(ng), sc.tri_mat[prim], ng.w};
}

// pR(i) of the path, from the window z_i (C), z_{i+1} (D), z_{i+2} (E): the
// density of reaching z_i from z_{i+1} (whose outgoing direction is towards
// z_{i+2}) as area density at z_i; z_k's emitter pdf and z_{k-1}'s emission
// density at the end of the path
__device__ __forceinline__ float path_pR(const SceneDev& sc, int i, int k, const PV& C,
                                         const PV& D, const PV& E) {
  float d2;
  if (i == k) return C.lpdf;
  if (i == k - 1) {
    const f3 w = dir_between(D.P, C.P, &d2);
    const float cl = dot3(D.ng, w);
    const float pe = cl > 0.0f ? cl * kInvPi : 0.0f;
    return (pe * fabsf(dot3(C.ng, w))) / d2;
  }
  const f3 wo = dir_between(D.P, E.P, &d2);
  const f3 wi = dir_between(D.P, C.P, &d2);
  f3 fc;
  float p;
  eval_facing(load_mat(sc.mats + 8 * (size_t)D.mat), D.ng, wo, wi, &fc, &p);
  return (p * fabsf(dot3(C.ng, wi))) / d2;
}

// The terms of a connection's weight that involve light vertices only, once
// per light vertex after the subpaths are traced (Sec. 5: the full-path
// weight sums over every strategy of the connected path; along its light
// side the densities and throughput factors below do not depend on the
// camera vertex).  For y_i of subpath r (y_0 its emitter point):
//   V2.w: the density of reaching y_i from y_{i-1} (incoming from y_{i-2}),
//         as area density at y_i; for y_1 the emission density of y_0;
//   V3:   for i < length, the BSDF at y_i towards y_{i-1} for a path arriving
//         from y_{i+1}: f cos / p per channel (-1 if p = 0) and the density
//         of reaching y_{i-1} (area density there).
// Both are evaluated by the same operations as the weight's walk would,
// so the weights do not change.
// One thread per subpath, walking it from y_1 with a window of four
// vertices (E = y_{i-2}, D = y_{i-1}, C = y_i, A = y_{i+1}), so that each
// vertex is fetched and decoded once.
__global__ __launch_bounds__(256) void light_walk_kernel(SceneDev sc, LightDev lt, uint32_t roots) {
  const uint32_t lm = (uint32_t)lt.lmax;
  for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < roots; r += gridDim.x * blockDim.x) {
    const int len = (int)lt.len[r].x;
    if (len < 1) continue;
    const size_t b = (size_t)r * lm;  // y_i at b + i - 1
    PV E{};
    PV D = light_vertex(sc, lt.Y0[r]);
    PV C = light_vertex(sc, lt.V0[b]);
    for (int i = 1; i <= len; ++i) {
      const size_t e = b + (size_t)(i - 1);
      float d2;
      float pR;
      if (i == 1) {
        const f3 w = dir_between(D.P, C.P, &d2);
        const float cl = dot3(D.ng, w);
        const float pe = cl > 0.0f ? cl * kInvPi : 0.0f;
        pR = (pe * fabsf(dot3(C.ng, w))) / d2;
      } else {
        const f3 wo = dir_between(D.P, E.P, &d2);
        const f3 wi = dir_between(D.P, C.P, &d2);
        f3 fc;
        float p;
        eval_facing(load_mat(sc.mats + 8 * (size_t)D.mat), D.ng, wo, wi, &fc, &p);
        pR = (p * fabsf(dot3(C.ng, wi))) / d2;
      }
      const float4 v2 = lt.V2[e];
      lt.V2[e] = make_float4(v2.x, v2.y, v2.z, pR);
      if (i == len) break;
      const PV A = light_vertex(sc, lt.V0[e + 1]);
      {
        const f3 wo = dir_between(C.P, A.P, &d2);
        const f3 wi = dir_between(C.P, D.P, &d2);
        f3 fc;
        float p;
        eval_facing(load_mat(sc.mats + 8 * (size_t)C.mat), C.ng, wo, wi, &fc, &p);
        const float pF = (p * fabsf(dot3(D.ng, wi))) / d2;
        lt.V3[e] = p > 0.0f ? make_float4(fc.x / p, fc.y / p, fc.z / p, pF)
                            : make_float4(-1.0f, -1.0f, -1.0f, pF);
      }
      E = D;
      D = C;
      C = A;
    }
  }
}
void k_light_walk(const SceneDev& sc, const LightDev& lt, uint32_t roots, hipStream_t s) {
  if (!roots || lt.lmax < 1) return;
  light_walk_kernel<<<(roots + 255) / 256, 256, 0, s>>>(sc, lt, roots);
}

// the strategies tt = d .. 2 of a path z_0..z_k through the camera vertex j
// of depth d (k > d: a connection or NEE sample there; k = d: z_d on an
// emitter), walking up the parent chain: pF of vertex tt and pR of vertex
// tt + 2 (tt <= d - 2) from the records (cur: those of z_d), the counts of
// vertex tt - 1; pR_d and pR_dm1 involve z_{d+1} and are passed in
__device__ __forceinline__ float camera_side_sum(const SceneDev& sc, const QueuesDev& q,
                                                 const IterDev& it, int d, int k, uint32_t j,
                                                 VRec cur, float pR_d, float pR_dm1, float tft,
                                                 float sum) {
  float rp = 1.0f, rb = 1.0f;
  uint32_t ecur = j;
  float prg1 = 0.0f, prg2 = 0.0f;
  for (int tt = d; tt >= 2; --tt) {
    const float pRt = tt == d ? pR_d : (tt == d - 1 ? pR_dm1 : prg2);
    const uint32_t epar = ubits(q.S0[(size_t)tt * q.cap + ecur].w);
    const VRec par = load_rec(q, tt - 1, epar);
    rp = rp * (pRt / cur.pF);
    rb = rb * mis_count(it, par.b0);
    // strategy tt: NEE at z_{k-1} (tt = k), else z_{tt-1} (par) connected to
    // the light vertex y_{k-tt}
    const float f = tt == k ? mis_count(it, par.b1)
                            : mis_count(it, lp_class_count(sc, par.b2, par.b3, par.b4, k - tt));
    sum = sum + rp * (f / (rb * tft));
    prg2 = prg1;
    prg1 = cur.pRg;
    cur = par;
    ecur = epar;
  }
  return sum;
}

// weight of the NEE sample of camera vertex j (depth d: zc, its parent zp,
// the camera for d = 1) on the emitter point y: strategy t = d + 1 of the
// path z_0..z_k, k = d + 1 (the sums above for t = k)
__device__ float bdpt_weight_nee(const SceneDev& sc, const QueuesDev& q, const IterDev& it, int d,
                                 uint32_t j, const PV& zc, const PV& zp, const PV& y) {
  const int k = d + 1;
  // pR of the camera vertex (y's emission density) and of its parent
  const float pR_d = d >= 2 ? path_pR(sc, d, k, zc, y, y) : 0.0f;
  const float pR_dm1 = d >= 3 ? path_pR(sc, d - 1, k, zp, zc, y) : 0.0f;
  // the NEE count at z_d (its record)
  const VRec rd = load_rec(q, d, j);
  const float tft = mis_count(it, rd.b1);
  if (!(tft > 0.0f)) return 0.0f;
  // strategy k + 1: the BSDF sample at z_d reaching y
  float d2;
  const f3 wo = dir_between(zc.P, zp.P, &d2);
  const f3 wi = dir_between(zc.P, y.P, &d2);
  f3 fc;
  float p;
  eval_facing(load_mat(sc.mats + 8 * (size_t)zc.mat), zc.ng, wo, wi, &fc, &p);
  const float pFk = (p * fabsf(dot3(y.ng, wi))) / d2;
  const float rp = 1.0f * (pFk / y.lpdf);
  const float rb = 1.0f * mis_count(it, rd.b0);
  float sum = 1.0f + (rp * rb) * (1.0f / tft);
  sum = camera_side_sum(sc, q, it, d, k, j, load_rec(q, d, j), pR_d, pR_dm1, tft, sum);
  if (!(sum < INFINITY)) return 0.0f;
  return 1.0f / sum;
}

// weight of the camera path z_0..z_k whose vertex z_k (queue entry j of
// depth k >= 2, zk) lies on an emitter: strategy k + 1, BSDF sampling at
// z_{k-1} (the sums above for t = k + 1).  pF(k) and pR(k - 2)
// involve z_k and are evaluated here; the rest comes from the records.
__device__ float bdpt_weight_hit(const SceneDev& sc, const QueuesDev& q, const IterDev& it, int k,
                                 uint32_t j, const PV& zk) {
  const uint32_t e1 = ubits(q.S0[(size_t)k * q.cap + j].w);
  const PV z1 = hit_vertex(sc, q, k - 1, e1);  // z_{k-1}
  PV z2{};                                      // z_{k-2} (the camera: position only)
  if (k == 2) z2.P = mk3(sc.cam_o[0], sc.cam_o[1], sc.cam_o[2]);
  else z2 = hit_vertex(sc, q, k - 2, ubits(q.S0[(size_t)(k - 1) * q.cap + e1].w));
  const Mat m1 = load_mat(sc.mats + 8 * (size_t)z1.mat);
  float d2;
  VRec cur{};
  {
    const f3 wo = dir_between(z1.P, z2.P, &d2);
    const f3 wi = dir_between(z1.P, zk.P, &d2);
    f3 fc;
    float p;
    eval_facing(m1, z1.ng, wo, wi, &fc, &p);
    cur.pF = (p * fabsf(dot3(zk.ng, wi))) / d2;
  }
  if (k >= 3) {
    const f3 wo = dir_between(z1.P, zk.P, &d2);
    const f3 wi = dir_between(z1.P, z2.P, &d2);
    f3 fc;
    float p;
    eval_facing(m1, z1.ng, wo, wi, &fc, &p);
    cur.pRg = (p * fabsf(dot3(z2.ng, wi))) / d2;
  }
  // pR(k - 1): the emission density of z_k towards z_{k-1}
  const f3 w = dir_between(zk.P, z1.P, &d2);
  const float cl = dot3(zk.ng, w);
  const float pe = cl > 0.0f ? cl * kInvPi : 0.0f;
  const float pR_km1 = (pe * fabsf(dot3(z1.ng, w))) / d2;
  const float sum = camera_side_sum(sc, q, it, k, k, j, cur, zk.lpdf, pR_km1, 1.0f, 1.0f);
  if (!(sum < INFINITY)) return 0.0f;
  return 1.0f / sum;
}

// weight of the light-path connection of camera vertex j (depth d: zc, its
// parent zp, the camera for d = 1) to the light vertex y_i (yi) of subpath
// r, strategy t = d + 1 of the path z_0..z_k, k = d + i + 1, whose light side
// z_{d+1}..z_k is y_i, .., y_1, y_0.  The sums above, in the order they
// state; the terms that involve light vertices only are read from the
// light walk (V2.w, V3) instead of evaluated.  ly: in learned-cache
// iterations, the network outputs at the subpath's vertices (y_h at
// ly[4 (h - 1)]).
__device__ float bdpt_weight_lp(const SceneDev& sc, const CacheDev& c, const QueuesDev& q,
                                const LightDev& lt, const IterDev& it, int d, uint32_t j,
                                const PV& zc, const PV& zp, const PV& yi, uint32_t r, int i,
                                const float* It, const float* ly) {
  const int k = d + i + 1, t = d + 1;
  const uint32_t base = r * (uint32_t)lt.lmax;  // y_h at base + h - 1
  const PV y0 = light_vertex(sc, lt.Y0[r]);
  const PV yn = i >= 2 ? light_vertex(sc, lt.V0[base + (uint32_t)(i - 2)]) : y0;  // y_{i-1}
  // pR of the camera vertex and of its parent, for the camera-side sums
  const float pR_d = d >= 2 ? path_pR(sc, d, k, zc, yi, yn) : 0.0f;
  const float pR_dm1 = d >= 3 ? path_pR(sc, d - 1, k, zp, zc, yi) : 0.0f;
  // counts at z_d (its record); t's own technique count
  const VRec rd = load_rec(q, d, j);
  f3 T = rd.T;
  float b[3] = {rd.b0, rd.b1, rd.b2};
  float bx[2] = {rd.b3, rd.b4};
  float nB_prev = mis_count(it, b[0]);
  const float tft = mis_count(it, lp_class_count(sc, b[2], bx[0], bx[1], k - t));
  if (!(tft > 0.0f)) return 0.0f;
  // the strategies u + 1 = t + 1 .. k + 1 along the light side, z_u = y_h:
  // pF(u) from the BSDF at z_{u-1} (evaluated for u <= d + 2, whose window
  // holds a camera vertex; read from V3 of y_{h+1} beyond), pR(u) of y_h
  // from V2.w (y_0: its emitter pdf), the counts at y_h along the
  // camera-prefix throughput continued through the light side
  float sum = 1.0f, rp = 1.0f, rb = 1.0f;
  const float lpdf0 = y0.lpdf;
  // one strategy u + 1 past z_u = y_h: pF(u) and the BSDF factor into z_u
  // (fcp; pos: p > 0), the counts at y_h along the continued throughput
  auto advance = [&](int u, bool pos, f3 fcp, float pFu) {
    const int h = k - u;
    float tf = 1.0f;  // strategy k + 1
    float nB_u = 0.0f;
    float pRu;
    if (u < k) {
      const float4 v2 = lt.V2[base + (uint32_t)(h - 1)];
      pRu = v2.w;
      if (pos && b[0] > 0.0f)
        T = mk3(T.x * ((fcp.x * 1.0f) / b[0]), T.y * ((fcp.y * 1.0f) / b[0]),
                T.z * ((fcp.z * 1.0f) / b[0]));
      else
        T = mk3(0.0f, 0.0f, 0.0f);
      const uint32_t cell = ubits(v2.z);
      // only the counts this walk reads: the BSDF count and the count of
      // strategy u + 1's technique (NEE, or the class of y_{h-1})
      const bool cls_x = sc.lp_classes == 3 && h - 1 >= 2;
      const uint32_t mask = 1u | (u == k - 1 ? 2u : (cls_x ? 0u : 4u));
      counts_at(sc, c, it, cell, T, It, u, b, mask);
      if (ly && mlp_active(c, it)) mlp_apply(it, T, It, ly + 4 * (h - 1), b, mask);
      if (cls_x && u != k - 1) counts_at_x(c, it, cell, T, It, bx, h - 1 == 2 ? 1u : 2u);
      nB_u = mis_count(it, b[0]);
      // strategy u + 1 connects z_u to the light vertex y_{h-1}
      tf = u == k - 1 ? mis_count(it, b[1])
                      : mis_count(it, lp_class_count(sc, b[2], bx[0], bx[1], h - 1));
    } else {
      pRu = lpdf0;
    }
    rp = rp * (pFu / pRu);
    rb = rb * nB_prev;
    sum = sum + (rp * rb) * (tf / tft);
    nB_prev = nB_u;
  };
  // u = d + 1 and d + 2: the BSDFs at the camera vertex and at y_i, whose
  // directions involve the camera vertex
  for (int u = d + 1; u <= d + 2; ++u) {
    const PV& B = u == d + 1 ? zc : yi;
    const PV& A = u == d + 1 ? zp : zc;
    const PV& C = u == d + 1 ? yi : yn;
    float d2;
    const f3 wo = dir_between(B.P, A.P, &d2);
    const f3 wi = dir_between(B.P, C.P, &d2);
    f3 fc;
    float p;
    eval_facing(load_mat(sc.mats + 8 * (size_t)B.mat), B.ng, wo, wi, &fc, &p);
    const bool pos = p > 0.0f;
    advance(u, pos, pos ? mk3(fc.x / p, fc.y / p, fc.z / p) : mk3(0.0f, 0.0f, 0.0f),
            (p * fabsf(dot3(C.ng, wi))) / d2);
  }
  // u >= d + 3: pF(u) and the factor from V3 of y_{h+1}, loaded a step ahead
  float4 w3 = d + 3 <= k ? lt.V3[base + (uint32_t)(k - d - 3)] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  for (int u = d + 3; u <= k; ++u) {
    const float4 w3c = w3;
    if (u + 1 <= k) w3 = lt.V3[base + (uint32_t)(k - u - 1)];
    advance(u, !(w3c.x < 0.0f), xyz(w3c), w3c.w);
  }
  sum = camera_side_sum(sc, q, it, d, k, j, load_rec(q, d, j), pR_d, pR_dm1, tft, sum);
  if (!(sum < INFINITY)) return 0.0f;
  return 1.0f / sum;
}

// shadow-entry requests written by the vertex kernel: kind in SH1.x, the
// camera vertex in SH1.w; NEE: emitter point and triangle in SH0; light
// path: subpath index and light vertex index in SH0.xy
constexpr uint32_t kConnNee = 1u, kConnLight = 2u;

// the light subpaths of the LP samples j = 0, 1, .. of a camera vertex, in
// turn: pool entry (b + j stride) mod npool, b the first word of the
// vertex's own random stream, so that the vertices of one path tree connect
// to unrelated light subpaths; walked by steps of stride mod npool (the same
// integers, without a 64-bit remainder per sample)
struct LpWalk {
  uint32_t idx, step, n;
  __device__ __forceinline__ LpWalk(uint32_t b, int32_t stride, uint32_t npool)
      : idx(npool ? b % npool : 0u), step(npool ? (uint32_t)stride % npool : 0u), n(npool) {}
  __device__ __forceinline__ uint32_t next() {
    const uint32_t r = idx;
    const uint32_t t = idx + step;  // < 2 npool
    idx = t >= n ? t - n : t;
    return r;
  }
};

// light vertices y_lo..y_hi a light-path sample of class cls connects to,
// of the imax its subpath offers within the path-length limit: every one
// with one light-path budget; with per-length budgets y_1, y_2 or y_3+
__device__ __forceinline__ void lp_class_range(const SceneDev& sc, int cls, int imax, int* lo,
                                               int* hi) {
  if (sc.lp_classes != 3) {
    *lo = 1;
    *hi = imax;
  } else {
    *lo = cls + 1;
    *hi = cls == 2 ? imax : min(cls + 1, imax);
  }
}

__global__ __launch_bounds__(kShadeBlock) void shade_bdpt_kernel(SceneDev sc, CacheDev c, QueuesDev q,
                                                         LightDev lt, Counters* cnt, IterDev it,
                                                         ImageDev img, DebugRec* dbg,
                                                         uint32_t dbg_cap, int d, uint32_t npool) {
  __shared__ uint32_t alloc_lds[4 * kShadeBlock / 64 + 2];
  if (group_overflowed(cnt)) return;
  const Key key{sc.key0, sc.key1};
  const uint32_t n = min(cnt->n_ray[d], (uint32_t)q.cap);
  const int lane = threadIdx.x & 63;
  const size_t L = (size_t)d * q.cap, Ln = (size_t)(d + 1) * q.cap;
  uint32_t my_vert = 0, my_samp = 0, my_ext = 0;
  for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
    const uint32_t j = base + threadIdx.x;
    const bool active = j < n;
    bool vert = false;
    f3 Ew = mk3(0.0f, 0.0f, 0.0f);
    uint32_t cell = kNoCell;
    // BSDF, NEE, light path (with per-length budgets: y_1, then y_2, y_3+)
    float beta[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    uint32_t gam[5] = {0u, 0u, 0u, 0u, 0u};
    f3 x = mk3(0, 0, 0), n_s = mk3(0, 0, 0), wo = mk3(0, 0, 0), T = mk3(0, 0, 0),
       ov = mk3(0, 0, 0);
    uint32_t prim = kMiss, pix = 0, root = 0, nconn = 0;
    uint2 strm = make_uint2(0, 0);
    float It[3] = {1.0f, 1.0f, 1.0f};
    if (active) {
      const uint2 h = q.H[L + j];
      prim = h.y;
      const float4 r1 = q.R1[L + j];
      pix = ubits(r1.w);
      const uint4 s3 = q.S3[L + j];
      root = s3.w;
      if (prim != kMiss) {
        const float t = fbits(h.x);
        const float4 r0 = q.R0[L + j];
        const f3 dir = xyz(r1);
        const float4 ngl = sc.tri_ng[prim];
        const f3 ng = xyz(ngl);
        const float* m = sc.mats + 8 * (size_t)sc.tri_mat[prim];
        x = mk3(r0.x + t * dir.x, r0.y + t * dir.y, r0.z + t * dir.z);
        It[0] = img.itilde[3 * (size_t)pix];
        It[1] = img.itilde[3 * (size_t)pix + 1];
        It[2] = img.itilde[3 * (size_t)pix + 2];
        const float cosl = -dot3(dir, ng);
        if (cosl > 0.0f && (m[5] > 0.0f || m[6] > 0.0f || m[7] > 0.0f)) {
          const float w = d > 1 ? bdpt_weight_hit(sc, q, it, d, j, PV{x, ng, sc.tri_mat[prim], ngl.w})
                                : 1.0f;
          Ew = mk3(w * m[5], w * m[6], w * m[7]);
        }
        if (d < sc.max_depth) {
          vert = true;
          n_s = dot3(ng, dir) < 0.0f ? ng : mk3(-ng.x, -ng.y, -ng.z);
          wo = mk3(-dir.x, -dir.y, -dir.z);
          ov = mk3(x.x + n_s.x * sc.eps, x.y + n_s.y * sc.eps, x.z + n_s.z * sc.eps);
          cell = cell_of(c.nodes, mk3(sc.oct_lo[0], sc.oct_lo[1], sc.oct_lo[2]), sc.oct_inv, x);
          T = xyz(q.S0[L + j]);
          counts_at(sc, c, it, cell, T, It, d, beta);
          if (sc.lp_classes == 3) counts_at_x(c, it, cell, T, It, beta + 3);
          bdpt_record(sc, c, q, it, d, j, x, ng, cell, It);
          mlp_counts(c, it, L + j, T, It, beta);
          strm = make_uint2(s3.x, s3.y);
          const float4 u = draw4(key, strm, 0);
          if (it.rounding) round_counts_independent(beta, u, gam);
          else if (sc.lp_classes == 3) round_counts_n<5>(beta, u.x, gam);
          else round_counts(beta, u.x, gam);
          mlp_record(c, strm, x, pix, ng, T);
          const int imax0 = sc.max_depth - d - 1;
          for (int cls = 0; cls < sc.lp_classes; ++cls) {
            LpWalk lw(strm.x, it.lp_stride, npool);
            for (uint32_t k = 0; k < gam[cls == 0 ? 2 : 2 + cls]; ++k) {
              const uint32_t lpi = lw.next();
              int lo, hi;
              lp_class_range(sc, cls, max(0, min(imax0, (int)lt.len[lpi].x)), &lo, &hi);
              nconn += (uint32_t)max(0, hi - lo + 1);
            }
          }
        }
      }
    }
    const uint32_t ncont = vert ? gam[0] : 0u, nsh = vert ? gam[1] + nconn : 0u;
    uint32_t cfirst, sfirst;
    group_alloc<kShadeBlock>(ncont, nsh, &cnt->n_ray[d + 1], &cnt->n_shadow[d], &cfirst, &sfirst,
                             alloc_lds);
    bool ovf = false;
    if (vert && ((size_t)cfirst + ncont > q.cap || (size_t)sfirst + nsh > q.scap)) {
      ovf = true;
      atomicMax(&cnt->overflow, 1u);
      atomicMax(&cnt->overflow_any, 1u);
    }
    if (!active) continue;
    q.V0[L + j] = make_float4(Ew.x, Ew.y, Ew.z, fbits(cell));
    q.V1[L + j] = make_float4(beta[0], beta[1], beta[2], fbits(vert ? gam[2] : 0u));
    if (q.V3)
      q.V3[L + j] = make_float4(beta[3], beta[4], fbits(vert ? gam[3] : 0u), fbits(vert ? gam[4] : 0u));
    q.V2[L + j] = ovf ? make_uint4(0, 0, 0, 0)
                      : make_uint4(sfirst, (vert ? gam[1] : 0u) | (nconn << 16), cfirst, ncont);
    if (d == 1) {
      img.beta1[3 * (size_t)root] = beta[0];
      img.beta1[3 * (size_t)root + 1] = beta[1];
      // per-length light paths: the light-path count is the sum over lengths
      img.beta1[3 * (size_t)root + 2] = sc.lp_classes == 3 ? (beta[2] + beta[3]) + beta[4] : beta[2];
    }
    if (!vert || ovf) continue;
    ++my_vert;
    my_samp += gam[0] + gam[1] + gam[2] + gam[3] + gam[4];
    if (d <= it.debug_depth && dbg) {
      const uint32_t k = atomicAdd(&cnt->n_debug, 1u);
      if (k < dbg_cap) {
        DebugRec r;
        r.root = root; r.depth = (uint32_t)d; r.stream_lo = strm.x; r.stream_hi = strm.y;
        r.cell = cell;
        for (int t = 0; t < 3; ++t) { r.beta[t] = beta[t]; r.gamma[t] = gam[t]; }
        r.beta_x[0] = beta[3]; r.beta_x[1] = beta[4]; r.gamma_x[0] = gam[3]; r.gamma_x[1] = gam[4];
        r.T[0] = T.x; r.T[1] = T.y; r.T[2] = T.z;
        dbg[k] = r;
      }
    }
    const Mat mat = load_mat(sc.mats + 8 * (size_t)sc.tri_mat[prim]);
    // NEE: the emitter point is drawn here; weight and contribution follow in
    // connect_bdpt_kernel, one thread per shadow entry
    for (uint32_t k = 0; k < gam[1]; ++k) {
      const uint2 ss = stream_child(key, strm, 1u, k, (uint32_t)d);
      const float4 u = draw4(key, ss, 1);
      int lo = 0, hi = sc.n_lights - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (u.x < sc.light_cdf[mid]) hi = mid; else lo = mid + 1;
      }
      const int li = sc.light_tri[lo];
      const float4* G = sc.tri_geo + (size_t)li * 3;
      const f3 v0 = xyz(G[0]), e1 = xyz(G[1]), e2 = xyz(G[2]);
      const float su = sqrtf(u.y);
      const float a = su * (1.0f - u.z), b = su * u.z;
      const f3 y = mk3((v0.x + a * e1.x) + b * e2.x, (v0.y + a * e1.y) + b * e2.y,
                       (v0.z + a * e1.z) + b * e2.z);
      const size_t e = sfirst + k;
      q.SH0[e] = make_float4(y.x, y.y, y.z, fbits((uint32_t)li));
      q.SH1[e] = make_float4(fbits(kConnNee), 0.0f, 0.0f, fbits(j));
    }
    // BSDF continuation (the only continuing technique: w_ind = 1)
    for (uint32_t k = 0; k < gam[0]; ++k) {
      const uint2 ss = stream_child(key, strm, 0u, k, (uint32_t)d);
      const float4 u = draw4(key, ss, 1);
      f3 w;
      bool ok = sample_bsdf(mat, n_s, wo, u.x, u.y, &w);
      f3 fc = mk3(0.0f, 0.0f, 0.0f);
      float pB = 0.0f;
      if (ok) {
        eval_bsdf(mat, n_s, wo, w, &fc, &pB);
        ok = (fc.x > 0.0f || fc.y > 0.0f || fc.z > 0.0f) && pB > 0.0f;
      }
      const size_t e = Ln + cfirst + k;
      if (ok) {
        const float c0 = fc.x / pB, c1 = fc.y / pB, c2 = fc.z / pB;
        const f3 Tc = mk3(T.x * ((c0 * 1.0f) / beta[0]), T.y * ((c1 * 1.0f) / beta[0]),
                          T.z * ((c2 * 1.0f) / beta[0]));
        q.R0[e] = make_float4(ov.x, ov.y, ov.z, 1.0f);
        q.S0[e] = make_float4(Tc.x, Tc.y, Tc.z, fbits(j));
        q.S1[e] = make_float4(c0, c1, c2, 1.0f);
        ++my_ext;
      } else {
        q.R0[e] = make_float4(ov.x, ov.y, ov.z, 0.0f);
        q.S0[e] = make_float4(0.0f, 0.0f, 0.0f, fbits(j));
        q.S1[e] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      }
      q.R1[e] = make_float4(w.x, w.y, w.z, fbits(pix));
      q.S2[e] = make_float4(0.0f, 0.0f, 0.0f, beta[0]);
      q.S3[e] = make_uint4(ss.x, ss.y, k, root);
    }
    // light-path connections: one shadow entry per (sample, light vertex),
    // the classes in order (sample k of every class on the same subpath)
    uint32_t slot = sfirst + gam[1];
    const int imax0 = sc.max_depth - d - 1;
    for (int cls = 0; cls < sc.lp_classes; ++cls) {
      LpWalk lw(strm.x, it.lp_stride, npool);
      for (uint32_t k = 0; k < gam[cls == 0 ? 2 : 2 + cls]; ++k) {
        const uint32_t lpi = lw.next();
        int lo, hi;
        lp_class_range(sc, cls, max(0, min(imax0, (int)lt.len[lpi].x)), &lo, &hi);
        for (int i = lo; i <= hi; ++i, ++slot) {
          const size_t e = slot;
          q.SH0[e] = make_float4(fbits(lpi), fbits((uint32_t)i), 0.0f, 0.0f);
          q.SH1[e] = make_float4(fbits(kConnLight), 0.0f, 0.0f, fbits(j));
        }
      }
    }
  }
  group_add<kShadeBlock, 3>({my_vert, my_samp, my_ext},
                            {&cnt->vertices, &cnt->samples, &cnt->rays_ext}, alloc_lds);
}

// NEE samples and light-path connections of the camera vertices of depth d,
// one thread per shadow entry: the full-path MIS weight and the weighted
// contribution, then the shadow ray.  Splitting gives vertices very uneven
// numbers of connections; this keeps the waves balanced.
__global__ __launch_bounds__(kConnectBlock) void connect_bdpt_kernel(SceneDev sc, CacheDev c, QueuesDev q,
                                                           LightDev lt, Counters* cnt, IterDev it,
                                                           ImageDev img, int d) {
  if (group_overflowed(cnt)) return;
  const uint32_t n = min(cnt->n_shadow[d], (uint32_t)q.scap);
  const size_t L = (size_t)d * q.cap, Ls = (size_t)d * q.scap;
  uint32_t my_sh = 0, my_conn = 0;
  // Each tile of blockDim.x entries is ranked by the length of its weight
  // walk (NEE first, then connections by light vertex index) with a
  // counting sort in LDS, and thread r takes the tile's r-th entry: a
  // wave's lanes then walk paths of about one length.  Which thread takes
  // an entry does not change what is computed for it.
  constexpr int kKeys = kMaxDepth + 2;
  __shared__ uint32_t key_count[kKeys];
  __shared__ uint16_t tile_order[kConnectBlock];
  for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
    {
      const uint32_t sr = base + threadIdx.x;
      uint32_t key = 0;
      if (sr < n) {
        if (ubits(q.SH1[sr].x) != kConnNee) key = min(ubits(q.SH0[sr].y), (uint32_t)kMaxDepth) + 1u;
      }
      if (threadIdx.x < kKeys) key_count[threadIdx.x] = 0u;
      __syncthreads();
      const uint32_t rank = sr < n ? atomicAdd(&key_count[key], 1u) : 0u;
      __syncthreads();
      if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int k = 0; k < kKeys; ++k) {
          const uint32_t c = key_count[k];
          key_count[k] = acc;
          acc += c;
        }
      }
      __syncthreads();
      if (sr < n) tile_order[key_count[key] + rank] = (uint16_t)threadIdx.x;
      __syncthreads();
    }
    const uint32_t ntile = min(n - base, (uint32_t)blockDim.x);
    const uint32_t s = base + ((uint32_t)threadIdx.x < ntile ? (uint32_t)tile_order[threadIdx.x] : 0u);
    if ((uint32_t)threadIdx.x >= ntile) continue;
    const size_t e = Ls + s;  // SH2; SH0 and SH1 hold one level, at s
    const float4 s0 = q.SH0[s], s1 = q.SH1[s];
    const uint32_t kind = ubits(s1.x), j = ubits(s1.w);
    // the camera vertex
    const uint2 h = q.H[L + j];
    const uint32_t prim = h.y;
    const float4 r0 = q.R0[L + j], r1 = q.R1[L + j];
    const float t = fbits(h.x);
    const f3 dir = xyz(r1);
    const uint32_t pix = ubits(r1.w);
    const float4 ngl = sc.tri_ng[prim];
    const f3 ng = xyz(ngl);
    const f3 x = mk3(r0.x + t * dir.x, r0.y + t * dir.y, r0.z + t * dir.z);
    float It[3];
    It[0] = img.itilde[3 * (size_t)pix];
    It[1] = img.itilde[3 * (size_t)pix + 1];
    It[2] = img.itilde[3 * (size_t)pix + 2];
    const f3 n_s = dot3(ng, dir) < 0.0f ? ng : mk3(-ng.x, -ng.y, -ng.z);
    const f3 wo = mk3(-dir.x, -dir.y, -dir.z);
    const f3 ov = mk3(x.x + n_s.x * sc.eps, x.y + n_s.y * sc.eps, x.z + n_s.z * sc.eps);
    const Mat mat = load_mat(sc.mats + 8 * (size_t)sc.tri_mat[prim]);
    // the camera vertex and its parent (the camera itself at depth 1)
    const PV zc = PV{x, ng, sc.tri_mat[prim], ngl.w};
    PV zp;
    if (d == 1) {
      zp = PV{mk3(sc.cam_o[0], sc.cam_o[1], sc.cam_o[2]), dir, 0u, 0.0f};
    } else {
      zp = hit_vertex(sc, q, d - 1, ubits(q.S0[L + j].w));
    }
    if (kind == kConnNee) {
      const f3 y = xyz(s0);
      const uint32_t li = ubits(s0.w);
      const f3 dv = sub3(y, ov);
      const float d2 = dot3(dv, dv);
      const float dist = sqrtf(d2);
      const f3 w = scl3(dv, 1.0f / dist);
      const float4 lng = sc.tri_ng[li];
      const float cl = -dot3(w, xyz(lng));
      f3 fc;
      float pB;
      eval_bsdf(mat, n_s, wo, w, &fc, &pB);
      float4 sh2 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      q.SH0[s] = make_float4(ov.x, ov.y, ov.z, dist * (1.0f - 1e-3f));
      q.SH1[s] = make_float4(w.x, w.y, w.z, fbits(j));
      if (cl > 0.0f && (fc.x > 0.0f || fc.y > 0.0f || fc.z > 0.0f)) {
        const float pN = (lng.w * d2) / cl;
        const f3 fp = mk3(fc.x / pN, fc.y / pN, fc.z / pN);
        const float wN = bdpt_weight_nee(sc, q, it, d, j, zc, zp, PV{y, xyz(lng), sc.tri_mat[li], lng.w});
        const float* Le = sc.mats + 8 * (size_t)sc.tri_mat[li] + 5;
        sh2 = make_float4(fp.x * (wN * Le[0]), fp.y * (wN * Le[1]), fp.z * (wN * Le[2]), 1.0f);
        ++my_sh;
      }
      q.SH2[e] = sh2;
    } else {
      const uint32_t lpi = ubits(s0.x);
      const int i = (int)ubits(s0.y);
      const size_t ye = (size_t)lpi * lt.lmax + (i - 1);
      const float4 y0v = lt.V0[ye], y1v = lt.V1[ye], y2v = lt.V2[ye];
      const f3 yP = xyz(y0v);
      const uint32_t yprim = ubits(y0v.w);
      const PV yv = prim_vertex(sc, yP, yprim);
      float d2;
      const f3 w = dir_between(x, yP, &d2);
      f3 fcC, fcL;
      float pc, pl;
      eval_bsdf(mat, n_s, wo, w, &fcC, &pc);
      const Mat ym = load_mat(sc.mats + 8 * (size_t)yv.mat);
      const f3 ywo = xyz(y1v);
      eval_facing(ym, yv.ng, ywo, mk3(-w.x, -w.y, -w.z), &fcL, &pl);
      float4 sh2 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if ((fcC.x > 0.0f || fcC.y > 0.0f || fcC.z > 0.0f) &&
          (fcL.x > 0.0f || fcL.y > 0.0f || fcL.z > 0.0f)) {
        // the shadow ray and the unweighted contribution first, so that
        // only the contribution stays live across the weight's walk
        const f3 ny = dot3(yv.ng, ywo) > 0.0f ? yv.ng : mk3(-yv.ng.x, -yv.ng.y, -yv.ng.z);
        const f3 yo = mk3(yP.x + ny.x * sc.eps, yP.y + ny.y * sc.eps, yP.z + ny.z * sc.eps);
        float sd2;
        const f3 sw = dir_between(ov, yo, &sd2);
        q.SH0[s] = make_float4(ov.x, ov.y, ov.z, sqrtf(sd2) * (1.0f - 1e-3f));
        q.SH1[s] = make_float4(sw.x, sw.y, sw.z, fbits(j));
        const f3 al = mk3(y1v.w, y2v.x, y2v.y);
        const f3 cv = mk3(((al.x * fcL.x) * fcC.x) / d2, ((al.y * fcL.y) * fcC.y) / d2,
                          ((al.z * fcL.z) * fcC.z) / d2);
        const float* ly = lt.y ? lt.y + (size_t)lpi * lt.lmax * 4 : nullptr;
        const float wc = bdpt_weight_lp(sc, c, q, lt, it, d, j, zc, zp, yv, lpi, i, It, ly);
        sh2 = make_float4(wc * cv.x, wc * cv.y, wc * cv.z, 1.0f);
        ++my_conn;
      } else {
        q.SH0[s] = make_float4(ov.x, ov.y, ov.z, 0.0f);
        q.SH1[s] = make_float4(w.x, w.y, w.z, fbits(j));
      }
      q.SH2[e] = sh2;
    }
  }
  __shared__ uint32_t stat_lds[2 * kConnectBlock / 64];
  group_add<kConnectBlock, 2>({my_sh, my_conn}, {&cnt->rays_shadow, &cnt->rays_conn}, stat_lds);
}

void k_shade_bdpt(const SceneDev& sc, const CacheDev& c, const QueuesDev& q, const LightDev& lt,
                  Counters* cnt, const IterDev& it, const ImageDev& img, DebugRec* dbg,
                  uint32_t dbg_cap, int d, uint32_t npool, hipStream_t s) {
  shade_bdpt_kernel<<<resident_grid(shade_bdpt_kernel, kShadeBlock), kShadeBlock, 0, s>>>(
      sc, c, q, lt, cnt, it, img, dbg, dbg_cap, d, npool);
}
void k_connect_bdpt(const SceneDev& sc, const CacheDev& c, const QueuesDev& q, const LightDev& lt,
                    Counters* cnt, const IterDev& it, const ImageDev& img, int d, hipStream_t s) {
  if (d < sc.max_depth)
    connect_bdpt_kernel<<<resident_grid(connect_bdpt_kernel, kConnectBlock), kConnectBlock, 0, s>>>(
        sc, c, q, lt, cnt, it, img, d);
}

// back-propagation for BDPT: NEE, BSDF and LP samples in that order
// (kLpLengths: per-length light-path budgets, the classes y_1, y_2, y_3+;
// an instantiation of its own so that the single-budget kernel keeps its
// registers)
template <bool kLpLengths>
__global__ __launch_bounds__(256) void backprop_bdpt_kernel(SceneDev sc, CacheDev c, QueuesDev q,
                                                            LightDev lt, const Counters* cnt,
                                                            IterDev it, ImageDev img, int d,
                                                            uint32_t npool) {
  __shared__ AggTable A;
  if (cnt->overflow) return;
  for (int k = threadIdx.x; k < kAggSlots; k += blockDim.x) {
    A.key[k] = kAggEmpty;
    for (int i = 0; i < kAggVals; ++i) A.val[k][i] = 0.0;
  }
  __syncthreads();
  const uint32_t n = min(cnt->n_ray[d], (uint32_t)q.cap);
  const size_t L = (size_t)d * q.cap, Ln = (size_t)(d + 1) * q.cap, Ls = (size_t)d * q.scap;
  const uint32_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const uint32_t j0 = blockIdx.x * chunk, j1 = min(n, j0 + chunk);
  for (uint32_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
    const float4 v0 = q.V0[L + j];
    const uint32_t cell = ubits(v0.w);
    f3 R = mk3(0.0f, 0.0f, 0.0f);
    uint32_t cost = 0;
    if (cell != kNoCell) {
      double st[3][8];
#pragma unroll
      for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int i = 0; i < 8; ++i) st[t][i] = 0.0;
      const uint4 v2 = q.V2[L + j];
      const float4 b = q.V1[L + j];
      const uint32_t nnee = v2.y & 0xFFFFu, glp = ubits(b.w);
      const uint32_t root = q.S3[L + j].w;
      auto record = [&](int t, f3 v, uint32_t cst) {
        const double x0 = (double)v.x, x1 = (double)v.y, x2 = (double)v.z;
        st[t][0] += x0; st[t][1] += x1; st[t][2] += x2;
        st[t][3] += x0 * x0; st[t][4] += x1 * x1; st[t][5] += x2 * x2;
        st[t][6] += 1.0; st[t][7] += (double)cst;
      };
      // loads issued four at a time, the sums taken in sample order
      for (uint32_t k0 = 0; k0 < nnee; k0 += 4) {
        float4 r4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          r4[u] = k0 + u < nnee ? q.SH2[Ls + v2.x + k0 + u] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (k0 + u >= nnee) break;
          const f3 v = xyz(r4[u]);
          R = mk3(R.x + v.x / b.y, R.y + v.y / b.y, R.z + v.z / b.y);
          cost += 1;
          record(1, v, 1u);
        }
      }
      for (uint32_t k0 = 0; k0 < v2.w; k0 += 2) {
        // the samples' values and costs, left by the launch of the next depth
        float4 sv2[2];
        float bt2[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const size_t e = Ln + v2.z + k0 + u;
          sv2[u] = k0 + u < v2.w ? q.RO[e] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
          bt2[u] = k0 + u < v2.w ? q.S2[e].w : 1.0f;
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          if (k0 + u >= v2.w) break;
          const f3 v = xyz(sv2[u]);
          const float bt = bt2[u];
          const uint32_t sc_ = ubits(sv2[u].w);
          R = mk3(R.x + v.x / bt, R.y + v.y / bt, R.z + v.z / bt);
          cost += sc_;
          record(0, v, sc_);
        }
      }
      uint32_t slot = v2.x + nnee;
      const int imax0 = sc.max_depth - d - 1;
      const float4 v3 = kLpLengths ? q.V3[L + j] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      for (int cls = 0; cls < (kLpLengths ? 3 : 1); ++cls) {
        // the class's count and rounded count: y_1 (or every light vertex)
        // in V1, the y_2 and y_3+ classes in V3, whose statistics are summed
        // apart and merged when the class is done
        const float bt = cls == 0 ? b.z : (cls == 1 ? v3.x : v3.y);
        const uint32_t g = cls == 0 ? glp : ubits(cls == 1 ? v3.z : v3.w);
        double sx[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        LpWalk lw(q.S3[L + j].x, it.lp_stride, npool);
        for (uint32_t k = 0; k < g; ++k) {
          const uint32_t lpi = lw.next();
          const uint2 ll = lt.len[lpi];
          int lo, hi;
          lp_class_range(sc, cls, max(0, min(imax0, (int)ll.x)), &lo, &hi);
          f3 v = mk3(0.0f, 0.0f, 0.0f);
          // an LP sample costs its connection rays (at least 1): the light
          // subpath is traced once per camera sample whatever the counts
          uint32_t sc_ = 0;
          for (int i0 = lo; i0 <= hi; i0 += 4) {
            float4 r4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
              r4[u] = i0 + u <= hi ? q.SH2[Ls + slot + (uint32_t)(i0 - lo + u)]
                                   : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const float4 r = r4[u];
              if (i0 + u <= hi && r.w != 0.0f) {
                sc_ += 1;
                v = mk3(v.x + r.x, v.y + r.y, v.z + r.z);
              }
            }
          }
          slot += (uint32_t)max(0, hi - lo + 1);
          sc_ = max(sc_, 1u);
          R = mk3(R.x + v.x / bt, R.y + v.y / bt, R.z + v.z / bt);
          cost += sc_;
          if (!kLpLengths || cls == 0) {
            record(2, v, sc_);
          } else {
            const double x0 = (double)v.x, x1 = (double)v.y, x2 = (double)v.z;
            sx[0] += x0; sx[1] += x1; sx[2] += x2;
            sx[3] += x0 * x0; sx[4] += x1 * x1; sx[5] += x2 * x2;
            sx[6] += 1.0; sx[7] += (double)sc_;
          }
        }
        if (kLpLengths && cls > 0 && sx[6] != 0.0) {
          double vals[kAggVals];
#pragma unroll
          for (int i = 0; i < 8; ++i) vals[i] = sx[i];
          vals[8] = 0.0;
          agg_add(A, c, (cell << 3) | (uint32_t)(2 + cls), vals);
        }
      }
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        if (t != 0 && st[t][6] == 0.0) continue;
        double vals[kAggVals];
#pragma unroll
        for (int i = 0; i < 8; ++i) vals[i] = st[t][i];
        vals[8] = t == 0 ? 1.0 : 0.0;
        agg_add(A, c, (cell << 3) | (uint32_t)t, vals);
      }
    }
    if (d >= 2) {
      // this entry as a BSDF sample of its parent vertex (depth d - 1): its
      // value with the factors the parent stored, and its cost (1 for a
      // sample whose direction was rejected)
      f3 v = mk3(0.0f, 0.0f, 0.0f);
      uint32_t sc_ = 1u;
      if (q.R0[L + j].w != 0.0f) {
        const float4 s1 = q.S1[L + j];
        v = mk3(s1.x * (v0.x + s1.w * R.x), s1.y * (v0.y + s1.w * R.y), s1.z * (v0.z + s1.w * R.z));
        sc_ = 1u + cost;
      }
      q.RO[L + j] = make_float4(v.x, v.y, v.z, fbits(sc_));
    }
    if (d == 1) {
      const uint32_t root = q.S3[L + j].w;
      img.Ls[3 * (size_t)root] = v0.x + R.x;
      img.Ls[3 * (size_t)root + 1] = v0.y + R.y;
      img.Ls[3 * (size_t)root + 2] = v0.z + R.z;
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kAggSlots; k += blockDim.x) {
    if (A.key[k] == kAggEmpty) continue;
    double vals[kAggVals];
    for (int i = 0; i < kAggVals; ++i) vals[i] = A.val[k][i];
    global_add_stats(c, A.key[k], vals);
  }
}
void k_init_launch_grids() {
  (void)resident_grid(shade_bdpt_kernel, kShadeBlock);
  (void)resident_grid(connect_bdpt_kernel, kConnectBlock);
  (void)resident_grid(backprop_bdpt_kernel<true>, 256);
  (void)resident_grid(backprop_bdpt_kernel<false>, 256);
  (void)resident_grid(backprop_pt_kernel, 256);
  (void)resident_grid(light_shade_kernel, 256);
}

void k_backprop_bdpt(const SceneDev& sc, const CacheDev& c, const QueuesDev& q,
                     const LightDev& lt, const Counters* cnt, const IterDev& it,
                     const ImageDev& img, int d, uint32_t npool, hipStream_t s) {
  if (sc.lp_classes == 3)
    backprop_bdpt_kernel<true><<<resident_grid(backprop_bdpt_kernel<true>, 256), 256, 0, s>>>(
        sc, c, q, lt, cnt, it, img, d, npool);
  else
    backprop_bdpt_kernel<false><<<resident_grid(backprop_bdpt_kernel<false>, 256), 256, 0, s>>>(
        sc, c, q, lt, cnt, it, img, d, npool);
}

// ---------------------------------------------------------------------------
// training targets of the learned cache, from the cells' updated factors:
//   y*_t = log(beta^_t) - log|T / I~|, beta^_t the resolved, unclamped
//   octree count of the vertex; weight min(n_t,c, 64) / 64 if the cell had at
//   least 4 samples of technique t in the iteration, else 0
// ---------------------------------------------------------------------------
__global__ void mlp_targets_kernel(SceneDev sc, CacheDev c, MlpDev m, ImageDev img, IterDev it,
                                   uint32_t cap, const uint32_t* skip) {
  SKIP_IF(skip);
  const uint32_t n = min(*m.n_rec, cap);
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const float4 a = m.rec[3 * (size_t)r], b = m.rec[3 * (size_t)r + 1], tt = m.rec[3 * (size_t)r + 2];
  const f3 P = xyz(a);
  const uint32_t pix = __float_as_uint(a.w);
  float* x = m.x6 + 6 * (size_t)r;
  x[0] = fminf(fmaxf((P.x - sc.oct_lo[0]) * sc.oct_inv, 0.0f), kOneMinus);
  x[1] = fminf(fmaxf((P.y - sc.oct_lo[1]) * sc.oct_inv, 0.0f), kOneMinus);
  x[2] = fminf(fmaxf((P.z - sc.oct_lo[2]) * sc.oct_inv, 0.0f), kOneMinus);
  x[3] = b.x; x[4] = b.y; x[5] = b.z;
  const float z0 = tt.x / img.itilde[3 * (size_t)pix], z1 = tt.y / img.itilde[3 * (size_t)pix + 1],
              z2 = tt.z / img.itilde[3 * (size_t)pix + 2];
  const float sm = sqrtf(((z0 * z0 + z1 * z1) + z2 * z2) * (1.0f / 3.0f));
  const uint32_t cell = cell_of(c.nodes, mk3(sc.oct_lo[0], sc.oct_lo[1], sc.oct_lo[2]), sc.oct_inv, P);
  const bool en[3] = {true, sc.nee != 0 && sc.n_lights > 0, sc.mode != 0};
  for (int t = 0; t < 3; ++t) {
    float y = 0.0f, w = 0.0f;
    const double cnt = c.acc[((size_t)cell * 3 + t) * 8 + 6];
    const float* aRR = c.fac + (size_t)cell * 18 + (0 * 3 + t) * 3;
    const float* aS = c.fac + (size_t)cell * 18 + (1 * 3 + t) * 3;
    if (en[t] && cnt >= 4.0 && aRR[0] >= 0.0f && sm > 0.0f) {
      const float sr = ((z0 * z0) * aRR[0] + (z1 * z1) * aRR[1]) + (z2 * z2) * aRR[2];
      const float ss = ((z0 * z0) * aS[0] + (z1 * z1) * aS[1]) + (z2 * z2) * aS[2];
      const float bRR = sqrtf(sr * (1.0f / 3.0f)), bS = sqrtf(ss * (1.0f / 3.0f));
      const float bh = bRR < 1.0f ? bRR : (bS > 1.0f ? bS : 1.0f);
      if (bh > 0.0f && isfinite(bh)) {
        y = logf(bh) - logf(sm);
        w = (float)(fmin(cnt, 64.0) / 64.0);
      }
    }
    m.tgt[3 * (size_t)r + t] = y;
    m.wt[3 * (size_t)r + t] = isfinite(y) ? w : 0.0f;
    if (!isfinite(y)) m.tgt[3 * (size_t)r + t] = 0.0f;
  }
}
void k_mlp_targets(const SceneDev& sc, const CacheDev& c, const MlpDev& m, const ImageDev& img,
                   const IterDev& it, uint32_t n, const uint32_t* skip, hipStream_t s) {
  if (n) mlp_targets_kernel<<<(n + 255) / 256, 256, 0, s>>>(sc, c, m, img, it, n, skip);
}

// ---------------------------------------------------------------------------
// per-pixel sums of the iteration (sample order) and the count map
// ---------------------------------------------------------------------------
__global__ void pixel_sums_kernel(ImageDev img, int npx, int spp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npx) return;
  float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, b0 = 0.0f, b1 = 0.0f, b2 = 0.0f;
  for (int s = 0; s < spp; ++s) {
    const size_t r = (size_t)i * spp + s;
    s0 += img.Ls[3 * r]; s1 += img.Ls[3 * r + 1]; s2 += img.Ls[3 * r + 2];
    b0 += img.beta1[3 * r]; b1 += img.beta1[3 * r + 1]; b2 += img.beta1[3 * r + 2];
  }
  img.iter_sum[3 * (size_t)i] = s0;
  img.iter_sum[3 * (size_t)i + 1] = s1;
  img.iter_sum[3 * (size_t)i + 2] = s2;
  img.count_map[3 * (size_t)i] = b0 / (float)spp;
  img.count_map[3 * (size_t)i + 1] = b1 / (float)spp;
  img.count_map[3 * (size_t)i + 2] = b2 / (float)spp;
}
void k_pixel_sums(const ImageDev& img, int npx, int spp, hipStream_t s) {
  pixel_sums_kernel<<<(npx + 255) / 256, 256, 0, s>>>(img, npx, spp);
}

// ---------------------------------------------------------------------------
// image estimates (Sec. 4.1 "Image estimates", Sec. 5.1):
//   I~ = 3x3 box filter (edge clamped) of the running mean image, floored
//   at 1e-3 x the image-mean channel value; V_I = mean over included pixels
//   of (1/spp) sum_s (1/3) sum_ch ((min(I_s, k I~) - I~) / I~)^2.
// red[0..2]: image-mean sums, red[3]: V_I sum, red[4]: included pixels,
// red[5]: inverse-variance weight sum, red[6]: samples per pixel so far.
// ---------------------------------------------------------------------------

// sum of v over the workgroup (fixed order), valid in thread 0
__device__ __forceinline__ double block_sum_d(double v) {
  __shared__ double part[16];
  v = wave_sum_d(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) part[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += part[k];
  __syncthreads();
  return s;
}
// red[first + j] for j < N: the sum of the previous kernel's per-workgroup
// partials part[b][first + j], computed by every workgroup that needs it in
// one fixed order (thread t sums partials t, t + blockDim, ... in turn, then
// the group sum), so all of them hold the same value and none waits on
// another.  Every thread must call it; out[] is valid in every thread.
template <int N>
__device__ __forceinline__ void sum_parts(const ImageDev& img, int first, double (&out)[N]) {
  __shared__ double res[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double s = 0.0;
    for (int b = threadIdx.x; b < kRedBlocks; b += blockDim.x) s += img.part[8 * b + first + j];
    s = block_sum_d(s);
    if (threadIdx.x == 0) res[j] = s;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < N; ++j) out[j] = res[j];
}

// running image: accum += iteration sums, mean = accum / total samples (the
// total after this iteration, red[6] + spp, stored by the per-cell update)
__global__ __launch_bounds__(256) void accum_mean_kernel(ImageDev img, int npx,
                                                         const double* total_spp, int spp,
                                                         const uint32_t* skip) {
  SKIP_IF(skip);
  const float tsp = (float)(*total_spp + (double)spp);
  double m[3] = {0.0, 0.0, 0.0};
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < npx; i += gridDim.x * blockDim.x)
    for (int ch = 0; ch < 3; ++ch) {
      const size_t e = 3 * (size_t)i + ch;
      const float a = img.accum[e] + img.iter_sum[e];
      img.accum[e] = a;
      const float mv = a / tsp;
      img.mean[e] = mv;
      m[ch] += (double)mv;
    }
  for (int ch = 0; ch < 3; ++ch) {
    const double s = block_sum_d(m[ch]);
    if (threadIdx.x == 0) img.part[8 * blockIdx.x + ch] = s;
  }
}

// I~ of pixel i (3x3 box filter of the running mean, edge clamped, floored)
// into itilde; returns the exclusion flag (1: floored), also stored
__device__ __forceinline__ uint8_t itilde_at(ImageDev& img, int W, int H, int i,
                                             const double (&msum)[3]) {
  const int y = i / W, x = i % W;
  const double npx = (double)W * (double)H;
  uint8_t ex = 0;
  for (int ch = 0; ch < 3; ++ch) {
    const float flo = fmaxf(1e-3f * (float)(msum[ch] / npx), 1e-6f);
    float s = 0.0f;
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int yy = min(max(y + dy, 0), H - 1), xx = min(max(x + dx, 0), W - 1);
        s += img.mean[3 * ((size_t)yy * W + xx) + ch];
      }
    s = s / 9.0f;
    if (!(s > flo)) {
      s = flo;
      ex = 1;
    }
    img.itilde[3 * (size_t)i + ch] = s;
  }
  img.excl[i] = ex;
  return ex;
}
// the image-mean sums (red[0..2]) from accum_mean's partials; stored by
// workgroup 0
__device__ __forceinline__ void mean_sums(ImageDev& img, double (&msum)[3]) {
  sum_parts<3>(img, 0, msum);
  if (blockIdx.x == 0 && threadIdx.x < 3) img.red[threadIdx.x] = msum[threadIdx.x];
}
__global__ __launch_bounds__(256) void itilde_kernel(ImageDev img, int W, int H,
                                                     const uint32_t* skip) {
  SKIP_IF(skip);
  double msum[3];
  mean_sums(img, msum);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= W * H) return;
  itilde_at(img, W, H, i, msum);
}

// BDPT: the 10 pixels with the largest iteration luminance leave V_I
// (Sec. 5.1); ties go to the lower index.  One workgroup, ten passes.
// the kBright brightest pixels of the iteration (luminance of the pixel sum,
// ties to the lower index): each chunk's top kBright, then the top kBright
// of the candidates.  Round r takes the best key strictly below round r-1's.
__device__ __forceinline__ bool ranks_above(float a, int ai, float b, int bi) {
  return a > b || (a == b && ai < bi);
}
template <int kThreads>
__device__ __forceinline__ void block_best(float* bl, int* bi, float& best, int& idx) {
  bl[threadIdx.x] = best;
  bi[threadIdx.x] = idx;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const float o = bl[threadIdx.x + s];
      const int oi = bi[threadIdx.x + s];
      if (o > bl[threadIdx.x] || (o == bl[threadIdx.x] && oi >= 0 &&
                                  (bi[threadIdx.x] < 0 || oi < bi[threadIdx.x]))) {
        bl[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  best = bl[0];
  idx = bi[0];
  __syncthreads();
}
__global__ __launch_bounds__(256) void brightest_part_kernel(ImageDev img, int npx,
                                                             const uint32_t* skip) {
  __shared__ float bl[256];
  __shared__ int bi[256];
  SKIP_IF(skip);
  const int lo = blockIdx.x * kBrightChunk, hi = min(npx, lo + kBrightChunk);
  float pl = INFINITY;
  int pi = -1;
  for (int r = 0; r < kBright; ++r) {
    float best = -1.0f;
    int idx = -1;
    for (int i = lo + (int)threadIdx.x; i < hi; i += 256) {
      const float l = lum(mk3(img.iter_sum[3 * (size_t)i], img.iter_sum[3 * (size_t)i + 1],
                              img.iter_sum[3 * (size_t)i + 2]));
      if (!ranks_above(pl, pi, l, i)) continue;
      if (l > best) { best = l; idx = i; }
    }
    block_best<256>(bl, bi, best, idx);
    if (threadIdx.x == 0) {
      img.bright_l[blockIdx.x * kBright + r] = best;
      img.bright_i[blockIdx.x * kBright + r] = idx;
    }
    if (idx < 0) {
      for (int q = r + 1 + (int)threadIdx.x; q < kBright; q += 256) {
        img.bright_l[blockIdx.x * kBright + q] = -1.0f;
        img.bright_i[blockIdx.x * kBright + q] = -1;
      }
      return;
    }
    pl = best;
    pi = idx;
  }
}
__global__ __launch_bounds__(1024) void brightest_final_kernel(ImageDev img, int ncand,
                                                               const uint32_t* skip) {
  __shared__ float bl[1024];
  __shared__ int bi[1024];
  SKIP_IF(skip);
  float pl = INFINITY;
  int pi = -1;
  for (int r = 0; r < kBright; ++r) {
    float best = -1.0f;
    int idx = -1;
    for (int c = threadIdx.x; c < ncand; c += 1024) {
      const int i = img.bright_i[c];
      if (i < 0) continue;
      const float l = img.bright_l[c];
      if (!ranks_above(pl, pi, l, i)) continue;
      if (l > best || (l == best && i < idx)) { best = l; idx = i; }
    }
    block_best<1024>(bl, bi, best, idx);
    if (idx < 0) return;
    if (threadIdx.x == 0) img.excl[idx] = 2;
    pl = best;
    pi = idx;
  }
}

// V_I partial sums; with_itilde: I~ and the exclusion flag of each pixel are
// computed here first (no brightest-pixel pass in between)
__global__ __launch_bounds__(256) void vi_kernel(ImageDev img, int W, int H, int spp, float kc,
                                                  int with_itilde, const uint32_t* skip) {
  SKIP_IF(skip);
  const int npx = W * H;
  double msum[3] = {0.0, 0.0, 0.0};
  if (with_itilde) mean_sums(img, msum);
  double e = 0.0, inc = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < npx; i += gridDim.x * blockDim.x) {
    const uint8_t ex = with_itilde ? itilde_at(img, W, H, i, msum) : img.excl[i];
    if (ex != 0) continue;
    const float* It = img.itilde + 3 * (size_t)i;
    double ep = 0.0;
    for (int s = 0; s < spp; ++s) {
      const float* l = img.Ls + 3 * ((size_t)i * spp + s);
      float dd[3];
      for (int ch = 0; ch < 3; ++ch) {
        const float xv = kc > 0.0f ? fminf(l[ch], kc * It[ch]) : l[ch];
        dd[ch] = (xv - It[ch]) / It[ch];
      }
      ep += (double)((dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2]);
    }
    e += ep / (3.0 * (double)spp);
    inc += 1.0;
  }
  const double se = block_sum_d(e), si = block_sum_d(inc);
  if (threadIdx.x == 0) {
    img.part[8 * blockIdx.x + 3] = se;
    img.part[8 * blockIdx.x + 4] = si;
  }
}
void k_update_image(const ImageDev& img, int W, int H, int spp, const double* total_spp, int bdpt,
                    float stat_clamp, const uint32_t* skip, hipStream_t s) {
  const int npx = W * H;
  accum_mean_kernel<<<kRedBlocks, 256, 0, s>>>(img, npx, total_spp, spp, skip);
  if (bdpt) {
    itilde_kernel<<<(npx + 255) / 256, 256, 0, s>>>(img, W, H, skip);
    const int nb = (npx + kBrightChunk - 1) / kBrightChunk;
    brightest_part_kernel<<<nb, 256, 0, s>>>(img, npx, skip);
    brightest_final_kernel<<<1, 1024, 0, s>>>(img, nb * kBright, skip);
  }
  vi_kernel<<<kRedBlocks, 256, 0, s>>>(img, W, H, spp, stat_clamp, bdpt ? 0 : 1, skip);
}

// ---------------------------------------------------------------------------
// fixed-point update (Sec. 3.1 "Optimization", supplement A.3): per cell and
// technique with samples, in binary64,
//   a^RR = C_I / (C_t V_I) E[v^2],  a^S = C_I / (C_t V_I) V[v]   per channel
// ---------------------------------------------------------------------------
__device__ __forceinline__ void ivw_at(ImageDev& img, int i, int spp, const double (&vs)[2]);
// Blocks [0, cell_blocks): per cell, the fixed point and (guided) the
// directional distribution; blocks after that: the inverse-variance weighted
// accumulation of the iteration's image, per pixel (npx pixels).
__global__ void fixed_point_kernel(CacheDev c, const int32_t* n_cells_dev, const double* red,
                                   double C_I, const Counters* cnt, double roots, int use_dev,
                                   double V_host, int guided, ImageDev img, int npx, int spp,
                                   int cell_blocks, const uint32_t* skip, int ears_mode) {
  SKIP_IF(skip);
  // V_I sums (red[3], red[4]) from vi's partials; workgroup 0 stores them
  // and advances the sample total (red[6]) by this iteration's spp
  double vs[2] = {0.0, 0.0};
  if (use_dev) {
    sum_parts<2>(img, 3, vs);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      img.red[3] = vs[0];
      img.red[4] = vs[1];
      if (npx > 0) img.red[6] += (double)spp;
    }
  }
  if ((int)blockIdx.x >= cell_blocks) {
    const int i = (blockIdx.x - cell_blocks) * blockDim.x + threadIdx.x;
    if (i < npx) ivw_at(img, i, spp, vs);
    return;
  }
  if (cnt) {
    const double rays = roots + (double)(cnt->rays_ext + cnt->rays_shadow + cnt->rays_light +
                                         cnt->rays_conn);
    C_I = rays / roots;
  }
  const int cidx = blockIdx.x * blockDim.x + threadIdx.x;
  if (cidx >= *n_cells_dev) return;
  const double V_I = use_dev ? (vs[1] > 0.0 ? vs[0] / vs[1] : 0.0) : V_host;
  if (V_I > 0.0 && C_I > 0.0) {
    for (int t = 0; t < 3; ++t) {
      const double* a = c.acc + ((size_t)cidx * 3 + t) * 8;
      const double n = a[6];
      if (!(n > 0.0)) continue;
      const double Ct = a[7] / n;
      if (!(Ct > 0.0)) continue;
      const double k = C_I / (Ct * V_I);
      for (int ch = 0; ch < 3; ++ch) {
        const double E1 = a[ch] / n, E2 = a[3 + ch] / n;
        double var = E2 - E1 * E1;
        if (var < 0.0) var = 0.0;
        c.fac[(size_t)cidx * 18 + (0 * 3 + t) * 3 + ch] = (float)(k * E2);
        c.fac[(size_t)cidx * 18 + (1 * 3 + t) * 3 + ch] = (float)(k * var);
      }
    }
    // per-length light paths: techniques 3 and 4, the same update
    for (int x = 0; c.acc_x && x < 2; ++x) {
      const double* a = c.acc_x + ((size_t)cidx * 2 + x) * 8;
      const double n = a[6];
      if (!(n > 0.0)) continue;
      const double Ct = a[7] / n;
      if (!(Ct > 0.0)) continue;
      const double k = C_I / (Ct * V_I);
      for (int ch = 0; ch < 3; ++ch) {
        const double E1 = a[ch] / n, E2 = a[3 + ch] / n;
        double var = E2 - E1 * E1;
        if (var < 0.0) var = 0.0;
        c.fac_x[(size_t)cidx * 12 + (0 * 2 + x) * 3 + ch] = (float)(k * E2);
        c.fac_x[(size_t)cidx * 12 + (1 * 2 + x) * 3 + ch] = (float)(k * var);
      }
    }
    if (ears_mode >= 0) {
      // EARS iterations: the shared factors of the cell into technique slot 0
      // (the fixed point restricted to beta_t = r_t lambda)
      double r[3], num[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}}, den = 0.0;
      ears_ratios(ears_mode, r);
      bool any = false;
      for (int t = 0; t < 3; ++t) {
        const double* a = c.acc + ((size_t)cidx * 3 + t) * 8;
        const double n = a[6];
        if (!(r[t] > 0.0) || !(n > 0.0)) continue;
        const double Ct = a[7] / n;
        if (!(Ct > 0.0)) continue;
        any = true;
        den = den + r[t] * Ct;
        for (int ch = 0; ch < 3; ++ch) {
          const double E1 = a[ch] / n, E2 = a[3 + ch] / n;
          double var = E2 - E1 * E1;
          if (var < 0.0) var = 0.0;
          num[0][ch] = num[0][ch] + E2 / r[t];
          num[1][ch] = num[1][ch] + var / r[t];
        }
      }
      if (any) {
        const double k = C_I / V_I;
        for (int ch = 0; ch < 3; ++ch) {
          c.fac[(size_t)cidx * 18 + (0 * 3 + 0) * 3 + ch] = (float)(k * (num[0][ch] / den));
          c.fac[(size_t)cidx * 18 + (1 * 3 + 0) * 3 + ch] = (float)(k * (num[1][ch] / den));
        }
      }
    }
  }
  if (!guided) return;
  // guided distribution of the next iteration: 0.9 learned + 0.1 uniform
  const double* h = c.hacc + 64 * (size_t)cidx;
  double tot = 0.0;
  for (int b = 0; b < 64; ++b) tot += h[b];
  if (!(tot > 0.0)) return;
  double run = 0.0;
  for (int b = 0; b < 64; ++b) {
    const double p = 0.9 * (h[b] / tot) + 0.1 / 64.0;
    run += p;
    c.pm[64 * (size_t)cidx + b] = (float)p;
    c.cdf[64 * (size_t)cidx + b] = b == 63 ? 1.0f : (float)run;
  }
}
// per cell: the fixed point, then (guided) the directional distribution;
// with img and npx > 0 also the inverse-variance weighted image (uses the
// device V_I)
void k_fixed_point(const CacheDev& c, const int32_t* n_cells_dev, const double* red, double C_I,
                   const Counters* cnt, double roots, int use_device_vi, double V_I_host,
                   int guided, int max_cells, const ImageDev* img, int npx, int spp,
                   const uint32_t* skip, hipStream_t s, int ears_mode) {
  const int cb = (max_cells + 255) / 256, pb = img ? (npx + 255) / 256 : 0;
  fixed_point_kernel<<<cb + pb, 256, 0, s>>>(c, n_cells_dev, red, C_I, cnt, roots, use_device_vi,
                                              V_I_host, guided, img ? *img : ImageDev{},
                                              img ? npx : 0, spp, cb, skip, ears_mode);
}

// ---------------------------------------------------------------------------
// octree refinement: leaves with more than split_visits visits and depth
// below the maximum split, in increasing leaf order, while the leaf budget
// allows.  One workgroup ranks the flagged leaves and advances the cell and
// node counts; then one wave per accepted leaf applies the split.
// scratch: [max_cells] ranks, then flagged total, old cell count, old node
// count.
// ---------------------------------------------------------------------------
constexpr int kScanRows = 16;  // rows of 1024 leaves per round
__global__ __launch_bounds__(1024) void scan_split_kernel(CacheDev c, int32_t* n_cells_dev,
                                                          int32_t* n_nodes_dev, uint32_t* rank,
                                                          uint32_t* tail, int split_visits,
                                                          int max_tree_depth, int max_cells,
                                                          const uint32_t* skip) {
  __shared__ uint32_t wcnt[kScanRows][16];  // flagged leaves per (row, wave), then prefixes
  __shared__ uint32_t rowbase[kScanRows + 1];
  __shared__ uint32_t carry;
  SKIP_IF(skip);
  const int n = *n_cells_dev;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, tid = threadIdx.x;
  if (tid == 0) carry = 0u;
  __syncthreads();
  for (int base = 0; base < n; base += 1024 * kScanRows) {
    // leaf base + 1024 k + tid of row k: coalesced loads, all issued first
    uint32_t vis[kScanRows], dep[kScanRows];
#pragma unroll
    for (int k = 0; k < kScanRows; ++k) {
      const int l = min(base + 1024 * k + tid, n - 1);
      vis[k] = c.visits[l];
      dep[k] = c.leaf_depth[l];
    }
    uint32_t flags = 0u, below[kScanRows];
#pragma unroll
    for (int k = 0; k < kScanRows; ++k) {
      const bool f = base + 1024 * k + tid < n && vis[k] > (uint32_t)split_visits &&
                     dep[k] < (uint32_t)max_tree_depth;
      const unsigned long long m = __ballot(f);
      below[k] = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
      if (f) flags |= 1u << k;
      if (lane == 0) wcnt[k][wid] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    // exclusive prefixes over the waves of each row, and of the rows
    if (tid < kScanRows) {
      uint32_t run = 0u;
      for (int w = 0; w < 16; ++w) {
        const uint32_t x = wcnt[tid][w];
        wcnt[tid][w] = run;
        run += x;
      }
      rowbase[tid + 1] = run;  // row total for now
    }
    __syncthreads();
    if (tid == 0) {
      uint32_t run = carry;
      for (int k = 0; k < kScanRows; ++k) {
        const uint32_t x = rowbase[k + 1];
        rowbase[k] = run;
        run += x;
      }
      rowbase[kScanRows] = run;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanRows; ++k) {
      const int l = base + 1024 * k + tid;
      if (l < n)
        rank[l] = ((flags >> k) & 1u) ? rowbase[k] + wcnt[k][wid] + below[k] : 0xFFFFFFFFu;
    }
    __syncthreads();
    if (tid == 0) carry = rowbase[kScanRows];
    __syncthreads();
  }
  if (tid == 0) {
    const int nn0 = *n_nodes_dev;
    const uint32_t room = max_cells > n ? (uint32_t)((max_cells - n) / 7) : 0u;
    const uint32_t acc = min(carry, room);
    tail[0] = acc;
    tail[1] = (uint32_t)n;
    tail[2] = (uint32_t)nn0;
    *n_cells_dev = n + 7 * (int)acc;
    *n_nodes_dev = nn0 + 8 * (int)acc;
  }
}
// one wave per leaf: lane 0 links the eight children into the tree, the
// lanes copy the parent's factors and distribution into the seven new cells
// and clear their statistics
__global__ __launch_bounds__(256) void apply_split_kernel(CacheDev c, const uint32_t* rank,
                                                          const uint32_t* tail,
                                                          const uint32_t* skip) {
  SKIP_IF(skip);
  const int lane = threadIdx.x & 63;
  const int l = (int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  const uint32_t acc = tail[0];
  const int n0 = (int)tail[1], nn0 = (int)tail[2];
  if (l >= n0) return;
  const uint32_t r = rank[l];
  if (r >= acc) return;  // not flagged (sentinel) or beyond the budget
  const uint32_t base = (uint32_t)nn0 + 8u * r;
  const uint32_t first = (uint32_t)n0 + 7u * r;  // ids of children 1..7
  if (lane == 0) {
    const uint32_t node = c.leaf_node[l];
    const uint32_t dep = c.leaf_depth[l] + 1u;
    c.nodes[node] = base;
    for (int ch = 0; ch < 8; ++ch) {
      const uint32_t id = ch == 0 ? (uint32_t)l : first + (uint32_t)(ch - 1);
      c.nodes[base + ch] = kLeafBit | id;
      c.leaf_node[id] = base + ch;
      c.leaf_depth[id] = dep;
    }
  }
  for (int k = lane; k < 7 * 18; k += 64)
    c.fac[(size_t)(first + k / 18) * 18 + k % 18] = c.fac[(size_t)l * 18 + k % 18];
  if (c.fac_x) {
    for (int k = lane; k < 7 * 12; k += 64)
      c.fac_x[(size_t)(first + k / 12) * 12 + k % 12] = c.fac_x[(size_t)l * 12 + k % 12];
    for (int k = lane; k < 7 * 16; k += 64) c.acc_x[(size_t)(first + k / 16) * 16 + k % 16] = 0.0;
  }
  for (int k = lane; k < 7 * 64; k += 64) {
    const size_t dst = (size_t)(first + k / 64) * 64 + k % 64, src = (size_t)l * 64 + k % 64;
    c.pm[dst] = c.pm[src];
    c.cdf[dst] = c.cdf[src];
    c.hacc[dst] = 0.0;
  }
  for (int k = lane; k < 7 * 24; k += 64) c.acc[(size_t)(first + k / 24) * 24 + k % 24] = 0.0;
  if (lane < 7) c.visits[first + lane] = 0u;
}
void k_refine(const CacheDev& c, int32_t* n_cells_dev, int32_t* n_nodes_dev, uint32_t* scratch,
              int split_visits, int max_tree_depth, int max_cells, const uint32_t* skip,
              hipStream_t s) {
  scan_split_kernel<<<1, 1024, 0, s>>>(c, n_cells_dev, n_nodes_dev, scratch, scratch + max_cells,
                                       split_visits, max_tree_depth, max_cells, skip);
  apply_split_kernel<<<(max_cells + 3) / 4, 256, 0, s>>>(c, scratch, scratch + max_cells, skip);
}

// per-scene summary of a batched iteration, gathered for one read-back:
// [0] overflow, [1..6] ray / vertex / sample totals, [7..14] image
// reductions, [15] cells, [16] nodes
__global__ void batch_summary_kernel(const Counters* cnt, const double* red,
                                     const int32_t* n_cells_dev, double* out) {
  const int t = threadIdx.x;
  if (t == 0) out[0] = (double)cnt->overflow_any;
  if (t == 1) out[1] = (double)cnt->rays_ext;
  if (t == 2) out[2] = (double)cnt->rays_shadow;
  if (t == 3) out[3] = (double)cnt->rays_light;
  if (t == 4) out[4] = (double)cnt->rays_conn;
  if (t == 5) out[5] = (double)cnt->vertices;
  if (t == 6) out[6] = (double)cnt->samples;
  if (t >= 7 && t < 15) out[t] = red[t - 7];
  if (t == 15) out[15] = (double)n_cells_dev[0];
  if (t == 16) out[16] = (double)n_cells_dev[1];
}
void k_batch_summary(const Counters* cnt, const double* red, const int32_t* n_cells_dev,
                     double* out, hipStream_t s) {
  batch_summary_kernel<<<1, 64, 0, s>>>(cnt, red, n_cells_dev, out);
}
__global__ void set_i32_kernel(int32_t* p, int32_t v) { *p = v; }
void k_set_i32(int32_t* p, int32_t v, hipStream_t s) { set_i32_kernel<<<1, 1, 0, s>>>(p, v); }

// inverse-variance weighted combination of the iterations (Sec. 5.1):
// iteration images weighted by spp / V_I
__device__ __forceinline__ void ivw_at(ImageDev& img, int i, int spp, const double (&vs)[2]) {
  const double V_I = vs[1] > 0.0 ? vs[0] / vs[1] : 0.0;
  if (!(V_I > 0.0)) return;
  const double w = (double)spp / V_I;
  if (i == 0) img.red[5] += w;
  for (int ch = 0; ch < 3; ++ch) {
    const size_t e = 3 * (size_t)i + ch;
    img.ivw_acc[e] += w * (double)(img.iter_sum[e] / (float)spp);
  }
}

// ---------------------------------------------------------------------------
// probes of the building blocks (tests)
// ---------------------------------------------------------------------------
__global__ void probe_kernel(int kind, int n, const void* in, void* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (kind == 0) {
    const uint32_t* a = (const uint32_t*)in + 6 * (size_t)i;
    const u4 o = philox10(a[0], a[1], u4{a[2], a[3], a[4], a[5]});
    uint32_t* b = (uint32_t*)out + 4 * (size_t)i;
    b[0] = o.a; b[1] = o.b; b[2] = o.c; b[3] = o.d;
  } else if (kind == 1) {
    float s, c;
    sincos_turns(((const float*)in)[i], &s, &c);
    ((float*)out)[2 * (size_t)i] = s;
    ((float*)out)[2 * (size_t)i + 1] = c;
  } else if (kind == 2) {
    const float* a = (const float*)in + 4 * (size_t)i;
    const float beta[3] = {a[0], a[1], a[2]};
    uint32_t g[3];
    round_counts(beta, a[3], g);
    uint32_t* b = (uint32_t*)out + 3 * (size_t)i;
    b[0] = g[0]; b[1] = g[1]; b[2] = g[2];
  }
}
void k_probe(int kind, int n, const void* in, void* out, hipStream_t s) {
  probe_kernel<<<(n + 255) / 256, 256, 0, s>>>(kind, n, in, out);
}

}  // namespace mars
