// Device building blocks of the MARS path (gfx950).
//
// Arithmetic is binary32 with the evaluation order written out (the library
// is compiled with -ffp-contract=off and correctly rounded division and
// square root), so that integer decisions taken from floats (cells, rounded
// sample counts) are reproducible on any IEEE implementation.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mars_internal.h"

namespace mars {

struct f3 {
  float x, y, z;
};
__device__ __forceinline__ f3 mk3(float x, float y, float z) { return f3{x, y, z}; }
__device__ __forceinline__ f3 sub3(f3 a, f3 b) { return mk3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ f3 add3(f3 a, f3 b) { return mk3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ f3 scl3(f3 a, float s) { return mk3(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ float dot3(f3 a, f3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
__device__ __forceinline__ f3 cross3(f3 a, f3 b) {
  return mk3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ f3 norm3(f3 a) {
  float il = 1.0f / sqrtf(dot3(a, a));
  return scl3(a, il);
}
__device__ __forceinline__ float lum(f3 c) { return (0.2126f * c.x + 0.7152f * c.y) + 0.0722f * c.z; }
__device__ __forceinline__ f3 xyz(float4 v) { return mk3(v.x, v.y, v.z); }

constexpr float kPi = 3.14159265358979323846f;
constexpr float kInvPi = 0.318309886183790671538f;
constexpr float kOneMinus = 0.99999994f;  // 1 - 2^-24
constexpr uint32_t kNoCell = 0xFFFFFFFFu;
constexpr uint32_t kMiss = 0xFFFFFFFFu;

// ---------------------------------------------------------------------------
// Philox4x32-10 counter-based generator (Salmon et al., SC'11): ten rounds of
// two 32x32->64 bit products, key bumped by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
struct u4 {
  uint32_t a, b, c, d;
};
__device__ __forceinline__ u4 philox10(uint32_t k0, uint32_t k1, u4 x) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t lo0 = 0xD2511F53u * x.a, hi0 = __umulhi(0xD2511F53u, x.a);
    uint32_t lo1 = 0xCD9E8D57u * x.c, hi1 = __umulhi(0xCD9E8D57u, x.c);
    x = u4{hi1 ^ x.b ^ k0, lo1, hi0 ^ x.d ^ k1, lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return x;
}

// random stream of a path-tree node: its identity is a pure function of the
// tree address, so the same sample gets the same numbers in any queue order
constexpr uint32_t kTagCam = 0x43000000u, kTagChild = 0x4B000000u, kTagDraw = 0x44000000u,
                   kTagLight = 0x4C000000u;

struct Key {
  uint32_t k0, k1;
};
__device__ __forceinline__ uint2 stream_root(Key k, uint32_t pix, uint32_t s, uint32_t iter,
                                             uint32_t tag) {
  u4 o = philox10(k.k0, k.k1, u4{pix, s, iter, tag});
  return make_uint2(o.a, o.b);
}
__device__ __forceinline__ uint2 stream_child(Key k, uint2 p, uint32_t tech, uint32_t idx,
                                              uint32_t depth) {
  u4 o = philox10(k.k0, k.k1,
                  u4{p.x, p.y, (tech << 16) | (idx & 0xFFFFu), kTagChild | (depth & 0xFFFFu)});
  return make_uint2(o.a, o.b);
}
__device__ __forceinline__ float to_unit(uint32_t x) {
  return (float)(x >> 8) * 5.9604644775390625e-8f;
}
__device__ __forceinline__ float4 draw4(Key k, uint2 s, uint32_t j) {
  u4 o = philox10(k.k0, k.k1, u4{s.x, s.y, j, kTagDraw});
  return make_float4(to_unit(o.a), to_unit(o.b), to_unit(o.c), to_unit(o.d));
}

// ---------------------------------------------------------------------------
// sin and cos of 2 pi u, u in [0, 1): quarter-turn reduction (exact for
// u = m 2^-24), Taylor series of sin/cos in theta = 2 pi r, |r| <= 1/8.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sincos_turns(float u, float* s_out, float* c_out) {
  const float q4 = floorf(u * 4.0f + 0.5f);
  const float r = u - q4 * 0.25f;
  const int quad = ((int)q4) & 3;
  const float th = r * 6.28318530717958647692f;
  const float t2 = th * th;
  float s = (float)(-1.0 / 39916800.0);
  s = s * t2 + (float)(1.0 / 362880.0);
  s = s * t2 + (float)(-1.0 / 5040.0);
  s = s * t2 + (float)(1.0 / 120.0);
  s = s * t2 + (float)(-1.0 / 6.0);
  const float sn = th + (th * t2) * s;
  float c = (float)(1.0 / 479001600.0);
  c = c * t2 + (float)(-1.0 / 3628800.0);
  c = c * t2 + (float)(1.0 / 40320.0);
  c = c * t2 + (float)(-1.0 / 720.0);
  c = c * t2 + (float)(1.0 / 24.0);
  c = c * t2 + (float)(-1.0 / 2.0);
  const float cs = 1.0f + t2 * c;
  float S = sn, C = cs;
  if (quad == 1) { S = cs; C = -sn; }
  else if (quad == 2) { S = -sn; C = -cs; }
  else if (quad == 3) { S = -cs; C = sn; }
  *s_out = S;
  *c_out = C;
}

// ---------------------------------------------------------------------------
// low-discrepancy stochastic rounding: a single uniform shared by all
// techniques; each technique takes floor(beta + r) samples and passes the
// fractional remainder on (supplement, Alg. 1)
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void round_counts_n(const float* beta, float u, uint32_t* g) {
  float r = u;
#pragma unroll
  for (int t = 0; t < N; ++t) {
    const float s = r + beta[t];
    const float f = floorf(s);
    g[t] = (uint32_t)f;
    r = s - f;
  }
}
__device__ __forceinline__ void round_counts(const float beta[3], float u, uint32_t g[3]) {
  round_counts_n<3>(beta, u, g);
}

// each count rounded with its own uniform (the scheme Alg. 1 improves on):
// gamma_t = floor(beta_t + u_t), which is ceil(beta_t) with probability
// beta_t - floor(beta_t)
__device__ __forceinline__ void round_counts_independent(const float beta[3], float4 u,
                                                         uint32_t g[3]) {
  g[0] = (uint32_t)floorf(beta[0] + u.x);
  g[1] = (uint32_t)floorf(beta[1] + u.y);
  g[2] = (uint32_t)floorf(beta[2] + u.z);
}

// ---------------------------------------------------------------------------
// shading frame (Duff et al. 2017, branchless orthonormal basis)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void frame(f3 n, f3* t, f3* b) {
  const float sgn = n.z >= 0.0f ? 1.0f : -1.0f;
  const float a = -1.0f / (sgn + n.z);
  const float bb = (n.x * n.y) * a;
  *t = mk3(1.0f + (sgn * (n.x * n.x)) * a, sgn * bb, -(sgn * n.x));
  *b = mk3(bb, sgn + (n.y * n.y) * a, -n.y);
}
__device__ __forceinline__ f3 local_to_world(f3 l, f3 t, f3 b, f3 n) {
  return mk3((l.x * t.x + l.y * b.x) + l.z * n.x, (l.x * t.y + l.y * b.y) + l.z * n.y,
             (l.x * t.z + l.y * b.z) + l.z * n.z);
}

// material record: kind, albedo rgb, alpha, emission rgb
struct Mat {
  float kind, r, g, b, alpha, er, eg, eb;
};

// direction from the BSDF sampling technique: cosine-weighted (Lambert) or
// GGX half-vector sampling (Walter et al. 2007) reflected about h.
__device__ __forceinline__ bool sample_bsdf(const Mat& m, f3 n, f3 wo, float u0, float u1,
                                            f3* wi) {
  f3 t, b;
  frame(n, &t, &b);
  float sn, cs;
  if (m.kind == 0.0f) {
    const float r = sqrtf(u0);
    sincos_turns(u1, &sn, &cs);
    *wi = local_to_world(mk3(r * cs, r * sn, sqrtf(fmaxf(0.0f, 1.0f - u0))), t, b, n);
  } else {
    const float a2 = m.alpha * m.alpha;
    const float t2 = (a2 * u0) / (1.0f - u0);
    const float ch = 1.0f / sqrtf(1.0f + t2);
    const float sh = sqrtf(fmaxf(0.0f, 1.0f - ch * ch));
    sincos_turns(u1, &sn, &cs);
    const f3 h = local_to_world(mk3(sh * cs, sh * sn, ch), t, b, n);
    const float d = dot3(wo, h);
    *wi = mk3((2.0f * d) * h.x - wo.x, (2.0f * d) * h.y - wo.y, (2.0f * d) * h.z - wo.z);
  }
  return dot3(n, *wi) > 0.0f;
}

// f(wo, wi) |cos theta_i| and the BSDF-sampling density of wi
__device__ __forceinline__ void eval_bsdf(const Mat& m, f3 n, f3 wo, f3 wi, f3* fcos,
                                          float* pdf) {
  const float ci = dot3(n, wi), co = dot3(n, wo);
  if (ci <= 0.0f || co <= 0.0f) {
    *fcos = mk3(0.0f, 0.0f, 0.0f);
    *pdf = 0.0f;
    return;
  }
  if (m.kind == 0.0f) {
    *fcos = mk3((m.r * kInvPi) * ci, (m.g * kInvPi) * ci, (m.b * kInvPi) * ci);
    *pdf = ci * kInvPi;
    return;
  }
  const float a2 = m.alpha * m.alpha;
  const f3 h = norm3(add3(wo, wi));
  const float ch = dot3(n, h), oh = dot3(wo, h);
  if (ch <= 0.0f || oh <= 0.0f) {
    *fcos = mk3(0.0f, 0.0f, 0.0f);
    *pdf = 0.0f;
    return;
  }
  const float k = (ch * ch) * (a2 - 1.0f) + 1.0f;
  const float D = a2 / ((kPi * k) * k);
  const float g1o = (2.0f * co) / (co + sqrtf(a2 + (1.0f - a2) * (co * co)));
  const float g1i = (2.0f * ci) / (ci + sqrtf(a2 + (1.0f - a2) * (ci * ci)));
  const float G = g1o * g1i;
  const float mm = fmaxf(0.0f, 1.0f - dot3(wi, h));
  const float m5 = ((mm * mm) * (mm * mm)) * mm;
  const float DG = D * G;
  const float den = 4.0f * co;
  *fcos = mk3((DG * (m.r + (1.0f - m.r) * m5)) / den, (DG * (m.g + (1.0f - m.g) * m5)) / den,
              (DG * (m.b + (1.0f - m.b) * m5)) / den);
  *pdf = (D * ch) / (4.0f * oh);
}

// ---------------------------------------------------------------------------
// guided technique: 8 x 8 equal-area histogram over the sphere (8 bins of
// cos(theta) in [-1, 1], 8 bins of phi), world frame
// ---------------------------------------------------------------------------
__device__ __forceinline__ int octant_of(float x, float y) {
  if (y >= 0.0f) {
    if (x > 0.0f) return (y < x) ? 0 : 1;
    return (y > -x) ? 2 : 3;
  }
  if (x < 0.0f) return (-y < -x) ? 4 : 5;
  return (-y > x) ? 6 : 7;
}
__device__ __forceinline__ int dir_bin(f3 w) {
  int bz = (int)floorf((w.z + 1.0f) * 4.0f);
  bz = bz < 0 ? 0 : (bz > 7 ? 7 : bz);
  return bz * 8 + octant_of(w.x, w.y);
}
__device__ __forceinline__ float guided_density(const float* pm, f3 w) {
  return pm[dir_bin(w)] * (float)(16.0 / 3.14159265358979323846);
}
__device__ __forceinline__ f3 guided_direction(const float* cdf, float u0, float u1, float u2) {
  int lo = 0, hi = 63;  // first bin with u0 < cdf[bin]
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (u0 < cdf[mid]) hi = mid; else lo = mid + 1;
  }
  const int bz = lo >> 3, bp = lo & 7;
  const float z = -1.0f + 0.25f * ((float)bz + u1);
  float sn, cs;
  sincos_turns(((float)bp + u2) * 0.125f, &sn, &cs);
  const float s = sqrtf(fmaxf(0.0f, 1.0f - z * z));
  return mk3(s * cs, s * sn, z);
}

// ---------------------------------------------------------------------------
// octree cache lookup: normalised position, one bit per axis per level
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t cell_of(const uint32_t* __restrict__ nodes, f3 lo, float inv,
                                            f3 p) {
  float qx = fminf(fmaxf((p.x - lo.x) * inv, 0.0f), kOneMinus);
  float qy = fminf(fmaxf((p.y - lo.y) * inv, 0.0f), kOneMinus);
  float qz = fminf(fmaxf((p.z - lo.z) * inv, 0.0f), kOneMinus);
  uint32_t v = nodes[0];
  while (!(v & kLeafBit)) {
    const uint32_t bx = qx >= 0.5f, by = qy >= 0.5f, bz = qz >= 0.5f;
    qx = qx * 2.0f - (float)bx;
    qy = qy * 2.0f - (float)by;
    qz = qz * 2.0f - (float)bz;
    v = nodes[v + (bx | (by << 1) | (bz << 2))];
  }
  return v & ~kLeafBit;
}

}  // namespace mars
