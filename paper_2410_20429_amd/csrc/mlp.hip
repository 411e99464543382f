// Learned cache: a small MLP that predicts the log sample count of every
// technique, relative to |T / I~|, from a vertex's position normalised to the
// octree's cube and its geometric normal as stored (sin/cos encoding with 6
// frequencies -> 72 features, padded to 80; three hidden layers of 64 ReLU
// units; 3 linear outputs).  Forward and backward
// run as bfloat16 matrix-core products with binary32 accumulation, one
// 16-sample tile per wave: training on v_mfma_f32_16x16x16_bf16, inference
// on gfx950's v_mfma_f32_16x16x32_bf16 (half the products per tile).  Master
// weights, biases and Adam moments are binary32.
//
// MFMA 16x16x16 operand layout (lane l = 0..63, element r = 0..3; the
// inference's 16x16x32 form is described with its kernels):
//   A (16 x 16, M x K): A[l % 16][4 (l / 16) + r]
//   B (16 x 16, K x N): B[4 (l / 16) + r][l % 16]
//   D (16 x 16, M x N): D[4 (l / 16) + r][l % 16]
#include <hip/hip_runtime.h>

#include <mutex>

#include "device_math.hpp"
#include "mars_internal.h"

namespace mars {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// binary32 -> bfloat16, round to nearest even (two neighbouring conversions
// become one packed gfx950 conversion)
__device__ __forceinline__ uint16_t to_bf16(float x) {
  return __builtin_bit_cast(uint16_t, (__bf16)x);
}
__device__ __forceinline__ void to_bf16x2(float x, float y, uint16_t* hx, uint16_t* hy) {
  *hx = to_bf16(x);
  *hy = to_bf16(y);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ v4f mma(v4s a, v4s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// bfloat16 copy of the weights (biases are read in binary32 from the master)
constexpr int qW1 = 0, qW2 = 5120, qW3 = 9216, qW4 = 13312, kQW = 14336;
__host__ __device__ constexpr int qindex(int p) {
  return p < kMlpB1 ? p
       : (p >= kMlpW2 && p < kMlpB2) ? qW2 + (p - kMlpW2)
       : (p >= kMlpW3 && p < kMlpB3) ? qW3 + (p - kMlpW3)
       : (p >= kMlpW4 && p < kMlpB4) ? qW4 + (p - kMlpW4) : -1;
}

// features of one vertex: x = (q.xyz, n.xyz); f[(d*6+k)*2 + s] = sin/cos(2^k pi x_d).
// Features k (even) and k + 1 are the sine and cosine of one angle; with k a
// multiple of 4, features k + 2, k + 3 belong to the same input and twice
// the angle.
__device__ __forceinline__ void feature_pair(const float* x, int k, float* fs, float* fc) {
  if (k >= 72) {
    *fs = 0.0f;
    *fc = 0.0f;
    return;
  }
  const int d = k / 12, kk = (k % 12) >> 1;
  const float a = ldexpf(x[d], kk);
  sincospif(a, fs, fc);
}

// Forward pass of one 16-sample tile by one wave, keeping what the backward
// pass needs.  x: this lane's sample inputs (sample = lane % 16).  wq: the
// bfloat16 weights (global memory or a copy in LDS).  Hidden activations go
// to hs[l][16][64] (bfloat16), features to xs[16][80] when xs != nullptr.
// Returns the output tile in D layout (rows = samples, columns = outputs).
// One-wave workgroups: the wave meets itself at workgroup barriers.
__device__ __forceinline__ v4f mlp_forward_tile(const float* __restrict__ master,
                                                const uint16_t* __restrict__ wq, const float* x,
                                                uint16_t (*hs)[16][64], uint16_t (*xs)[80]) {
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  v4f acc[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) acc[nt] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int ks = 0; ks < 5; ++ks) {
    v4s a;
    // this lane's features k0 .. k0 + 3, k0 = 16 ks + 4 lg: the sine and
    // cosine of one angle 2^kk pi x_d (kk even) and of its double, the
    // latter from the double-angle identities
    const int k0 = 16 * ks + 4 * lg;
    float fs, fc, gs, gc;
    feature_pair(x, k0, &fs, &fc);
    if (k0 < 72) {
      gs = 2.0f * (fs * fc);
      gc = (fc - fs) * (fc + fs);
    } else {
      gs = 0.0f;
      gc = 0.0f;
    }
    uint16_t h[4];
    to_bf16x2(fs, fc, &h[0], &h[1]);
    to_bf16x2(gs, gc, &h[2], &h[3]);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      a[r] = (short)h[r];
      if (xs) xs[lr][k0 + r] = h[r];
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const uint16_t* w = wq + qW1 + (16 * nt + lr) * 80 + 16 * ks + 4 * lg;
      const v4s b = {(short)w[0], (short)w[1], (short)w[2], (short)w[3]};
      acc[nt] = mma(a, b, acc[nt]);
    }
  }
  int boff[3] = {kMlpB1, kMlpB2, kMlpB3};
  int woff[3] = {qW2, qW3, qW4};
  for (int l = 0; l < 3; ++l) {
    const int hb = l;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int j = 16 * nt + lr;
      const float bj = master[boff[l] + j];
#pragma unroll
      for (int r = 0; r < 4; r += 2) {
        uint16_t h0, h1;
        to_bf16x2(fmaxf(acc[nt][r] + bj, 0.0f), fmaxf(acc[nt][r + 1] + bj, 0.0f), &h0, &h1);
        hs[hb][4 * lg + r][j] = h0;
        hs[hb][4 * lg + r + 1][j] = h1;
      }
    }
    __syncthreads();
    const int ntn = l < 2 ? 4 : 1;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const uint16_t* hr = &hs[hb][lr][16 * ks + 4 * lg];
      const v4s a = {(short)hr[0], (short)hr[1], (short)hr[2], (short)hr[3]};
      for (int nt = 0; nt < ntn; ++nt) {
        const uint16_t* w = wq + woff[l] + (16 * nt + lr) * 64 + 16 * ks + 4 * lg;
        const v4s b = {(short)w[0], (short)w[1], (short)w[2], (short)w[3]};
        acc[nt] = mma(a, b, acc[nt]);
      }
    }
  }
  v4f y = acc[0];
  const float b4 = master[kMlpB4 + lr];
#pragma unroll
  for (int r = 0; r < 4; ++r) y[r] += b4;
  return y;
}

// ---------------------------------------------------------------------------
// Inference.  Every layer is computed transposed, Z^T = W H^T, with the
// weights as the A operand and the activations as the B operand, on gfx950's
// 16x16x32 bfloat16 matrix-core product (v_mfma_f32_16x16x32_bf16): lane l
// holds elements e = 0..7 of row l % 16 of A and of column l % 16 of B in
// the K positions of its lane group l / 16, the same positions for A and B.
// Which of the 32 products a position stands for is the caller's choice as
// long as A and B agree: here element e of lane group g in chunk c stands for
// input 16 (2c + e / 4) + 4g + e % 4.  The output tile D[neuron 16 nt +
// 4 (l / 16) + r][sample l % 16] of output block nt is, after bias, ReLU and
// rounding, elements 4 (nt % 2) .. 4 (nt % 2) + 3 of the B operand of chunk
// nt / 2 of the next layer, so activations stay in registers.  (The same
// products as mlp_forward_tile; only the order of each binary32 matrix-core
// accumulation may differ.)
//
// The weights are staged in LDS in fragment order: the A operand of every
// (layer, output block, chunk) as 64 consecutive 16-byte lane fragments,
// so that each operand is one conflict-free 1 KB read.  Blocks: layer 1
// 3 nt + c (nt < 4, c < 3; inputs 80 .. 95 are zero), layer 2 12 + 2 nt + c,
// layer 3 20 + 2 nt + c, output layer 28 + c (one output block); 30 KB.
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef short v8s __attribute__((ext_vector_type(8)));
__device__ __forceinline__ v4f mma32(v8s a, v8s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a),
                                                 __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}
__device__ __forceinline__ v8s cat8(v4s lo, v4s hi) {
  return v8s{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}

constexpr int kFragBlocks = 30;
constexpr int kInferWaves = 8;            // waves per inference workgroup
constexpr uint32_t kNoTile = 0xFFFFFFFFu;

// Stages the fragments: fragment f (block f / 64, lane f % 64) is two runs of
// four consecutive weights, inputs 16 (2c) + 4g .. + 3 and 16 (2c + 1) + 4g
// .. + 3 of output row 16 nt + l % 16 (a run past input 79 of layer 1 is
// zero).  Every thread loads all of its fragments before it writes any.
template <int kThreads>
__device__ __forceinline__ void stage_fragments(const uint16_t* __restrict__ wq, uint4* wf) {
  constexpr int kN = kFragBlocks * 64, kPer = (kN + kThreads - 1) / kThreads;
  uint4 v[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int f = threadIdx.x + j * kThreads;
    v[j] = make_uint4(0u, 0u, 0u, 0u);
    if (f < kN) {
      const int blk = f >> 6, ln = f & 63, lr = ln & 15, lg = ln >> 4;
      int base, stride, nt, c, nin;
      if (blk < 12) {
        base = qW1; stride = 80; nin = 80; nt = blk / 3; c = blk % 3;
      } else if (blk < 28) {
        const int b = (blk - 12) & 7;
        base = blk < 20 ? qW2 : qW3; stride = 64; nin = 64; nt = b >> 1; c = b & 1;
      } else {
        base = qW4; stride = 64; nin = 64; nt = 0; c = blk - 28;
      }
      const int row = base + (16 * nt + lr) * stride, k0 = 32 * c + 4 * lg, k1 = k0 + 16;
      const uint2 lo = *reinterpret_cast<const uint2*>(wq + row + k0);
      const uint2 hi = k1 < nin ? *reinterpret_cast<const uint2*>(wq + row + k1) : make_uint2(0u, 0u);
      v[j] = make_uint4(lo.x, lo.y, hi.x, hi.y);
    }
  }
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int f = threadIdx.x + j * kThreads;
    if (f < kN) wf[f] = v[j];
  }
}

// the biases b1, b2, b3 (64 each) and b4 (16) as 52 float4 in LDS
__device__ __forceinline__ void stage_biases(const float* __restrict__ master, float4* bl) {
  float* b = reinterpret_cast<float*>(bl);
  for (int k = threadIdx.x; k < 208; k += blockDim.x)
    b[k] = k < 192 ? master[(k < 64 ? kMlpB1 : (k < 128 ? kMlpB2 : kMlpB3)) + (k & 63)]
                   : master[kMlpB4 + (k - 192)];
}

__device__ __forceinline__ v8s frag(const uint4* wf, int blk, int lane) {
  return __builtin_bit_cast(v8s, wf[blk * 64 + lane]);
}

// bias, ReLU and bfloat16 rounding of one output block (neurons 16 nt +
// 4 (l / 16) + r of sample l % 16): half of the next layer's B operand
__device__ __forceinline__ v4s relu_bf16(const v4f& z, float4 b) {
  uint16_t h[4];
  to_bf16x2(fmaxf(z[0] + b.x, 0.0f), fmaxf(z[1] + b.y, 0.0f), &h[0], &h[1]);
  to_bf16x2(fmaxf(z[2] + b.z, 0.0f), fmaxf(z[3] + b.w, 0.0f), &h[2], &h[3]);
  return v4s{(short)h[0], (short)h[1], (short)h[2], (short)h[3]};
}

// features k0 .. k0 + 3 of a sample, k0 a multiple of 4: the sine and cosine
// of one angle 2^kk pi x_d (kk even) and of its double, the latter from the
// double-angle identities (zero past feature 71)
__device__ __forceinline__ v4s feature_quad(const float* x, int k0) {
  float fs, fc, gs, gc;
  feature_pair(x, k0, &fs, &fc);
  if (k0 < 72) {
    gs = 2.0f * (fs * fc);
    gc = (fc - fs) * (fc + fs);
  } else {
    gs = 0.0f;
    gc = 0.0f;
  }
  uint16_t h[4];
  to_bf16x2(fs, fc, &h[0], &h[1]);
  to_bf16x2(gs, gc, &h[2], &h[3]);
  return v4s{(short)h[0], (short)h[1], (short)h[2], (short)h[3]};
}

// One 16-sample tile by one wave.  x: the inputs of sample l % 16 (the same
// in the four lanes that hold it).  Returns D[output 4 (l / 16) + r][sample
// l % 16]: the lanes l < 16 hold outputs 0..3 of sample l.
__device__ __forceinline__ v4f mlp_infer_tile(const uint4* wf, const float4* bl, const float* x) {
  const int lane = threadIdx.x & 63, lg = lane >> 4;
  v4f acc[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) acc[nt] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const v8s b = cat8(feature_quad(x, 32 * c + 4 * lg), feature_quad(x, 32 * c + 16 + 4 * lg));
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = mma32(frag(wf, 3 * nt + c, lane), b, acc[nt]);
  }
  v4s hb[4];
#pragma unroll
  for (int l = 0; l < 2; ++l) {
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) hb[nt] = relu_bf16(acc[nt], bl[16 * l + 4 * nt + lg]);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const v8s b = cat8(hb[2 * c], hb[2 * c + 1]);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
        acc[nt] = mma32(frag(wf, 12 + 8 * l + 2 * nt + c, lane), b, acc[nt]);
    }
  }
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) hb[nt] = relu_bf16(acc[nt], bl[32 + 4 * nt + lg]);
  v4f y = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int c = 0; c < 2; ++c) y = mma32(frag(wf, 28 + c, lane), cat8(hb[2 * c], hb[2 * c + 1]), y);
  const float4 b4 = bl[48 + lg];
  y[0] += b4.x;
  y[1] += b4.y;
  y[2] += b4.z;
  y[3] += b4.w;
  return y;
}

// s_waitcnt vmcnt(0) (expcnt and lgkmcnt left at their maxima, the gfx9
// encoding): every vector memory operation issued so far has completed.  At
// the top of a pipelined loop this costs nothing (what is outstanding was
// issued a tile's computation earlier) and tells the compiler's wait
// insertion that nothing is outstanding, which it cannot prove by itself
// where loads are conditional and the first iteration's come from before the
// loop; otherwise it waits, in the middle of the tile, for the stores and
// loads the tile has just issued.
__device__ __forceinline__ void wait_vector_memory() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Inference kernels: the fragments and biases are staged once per
// workgroup; each of its kInferWaves waves then runs 16-sample tiles (31 KB
// of LDS per workgroup).  Every global access of a tile is issued a whole
// tile's computation before it is needed: the records two tiles ahead, the
// normals one tile ahead, and the outputs are stored one tile late.  (Vector
// memory operations complete in the order they are issued, stores included,
// so a wait for any of them is a wait for all that were issued before it.)

// inference over a list of vertices given as (q, n)
__global__ __launch_bounds__(64 * kInferWaves) void mlp_infer_inputs_kernel(MlpDev m, const float* x6,
                                                                            int n, float* y3) {
  __shared__ uint4 wf[kFragBlocks * 64];
  __shared__ float4 bl[52];
  stage_fragments<64 * kInferWaves>(m.wq, wf);
  stage_biases(m.master, bl);
  __syncthreads();
  const int lane = threadIdx.x & 63, lr = lane & 15, w = threadIdx.x >> 6;
  for (int tile = blockIdx.x * kInferWaves + w; tile * 16 < n; tile += gridDim.x * kInferWaves) {
    const int s = tile * 16 + lr;
    float x[6] = {0, 0, 0, 0, 0, 0};
    if (s < n)
      for (int k = 0; k < 6; ++k) x[k] = x6[6 * (size_t)s + k];
    const v4f y = mlp_infer_tile(wf, bl, x);
    if (s < n && lane < 16)
      for (int t = 0; t < 3; ++t) y3[3 * (size_t)s + t] = y[t];
  }
}
void k_mlp_forward(const MlpDev& m, const float* x6, int n, float* y3, hipStream_t s) {
  const int tiles = (n + 15) / 16;
  const int blocks = std::max(1, std::min((tiles + kInferWaves - 1) / kInferWaves, 2048));
  mlp_infer_inputs_kernel<<<blocks, 64 * kInferWaves, 0, s>>>(m, x6, n, y3);
}

// network inputs of a vertex: position normalised to the octree cube, and
// the geometric normal as stored
__device__ __forceinline__ void mlp_input(const SceneDev& sc, f3 p, f3 ng, float* x) {
  x[0] = fminf(fmaxf((p.x - sc.oct_lo[0]) * sc.oct_inv, 0.0f), kOneMinus);
  x[1] = fminf(fmaxf((p.y - sc.oct_lo[1]) * sc.oct_inv, 0.0f), kOneMinus);
  x[2] = fminf(fmaxf((p.z - sc.oct_lo[2]) * sc.oct_inv, 0.0f), kOneMinus);
  x[3] = ng.x; x[4] = ng.y; x[5] = ng.z;
}

// inference at the vertices of one depth's queue (hits with d < D): inputs
// from the hit point and the geometric normal, outputs to m.y[d * cap + j].
struct InferRec {
  uint2 h;       // hit (t bits, primitive); primitive kMiss: no sample
  float4 r0, r1;
};

__global__ __launch_bounds__(64 * kInferWaves) void mlp_infer_queue_kernel(SceneDev sc,
                                                                           QueuesDev q, MlpDev m,
                                                                           const Counters* cnt,
                                                                           int d) {
  __shared__ uint4 wf[kFragBlocks * 64];
  __shared__ float4 bl[52];
  if (cnt->overflow) return;
  const uint32_t n = min(cnt->n_ray[d], (uint32_t)q.cap);
  if ((size_t)blockIdx.x * kInferWaves * 16 >= n) return;  // no tile for this workgroup
  stage_fragments<64 * kInferWaves>(m.wq, wf);
  stage_biases(m.master, bl);
  __syncthreads();
  const int lane = threadIdx.x & 63, lr = lane & 15, w = threadIdx.x >> 6;
  const size_t L = (size_t)d * q.cap;
  const uint32_t stride = gridDim.x * kInferWaves;
  const float4 zero4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  // this lane's sample (lr) of a tile
  auto fetch = [&](uint32_t tile) {
    InferRec r{make_uint2(0u, kMiss), zero4, zero4};
    const uint32_t s = tile * 16 + lr;
    if (tile < kNoTile / 16 && s < n) {
      r.h = q.H[L + s];
      r.r0 = q.R0[L + s];
      r.r1 = q.R1[L + s];
    }
    return r;
  };
  auto normal = [&](const InferRec& r) { return r.h.y != kMiss ? sc.tri_ng[r.h.y] : zero4; };
  // outputs 0..3 of sample s (the fourth is padding) from the lanes < 16
  auto store = [&](uint32_t tile, const v4f& y) {
    const uint32_t s = tile * 16 + lr;
    if (lane < 16 && s < n)
      reinterpret_cast<float4*>(m.y)[L + s] = make_float4(y[0], y[1], y[2], y[3]);
  };
  uint32_t tile = blockIdx.x * kInferWaves + w;
  InferRec cur = fetch(tile);
  float4 ng = normal(cur);
  InferRec nxt = fetch(tile + stride);
  v4f yp = v4f{0.0f, 0.0f, 0.0f, 0.0f};
  uint32_t tp = kNoTile;  // the tile yp belongs to
  for (; tile * 16 < n; tile += stride) {
    wait_vector_memory();
    if (tp != kNoTile) store(tp, yp);
    float x[6] = {0, 0, 0, 0, 0, 0};
    if (cur.h.y != kMiss) {
      const float t = __uint_as_float(cur.h.x);
      const f3 p = mk3(cur.r0.x + t * cur.r1.x, cur.r0.y + t * cur.r1.y, cur.r0.z + t * cur.r1.z);
      mlp_input(sc, p, xyz(ng), x);
    }
    const float4 ngn = normal(nxt);
    const InferRec nn = fetch(tile + 2 * stride);
    yp = mlp_infer_tile(wf, bl, x);
    tp = tile;
    cur = nxt;
    ng = ngn;
    nxt = nn;
  }
  if (tp != kNoTile) store(tp, yp);
}
void k_mlp_infer_queue(const SceneDev& sc, const QueuesDev& q, const MlpDev& m, const Counters* cnt,
                       int d, int grid, hipStream_t s) {
  // grid = 32 per CU.  At up to 128 VGPRs, four waves per SIMD: two
  // eight-wave workgroups per CU, all resident at once
  mlp_infer_queue_kernel<<<std::max(1, grid / 16), 64 * kInferWaves, 0, s>>>(sc, q, m, cnt, d);
}

// inference at the light vertices of bounce i (bidirectional learned-cache
// iterations), on the light queue (level 0) between its traversal and the
// light shading: a hit of the light ray of root r is light vertex i of r's
// subpath, and its outputs go to lt.y[4 (r * lmax + i - 1)] (each root has
// one light ray per bounce).  The MIS weights evaluate the network's counts
// there as if the vertex were on the camera side.
__global__ __launch_bounds__(64 * kInferWaves) void mlp_infer_light_kernel(SceneDev sc, QueuesDev q,
                                                                           MlpDev m, LightDev lt,
                                                                           const Counters* cnt,
                                                                           int i) {
  __shared__ uint4 wf[kFragBlocks * 64];
  __shared__ float4 bl[52];
  const uint32_t n = min(cnt->n_ray[0], (uint32_t)q.cap);
  if ((size_t)blockIdx.x * kInferWaves * 16 >= n) return;
  stage_fragments<64 * kInferWaves>(m.wq, wf);
  stage_biases(m.master, bl);
  __syncthreads();
  const int lane = threadIdx.x & 63, lr = lane & 15, w = threadIdx.x >> 6;
  const uint32_t stride = gridDim.x * kInferWaves;
  const float4 zero4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  // the light ray and hit of this lane's sample (lr) of a tile; the same
  // pipeline as the queue kernel's
  auto fetch = [&](uint32_t tile) {
    InferRec r{make_uint2(0u, kMiss), zero4, zero4};
    const uint32_t s = tile * 16 + lr;
    if (tile < kNoTile / 16 && s < n) {
      r.r0 = q.R0[s];
      r.h = q.H[s];
      r.r1 = q.R1[s];
    }
    return r;
  };
  auto is_hit = [](const InferRec& r) { return r.r0.w != 0.0f && r.h.y != kMiss; };
  auto normal = [&](const InferRec& r) { return is_hit(r) ? sc.tri_ng[r.h.y] : zero4; };
  uint32_t tile = blockIdx.x * kInferWaves + w;
  InferRec cur = fetch(tile);
  float4 ng = normal(cur);
  InferRec nxt = fetch(tile + stride);
  v4f yp = v4f{0.0f, 0.0f, 0.0f, 0.0f};
  uint32_t rootp = 0u;    // the root of this lane's sample of tile tp
  uint32_t tp = kNoTile;  // the tile yp belongs to
  // outputs 0..3 of the sample (the fourth is padding) from the lanes < 16
  auto store = [&]() {
    const uint32_t s = tp * 16 + lr;
    if (lane < 16 && s < n)
      reinterpret_cast<float4*>(lt.y)[(size_t)rootp * lt.lmax + (i - 1)] =
          make_float4(yp[0], yp[1], yp[2], yp[3]);
  };
  for (; tile * 16 < n; tile += stride) {
    wait_vector_memory();
    if (tp != kNoTile) store();
    tp = kNoTile;
    const bool hit = is_hit(cur);
    float x[6] = {0, 0, 0, 0, 0, 0};
    if (hit) {
      const float t = __uint_as_float(cur.h.x);
      const f3 p = mk3(cur.r0.x + t * cur.r1.x, cur.r0.y + t * cur.r1.y, cur.r0.z + t * cur.r1.z);
      mlp_input(sc, p, xyz(ng), x);
    }
    const float4 ngn = normal(nxt);
    const InferRec nn = fetch(tile + 2 * stride);
    if (__any(hit)) {  // else no light vertex in the tile (wave-uniform)
      yp = mlp_infer_tile(wf, bl, x);
      rootp = __float_as_uint(cur.r1.w);
      tp = tile;
    }
    cur = nxt;
    ng = ngn;
    nxt = nn;
  }
  if (tp != kNoTile) store();
}
void k_mlp_infer_light(const SceneDev& sc, const QueuesDev& q, const MlpDev& m, const LightDev& lt,
                       const Counters* cnt, int i, int grid, hipStream_t s) {
  mlp_infer_light_kernel<<<std::max(1, grid / 16), 64 * kInferWaves, 0, s>>>(sc, q, m, lt, cnt, i);
}

// ---------------------------------------------------------------------------
// training: loss L = (1/N) sum_i sum_t w_it (y_it - y*_it)^2 over a batch of
// N samples taken cyclically from the training set starting at `offset`.
// One wave per workgroup walks a contiguous chunk of tiles and accumulates
// the gradient in LDS (binary32, fixed order); each workgroup writes its
// partial gradient; the Adam kernel sums the partials in workgroup order.
// ---------------------------------------------------------------------------
struct TrainLds {
  uint16_t xs[16][80];
  uint16_t hs[3][16][64];
  uint16_t dz[16][64];
  float g[kMlpParams];
  float loss;
};

__device__ __forceinline__ void dense_backward(const uint16_t* __restrict__ wq, int qoff, int nout,
                                               int nin, const uint16_t* hprev, int hstride,
                                               float* gW, float* gb, v4f* dz_in,
                                               uint16_t (*dzs)[64], v4f* dprev, bool want_prev) {
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const int nto = nout / 16, nti = nin / 16;
  // dZ to LDS (bfloat16) and the bias gradient
  for (int nt = 0; nt < nto; ++nt) {
    float sacc = 0.0f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      dzs[4 * lg + r][16 * nt + lr] = to_bf16(dz_in[nt][r]);
      sacc += dz_in[nt][r];
    }
    sacc += __shfl_xor(sacc, 16, 64);
    sacc += __shfl_xor(sacc, 32, 64);
    if (lg == 0) gb[16 * nt + lr] += sacc;
  }
  __syncthreads();
  // weight gradient: dW[o][i] += sum_samples dZ[s][o] Hprev[s][i]
  for (int mt = 0; mt < nto; ++mt)
    for (int nt = 0; nt < nti; ++nt) {
      v4s a, b;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        a[r] = (short)dzs[4 * lg + r][16 * mt + lr];
        b[r] = (short)hprev[(4 * lg + r) * hstride + 16 * nt + lr];
      }
      const v4f d = mma(a, b, v4f{0.0f, 0.0f, 0.0f, 0.0f});
#pragma unroll
      for (int r = 0; r < 4; ++r) gW[(16 * mt + 4 * lg + r) * nin + 16 * nt + lr] += d[r];
    }
  if (!want_prev) return;
  // dHprev[s][i] = sum_o dZ[s][o] W[o][i], then the ReLU mask of Hprev
  for (int nt = 0; nt < nti; ++nt) {
    v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int ks = 0; ks < nto; ++ks) {
      v4s a, b;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        a[r] = (short)dzs[lr][16 * ks + 4 * lg + r];
        b[r] = (short)wq[qoff + (16 * ks + 4 * lg + r) * nin + 16 * nt + lr];
      }
      acc = mma(a, b, acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float hp = from_bf16(hprev[(4 * lg + r) * hstride + 16 * nt + lr]);
      acc[r] = hp > 0.0f ? acc[r] : 0.0f;
    }
    dprev[nt] = acc;
  }
  __syncthreads();
}

__global__ __launch_bounds__(64) void mlp_train_kernel(MlpDev m, const float* x6, const float* tgt,
                                                       const float* wt, int n_set, int offset,
                                                       int batch, int tiles_per_block) {
  __shared__ TrainLds S;
  // the bfloat16 weights, read by every product of the forward and backward
  // passes, copied once into LDS
  __shared__ uint4 wl4[kQW / 8];
  const int lane = threadIdx.x, lr = lane & 15, lg = lane >> 4;
  for (int p = lane; p < kMlpParams; p += 64) S.g[p] = 0.0f;
  for (int k = lane; k < kQW / 8; k += 64) wl4[k] = reinterpret_cast<const uint4*>(m.wq)[k];
  if (lane == 0) S.loss = 0.0f;
  __syncthreads();
  const uint16_t* wl = reinterpret_cast<const uint16_t*>(wl4);
  const int ntiles = (batch + 15) / 16;
  const int t0 = blockIdx.x * tiles_per_block, t1 = min(ntiles, t0 + tiles_per_block);
  const float inv_n = 1.0f / (float)batch;
  float lsum = 0.0f;
  for (int tile = t0; tile < t1; ++tile) {
    const int bi = tile * 16 + lr;
    float x[6] = {0, 0, 0, 0, 0, 0};
    if (bi < batch) {
      const size_t s = (size_t)((offset + bi) % n_set);
      for (int k = 0; k < 6; ++k) x[k] = x6[6 * s + k];
    }
    const v4f y = mlp_forward_tile(m.master, wl, x, S.hs, S.xs);
    v4f dz[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int bs = tile * 16 + 4 * lg + r;
      float g = 0.0f;
      if (bs < batch && lr < 3) {
        const size_t s = (size_t)((offset + bs) % n_set);
        const float w = wt[3 * s + lr];
        const float df = y[r] - tgt[3 * s + lr];
        g = (2.0f * w * df) * inv_n;
        lsum += (w * df * df) * inv_n;
      }
      dz[0][r] = g;
    }
    v4f dp[5];
    dense_backward(wl, qW4, 16, 64, &S.hs[2][0][0], 64, S.g + kMlpW4, S.g + kMlpB4, dz, S.dz, dp,
                   true);
    dense_backward(wl, qW3, 64, 64, &S.hs[1][0][0], 64, S.g + kMlpW3, S.g + kMlpB3, dp, S.dz, dz,
                   true);
    dense_backward(wl, qW2, 64, 64, &S.hs[0][0][0], 64, S.g + kMlpW2, S.g + kMlpB2, dz, S.dz, dp,
                   true);
    dense_backward(wl, qW1, 64, 80, &S.xs[0][0], 80, S.g + kMlpW1, S.g + kMlpB1, dp, S.dz, dz,
                   false);
    __syncthreads();
  }
  lsum += __shfl_xor(lsum, 1, 64);
  lsum += __shfl_xor(lsum, 2, 64);
  lsum += __shfl_xor(lsum, 4, 64);
  lsum += __shfl_xor(lsum, 8, 64);
  lsum += __shfl_xor(lsum, 16, 64);
  lsum += __shfl_xor(lsum, 32, 64);
  float* out = m.partial + (size_t)blockIdx.x * (kMlpParams + 1);
  for (int p = lane; p < kMlpParams; p += 64) out[p] = S.g[p];
  if (lane == 0) out[kMlpParams] = lsum;
}

// sum over the workgroup partials of parameter p, in workgroup order; the
// loads of eight partials are issued before their additions
__device__ __forceinline__ float sum_partials(const float* __restrict__ partial, int nblocks,
                                              int p) {
  float g = 0.0f;
  int b = 0;
  for (; b + 8 <= nblocks; b += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = partial[(size_t)(b + u) * (kMlpParams + 1) + p];
#pragma unroll
    for (int u = 0; u < 8; ++u) g += v[u];
  }
  for (; b < nblocks; ++b) g += partial[(size_t)b * (kMlpParams + 1) + p];
  return g;
}

// Adam (binary32): the gradient is the sum of the workgroup partials in
// workgroup order
// Adam over the summed workgroup partials: a workgroup of kAdamWaves waves
// takes 64 parameters (index kMlpParams: the loss), wave w summing the
// partials of workgroups w, w + kAdamWaves, ... and the waves' sums then
// added in wave order, so that the gradient does not depend on scheduling
constexpr int kAdamWaves = 8;
__global__ __launch_bounds__(64 * kAdamWaves) void mlp_adam_kernel(MlpDev m, int nblocks,
                                                                  const float* ext_grad, float lr,
                                                                  float bc1, float bc2,
                                                                  float* loss_out) {
  __shared__ float part[kAdamWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int p = blockIdx.x * 64 + lane;
  float g = 0.0f;
  if (p <= kMlpParams && (!ext_grad || p == kMlpParams)) {
    const float* __restrict__ src = m.partial + p;
    constexpr size_t kRow = (size_t)kMlpParams + 1;
    int b = w;
    for (; b + 7 * kAdamWaves < nblocks; b += 8 * kAdamWaves) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = src[(size_t)(b + u * kAdamWaves) * kRow];
#pragma unroll
      for (int u = 0; u < 8; ++u) g += v[u];
    }
    for (; b < nblocks; b += kAdamWaves) g += src[(size_t)b * kRow];
  }
  part[w][lane] = g;
  __syncthreads();
  if (w != 0 || p > kMlpParams) return;
  float gs = part[0][lane];
#pragma unroll
  for (int k = 1; k < kAdamWaves; ++k) gs += part[k][lane];
  if (p == kMlpParams) {
    if (loss_out) *loss_out = gs;
    return;
  }
  if (ext_grad) gs = ext_grad[p];
  const float b1 = 0.9f, b2 = 0.99f, c1 = (float)(1.0 - 0.9), c2 = (float)(1.0 - 0.99);
  const float mm = b1 * m.m[p] + c1 * gs;
  const float vv = b2 * m.v[p] + c2 * gs * gs;
  m.m[p] = mm;
  m.v[p] = vv;
  const float mh = mm / bc1, vh = vv / bc2;
  const float wn = m.master[p] - (lr * mh) / (sqrtf(vh) + 1e-8f);
  m.master[p] = wn;
  const int qi = qindex(p);
  if (qi >= 0) m.wq[qi] = to_bf16(wn);
}

// gradient only (tests): the partials summed in workgroup order
__global__ void mlp_sum_partials_kernel(MlpDev m, int nblocks, float* grad, float* loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kMlpParams) return;
  const float g = sum_partials(m.partial, nblocks, p);
  if (p < kMlpParams) grad[p] = g;
  else *loss = g;
}

void k_mlp_train_pass(const MlpDev& m, const float* x6, const float* tgt, const float* wt, int n_set,
                      int offset, int batch, int* nblocks_out, hipStream_t s) {
  const int ntiles = (batch + 15) / 16;
  const int tpb = std::max(1, (ntiles + kMlpMaxBlocks - 1) / kMlpMaxBlocks);
  const int nb = (ntiles + tpb - 1) / tpb;
  mlp_train_kernel<<<nb, 64, 0, s>>>(m, x6, tgt, wt, n_set, offset, batch, tpb);
  *nblocks_out = nb;
}
void k_mlp_adam(const MlpDev& m, int nblocks, const float* ext_grad, float lr, float bc1, float bc2,
                float* loss_out, hipStream_t s) {
  // 64 parameters (and the loss) per workgroup: 228 of them
  mlp_adam_kernel<<<(kMlpParams + 1 + 63) / 64, 64 * kAdamWaves, 0, s>>>(m, nblocks, ext_grad, lr,
                                                                         bc1, bc2, loss_out);
}
void k_mlp_sum_partials(const MlpDev& m, int nblocks, float* grad, float* loss, hipStream_t s) {
  mlp_sum_partials_kernel<<<(kMlpParams + 64) / 64, 64, 0, s>>>(m, nblocks, grad, loss);
}

// ---------------------------------------------------------------------------
// Allocation-free gradient pass: the per-workgroup partial gradients of
// mars_mlp_grad_noalloc live in this fixed array (one per device, kept until
// the process ends) instead of scene memory.  Host code never passes the
// array's name to a kernel: it is a host-side stand-in; the device address
// comes from hipGetSymbolAddress, taken once per device with that device
// current.
// ---------------------------------------------------------------------------
static __device__ __align__(256) float scratch[kNoAllocScratchFloats];

namespace {
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_address(int device, float** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = (float*)p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

// bfloat16 copy of freshly written master weights
__global__ void mlp_quantize_kernel(MlpDev m) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpParams) return;
  const int qi = qindex(p);
  if (qi >= 0) m.wq[qi] = to_bf16(m.master[p]);
}
void k_mlp_quantize(const MlpDev& m, hipStream_t s) {
  mlp_quantize_kernel<<<(kMlpParams + 255) / 256, 256, 0, s>>>(m);
}

// probe of the matrix-core lane layout: D = A B for one 16 x 16 x 16 tile
// (A, B given as bfloat16 bit patterns, row-major)
__global__ void mfma_probe_kernel(const uint16_t* A, const uint16_t* B, float* D) {
  const int lane = threadIdx.x, lr = lane & 15, lg = lane >> 4;
  v4s a, b;
  for (int r = 0; r < 4; ++r) {
    a[r] = (short)A[lr * 16 + 4 * lg + r];
    b[r] = (short)B[(4 * lg + r) * 16 + lr];
  }
  const v4f d = mma(a, b, v4f{0.0f, 0.0f, 0.0f, 0.0f});
  for (int r = 0; r < 4; ++r) D[(4 * lg + r) * 16 + lr] = d[r];
}
void k_mfma_probe(const uint16_t* A, const uint16_t* B, float* D, hipStream_t s) {
  mfma_probe_kernel<<<1, 64, 0, s>>>(A, B, D);
}

}  // namespace mars
