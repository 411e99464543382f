// Learned cache: a small MLP that predicts the log sample count of every
// technique, relative to |T / I~|, from a vertex's position normalised to the
// octree's cube and its geometric normal as stored (sin/cos encoding with 6
// frequencies -> 72 features, padded to 80; three hidden layers of 64 ReLU
// units; 3 linear outputs).  Forward and backward
// run as bfloat16 matrix-core products with binary32 accumulation
// (v_mfma_f32_16x16x16_bf16), one 16-sample tile per wave.  Master weights,
// biases and Adam moments are binary32.
//
// MFMA 16x16x16 operand layout (lane l = 0..63, element r = 0..3):
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
// Features k (even) and k + 1 are the sine and cosine of one angle.
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

// LDS written by some lanes of a wave and read by others of the same wave
// (the workgroups using it hold several waves that do not meet): the wave's
// own writes completed (workgroup-scope release), no code motion across it
// (wave barrier), then the reads (acquire)
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Forward pass of one 16-sample tile by one wave.  x: this lane's sample
// inputs (sample = lane % 16).  wq: the bfloat16 weights (global memory or a
// copy in LDS).  Hidden activations go to hs[l][16][64] (bfloat16), features
// to xs[16][80] when xs != nullptr.  Returns the output tile in D layout (rows
// = samples, columns = outputs).  kGroupSync: one-wave workgroups meet at
// workgroup barriers; otherwise only the wave's own order is kept.
template <bool kGroupSync>
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
#pragma unroll
    for (int r = 0; r < 4; r += 2) {
      const int k = 16 * ks + 4 * lg + r;
      float fs, fc;
      feature_pair(x, k, &fs, &fc);
      uint16_t hs0, hc0;
      to_bf16x2(fs, fc, &hs0, &hc0);
      a[r] = (short)hs0;
      a[r + 1] = (short)hc0;
      if (xs) {
        xs[lr][k] = hs0;
        xs[lr][k + 1] = hc0;
      }
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
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int j = 16 * nt + lr;
      const float bj = master[boff[l] + j];
#pragma unroll
      for (int r = 0; r < 4; r += 2) {
        uint16_t h0, h1;
        to_bf16x2(fmaxf(acc[nt][r] + bj, 0.0f), fmaxf(acc[nt][r + 1] + bj, 0.0f), &h0, &h1);
        hs[l][4 * lg + r][j] = h0;
        hs[l][4 * lg + r + 1][j] = h1;
      }
    }
    if (kGroupSync) __syncthreads();
    else wave_lds_sync();
    const int ntn = l < 2 ? 4 : 1;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const uint16_t* hr = &hs[l][lr][16 * ks + 4 * lg];
      const v4s a = {(short)hr[0], (short)hr[1], (short)hr[2], (short)hr[3]};
      for (int nt = 0; nt < ntn; ++nt) {
        const uint16_t* w = wq + woff[l] + (16 * nt + lr) * 64 + 16 * ks + 4 * lg;
        const v4s b = {(short)w[0], (short)w[1], (short)w[2], (short)w[3]};
        acc[nt] = mma(a, b, acc[nt]);
      }
    }
  }
  v4f y = acc[0];
#pragma unroll
  for (int r = 0; r < 4; ++r) y[r] += master[kMlpB4 + lr];
  return y;
}

// inference over a list of vertices given as (q, n); 64-thread workgroups
__global__ __launch_bounds__(64) void mlp_infer_inputs_kernel(MlpDev m, const float* x6, int n,
                                                              float* y3) {
  __shared__ uint16_t hs[3][16][64];
  const int lane = threadIdx.x, lr = lane & 15, lg = lane >> 4;
  for (int tile = blockIdx.x; tile * 16 < n; tile += gridDim.x) {
    const int s = tile * 16 + lr;
    float x[6] = {0, 0, 0, 0, 0, 0};
    if (s < n)
      for (int k = 0; k < 6; ++k) x[k] = x6[6 * (size_t)s + k];
    const v4f y = mlp_forward_tile<true>(m.master, m.wq, x, hs, nullptr);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int si = tile * 16 + 4 * lg + r;
      if (si < n && lr < 3) y3[3 * (size_t)si + lr] = y[r];
    }
    __syncthreads();
  }
}
void k_mlp_forward(const MlpDev& m, const float* x6, int n, float* y3, hipStream_t s) {
  const int tiles = (n + 15) / 16;
  mlp_infer_inputs_kernel<<<std::min(tiles, 8192), 64, 0, s>>>(m, x6, n, y3);
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
// The bfloat16 weights are copied once per workgroup into LDS; each of its
// four waves then runs 16-sample tiles of the queue.
constexpr int kInferWaves = 4;
__global__ __launch_bounds__(64 * kInferWaves) void mlp_infer_queue_kernel(SceneDev sc,
                                                                           QueuesDev q, MlpDev m,
                                                                           const Counters* cnt,
                                                                           int d) {
  __shared__ uint4 wl4[kQW / 8];
  __shared__ uint16_t hs[kInferWaves][3][16][64];
  if (cnt->overflow) return;
  const uint32_t n = min(cnt->n_ray[d], (uint32_t)q.cap);
  if ((size_t)blockIdx.x * kInferWaves * 16 >= n) return;  // no tile for this workgroup
  for (int k = threadIdx.x; k < kQW / 8; k += blockDim.x)
    wl4[k] = reinterpret_cast<const uint4*>(m.wq)[k];
  __syncthreads();
  const uint16_t* wl = reinterpret_cast<const uint16_t*>(wl4);
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4, w = threadIdx.x >> 6;
  const size_t L = (size_t)d * q.cap;
  for (uint32_t tile = blockIdx.x * kInferWaves + w; tile * 16 < n;
       tile += gridDim.x * kInferWaves) {
    const uint32_t s = tile * 16 + lr;
    float x[6] = {0, 0, 0, 0, 0, 0};
    if (s < n) {
      const uint2 h = q.H[L + s];
      if (h.y != kMiss) {
        const float4 r0 = q.R0[L + s], r1 = q.R1[L + s];
        const float t = __uint_as_float(h.x);
        const f3 ng = xyz(sc.tri_ng[h.y]);
        const f3 p = mk3(r0.x + t * r1.x, r0.y + t * r1.y, r0.z + t * r1.z);
        mlp_input(sc, p, ng, x);
      }
    }
    const v4f y = mlp_forward_tile<false>(m.master, wl, x, hs[w], nullptr);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t si = tile * 16 + 4 * lg + r;
      if (si < n && lr < 3) m.y[(L + si) * 4 + lr] = y[r];
    }
    // the next tile rewrites hs[w] only after every lane has read it
    wave_lds_sync();
  }
}
void k_mlp_infer_queue(const SceneDev& sc, const QueuesDev& q, const MlpDev& m, const Counters* cnt,
                       int d, int grid, hipStream_t s) {
  // three workgroups (53 KB of LDS each) per CU; grid = 32 per CU
  mlp_infer_queue_kernel<<<std::max(1, grid * 3 / 32), 64 * kInferWaves, 0, s>>>(sc, q, m, cnt, d);
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
  __shared__ uint4 wl4[kQW / 8];
  __shared__ uint16_t hs[kInferWaves][3][16][64];
  const uint32_t n = min(cnt->n_ray[0], (uint32_t)q.cap);
  if ((size_t)blockIdx.x * kInferWaves * 16 >= n) return;
  for (int k = threadIdx.x; k < kQW / 8; k += blockDim.x)
    wl4[k] = reinterpret_cast<const uint4*>(m.wq)[k];
  __syncthreads();
  const uint16_t* wl = reinterpret_cast<const uint16_t*>(wl4);
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4, w = threadIdx.x >> 6;
  for (uint32_t tile = blockIdx.x * kInferWaves + w; tile * 16 < n;
       tile += gridDim.x * kInferWaves) {
    const uint32_t s = tile * 16 + lr;
    float x[6] = {0, 0, 0, 0, 0, 0};
    float4 r0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    uint2 h = make_uint2(0u, kMiss);
    if (s < n) {
      r0 = q.R0[s];
      h = q.H[s];
    }
    const bool hit = r0.w != 0.0f && h.y != kMiss;
    if (!__any(hit)) continue;  // no light vertex in the tile (wave-uniform)
    if (hit) {
      const float4 r1 = q.R1[s];
      const float t = __uint_as_float(h.x);
      const f3 p = mk3(r0.x + t * r1.x, r0.y + t * r1.y, r0.z + t * r1.z);
      mlp_input(sc, p, xyz(sc.tri_ng[h.y]), x);
    }
    const v4f y = mlp_forward_tile<false>(m.master, wl, x, hs[w], nullptr);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t si = tile * 16 + 4 * lg + r;
      if (si < n && lr < 3) {
        const uint32_t root = __float_as_uint(q.R1[si].w);
        lt.y[((size_t)root * lt.lmax + (i - 1)) * 4 + lr] = y[r];
      }
    }
    wave_lds_sync();
  }
}
void k_mlp_infer_light(const SceneDev& sc, const QueuesDev& q, const MlpDev& m, const LightDev& lt,
                       const Counters* cnt, int i, int grid, hipStream_t s) {
  mlp_infer_light_kernel<<<std::max(1, grid * 3 / 32), 64 * kInferWaves, 0, s>>>(sc, q, m, lt, cnt, i);
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
    const v4f y = mlp_forward_tile<true>(m.master, wl, x, S.hs, S.xs);
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

// Adam (binary32): the gradient is the sum of the workgroup partials in
// workgroup order
__global__ void mlp_adam_kernel(MlpDev m, int nblocks, const float* ext_grad, float lr, float bc1,
                                float bc2, float* loss_out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0 && loss_out) {
    float l = 0.0f;
    for (int b = 0; b < nblocks; ++b) l += m.partial[(size_t)b * (kMlpParams + 1) + kMlpParams];
    *loss_out = l;
  }
  if (p >= kMlpParams) return;
  float g = 0.0f;
  if (ext_grad) {
    g = ext_grad[p];
  } else {
    for (int b = 0; b < nblocks; ++b) g += m.partial[(size_t)b * (kMlpParams + 1) + p];
  }
  const float b1 = 0.9f, b2 = 0.99f, c1 = (float)(1.0 - 0.9), c2 = (float)(1.0 - 0.99);
  const float mm = b1 * m.m[p] + c1 * g;
  const float vv = b2 * m.v[p] + c2 * g * g;
  m.m[p] = mm;
  m.v[p] = vv;
  const float mh = mm / bc1, vh = vv / bc2;
  const float w = m.master[p] - (lr * mh) / (sqrtf(vh) + 1e-8f);
  m.master[p] = w;
  const int qi = qindex(p);
  if (qi >= 0) m.wq[qi] = to_bf16(w);
}

// gradient only (tests): the partials summed in workgroup order
__global__ void mlp_sum_partials_kernel(MlpDev m, int nblocks, float* grad, float* loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kMlpParams) return;
  float g = 0.0f;
  for (int b = 0; b < nblocks; ++b) g += m.partial[(size_t)b * (kMlpParams + 1) + p];
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
  mlp_adam_kernel<<<(kMlpParams + 255) / 256, 256, 0, s>>>(m, nblocks, ext_grad, lr, bc1, bc2,
                                                           loss_out);
}
void k_mlp_sum_partials(const MlpDev& m, int nblocks, float* grad, float* loss, hipStream_t s) {
  mlp_sum_partials_kernel<<<(kMlpParams + 256) / 256, 256, 0, s>>>(m, nblocks, grad, loss);
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
