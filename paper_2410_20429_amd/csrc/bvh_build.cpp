// Host BVH builder: binned SAH (16 bins per axis), at most 4 triangles per
// leaf unless a split cannot separate them (then up to 15), depth bounded so
// that the traversal's 32-entry stack always suffices (median splits take
// over when the remaining triangles could otherwise exceed the bound).
// Output layout (64 B per inner node, depth-first order):
//   float4 (c0.lo.xyz, c0.hi.x), (c0.hi.yz, c1.lo.xy), (c1.lo.z, c1.hi.xyz),
//   (child0, child1, 0, 0) as int bits; child >= 0: inner node index,
//   child < 0: leaf = -1 - (first << 4 | count).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "bvh_build.h"

namespace mars {
namespace {

struct Box {
  float lo[3], hi[3];
  void reset() {
    for (int a = 0; a < 3; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
  }
  void grow(const float* p) {
    for (int a = 0; a < 3; ++a) { lo[a] = std::min(lo[a], p[a]); hi[a] = std::max(hi[a], p[a]); }
  }
  void grow(const Box& b) {
    for (int a = 0; a < 3; ++a) { lo[a] = std::min(lo[a], b.lo[a]); hi[a] = std::max(hi[a], b.hi[a]); }
  }
  float area() const {
    const float dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
    if (!(dx >= 0.0f)) return 0.0f;
    return 2.0f * (dx * dy + dy * dz + dz * dx);
  }
};

struct Node {
  Box box;
  int left = -1, right = -1;
  int first = 0, count = 0;
};

struct Builder {
  const float* V;
  std::vector<Box> tb;
  std::vector<float> cent;
  std::vector<int32_t> idx;
  std::vector<Node> nodes;
  int max_depth_seen = 0;

  static int ceil_log2(int n) {
    int k = 0;
    while ((1 << k) < n) ++k;
    return k;
  }

  int build(int first, int count, int depth) {
    const int id = (int)nodes.size();
    nodes.emplace_back();
    Box b, cb;
    b.reset();
    cb.reset();
    for (int k = first; k < first + count; ++k) {
      b.grow(tb[idx[k]]);
      cb.grow(&cent[3 * (size_t)idx[k]]);
    }
    nodes[id].box = b;
    max_depth_seen = std::max(max_depth_seen, depth);
    if (count <= 4) {
      nodes[id].first = first;
      nodes[id].count = count;
      return id;
    }
    int axis = 0;
    float ext[3];
    for (int a = 0; a < 3; ++a) ext[a] = cb.hi[a] - cb.lo[a];
    if (ext[1] > ext[axis]) axis = 1;
    if (ext[2] > ext[axis]) axis = 2;
    int mid = -1;
    const bool force_median = depth + ceil_log2((count + 3) / 4) >= 30;
    if (!force_median && ext[axis] > 0.0f) {
      constexpr int NB = 16;
      float best_cost = INFINITY;
      int best_axis = -1, best_split = -1;
      for (int a = 0; a < 3; ++a) {
        if (!(ext[a] > 0.0f)) continue;
        Box bins[NB];
        int cnt[NB] = {0};
        for (int k = 0; k < NB; ++k) bins[k].reset();
        const float scale = NB / ext[a];
        for (int k = first; k < first + count; ++k) {
          const int t = idx[k];
          int bi = (int)((cent[3 * (size_t)t + a] - cb.lo[a]) * scale);
          bi = std::min(NB - 1, std::max(0, bi));
          bins[bi].grow(tb[t]);
          ++cnt[bi];
        }
        float ra[NB];
        int rc[NB];
        Box acc;
        acc.reset();
        int c = 0;
        for (int k = NB - 1; k > 0; --k) {
          acc.grow(bins[k]);
          c += cnt[k];
          ra[k] = acc.area();
          rc[k] = c;
        }
        acc.reset();
        c = 0;
        for (int k = 0; k < NB - 1; ++k) {
          acc.grow(bins[k]);
          c += cnt[k];
          if (c == 0 || rc[k + 1] == 0) continue;
          const float cost = acc.area() * c + ra[k + 1] * rc[k + 1];
          if (cost < best_cost) {
            best_cost = cost;
            best_axis = a;
            best_split = k;
          }
        }
      }
      if (best_axis >= 0) {
        const float scale = NB / ext[best_axis];
        auto it = std::partition(idx.begin() + first, idx.begin() + first + count, [&](int32_t t) {
          int bi = (int)((cent[3 * (size_t)t + best_axis] - cb.lo[best_axis]) * scale);
          bi = std::min(NB - 1, std::max(0, bi));
          return bi <= best_split;
        });
        mid = (int)(it - idx.begin());
        if (mid == first || mid == first + count) mid = -1;
      }
    }
    if (mid < 0) {
      // median split along the longest centroid axis (ties by index)
      mid = first + count / 2;
      std::nth_element(idx.begin() + first, idx.begin() + mid, idx.begin() + first + count,
                       [&](int32_t x, int32_t y) {
                         const float cx = cent[3 * (size_t)x + axis], cy = cent[3 * (size_t)y + axis];
                         return cx < cy || (cx == cy && x < y);
                       });
    }
    const int l = build(first, mid - first, depth + 1);
    const int r = build(mid, first + count - mid, depth + 1);
    nodes[id].left = l;
    nodes[id].right = r;
    return id;
  }
};

}  // namespace

BvhResult build_bvh(const float* V, int n_tris, float pad) {
  Builder B;
  B.V = V;
  B.tb.resize(n_tris);
  B.cent.resize(3 * (size_t)n_tris);
  B.idx.resize(n_tris);
  for (int i = 0; i < n_tris; ++i) {
    const float* p = V + 9 * (size_t)i;
    B.tb[i].reset();
    for (int v = 0; v < 3; ++v) B.tb[i].grow(p + 3 * v);
    for (int a = 0; a < 3; ++a) B.cent[3 * (size_t)i + a] = (p[a] + p[3 + a] + p[6 + a]) / 3.0f;
    B.idx[i] = i;
  }
  B.nodes.reserve(2 * (size_t)n_tris);
  B.build(0, n_tris, 0);

  BvhResult out;
  out.max_depth = B.max_depth_seen;
  out.prim_order = B.idx;
  // depth-first numbering of inner nodes
  std::vector<int> gpu_id(B.nodes.size(), -1);
  std::vector<int> order;
  std::vector<int> st{0};
  const bool root_leaf = B.nodes[0].left < 0;
  if (!root_leaf) {
    while (!st.empty()) {
      const int n = st.back();
      st.pop_back();
      gpu_id[n] = (int)order.size();
      order.push_back(n);
      const Node& nd = B.nodes[n];
      if (B.nodes[nd.right].left >= 0) st.push_back(nd.right);
      if (B.nodes[nd.left].left >= 0) st.push_back(nd.left);
    }
  }
  auto child_ref = [&](int n) -> int32_t {
    const Node& c = B.nodes[n];
    if (c.left >= 0) return gpu_id[n];
    return -1 - (int32_t)(((uint32_t)c.first << 4) | (uint32_t)c.count);
  };
  auto put_box = [&](const Box& b, float* lo, float* hi) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = b.lo[a] - pad;
      hi[a] = b.hi[a] + pad;
    }
  };
  const size_t nn = root_leaf ? 1 : order.size();
  out.nodes.assign(nn * 16, 0.0f);
  for (size_t g = 0; g < nn; ++g) {
    float lo0[3], hi0[3], lo1[3], hi1[3];
    int32_t r0, r1;
    if (root_leaf) {
      put_box(B.nodes[0].box, lo0, hi0);
      r0 = -1 - (int32_t)(((uint32_t)0 << 4) | (uint32_t)B.nodes[0].count);
      for (int a = 0; a < 3; ++a) { lo1[a] = INFINITY; hi1[a] = -INFINITY; }
      r1 = -1;  // empty leaf
    } else {
      const Node& nd = B.nodes[order[g]];
      put_box(B.nodes[nd.left].box, lo0, hi0);
      put_box(B.nodes[nd.right].box, lo1, hi1);
      r0 = child_ref(nd.left);
      r1 = child_ref(nd.right);
    }
    float* f = &out.nodes[g * 16];
    f[0] = lo0[0]; f[1] = lo0[1]; f[2] = lo0[2]; f[3] = hi0[0];
    f[4] = hi0[1]; f[5] = hi0[2]; f[6] = lo1[0]; f[7] = lo1[1];
    f[8] = lo1[2]; f[9] = hi1[0]; f[10] = hi1[1]; f[11] = hi1[2];
    uint32_t u0 = (uint32_t)r0, u1 = (uint32_t)r1;
    std::memcpy(&f[12], &u0, 4);
    std::memcpy(&f[13], &u1, 4);
  }
  // triangles in leaf order: (v0, prim), (e1, 0), (e2, 0)
  out.tris.assign((size_t)n_tris * 12, 0.0f);
  for (int k = 0; k < n_tris; ++k) {
    const int t = B.idx[k];
    const float* p = V + 9 * (size_t)t;
    float* d = &out.tris[(size_t)k * 12];
    d[0] = p[0]; d[1] = p[1]; d[2] = p[2];
    const uint32_t pb = (uint32_t)t;
    std::memcpy(&d[3], &pb, 4);
    d[4] = p[3] - p[0]; d[5] = p[4] - p[1]; d[6] = p[5] - p[2]; d[7] = 0.0f;
    d[8] = p[6] - p[0]; d[9] = p[7] - p[1]; d[10] = p[8] - p[2]; d[11] = 0.0f;
  }
  return out;
}

}  // namespace mars
