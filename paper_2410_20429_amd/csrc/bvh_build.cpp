// Host BVH builder: binned SAH (16 bins per axis) binary tree, at most 4
// triangles per leaf (a median split separates any larger set), depth
// bounded by 30 (median splits take over when the remaining triangles
// could otherwise exceed the bound), then collapsed to a 4-wide tree: each
// node takes up to four descendants, expanding the inner child of largest
// surface area first.
// Output layout (128 B = one cache line per node, depth-first order): four
// 32-byte child records, child k at bytes [32k, 32k + 32):
//   float lo.x, lo.y, lo.z, int32 reference, float hi.x, hi.y, hi.z, unused;
//   reference >= 0: node index; < 0: leaf = -1 - (first << 4 | count);
//   kBvhEmpty: no child (its box is empty: lo = +inf, hi = -inf).
// A child's record is two aligned 16-byte words, so the lane that tests it
// fetches it with two vector loads.
// Traversal pushes at most 3 children per visited node and the 4-wide depth
// is at most the binary depth, so the stack never exceeds 3 x 30 entries;
// max_stack reports the exact bound of the built tree.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <functional>
#include <utility>
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
  auto area = [&](int n) { return B.nodes[n].box.area(); };
  auto is_leaf = [&](int n) { return B.nodes[n].left < 0; };
  auto leaf_ref = [&](int n) -> int32_t {
    const Node& c = B.nodes[n];
    return -1 - (int32_t)(((uint32_t)c.first << 4) | (uint32_t)c.count);
  };
  // returns (node index, stack bound of its subtree)
  std::function<std::pair<int, int>(int)> emit = [&](int n) -> std::pair<int, int> {
    const int id = (int)(out.nodes.size() / 32);
    out.nodes.resize(out.nodes.size() + 32, 0.0f);
    std::vector<int> ch;
    if (is_leaf(n)) {
      ch.push_back(n);  // a root that is a leaf
    } else {
      ch = {B.nodes[n].left, B.nodes[n].right};
      while (ch.size() < 4) {
        int best = -1;
        float ba = -1.0f;
        for (size_t i = 0; i < ch.size(); ++i)
          if (!is_leaf(ch[i]) && area(ch[i]) > ba) { ba = area(ch[i]); best = (int)i; }
        if (best < 0) break;
        const int x = ch[best];
        ch[best] = B.nodes[x].left;
        ch.insert(ch.begin() + best + 1, B.nodes[x].right);
      }
    }
    int32_t ref[4] = {kBvhEmpty, kBvhEmpty, kBvhEmpty, kBvhEmpty};
    float lo[3][4], hi[3][4];
    int inner = 0, sub = 0;
    for (int k = 0; k < 4; ++k)
      for (int a = 0; a < 3; ++a) { lo[a][k] = INFINITY; hi[a][k] = -INFINITY; }
    for (size_t k = 0; k < ch.size(); ++k) {
      const Box& b = B.nodes[ch[k]].box;
      for (int a = 0; a < 3; ++a) { lo[a][k] = b.lo[a] - pad; hi[a][k] = b.hi[a] + pad; }
      if (is_leaf(ch[k])) {
        ref[k] = leaf_ref(ch[k]);
      } else {
        const auto r = emit(ch[k]);
        ref[k] = r.first;
        sub = std::max(sub, r.second);
        ++inner;
      }
    }
    float* f = &out.nodes[(size_t)id * 32];
    for (int k = 0; k < 4; ++k) {
      float* c = f + 8 * k;
      for (int a = 0; a < 3; ++a) {
        c[a] = lo[a][k];
        c[4 + a] = hi[a][k];
      }
      const uint32_t u = (uint32_t)ref[k];
      std::memcpy(&c[3], &u, 4);
    }
    return {id, std::max(0, inner - 1) + sub};
  };
  out.nodes.reserve((size_t)n_tris * 16);
  out.max_stack = emit(0).second;
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
