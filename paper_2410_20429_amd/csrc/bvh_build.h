// Host BVH builder interface.
#pragma once
#include <cstdint>
#include <vector>

namespace mars {

struct BvhResult {
  std::vector<float> nodes;        // [n_nodes][16] floats (64 B per node)
  std::vector<float> tris;         // [n_tris][12] floats, leaf order
  std::vector<int32_t> prim_order; // leaf order -> primitive index
  int max_depth = 0;
};

// V: [n_tris][9] vertices; pad: absolute padding added to every child box
BvhResult build_bvh(const float* V, int n_tris, float pad);

}  // namespace mars
