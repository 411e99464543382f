// Host BVH builder interface.
#pragma once
#include <cstdint>
#include <vector>

namespace mars {

// child reference of an unused slot of a 4-wide node
constexpr int32_t kBvhEmpty = 0x7FFFFFFF;

struct BvhResult {
  std::vector<float> nodes;        // [n_nodes][4 children][8] floats (128 B per 4-wide node)
  std::vector<float> tris;         // [n_tris][12] floats, leaf order
  std::vector<int32_t> prim_order; // leaf order -> primitive index
  int max_depth = 0;  // of the binary tree
  int max_stack = 0;  // traversal stack entries the 4-wide tree can need
};

// V: [n_tris][9] vertices; pad: absolute padding added to every child box
BvhResult build_bvh(const float* V, int n_tris, float pad);

}  // namespace mars
