// bvh_build.h -- host BVH construction for librtq.
//
// Top-down construction (the splitting approach of §6.2, BVH construction
// paragraph) with binned surface-area-heuristic splits (Wald 2007, the
// top-down method the paper cites), producing a binary tree that is then
// collapsed into a W-wide tree (§6.2: wide trees of branching factor 4 or 8)
// and laid out as in rt_layout.h.  The cost the paper names -- the sum of the
// internal nodes' surface areas -- is reported for every tree.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "rt_layout.h"

namespace rtb {

struct Box {
  float lo[3], hi[3];
};

struct BuildInput {
  const float* vertices;     // host, vertex_count * 3 (compact)
  const uint32_t* indices;   // host, triangle_count * 3 (compact)
  uint32_t vertex_count;
  uint32_t triangle_count;
};

struct WideTree {
  int width = 4;
  std::vector<float> nodes;          // node_count * 8W floats (layout of rt_layout.h)
  std::vector<rt_tri_rec> tris;      // leaf order
  uint32_t node_count = 0;
  uint32_t root = RT_CHILD_EMPTY;    // child reference of the root (internal node 0 or empty)
  uint32_t max_depth = 0;            // nodes on the longest root-to-leaf path
  uint32_t max_stack = 0;            // stack entries a traversal may need
  uint32_t leaf_count = 0;
  uint32_t stored_triangles = 0;
  std::vector<uint32_t> node_depth;  // depth of each wide node (root = 1)
  double sah_cost = 0.0;             // sum of internal-node areas / root area
  Box bounds{};
};

// Builds the bottom-level tree of one mesh.  Degenerate triangles (zero
// float64 normal, non-finite vertices) are dropped.  Returns false and sets
// `err` on invalid input (an index out of range).
bool build_mesh(const BuildInput& in, int width, int max_leaf, WideTree& out, std::string& err,
                int threads);

// Builds the top-level tree over instance boxes; leaf i refers to instance
// ids[i] (instance leaves, one instance per leaf).
void build_instances(const std::vector<Box>& boxes, int width, WideTree& out, int threads);

}  // namespace rtb
