// bvh_device.h -- device-side BVH construction of one mesh (librtq internal).
//
// A bottom-up, clustering build on the GPU (§6.2 construction paragraph:
// every triangle starts as a cluster and clusters are merged until one
// remains), by PLOC (Meister & Bittner 2018), the family of the paper's
// balanced builder: triangles are ordered along a 30-bit Morton curve of
// their box centres; in each pass every cluster finds the cluster within 32
// places on either side whose merged box has the least surface area, mutual
// pairs merge, and the list is compacted.  The binary tree is collapsed level
// by level into the W-wide layout of rt_layout.h, leaves holding subtrees of
// up to max_leaf triangles, stored contiguously.  It trades some tree
// quality for build speed against the host binned-SAH build.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "rt_layout.h"

namespace rtd {

struct Input {
  const float* vertices;     // device, vertex_count records of vertex_stride bytes
  uint32_t vertex_count, vertex_stride;
  const uint32_t* indices;   // device, triangle_count records of index_stride bytes
  uint32_t triangle_count, index_stride;
  int width;                 // 2, 4 or 8
  int max_leaf;              // 1..15
};

// Device arrays are allocated with hipMalloc and handed to the caller, who
// frees them (listed in `owned`).
struct Output {
  float* nodes = nullptr;               // node_count * 8 * width floats
  rt_tri_rec* tris = nullptr;           // tri_count records, leaf order
  float* vertices = nullptr;            // compact copy, vertex_count * 3
  uint32_t* indices = nullptr;          // compact copy, triangle_count * 3
  uint32_t* refit_nodes = nullptr;      // wide node ids, deepest level first
  std::vector<uint32_t> refit_levels;   // level boundaries in refit_nodes
  std::vector<void*> owned;
  uint64_t owned_bytes = 0;
  uint32_t node_count = 0, tri_count = 0, leaf_count = 0, max_depth = 0, max_stack = 0;
  uint32_t root = RT_CHILD_EMPTY;
  double sah_cost = 0.0;
  float bounds[6] = {0, 0, 0, -1, -1, -1};  // box of all triangles (lo xyz, hi xyz; inverted when empty)
};

// Returns hipSuccess and fills `out`, or an error (then `out.owned` may hold
// allocations the caller frees).  `index_error` is set when an index is
// >= vertex_count (nothing else is valid then).
hipError_t build(const Input& in, Output& out, bool& index_error, hipStream_t stream);

// Adds node_base to the internal-node references and tri_base to the first
// record of the triangle-leaf references of node_count W-wide nodes (device),
// so that a tree can be placed at those offsets of larger node and record
// arrays.  Instance-leaf and empty references are left as they are.
hipError_t relocate(float* nodes, uint32_t node_count, int width, uint32_t node_base, uint32_t tri_base,
                    hipStream_t stream);

}  // namespace rtd
