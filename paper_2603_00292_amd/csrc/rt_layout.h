// rt_layout.h -- device data layout of the acceleration structure, shared by
// the host builder and the HIP kernels of librtq.
//
// Node of a W-wide BVH (W = 2, 4, 8), 32*W bytes, 16-byte aligned:
//   float lo_x[W], hi_x[W], lo_y[W], hi_y[W], lo_z[W], hi_z[W];  child boxes
//   uint32 child[W];                                             child refs
//   uint32 pad[W];
// Child boxes are the exact min/max of the float32 vertices below them, so a
// conservative slab test never culls a box that holds a hit.  Empty slots
// carry an inverted box (lo = +inf, hi = -inf), which every slab test
// rejects, and child = RT_CHILD_EMPTY.
//
// Child reference encoding (32 bits):
//   bit 31 = 0               internal node, bits 30..0 = node index
//   bit 31 = 1, bit 30 = 0   triangle leaf: bits 29..26 = count (1..15),
//                            bits 25..0 = first triangle record
//   bit 31 = 1, bit 30 = 1   instance leaf: bits 29..0 = instance index
//   0xFFFFFFFF               empty slot
//
// Triangle record (48 bytes, leaf order): three float4
//   (p0.xyz, prim id bits), (p1.xyz, order), (p2.xyz, 0)
// with the vertices sorted lexicographically (x, then y, then z), p0 < p1 <
// p2, so every edge is evaluated from its smaller endpoint on both triangles
// sharing it (bit-identical edge functions, no cracks).  The inside test and
// t do not depend on the vertex order; u, v are recomputed in float64 from
// the original vertex order at the end of a query: bits 2c..2c+1 of `order`
// give the sorted slot of the triangle's corner c.
//
// Instance record (64 bytes): float32 rows of the world->object affine map
// (3 x float4: r0, r1, r2 with object = R3x3 * world + c in .w), blas root
// ref, mesh id, visibility mask, 1 pad word.
#pragma once
#include <stdint.h>

#define RT_CHILD_EMPTY 0xFFFFFFFFu
#define RT_LEAF_BIT 0x80000000u
#define RT_INST_BIT 0x40000000u
#define RT_LEAF_COUNT_SHIFT 26
#define RT_LEAF_COUNT_MASK 0xFu
#define RT_LEAF_FIRST_MASK 0x03FFFFFFu
#define RT_INST_INDEX_MASK 0x3FFFFFFFu
#define RT_MAX_LEAF_SIZE 15u
#define RT_MAX_TRI_RECORDS (RT_LEAF_FIRST_MASK + 1u)

static inline uint32_t rt_make_leaf(uint32_t first, uint32_t count) {
  return RT_LEAF_BIT | (count << RT_LEAF_COUNT_SHIFT) | first;
}
static inline uint32_t rt_make_inst(uint32_t inst) { return RT_LEAF_BIT | RT_INST_BIT | inst; }

struct rt_tri_rec {
  float p0x, p0y, p0z;
  uint32_t prim;
  float p1x, p1y, p1z;
  uint32_t order;  // sorted slot of corner c in bits 2c..2c+1
  float p2x, p2y, p2z;
  uint32_t pad2;
};

struct rt_inst_rec {
  float r0[4];
  float r1[4];
  float r2[4];
  uint32_t root;
  uint32_t mesh;
  uint32_t mask;   // visibility mask, ANDed with a ray's mask (all ones by default)
  uint32_t pad;
};

// float64 world->object map of an instance, used by the float64 finalize
struct rt_inst_rec64 {
  double m[12];  // rows r0, r1, r2: (m00 m01 m02 c0) ...
};

// Per-mesh data needed by the float64 finalize and by the adjoint: the
// original vertices and indices (compact, stride 12).
struct rt_mesh_dev {
  const float* vertices;
  const uint32_t* indices;
  uint32_t vertex_count;
  uint32_t triangle_count;
};
