// rt_kernels.h -- kernel parameter blocks and launch entry points of librtq
// (internal to the library; not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rt.h"
#include "accumulate.h"
#include "rt_layout.h"

// One batch entry of a batched plan (device copy).
struct BatchDesc {
  const float* nodes;
  const rt_tri_rec* tris;
  const rt_mesh_dev* meshes;
  const rt_ray* rays;
  rt_hit* hits;
  uint32_t root;
  uint32_t count;
  const rt_inst_rec* insts;      // two-level plans
  const rt_inst_rec64* insts64;  // two-level plans
  uint32_t* inst_ids;            // two-level plans: instance ids out (may be null)
};

struct TraceParams {
  const float* nodes;
  const rt_tri_rec* tris;
  const rt_inst_rec* insts;
  const rt_inst_rec64* insts64;
  const rt_mesh_dev* meshes;
  const rt_ray* rays;
  rt_hit* hits;
  uint32_t* inst_ids;
  uint8_t* occluded;
  uint32_t* counter;     // ray queue head, zero before the launch
  uint32_t* gstack;      // global stack: (max_stack - S) * gstride entries
  const BatchDesc* batches;
  const uint32_t* batch_offsets;  // batch_count + 1 prefix sums of counts
  uint32_t batch_count;
  uint32_t root;
  uint32_t n;            // rays in the launch (batched: total)
  uint32_t max_stack;    // stack entries a lane may need
  uint32_t gstride;      // threads in the grid
  uint32_t refill_min;   // refill a wave once this many lanes are idle
  uint64_t* counters;    // counting variants: node visits, triangle tests, spills
  uint32_t phase_counters;  // counting variants: also the wave-level loop counts (counters[4..7])
                         // (sums) and the deepest stack fill (maximum)
  uint32_t* status;      // host-mapped word: a lane of a counting variant
                         // sets it to 1 when a push would exceed max_stack
  // query options (modes 2 and 3; each may be null)
  const uint32_t* ray_masks;
  const uint32_t* skip_inst;
  const uint32_t* skip_prim;
  uint32_t* counts;      // mode 3: hits per ray
  uint32_t cap;          // mode 3: list entries per ray
  // closest queries on one accel (mode 0): the float64 finalize runs in the
  // traversal kernel, each wave finalizing the ray
  // ranges it took from the queue once they are all finished.  ranges: kRtRangesPerWave (first, count) pairs per
  // wave of the grid; a wave whose list is full appends further ranges to
  // ovf (ovf_cap pairs, their number in counter[1], zero before the launch),
  // finalized by a follow-up kernel.
  uint32_t* ranges;
  uint32_t* ovf;
  uint32_t ovf_cap;
};

// per-wave ray ranges kept for the finalize inside the closest-hit traversal
constexpr uint32_t kRtRangesPerWave = 128;

// Single-level adjoint (a workgroup of 1024 threads per tile of rta::kTile
// rays): writes the ray gradients and places each hit ray's record in its
// bucket for the vertex accumulation of accumulate.h.
struct BackwardParams {
  rt_mesh_dev mesh;
  const float* tri_vertices;   // 9 floats per triangle: its vertices in index order
  const rt_ray* rays;
  const rt_hit* hits;
  const float* d_tuv;
  uint32_t n;
  float* d_origins;
  float* d_directions;
  rta::Bucketing bk;
};

// Adjoint of two-level closest hits (one thread per ray, two phases as
// above).  Vertex rows: vertex_base[mesh] + vertex id; frame rows:
// frame_row0 + 4 * instance + part, parts holding (S xyz), (q xyz),
// (q w, T x, T y), (T z, -, -).
struct BackwardInstParams {
  const rt_mesh_dev* meshes;      // device mesh records (the accel's copies)
  const uint64_t* vertex_base;    // first gradient row of each mesh
  const rt_inst_rec* insts;       // mesh of each instance
  const rt_inst_rec64* insts64;   // float64 world-to-object maps
  const rt_srt* srts;             // frames as given to the build
  uint32_t inst_count;
  const rt_ray* rays;
  const rt_hit* hits;
  const uint32_t* inst_ids;
  const float* d_tuv;
  uint32_t n;
  float* d_origins;
  float* d_directions;
  rta::Acc acc;
  uint32_t want_vertices;         // add vertex rows
  uint32_t want_frames;           // add frame rows
  uint32_t frame_row0;
  // bucketed form (backward_inst_tile_kernel): global-triangle vertex copy,
  // each instance's (first global triangle, triangle count), placements
  const float* tri_vertices;
  const uint2* inst_tris;
  rta::Bucketing vb, fb;
};

// Ambient-occlusion rays from closest hits (one thread per ray sample).
struct AoParams {
  rt_mesh_dev mesh;       // single level
  const rt_mesh_dev* meshes;  // two-level (device): every mesh
  const rt_inst_rec* insts;   // two-level: instance records (mesh id)
  const rt_srt* srts;         // two-level: frames
  const uint32_t* inst_ids;   // two-level: instance of each hit; null for single level
  uint32_t inst_count;
  const rt_ray* rays;
  const rt_hit* hits;
  const float* xi;        // n * samples * 2 uniforms
  rt_ray* out;            // n * samples rays
  uint32_t n;
  uint32_t samples;
  double offset;
  float radius;
};

// Kernel handle for a variant (mode 0: one accel, mode 1: batched closest,
// mode 2: one accel with query options, mode 3: all hits with query options;
// modes 2 and 3 exist for stack 16 / workgroup 256 only); nullptr when the
// combination is not compiled.
const void* rtk_trace_kernel(int width, int stack, int wg, bool any, bool inst, int mode);
const void* rtk_count_kernel(int width, bool any, bool inst);
hipError_t rtk_launch_trace(const void* kern, uint32_t grid, uint32_t wg, const TraceParams& p,
                            hipStream_t stream);
// float64 finalize of closest hits written by a trace launch with the same params
hipError_t rtk_launch_finalize(bool inst, int mode, const TraceParams& p, hipStream_t stream);
// true when the traversal kernel of (any, inst, mode) finalizes its own hits
// (it then needs p.ranges / p.ovf and rtk_launch_finalize_ovf afterwards)
bool rtk_trace_fuses_finalize(bool any, bool inst, int mode);
// float64 finalize of the overflow ranges of a fused traversal launch
hipError_t rtk_launch_finalize_ovf(bool inst, const TraceParams& p, hipStream_t stream);
// float64 finalize of the hit lists of an all-hits launch (n * cap entries)
hipError_t rtk_launch_finalize_all(bool inst, const TraceParams& p, hipStream_t stream);
hipError_t rtk_launch_backward(const BackwardParams& p, hipStream_t stream);
hipError_t rtk_launch_backward_inst(const BackwardInstParams& p, int phase, hipStream_t stream);
// the bucketed two-level adjoint (p.vb / p.fb placements; grid of kTile-ray tiles)
hipError_t rtk_launch_backward_inst_tiles(const BackwardInstParams& p, hipStream_t stream);
hipError_t rtk_launch_refit_tris(rt_tri_rec* tris, uint32_t n, const rt_mesh_dev& mesh,
                                 hipStream_t stream);
hipError_t rtk_launch_refit_nodes(int width, float* nodes, const rt_tri_rec* tris,
                                  const uint32_t* node_ids, uint32_t count, hipStream_t stream);
hipError_t rtk_launch_fill(uint32_t* ptr, uint32_t n, uint32_t value, hipStream_t stream);
hipError_t rtk_launch_ao_rays(const AoParams& p, hipStream_t stream);
hipError_t rtk_launch_ao_resolve(const uint8_t* occluded, uint32_t n, uint32_t samples, float* ao,
                                 hipStream_t stream);
