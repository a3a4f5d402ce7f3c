/* rt.h -- C ABI of the MI355X ray-query library (librtq.so).
 *
 * The library answers ray queries against triangle meshes: the closest hit
 * (t, triangle id, barycentrics u, v), any hit (occlusion) and the adjoint of
 * the closest hit.  It implements the data-parallel hot path of the method in
 * arxiv 2603.00292 ("Ray Tracing using HIP"): traversal of a bounding-volume
 * hierarchy with ray/triangle tests (§6.2 and its traversal paragraph), over
 * indexed triangle meshes given as float3 vertices and uint3 indices (§7.2),
 * optionally instanced with scale/rotation/translation frames in a two-level
 * hierarchy (§6.2 two-level paragraph, §7.3).
 *
 * Conventions for every function below
 *  - Buffers called "device" are HIP device pointers owned by the caller;
 *    "host" pointers are ordinary host memory read before the call returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Query calls only enqueue work on it and return; results are valid once
 *    the stream has reached that point.
 *  - Every function returns an rt_status.  Argument errors are detected on the
 *    host and returned before anything is enqueued; a device fault surfaces as
 *    RT_ERROR_HIP from a later call.  No C++ exception crosses the boundary.
 *    rt_last_error_message() gives a thread-local detail string.
 *    In every function: a NULL handle (context, accel, plan), or a NULL
 *    pointer that the call would read or write (a query with n = 0 touches
 *    no buffer), is RT_ERROR_INVALID_VALUE, a failed device or host
 *    allocation RT_ERROR_OUT_OF_MEMORY, a failed HIP call RT_ERROR_HIP.  A
 *    handle used while another device is current is not an error: the call
 *    makes the handle's device current for the calling thread, and it stays
 *    current afterwards.  The "Errors:" line of each function lists its
 *    other conditions.
 *  - A traversal lane whose stack would grow past the accel's bound
 *    (rt_accel_info.max_stack, the builder's bound on the entries any ray
 *    can need, which the global spill stack is sized for) drops the entry,
 *    so memory stays in bounds.  The counting variant (rt_trace_counters)
 *    checks the bound: it reports the deepest fill, and a dropped entry
 *    flags the context, so that the next query or batch launch on it returns
 *    RT_ERROR_STACK_OVERFLOW without enqueuing anything (clearing the flag).
 *    The query kernels do not check (it costs them about 1%).
 *  - Ray record (32 bytes, float32): origin o, tmin, direction d, tmax.  The
 *    ray is R(t) = o + t d (§3.1); t is measured in units of the given d (d is
 *    never normalised); a hit needs tmin <= t <= tmax (both inclusive, the
 *    MIN_T/MAX_T of the §3.1 listing).  A ray with a NaN, a zero direction or
 *    tmin > tmax is a miss, never an error.
 *  - Triangles are two-sided; edges and vertices are inclusive.  Degenerate
 *    triangles (zero normal or non-finite vertices) are never hit.
 *  - Closest hit = lexicographic minimum of (t, instance id, triangle id)
 *    (the strict "t < minT" linear search of §3.3 visits ids in ascending
 *    order, so the lowest id wins a tie in t).  A miss reports
 *    t = +inf, prim_id = RT_INVALID_ID, u = v = 0.
 *  - (u, v) are the barycentric weights of v1 and v2: the hit point is
 *    (1-u-v) v0 + u v1 + v v2 (the paper names u, v without defining them).
 *  - Traversal and the hit search run in float32; the reported (t, u, v) of
 *    the winning triangle is recomputed in float64 from the float32 inputs and
 *    rounded once to float32.
 */
#ifndef RTQ_RT_H
#define RTQ_RT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rt_status {
  RT_SUCCESS = 0,
  RT_ERROR_INVALID_VALUE = 1,      /* null pointer with n > 0, bad stride/scale/option */
  RT_ERROR_OUT_OF_MEMORY = 2,      /* a device or host allocation failed */
  RT_ERROR_NO_DEVICE = 3,          /* no HIP device, or the device id is out of range */
  RT_ERROR_HIP = 4,                /* a HIP runtime call failed (detail in the message) */
  RT_ERROR_UNSUPPORTED = 5,        /* a valid request the library does not implement */
  RT_ERROR_INDEX_OUT_OF_RANGE = 6, /* a triangle index >= vertex_count, a mesh id >= mesh_count */
  RT_ERROR_STACK_OVERFLOW = 7      /* an earlier counting traversal (rt_trace_counters) on this
                                      context needed more stack entries than the accel's bound
                                      (rt_accel_info.max_stack); its results may lack hits */
} rt_status;

/* Miss / no instance (the linear search of §3.3 starts from triIdx = -1). */
#define RT_INVALID_ID 0xFFFFFFFFu

typedef struct rt_context_s* rt_context;
typedef struct rt_accel_s* rt_accel;
typedef struct rt_batch_plan_s* rt_batch_plan;

/* 32-byte ray (ray fields of §7.5: origin, direction, minT, maxT). */
typedef struct rt_ray {
  float ox, oy, oz, tmin;
  float dx, dy, dz, tmax;
} rt_ray;

/* 16-byte closest-hit record. */
typedef struct rt_hit {
  float t;
  uint32_t prim_id;
  float u, v;
} rt_hit;

/* Instance frame (§7.3 lists scale, rotation, translation components):
 * world = T + R(q/|q|) (S * x), S per axis (non-zero, finite), q = (x,y,z,w)
 * a non-zero quaternion, normalised by the library. */
typedef struct rt_srt {
  float sx, sy, sz;
  float qx, qy, qz, qw;
  float tx, ty, tz;
} rt_srt;

/* Indexed triangle mesh (§7.2): device pointers; strides in bytes (>= 12).
 * vertices: vertex_count records of 3 float32; indices: triangle_count
 * records of 3 uint32. */
typedef struct rt_mesh_desc {
  const float* vertices;
  uint32_t vertex_count;
  uint32_t vertex_stride;
  const uint32_t* indices;
  uint32_t triangle_count;
  uint32_t index_stride;
} rt_mesh_desc;

/* Build options.  node_width: 0 = default (4), or 2, 4, 8 (§6.2: wide trees
 * of branching factor 4 or 8).  max_leaf_size: 0 = default (4), at most 15.
 * flags: 0 (host binned-SAH build) or RT_BUILD_DEVICE. */
/* Build the trees on the GPU (§6.2 construction paragraph: bottom-up
 * clustering from one cluster per triangle), by PLOC: clusters in Morton
 * order of the triangle centres, repeatedly merged with their mutual nearest
 * neighbour by merged-box surface area, then collapsed to node_width.  Much
 * faster to build than the host SAH build, with a tree that traces somewhat
 * slower.  With instances, every mesh's tree is built on the GPU and the
 * top-level tree over the instance boxes on the host.  Vertex and index
 * pointers and strides must be multiples of 4 bytes. */
#define RT_BUILD_DEVICE 0x1u

typedef struct rt_build_options {
  uint32_t node_width;
  uint32_t max_leaf_size;
  uint32_t flags;
} rt_build_options;

/* Trace variant (launch configuration of the traversal kernels):
 * stack_entries = per-lane traversal stack kept in LDS (8, 16, 32; deeper
 * entries spill to a global stack), workgroup = threads per workgroup (64,
 * 128, 256).  The defaults are 16 and 256.  Results do not depend on the
 * variant (§7.5 notes that stack and block sizes are compile-time choices). */
typedef struct rt_variant {
  uint32_t stack_entries;
  uint32_t workgroup;
} rt_variant;

/* Statistics of a built acceleration structure (host-side copy). */
typedef struct rt_accel_info {
  uint32_t node_width;
  uint32_t node_count;         /* all levels */
  uint32_t triangle_count;     /* triangles stored (degenerate ones are dropped) */
  uint32_t input_triangles;    /* triangles given */
  uint32_t instance_count;
  uint32_t max_depth;          /* longest root-to-leaf path in nodes, over both levels */
  uint32_t max_stack;          /* traversal stack entries a lane can need */
  uint32_t leaf_count;
  double sah_cost;             /* sum of internal-node surface areas / root area (§6.2) */
  uint64_t device_bytes;       /* device memory owned by the accel */
} rt_accel_info;

/* ---- context (§7.1) ---------------------------------------------------- */

/* Creates a context on HIP device `hip_device` and makes it current for the
 * calling thread's later library calls.  Errors: RT_ERROR_NO_DEVICE,
 * RT_ERROR_INVALID_VALUE (out == NULL), RT_ERROR_OUT_OF_MEMORY, RT_ERROR_HIP.
 * Test hook for the out-of-memory paths: with the environment variable
 * RT_FAULT_ALLOC = k (k >= 1) set at this call, the k-th device or pinned
 * allocation the library makes after it (by any context) fails once; the
 * call that made it returns RT_ERROR_OUT_OF_MEMORY and frees what it had
 * allocated, and objects it was to create are not created.  Unset or 0:
 * no failure (this call disarms an earlier one). */
rt_status rt_context_create(int hip_device, rt_context* out);
/* Frees the context's scratch (global stacks, queue counters, the ray-range
 * lists of rt_trace_closest).  An accel
 * keeps the context it was built with and traces with that context's
 * variant and scratch, so destroy every accel and batch plan of a context
 * before the context.  Trace calls of one context on different streams are
 * ordered one after another (they share the scratch). */
rt_status rt_context_destroy(rt_context ctx);
/* Sets the variant used by later trace calls on this context (see
 * rt_variant); RT_ERROR_INVALID_VALUE for unsupported values. */
rt_status rt_context_set_variant(rt_context ctx, const rt_variant* v);
rt_status rt_context_get_variant(rt_context ctx, rt_variant* out);

/* Traversal-kernel timing.  Measurement support, no operation of the paper:
 * it lets a caller relate a query's traversal kernel alone (without the
 * queue reset and, except for rt_trace_closest, whose traversal kernel runs
 * it, without the float64 finalize) to the bytes and
 * instructions it needs.  With slots > 0, every later rt_trace_closest / rt_trace_any /
 * rt_trace_closest_ex / rt_trace_any_ex / rt_trace_all / rt_trace_counters
 * call on this context records a pair of HIP events on its stream directly
 * before and after its traversal kernel, into the next of `slots` pairs used
 * round-robin; slots == 0 turns this off.  The events are owned by the
 * context; a new call waits for the recorded ones and replaces them.
 * Batched plans record nothing.
 * Errors: RT_ERROR_INVALID_VALUE (NULL context, slots > RT_TIMING_MAX_SLOTS),
 * RT_ERROR_HIP. */
#define RT_TIMING_MAX_SLOTS 4096u
rt_status rt_context_set_timing(rt_context ctx, uint32_t slots);
/* Waits for the timed launches recorded since the last read (at most the
 * last `slots` of them) and writes their traversal-kernel durations in
 * milliseconds, oldest first, into ms[0 .. min(that number, capacity)) (HOST),
 * and that count into *count (HOST); the launches not returned are dropped.
 * *count is 0 when timing is off.
 * Errors: RT_ERROR_INVALID_VALUE (NULL ctx or count, or NULL ms with
 * capacity > 0), RT_ERROR_HIP. */
rt_status rt_context_read_timing(rt_context ctx, float* ms, uint32_t capacity, uint32_t* count);

/* ---- build (§7.2, §7.3; top-down construction of §6.2) ----------------- */

/* Builds an acceleration structure.
 *  instance_count == 0: a single-level BVH over meshes[0] (mesh_count must
 *    be 1); instance_mesh / instance_srt must be NULL.
 *  instance_count > 0: a bottom-level BVH per mesh and a top-level BVH over
 *    the instances; instance_mesh[j] (HOST) < mesh_count selects the mesh of
 *    instance j and instance_srt[j] (HOST) its frame.
 * The mesh buffers are read on `stream`; the call returns after the build
 * has completed, and the caller may then free or modify them (the accel
 * keeps its own copies).  Triangles whose normal is zero or whose vertices
 * are not finite are not stored (they can never be hit).
 * Errors: RT_ERROR_INVALID_VALUE (null pointers, stride < 12, mesh_count
 * mismatch, zero/non-finite scale, zero quaternion, bad options),
 * RT_ERROR_INDEX_OUT_OF_RANGE (an index >= vertex_count, a mesh id >=
 * mesh_count), RT_ERROR_OUT_OF_MEMORY, RT_ERROR_HIP. */
rt_status rt_build(rt_context ctx, const rt_mesh_desc* meshes, uint32_t mesh_count,
                   const uint32_t* instance_mesh, const rt_srt* instance_srt,
                   uint32_t instance_count, const rt_build_options* options, void* stream,
                   rt_accel* out);
rt_status rt_accel_destroy(rt_accel accel);
rt_status rt_accel_get_info(rt_accel accel, rt_accel_info* out);

/* ---- queries (§6.2 traversal paragraph; §7.5 closest and any-hit) ------- */

/* Closest hit for n rays (device) into hits (device, n records).
 * inst_ids (device, n uint32, nullable): instance of the hit, RT_INVALID_ID
 * on a miss (0 on hits of a single-level accel).  n == 0 does nothing. */
rt_status rt_trace_closest(rt_accel accel, const rt_ray* rays, uint32_t n, rt_hit* hits,
                           uint32_t* inst_ids, void* stream);

/* rt_trace_closest for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, same kernels and bit-identical results, but
 * the launch's scratch (ray-queue counters, the per-wave ray-range lists of
 * the float64 finalize and the global spill stack) lives in a fixed device
 * array of RT_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it
 * runs on until the process ends; the call allocates nothing.  The grid is
 * narrowed when the spill stack of a full grid would not fit.  Every call on
 * a GPU shares that GPU's array: calls that overlap on one GPU (from
 * different contexts, or on streams the caller does not order) race and
 * must not be issued; calls of one context are ordered as usual.
 * Errors: as rt_trace_closest, and RT_ERROR_INVALID_VALUE when n rays need
 * more scratch than the array holds (about 2^28 rays at the default refill
 * setting). */
#define RT_NOALLOC_SCRATCH_BYTES (64u << 20)
rt_status rt_trace_closest_noalloc(rt_accel accel, const rt_ray* rays, uint32_t n, rt_hit* hits,
                                   uint32_t* inst_ids, void* stream);

/* Any hit (§4.2: stop at the first hit found within the ray's length):
 * occluded[i] (device, n bytes) = 1 when some triangle is hit with
 * t in [tmin, tmax], else 0. */
rt_status rt_trace_any(rt_accel accel, const rt_ray* rays, uint32_t n, uint8_t* occluded,
                       void* stream);

/* ---- ambient occlusion (§4), a workload driving the queries ------------- */

/* Ambient-occlusion rays for the closest hits of a single-level accel.  For
 * ray i with hit (hits[i], as written by rt_trace_closest) and sample k,
 * with the uniforms xi[2(i*samples + k) + {0,1}] (DEVICE, float32 in [0,1)):
 * shading point p = o + t d; unit geometric normal n of the hit triangle
 * turned toward the incoming ray; tangent t0 = (v1 - v0)/|v1 - v0| and
 * bi-tangent t1 = n x t0 (§4.1); the cosine-weighted direction of §4.1
 * (phi = 2 pi xi0, rr = sqrt(xi1); (rr cos phi, sqrt(1 - rr^2), rr sin phi)
 * in the (t0, n, t1) frame); origin p + offset n (§4.2 self-intersection
 * offset); t in [0, radius] (§4.2 limited length).  Written to
 * ao_rays[i*samples + k] (DEVICE); a miss gives void rays (tmin 1 > tmax 0,
 * never occluded).  Computed in float64, rounded once to float32.
 * Errors: RT_ERROR_UNSUPPORTED on a two-level accel; RT_ERROR_INVALID_VALUE
 * for samples < 1, a negative or non-finite offset, a negative radius,
 * n * samples >= 2^31, NULL buffers with n > 0, misaligned records. */
rt_status rt_ao_rays(rt_accel accel, const rt_ray* rays, const rt_hit* hits, uint32_t n,
                     uint32_t samples, const float* xi, float offset, float radius,
                     rt_ray* ao_rays, void* stream);

/* The same for the closest hits of a two-level accel: inst_ids[i] (DEVICE,
 * as written by rt_trace_closest) names the instance of ray i's hit, whose
 * frame maps the hit triangle's corners to world space (world = T +
 * R(qhat)(S x), §7.3) before the normal and tangent frame are formed; a hit
 * with an instance id >= instance_count gives void rays.  Errors:
 * RT_ERROR_UNSUPPORTED on a single-level accel; otherwise as rt_ao_rays
 * (inst_ids may not be NULL with n > 0). */
rt_status rt_ao_rays_instances(rt_accel accel, const rt_ray* rays, const rt_hit* hits, const uint32_t* inst_ids,
                               uint32_t n, uint32_t samples, const float* xi, float offset, float radius,
                               rt_ray* ao_rays, void* stream);

/* ao[i] = (number of k < samples with occluded[i*samples + k] != 0) /
 * samples (DEVICE buffers): the occluded fraction of §4's listing. */
rt_status rt_ao_resolve(const uint8_t* occluded, uint32_t n, uint32_t samples, float* ao,
                        void* stream);

/* ---- query variants (§6.2: a stack traversal finds the nearest, any or
 * all intersections; §7.5 names ray masks and intersection filters) ------- */

/* Options of the _ex and all-hit queries (all DEVICE arrays of n entries;
 * each may be NULL):
 *   ray_masks: ray i may hit instance j only when ray_masks[i] & mask_j != 0
 *     (instance masks default to 0xFFFFFFFF, see
 *     rt_accel_set_instance_masks; a single-level accel is one geometry of
 *     mask 0xFFFFFFFF, so a zero ray mask hits nothing).  NULL: all ones.
 *   skip_prim / skip_inst: ray i ignores the one triangle
 *     (skip_inst[i], skip_prim[i]), e.g. the triangle a secondary ray leaves
 *     (self-intersection filter).  skip_prim[i] = RT_INVALID_ID filters
 *     nothing; skip_inst is not read for single-level accels and may be NULL
 *     for them.  For a two-level accel with skip_prim set, skip_inst is
 *     required. */
typedef struct rt_query_options {
  const uint32_t* ray_masks;
  const uint32_t* skip_inst;
  const uint32_t* skip_prim;
} rt_query_options;

/* Largest list length of rt_trace_all. */
#define RT_MAX_HIT_CAPACITY 64u

/* Sets the visibility masks of a two-level accel's instances (masks: HOST
 * array of instance_count entries).  Returns after the update is visible to
 * later queries on any stream.  Errors: RT_ERROR_UNSUPPORTED on a
 * single-level accel; RT_ERROR_INVALID_VALUE for NULL masks. */
rt_status rt_accel_set_instance_masks(rt_accel accel, const uint32_t* masks, void* stream);

/* Moves the instances of a two-level accel (§6.2 construction paragraph:
 * for changed geometry, keep the tree's topology and refit its boxes
 * bottom-up; §7.3 instance frames).  instance_srt: HOST array of
 * instance_count new frames, under rt_build's rules.  The instance records
 * are recomputed (meshes and masks kept) and the boxes of the top-level tree
 * refit over its unchanged topology; the meshes' trees are untouched.  The
 * tree's quality may degrade for large motions; a new rt_build restores it.
 * Returns after the update is visible to later queries on any stream; the
 * caller makes sure no query of this accel is still running.  Errors:
 * RT_ERROR_UNSUPPORTED on a single-level accel, RT_ERROR_INVALID_VALUE for
 * a NULL array or an invalid frame (nothing is changed then). */
rt_status rt_update_instances(rt_accel accel, const rt_srt* instance_srt, void* stream);

/* rt_trace_closest / rt_trace_any with options (NULL options: none).  These
 * queries run the stack-16 / workgroup-256 variant of the context's node
 * width whatever the context's variant is. */
rt_status rt_trace_closest_ex(rt_accel accel, const rt_ray* rays, uint32_t n,
                              const rt_query_options* options, rt_hit* hits, uint32_t* inst_ids,
                              void* stream);
rt_status rt_trace_any_ex(rt_accel accel, const rt_ray* rays, uint32_t n,
                          const rt_query_options* options, uint8_t* occluded, void* stream);

/* All hits: for each ray, every triangle hit with t in [tmin, tmax] (after
 * masks and the filter) is counted in counts[i] (DEVICE, n uint32), and the
 * `capacity` nearest, sorted by (t, instance, prim_id), are written to
 * hits[i * capacity + k] (DEVICE, n * capacity records; entries past
 * min(counts[i], capacity) are misses: t = +inf, prim_id = RT_INVALID_ID)
 * with t, u, v as for rt_trace_closest; inst_ids (DEVICE, n * capacity,
 * nullable) gets the instance of each entry.  The traversal does not stop
 * at the nearest hit: its cost grows with the number of boxes the whole ray
 * crosses.  Runs the stack-16 / workgroup-256 variant.
 * Errors: RT_ERROR_INVALID_VALUE for capacity outside
 * [1, RT_MAX_HIT_CAPACITY], n * capacity >= 2^31, NULL buffers with n > 0,
 * rays/hits not 16-byte aligned. */
rt_status rt_trace_all(rt_accel accel, const rt_ray* rays, uint32_t n,
                       const rt_query_options* options, uint32_t capacity, rt_hit* hits,
                       uint32_t* inst_ids, uint32_t* counts, void* stream);

/* Adjoint of the closest hit at fixed triangles (single-level accels).
 * For each ray with hits[i].prim_id != RT_INVALID_ID and g = d_tuv[3i..3i+2]
 * = dL/d(t,u,v): with M = [-d | v1-v0 | v2-v0] and lambda = M^-T g,
 *   d_origins[i] = lambda, d_directions[i] = t lambda,
 *   d_vertices[v_k] += -w_k lambda  (w = (1-u-v, u, v))
 * using the accel's copy of the vertices it was built from.  d_vertices
 * (device, vertex_count*3 float32) is ACCUMULATED deterministically, without
 * global atomics: the hit rays are grouped by triangle range, each
 * (triangle, corner) sums its rays' float64 contributions exactly, as 64-bit
 * integers at the row's binary scale, each vertex adds its corners' values
 * in (triangle, corner) order, and the float64 sum is rounded once to
 * float32 and added; repeated calls, and calls with the rays permuted, give
 * bit-identical results.  The first call on an accel builds its vertex ->
 * corner lists and a per-triangle copy of the vertices (4 bytes per vertex
 * and 120 per triangle; rt_refit marks the copy stale and the next call
 * refreshes it); the context keeps 48 bytes per ray plus 4 per (4096-ray
 * tile, triangle range) of sort buffers, grown stream-ordered on `stream`
 * when n exceeds them.
 * d_origins / d_directions (device, n*3 float32) are overwritten (zero for
 * misses).  t, u, v are recomputed in float64 from the triangle, so `hits`
 * contributes only the triangle id.
 * Errors: RT_ERROR_INVALID_VALUE for a NULL accel, NULL rays, hits, d_tuv,
 * d_vertices, d_origins or d_directions with n > 0, or rays/hits not 16-byte
 * aligned; RT_ERROR_UNSUPPORTED on a two-level accel (use
 * rt_trace_backward_instances) or a mesh of more than 16,777,216 triangles
 * (16,384 groups of at most 1,024); RT_ERROR_OUT_OF_MEMORY when the lists,
 * the vertex copy or the sort buffers cannot be allocated. */
rt_status rt_trace_backward(rt_accel accel, const rt_ray* rays, const rt_hit* hits,
                            const float* d_tuv, uint32_t n, float* d_vertices, float* d_origins,
                            float* d_directions, void* stream);

/* Adjoint of two-level closest hits (§6.2 two-level hierarchy: a hit on an
 * instance is the hit of the ray taken to object space by the inverse of
 * the instance frame, so t, u, v are those of the world ray against the
 * world-space triangle T + R(q/|q|)(S v_k)).  For ray i with
 * hits[i].prim_id != RT_INVALID_ID on instance inst_ids[i] (the ids written
 * by rt_trace_closest) and g = d_tuv[3i..3i+2] = dL/d(t,u,v), with lambda =
 * M^-T g for the world-space M = [-d | W1-W0 | W2-W0]:
 *   d_origins[i] = lambda, d_directions[i] = t lambda (world space,
 *     device, n*3 float32, OVERWRITTEN; zero for misses);
 *   d_vertices (device, float32, nullable): gradients of the base meshes'
 *     object-space vertices, ACCUMULATED; mesh m's rows start at the sum of
 *     the vertex counts of meshes 0..m-1 (the mesh order of rt_build), so
 *     the buffer holds 3 * (total vertex count) floats (RT_ERROR_UNSUPPORTED
 *     when that count reaches 2^32 - 1);
 *   d_srt (device, instance_count*10 float32, nullable): gradients of each
 *     instance's (sx,sy,sz, qx,qy,qz,qw, tx,ty,tz) as given to rt_build,
 *     ACCUMULATED; the quaternion part is the gradient with respect to the
 *     unnormalised q (orthogonal to q).
 * Both accumulations are deterministic and independent of the order of the
 * rays, as in rt_trace_backward: the hit rays are grouped by triangle range
 * of the meshes' triangles taken one after another, and by instance; each
 * (triangle, corner) and each frame row sums its rays' float64
 * contributions exactly, as 64-bit integers at the row's binary scale, and
 * is rounded once.  The first call on an accel builds the vertex -> corner
 * lists of all meshes and a per-triangle copy of the object-space vertices
 * (4 bytes per vertex row, 120 per triangle, 8 per instance; rt_refit marks
 * the copy stale and the next call refreshes it); the context's sort
 * buffers (48 bytes per ray for each of the two groupings, plus 4 per
 * (4096-ray tile, group)) grow stream-ordered on `stream`.  Accels with
 * more than 16,384 instances (or any accel on a context created with the
 * environment variable RT_BACKWARD_ATOMIC=1) sum into fixed-point rows with
 * device atomics instead (the same row scale and rounding; the first such
 * call allocates 260 bytes per vertex row and 4 x 260 per instance).
 * t, u, v are recomputed in float64 with the accel's copies of the meshes
 * and frames.  A hit whose instance id is not an instance of
 * the accel, or whose prim_id is not a triangle of that instance's mesh,
 * contributes nothing (zero ray gradients).
 * Errors: RT_ERROR_UNSUPPORTED on a single-level accel (use
 * rt_trace_backward), or with d_vertices on an accel of 2^32 - 1 or more
 * vertex rows; RT_ERROR_INVALID_VALUE for a NULL accel, NULL rays, hits,
 * inst_ids, d_tuv, d_origins or d_directions with n > 0, or rays/hits not
 * 16-byte aligned; RT_ERROR_OUT_OF_MEMORY when the lists, the vertex copy,
 * the sort buffers or the atomic rows cannot be allocated. */
rt_status rt_trace_backward_instances(rt_accel accel, const rt_ray* rays, const rt_hit* hits,
                                      const uint32_t* inst_ids, const float* d_tuv, uint32_t n,
                                      float* d_vertices, float* d_srt, float* d_origins,
                                      float* d_directions, void* stream);

/* Diagnostics: the query of rt_trace_closest (any == 0, into hits) or
 * rt_trace_any (any != 0, into occluded) run with a counting kernel variant
 * (stack 16, workgroup 256).  counters (device, 4 uint64): the call ADDS
 * node visits (both levels of a two-level accel), triangle tests and stack
 * entries spilled to global memory to counters[0..2], and raises counters[3]
 * to the deepest stack fill any ray reached (entries, instance markers
 * included; at most rt_accel_info.max_stack).  Used to measure the bytes a
 * query fetches per ray.  The instance ids of a two-level closest query are
 * not written. */
rt_status rt_trace_counters(rt_accel accel, const rt_ray* rays, uint32_t n, int any, rt_hit* hits,
                            uint8_t* occluded, uint64_t* counters, void* stream);

/* rt_trace_counters with n_counters (4 or 8) uint64 counters.  With 8 the
 * call also ADDS the counting kernel's wave-level loop counts to
 * counters[4..7]: passes of its outer loop (refill check, node phase, leaf
 * phase), refills, node-loop iterations and leaf-loop iterations, every
 * iteration of a wave counted once.  A wave iteration issues its
 * instructions for all 64 lanes, so node visits / (64 x node-loop
 * iterations) is the node phase's lane occupancy, triangle tests / (64 x
 * leaf-loop iterations) the leaf phase's.  A diagnostic of how the work of
 * §7.5's stack traversal spreads over the lanes of a wave.
 * Errors: as rt_trace_counters; RT_ERROR_INVALID_VALUE for another
 * n_counters. */
rt_status rt_trace_counters_ex(rt_accel accel, const rt_ray* rays, uint32_t n, int any, rt_hit* hits,
                               uint8_t* occluded, uint64_t* counters, uint32_t n_counters, void* stream);

/* Refit (§6.2 construction paragraph: keep the topology of the hierarchy and
 * fit the bounding volumes to the current geometry, bottom-up): replaces the
 * accel's vertices by `vertices` (device, compact records of 3 float32) and
 * recomputes every triangle record and child box on `stream`.  Single level:
 * vertex_count records, enqueued without a host round trip.  Two-level: the
 * vertex_count records of every mesh one after another in build order (the
 * row layout of rt_trace_backward_instances); the meshes' trees are refit on
 * the device, their root boxes read back and the top-level boxes refit for
 * the current frames on the host, so the call returns after the update is
 * visible to later queries on any stream.  Triangles that were degenerate or
 * non-finite when the accel was built stay out of it; triangles that become
 * degenerate or non-finite are disabled (never hit) until a refit makes them
 * valid again.  Query results after a refit equal those of a fresh build on
 * the same vertices (up to ties between distinct triangles at equal t);
 * traversal cost grows as the geometry departs from the one the topology was
 * built for. */
rt_status rt_refit(rt_accel accel, const float* vertices, void* stream);

/* ---- batched queries (many meshes, one persistent launch) --------------- */

/* Plans closest-hit queries for batch_count (accel, rays, hits, count)
 * tuples: accels, rays, hits and counts are HOST arrays of length
 * batch_count whose rays/hits entries are device pointers.  The accels
 * belong to ctx's device, share one node width, and are either all
 * single-level or all two-level (RT_ERROR_INVALID_VALUE otherwise).  The
 * plan copies its descriptors to the device once; the buffers must stay
 * valid while the plan is used.  The plan keeps the context's variant at
 * creation (rt_context_set_variant afterwards does not affect it). */
rt_status rt_batch_plan_create(rt_context ctx, const rt_accel* accels, const rt_ray* const* rays,
                               rt_hit* const* hits, const uint32_t* counts, uint32_t batch_count,
                               rt_batch_plan* out);
/* The same, also writing instance ids for two-level accels: inst_ids is a
 * HOST array of batch_count device pointers, each NULL (no ids) or an array
 * of counts[b] uint32 written as by rt_trace_closest.  inst_ids may be NULL;
 * a non-NULL entry for a single-level accel is RT_ERROR_INVALID_VALUE. */
rt_status rt_batch_plan_create_instances(rt_context ctx, const rt_accel* accels, const rt_ray* const* rays,
                                         rt_hit* const* hits, uint32_t* const* inst_ids, const uint32_t* counts,
                                         uint32_t batch_count, rt_batch_plan* out);
/* Enqueues the whole batch: a queue reset and one persistent kernel launch. */
rt_status rt_batch_plan_launch(rt_batch_plan plan, void* stream);
/* Captures the launch into a HIP graph (queue reset by a fill kernel, not a
 * memset node) and instantiates it; *out is a hipGraphExec_t owned by the
 * plan (freed by rt_batch_plan_destroy).  Replay it with hipGraphLaunch. */
rt_status rt_batch_plan_graph(rt_batch_plan plan, void* stream, void** out_graph_exec);
rt_status rt_batch_plan_destroy(rt_batch_plan plan);

/* ---- autotuning ---------------------------------------------------------- */

/* One measured configuration. */
typedef struct rt_tune_entry {
  uint32_t node_width;
  uint32_t stack_entries;
  uint32_t workgroup;
  float ms;                   /* median of the timed closest-hit launches */
} rt_tune_entry;

/* Picks node width, stack entries and workgroup size for closest-hit
 * queries on `mesh` by measurement: the mesh is built at each candidate
 * node width (2, 4, 8) and every variant is timed with HIP events on
 * `stream` on the n_probe probe rays (device), median of `repeats` launches
 * after one warm-up.  On return *best holds the fastest configuration (the
 * default, node width 4 / stack 16 / workgroup 256, unless another is faster
 * by more than 1%), the context's variant is set to it, and table (HOST, capacity table_cap,
 * nullable) receives up to table_cap measured entries (*table_len = how many
 * were measured).  The caller builds its accel with best->node_width.
 * Synchronises the stream.  Errors as rt_build and rt_trace_closest. */
rt_status rt_autotune(rt_context ctx, const rt_mesh_desc* mesh, const rt_ray* probe_rays,
                      uint32_t n_probe, uint32_t repeats, void* stream, rt_tune_entry* best,
                      rt_tune_entry* table, uint32_t table_cap, uint32_t* table_len);

/* ---- diagnostics -------------------------------------------------------- */

const char* rt_status_string(rt_status s);
const char* rt_last_error_message(void);
/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
uint32_t rt_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RTQ_RT_H */
