/* rt_oracle.h -- FP64 CPU reference for ray/triangle queries.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path never
 * links, loads or calls it, and it shares no code with the HIP library.
 *
 * Everything is computed in double precision from float32 inputs promoted
 * exactly to double.  The queries are defined by the plain linear search over
 * every triangle (the paper's §3.3 search for the closest hit), using the
 * plane-then-edge ray/triangle test of §3.1.  A scene may carry an FP64 BVH
 * (orc_bvh_create): a median-split binary tree that only skips triangles
 * whose boxes provably hold no wanted pair, so the answers are identical bit
 * for bit to the linear search (§6.2: the hierarchy accelerates, it does not
 * change, the search).  No blocking or reordering of the arithmetic is used.
 *
 * Shared array conventions:
 *   vertices  float[nv*3]           (x,y,z) per vertex
 *   indices   uint32[nt*3]          three vertex indices per triangle
 *   rays      float[nr*8]           (ox,oy,oz,tmin, dx,dy,dz,tmax)
 *   srt       float[ninst*10]       (sx,sy,sz, qx,qy,qz,qw, tx,ty,tz):
 *                                   world = T + R(q/|q|)(S*x)
 *   prim/inst outputs use 0xFFFFFFFF for "none" (a miss).
 * Return value: 0 on success, -1 on invalid arguments (an index >= nv, a
 * null pointer with a non-zero count, a mesh id >= mesh count).
 */
#ifndef RT_ORACLE_H
#define RT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NONE 0xFFFFFFFFu

typedef struct orc_bvh_s orc_bvh;

/* A scene: n_mesh meshes; either no instances (n_inst == 0: mesh 0 is traced
 * in world space) or n_inst instances of the meshes with SRT frames.  bvh:
 * NULL for the linear search, or a hierarchy built from this very scene
 * (same arrays) by orc_bvh_create. */
typedef struct {
  int32_t n_mesh;
  const float* const* vertices;   /* [n_mesh] */
  const int64_t* n_vertices;      /* [n_mesh] */
  const uint32_t* const* indices; /* [n_mesh] */
  const int64_t* n_triangles;     /* [n_mesh] */
  int64_t n_inst;
  const uint32_t* inst_mesh;      /* [n_inst] */
  const float* inst_srt;          /* [n_inst*10] */
  const orc_bvh* bvh;
} orc_scene;

/* FP64 BVH of a scene: one median-split binary tree per mesh (boxes: exact
 * min/max of the float32 vertices) and, with instances, one over the
 * instances' world boxes.  It keeps pointers into the scene's arrays, which
 * must outlive it.  Returns 0, or -1 on invalid scenes or allocation failure. */
int orc_bvh_create(const orc_scene* s, orc_bvh** out);
void orc_bvh_destroy(orc_bvh* b);
/* out[4]: tree nodes over all meshes, triangles without a finite box, the
 * deepest leaf, nodes of the instance tree */
int orc_bvh_stats(const orc_bvh* b, int64_t* out);
/* The culling invariant, checked pair by pair against the linear search:
 * every box above a wanted pair (kind 0: a hit; kind 1: a sure or maybe pair
 * of the tolerance model with slack delta) admits it with a key no larger
 * than its t (its lowest possible t).  out[2] = pairs checked, violations. */
int orc_bvh_check(const orc_scene* s, const float* rays, int64_t nr, int kind, double delta,
                  int64_t* out);

/* Query options.  §7.5 names ray masks and intersection filters as options
 * of a traversal without fixing their semantics; the readings here:
 *   ray r may hit instance j only when ray_mask[r] & inst_mask[j] != 0 (a
 *     single-level scene is one geometry of mask 0xFFFFFFFF, so a zero ray
 *     mask hits nothing);
 *   ray r ignores the one triangle (skip_inst[r], skip_prim[r]) (the
 *     self-intersection filter of a ray leaving a surface); skip_prim[r] =
 *     ORC_NONE filters nothing and skip_inst is not used in single-level
 *     scenes.
 * Any pointer may be NULL (no masks, no filter). */
typedef struct {
  const uint32_t* inst_mask;  /* [n_inst] */
  const uint32_t* ray_mask;   /* [nr] */
  const uint32_t* skip_inst;  /* [nr] */
  const uint32_t* skip_prim;  /* [nr] */
} orc_opts;

/* Closest hit: lexicographic minimum of (t, inst, prim) over all hits.
 * Miss: inst = prim = ORC_NONE, t = +inf, u = v = 0.  inst_out may be NULL. */
int orc_closest(const orc_scene* s, const float* rays, int64_t nr,
                uint32_t* inst_out, uint32_t* prim_out, double* tuv_out /* nr*3 */);

int orc_closest_ex(const orc_scene* s, const float* rays, int64_t nr, const orc_opts* opts,
                   uint32_t* inst_out, uint32_t* prim_out, double* tuv_out);

/* Any hit: 1 when some triangle is hit with t in [tmin, tmax]. */
int orc_any(const orc_scene* s, const float* rays, int64_t nr, uint8_t* occluded);
int orc_any_ex(const orc_scene* s, const float* rays, int64_t nr, const orc_opts* opts,
               uint8_t* occluded);

/* All hits (§6.2: the stack traversal finds the nearest, any or all
 * intersections): every (inst, prim) hit within [tmin, tmax], sorted by
 * (t, inst, prim).  count[r] = number of hits; the first K are stored
 * (inst/prim ORC_NONE, t = +inf beyond the count).  inst_out may be NULL. */
int orc_all(const orc_scene* s, const float* rays, int64_t nr, const orc_opts* opts, int32_t K,
            int64_t* count, uint32_t* inst_out, uint32_t* prim_out, double* tuv_out /* nr*K*3 */);

/* Acceptable sets of the FP32 tolerance model (delta = relative slack).
 * For each ray: miss_ok (1 when no pair is a sure hit), count (number of
 * acceptable (inst, prim) pairs; may exceed K, then only the K smallest by
 * (t, inst, prim) are stored), the pairs and their FP64 (t,u,v) and the
 * scale s used in the t tolerance.  any_class: 1 = must be occluded,
 * 0 = must not be occluded, 2 = either (for an any-hit query). */
int orc_accept(const orc_scene* s, const float* rays, int64_t nr, double delta, int32_t K,
               uint8_t* miss_ok, int32_t* count, uint32_t* acc_inst /* nr*K */,
               uint32_t* acc_prim /* nr*K */, double* acc_tuv /* nr*K*3 */,
               double* acc_scale /* nr*K */, uint8_t* any_class);

int orc_accept_ex(const orc_scene* s, const float* rays, int64_t nr, const orc_opts* opts,
                  double delta, int32_t K, uint8_t* miss_ok, int32_t* count,
                  uint32_t* acc_inst, uint32_t* acc_prim, double* acc_tuv, double* acc_scale,
                  uint8_t* any_class);

/* Every candidate of the tolerance model for all-hit queries: count[r]
 * sure-or-maybe pairs (n_sure[r] of them sure), sorted by (t, inst, prim),
 * with the range [lo, hi] a float32 t of the pair may take; the first K are
 * stored. */
int orc_classify_all(const orc_scene* s, const float* rays, int64_t nr, const orc_opts* opts,
                     double delta, int32_t K, int32_t* count, int32_t* n_sure, uint32_t* acc_inst,
                     uint32_t* acc_prim, double* acc_tuv, double* acc_scale, double* acc_lo,
                     double* acc_hi, uint8_t* acc_sure);

/* Adjoint of (t,u,v) at fixed triangles, single-level scenes only.
 * prim[r] = ORC_NONE contributes nothing.  g = dL/d(t,u,v) per ray (nr*3).
 * d_vertices (nv*3) is ACCUMULATED; d_orig / d_dir (nr*3) are overwritten. */
int orc_adjoint(const orc_scene* s, const float* rays, const uint32_t* prim, int64_t nr,
                const double* g, double* d_vertices, double* d_orig, double* d_dir);

/* Central finite differences (step h) of l = g.(t,u,v) evaluated at the fixed
 * triangle prim[r] with the plane formula of §3.1 (no inside or range test).
 * Output per ray: 15 derivatives: v0.xyz, v1.xyz, v2.xyz, o.xyz, d.xyz. */
int orc_fd(const orc_scene* s, const float* rays, const uint32_t* prim, int64_t nr,
           const double* g, double h, double* out /* nr*15 */);

/* (t,u,v) of ray r against triangle prim[r] by the plane formula, no tests. */
int orc_fixed_tuv(const orc_scene* s, const float* rays, const uint32_t* prim, int64_t nr,
                  double* tuv);

/* Adjoint of (t,u,v) of two-level hits at fixed (inst[r], prim[r]): the
 * gradients reach the base mesh's object-space vertices and the instance's
 * ten frame parameters.  d_vertices: n_mesh pointers (the array or an entry
 * may be NULL: not wanted), mesh m holding nv_m*3 doubles, ACCUMULATED;
 * d_srt (n_inst*10, may be NULL) ACCUMULATED; d_orig / d_dir (nr*3)
 * overwritten.  prim[r] = ORC_NONE contributes nothing. */
int orc_adjoint_inst(const orc_scene* s, const float* rays, const uint32_t* inst,
                     const uint32_t* prim, int64_t nr, const double* g,
                     double* const* d_vertices, double* d_srt, double* d_orig, double* d_dir);

/* Central finite differences for two-level hits.  Output per ray: 25
 * derivatives: v0, v1, v2 (object space), the frame (sx,sy,sz, qx,qy,qz,qw,
 * tx,ty,tz), o.xyz, d.xyz. */
int orc_fd_inst(const orc_scene* s, const float* rays, const uint32_t* inst, const uint32_t* prim,
                int64_t nr, const double* g, double h, double* out /* nr*25 */);

/* Ambient-occlusion rays of §4 for single-level scenes: N per primary ray
 * from its closest hit (prim, tuv as returned by orc_closest) and the
 * uniforms xi (nr*N*2): cosine-weighted about the geometric normal facing
 * the incoming ray, tangent frame (v1-v0 normalised, n x tangent), origin
 * offset along the normal, t in [0, radius].  Misses give void rays
 * (tmin 1 > tmax 0).  out: nr*N*8 floats, ray r's sample k at r*N + k. */
int orc_ao_rays(const orc_scene* s, const float* rays, const uint32_t* prim, const double* tuv,
                int64_t nr, int32_t N, const float* xi, double offset, double radius,
                float* out);

/* The same for two-level scenes: inst[r] is the instance of ray r's closest
 * hit (as returned by orc_closest); the hit triangle's corners are mapped to
 * world space by that instance's frame before the normal and tangent frame
 * are formed. */
int orc_ao_rays_inst(const orc_scene* s, const float* rays, const uint32_t* inst, const uint32_t* prim,
                     const double* tuv, int64_t nr, int32_t N, const float* xi, double offset,
                     double radius, float* out);

int orc_num_threads(void);
void orc_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
