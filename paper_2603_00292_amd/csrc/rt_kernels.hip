// rt_kernels.hip -- traversal, adjoint and batched kernels of librtq (gfx950).
//
// One ray per lane (the paper's §3.3 observes that rays through pixels are
// independent and map to parallel threads).  Waves are persistent: lanes
// whose ray is finished take new rays from a global counter, one atomic per
// wave, with lane offsets from a ballot and a prefix popcount (wave-level
// compaction).  Each lane walks a W-wide BVH (§6.2) with a stack (the
// traversal paragraph of §6.2) whose top S entries live in LDS and whose
// deeper entries spill to a global buffer (§7.5 describes the shared-memory
// stack with a global fallback).  Internal nodes are visited until every
// live lane of the wave has reached a leaf, then the leaves are tested
// (Aila & Laine 2009, "while-while").  No matrix cores: this is pointer
// chasing, not a dense contraction.
//
// Numerics: float32 traversal with a conservative slab test (boxes are exact
// float32 bounds; the far distance is widened by 2*gamma(3), Ize 2013) and a
// watertight float32 ray/triangle test on canonically ordered edges (each
// shared edge is evaluated from the same endpoint with the same operations
// on both triangles, so no ray passes between them).  The winning triangle's
// (t, u, v) is recomputed in float64 from the float32 inputs.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rt_kernels.h"
#include "rt_layout.h"

namespace rtk {

// 1 + 2 gamma(3), gamma(n) = n u / (1 - n u), u = 2^-24, rounded up
__device__ constexpr float kSlabWiden = 3.5762793e-7f;
// relative widening of the best distance in the box test, so that a box
// holding an exact tie in t with a lower id is still visited
__device__ constexpr float kTieWiden = 9.5367432e-7f;  // 2^-20

#define RT_STACK_MARKER 0xFFFFFFFEu  // "leave the instance, restore the world ray"

struct RayState {
  float ox, oy, oz, dx, dy, dz;
  float ix, iy, iz;
  float tmin, tmax;
  uint32_t sx, sy, sz;  // 1 when the direction's sign bit is set
};

__device__ __forceinline__ void ray_setup(RayState& r) {
  r.ix = 1.0f / r.dx;
  r.iy = 1.0f / r.dy;
  r.iz = 1.0f / r.dz;
  r.sx = __float_as_uint(r.dx) >> 31;
  r.sy = __float_as_uint(r.dy) >> 31;
  r.sz = __float_as_uint(r.dz) >> 31;
}

// Rays that can never hit: a NaN, a zero direction, or tmin > tmax.
__device__ __forceinline__ bool ray_void(const rt_ray& q) {
  bool nan = (q.ox != q.ox) | (q.oy != q.oy) | (q.oz != q.oz) | (q.dx != q.dx) | (q.dy != q.dy) |
             (q.dz != q.dz) | (q.tmin != q.tmin) | (q.tmax != q.tmax);
  bool zero = (q.dx == 0.0f) & (q.dy == 0.0f) & (q.dz == 0.0f);
  return nan | zero | (q.tmin > q.tmax);
}

__device__ __forceinline__ rt_ray load_ray(const rt_ray* rays, uint32_t i) {
  const float4* p = reinterpret_cast<const float4*>(rays + i);
  float4 a = p[0], b = p[1];
  rt_ray q;
  q.ox = a.x; q.oy = a.y; q.oz = a.z; q.tmin = a.w;
  q.dx = b.x; q.dy = b.y; q.dz = b.z; q.tmax = b.w;
  return q;
}

// ---------------------------------------------------------------------------
// per-lane traversal stack: top S entries in LDS, the rest in global memory
// ---------------------------------------------------------------------------
// Entry i of a lane's stack lives in LDS slot (i mod S) while it is one of the
// S newest entries; older entries live at gstack[(i - S) * gstride + gtid].
// A push beyond `cap` (the builder's bound on the entries a ray can need,
// which the global stack is sized for; never below S) is not stored.  The
// counting variant (CHECK) also remembers it and raises the launch's
// host-mapped status word at the end, which the host turns into an error on
// the context's next call, and records the deepest fill.  The query kernels
// do neither: any observable action on that branch (a flag carried through
// the loop, a store of any kind) measured 1.3% on the closest-hit kernel.
template <int S, int WG, bool CHECK = false>
struct Stack {
  uint32_t* lds;       // this lane's column: lds[slot * WG]
  uint32_t* glob;      // this lane's column: glob[i * gstride]
  uint32_t gstride;
  uint32_t cap;        // total entries this lane may hold (at least S)
  uint32_t sp;
  uint32_t peak;       // CHECK: the largest sp reached
  bool over;           // CHECK: a push was dropped

  __device__ __forceinline__ void push(uint32_t v) {
    uint32_t slot = sp & (S - 1);
    if (sp >= S) {
      // only a stack that spills can reach the bound (cap >= S)
      if (sp >= cap) {
        if constexpr (CHECK) over = true;
        return;
      }
      glob[(size_t)(sp - S) * gstride] = lds[slot * WG];
    }
    lds[slot * WG] = v;
    ++sp;
    if constexpr (CHECK) peak = max(peak, sp);
  }
  __device__ __forceinline__ uint32_t pop() {
    if (sp == 0) return RT_CHILD_EMPTY;
    --sp;
    uint32_t slot = sp & (S - 1);
    uint32_t v = lds[slot * WG];
    if (sp >= S) lds[slot * WG] = glob[(size_t)(sp - S) * gstride];
    return v;
  }
};

// ---------------------------------------------------------------------------
// geometry access
// ---------------------------------------------------------------------------
struct Geo {
  const float* nodes;          // node_count * 8W floats
  const float4* tris;          // 3 float4 per record
  const rt_inst_rec* insts;    // two-level only
  const rt_inst_rec64* insts64;
  const rt_mesh_dev* meshes;
  uint32_t root;
  uint32_t max_stack;
};

// W-wide node visit: returns the child refs that the ray enters, nearest
// first, in keys k[0..W-1] (0xFFFFFFFF = no child).
// DIRECT (4-wide nodes only): each lane loads its near and far plane
// vectors at lane-dependent addresses (lo or hi by the sign of the ray's
// direction) instead of loading both and selecting; it needs more registers,
// which pays only where they are free (the single-level any-hit kernel:
// +2%; the closest-hit kernel loses a wave per SIMD and 5%).
template <int W, bool DIRECT = false>
__device__ __forceinline__ void visit_node(const float* nodes, uint32_t idx, const RayState& r,
                                           float tcull, uint32_t* out_ref, int& n_out) {
  constexpr int NF4 = (W == 2) ? 4 : (7 * W) / 4;  // skip trailing pad when it fills a float4
  constexpr bool PRE = DIRECT && W == 4;            // planes loaded in (near, far) order
  const float4* p = reinterpret_cast<const float4*>(nodes + (size_t)idx * (8 * W));
  float nd[4 * NF4];
  if constexpr (PRE) {
    float4 v[7];
    v[0] = p[r.sx];
    v[1] = p[1u - r.sx];
    v[2] = p[2u + r.sy];
    v[3] = p[3u - r.sy];
    v[4] = p[4u + r.sz];
    v[5] = p[5u - r.sz];
    v[6] = p[6];
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      nd[4 * i + 0] = v[i].x;
      nd[4 * i + 1] = v[i].y;
      nd[4 * i + 2] = v[i].z;
      nd[4 * i + 3] = v[i].w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < NF4; ++i) {
      float4 v = p[i];
      nd[4 * i + 0] = v.x;
      nd[4 * i + 1] = v.y;
      nd[4 * i + 2] = v.z;
      nd[4 * i + 3] = v.w;
    }
  }
  constexpr int SH = (W == 2) ? 1 : ((W == 4) ? 2 : 3);
  uint32_t key[W];
#pragma unroll
  for (int i = 0; i < W; ++i) {
    float lox = nd[0 * W + i], hix = nd[1 * W + i];
    float loy = nd[2 * W + i], hiy = nd[3 * W + i];
    float loz = nd[4 * W + i], hiz = nd[5 * W + i];
    float nx = PRE ? lox : (r.sx ? hix : lox), fx = PRE ? hix : (r.sx ? lox : hix);
    float ny = PRE ? loy : (r.sy ? hiy : loy), fy = PRE ? hiy : (r.sy ? loy : hiy);
    float nz = PRE ? loz : (r.sz ? hiz : loz), fz = PRE ? hiz : (r.sz ? loz : hiz);
    float tnx = (nx - r.ox) * r.ix, tfx = (fx - r.ox) * r.ix;
    float tny = (ny - r.oy) * r.iy, tfy = (fy - r.oy) * r.iy;
    float tnz = (nz - r.oz) * r.iz, tfz = (fz - r.oz) * r.iz;
    // fmaxf/fminf ignore a NaN operand (0 * inf on a slab boundary with a
    // zero direction component), which is the correct "no constraint".
    float tn = fmaxf(fmaxf(tnx, tny), fmaxf(tnz, r.tmin));
    float tf = fminf(fminf(tfx, tfy), tfz);
    // cull first, then widen: a far distance of -inf (a zero direction
    // component with the origin outside that slab) widens to NaN, which
    // fails the test below; widened first, the NaN would be dropped by the
    // NaN-ignoring fminf and the box kept
    tf = fminf(tf, tcull);
    tf = fmaf(fabsf(tf), kSlabWiden, tf);
    bool hit = (tn <= tf) & (tn < __int_as_float(0x7f800000));
    key[i] = hit ? ((__float_as_uint(tn) & ~((1u << SH) - 1u)) | (uint32_t)i) : 0xFFFFFFFFu;
  }
  // sort (key, child) pairs by key, nearest first; missed children (key
  // 0xFFFFFFFF) sort last.  Moving the child reference with its key costs two
  // selects per exchange and saves looking it up by slot afterwards.
  uint32_t ref[W];
#pragma unroll
  for (int i = 0; i < W; ++i) ref[i] = __float_as_uint(nd[6 * W + i]);
#define RT_CSWAP(a, b)                                  \
  {                                                     \
    bool s_ = key[b] < key[a];                          \
    uint32_t k0_ = s_ ? key[b] : key[a];                \
    uint32_t k1_ = s_ ? key[a] : key[b];                \
    uint32_t r0_ = s_ ? ref[b] : ref[a];                \
    uint32_t r1_ = s_ ? ref[a] : ref[b];                \
    key[a] = k0_;                                       \
    key[b] = k1_;                                       \
    ref[a] = r0_;                                       \
    ref[b] = r1_;                                       \
  }
  if constexpr (W == 2) {
    RT_CSWAP(0, 1);
  } else if constexpr (W == 4) {
    RT_CSWAP(0, 1); RT_CSWAP(2, 3); RT_CSWAP(0, 2); RT_CSWAP(1, 3); RT_CSWAP(1, 2);
  } else {
    // Batcher odd-even merge sort for 8 keys (19 compare-exchanges)
    RT_CSWAP(0, 1); RT_CSWAP(2, 3); RT_CSWAP(4, 5); RT_CSWAP(6, 7);
    RT_CSWAP(0, 2); RT_CSWAP(1, 3); RT_CSWAP(4, 6); RT_CSWAP(5, 7);
    RT_CSWAP(1, 2); RT_CSWAP(5, 6);
    RT_CSWAP(0, 4); RT_CSWAP(1, 5); RT_CSWAP(2, 6); RT_CSWAP(3, 7);
    RT_CSWAP(2, 4); RT_CSWAP(3, 5);
    RT_CSWAP(1, 2); RT_CSWAP(3, 4); RT_CSWAP(5, 6);
  }
#undef RT_CSWAP
  n_out = 0;
#pragma unroll
  for (int i = 0; i < W; ++i) {
    out_ref[i] = ref[i];
    n_out += (key[i] != 0xFFFFFFFFu) ? 1 : 0;
  }
}

// Watertight float32 ray/triangle test.  The record's vertices are sorted
// (p0 < p1 < p2 lexicographically), so each edge function
//   g(P,Q) = d . ((Q - P) x (P - o)),  P < Q,
// is computed from the same operands wherever the edge appears.  The edge
// functions of the triangle are F0 = -g(p1,p2), F1 = g(p0,p2), F2 = -g(p0,p1)
// (F_k is proportional to the weight of p_k); the ray crosses the closed
// triangle when they share a sign and their sum d.n is non-zero.  Then
// t = n.(p0 - o) / n.d with n = (p1 - p0) x (p2 - p0) (§3.1, plane solution).
// The denominator is n.d from the short edge vectors, not the sum of the
// edge functions: those are formed against the (possibly distant) origin and
// their sum carries a cancellation error of order u |e| |p - o| |d|, which for
// grazing rays from afar would reach 1e-4 of t.
__device__ __forceinline__ bool tri_test(const float4& A, const float4& B, const float4& C,
                                         const RayState& r, float& t_out) {
  float w0x = A.x - r.ox, w0y = A.y - r.oy, w0z = A.z - r.oz;
  float w1x = B.x - r.ox, w1y = B.y - r.oy, w1z = B.z - r.oz;
  float e01x = B.x - A.x, e01y = B.y - A.y, e01z = B.z - A.z;
  float e12x = C.x - B.x, e12y = C.y - B.y, e12z = C.z - B.z;
  float e02x = C.x - A.x, e02y = C.y - A.y, e02z = C.z - A.z;
  // c = e x w, g = d . c
  float g01 = r.dx * (e01y * w0z - e01z * w0y) + r.dy * (e01z * w0x - e01x * w0z) +
              r.dz * (e01x * w0y - e01y * w0x);
  float g12 = r.dx * (e12y * w1z - e12z * w1y) + r.dy * (e12z * w1x - e12x * w1z) +
              r.dz * (e12x * w1y - e12y * w1x);
  float g02 = r.dx * (e02y * w0z - e02z * w0y) + r.dy * (e02z * w0x - e02x * w0z) +
              r.dz * (e02x * w0y - e02y * w0x);
  float F0 = -g12, F1 = g02, F2 = -g01;
  bool pos = (F0 >= 0.0f) & (F1 >= 0.0f) & (F2 >= 0.0f);
  bool neg = (F0 <= 0.0f) & (F1 <= 0.0f) & (F2 <= 0.0f);
  float det = F0 + F1 + F2;
  if (!((pos | neg) & (det != 0.0f))) return false;
  float nx = e01y * e02z - e01z * e02y;
  float ny = e01z * e02x - e01x * e02z;
  float nz = e01x * e02y - e01y * e02x;
  float T = nx * w0x + ny * w0y + nz * w0z;
  float nd = nx * r.dx + ny * r.dy + nz * r.dz;
  if (nd == 0.0f) return false;
  t_out = T / nd;
  return true;
}

// float64 (t, u, v) of the triangle of record `rec` in its original vertex
// order (Moeller-Trumbore solution of o + t d = (1-u-v) v0 + u v1 + v v2);
// the record holds the float32 vertices sorted and the slot of each corner.
__device__ __forceinline__ bool finalize64(const float4* tris, uint32_t rec, double ox, double oy,
                                           double oz, double dx, double dy, double dz, float& t,
                                           float& u, float& v) {
  const float4* tp = tris + 3 * (size_t)rec;
  float4 P0 = tp[0], P1 = tp[1], P2 = tp[2];
  uint32_t order = __float_as_uint(P1.w);
  auto slot = [&](uint32_t k) -> float4 { return k == 0u ? P0 : (k == 1u ? P1 : P2); };
  float4 C0 = slot(order & 3u), C1 = slot((order >> 2) & 3u), C2 = slot((order >> 4) & 3u);
  double v0x = C0.x, v0y = C0.y, v0z = C0.z;
  double e1x = C1.x - v0x, e1y = C1.y - v0y, e1z = C1.z - v0z;
  double e2x = C2.x - v0x, e2y = C2.y - v0y, e2z = C2.z - v0z;
  double px = dy * e2z - dz * e2y, py = dz * e2x - dx * e2z, pz = dx * e2y - dy * e2x;
  double det = e1x * px + e1y * py + e1z * pz;
  if (det == 0.0) return false;
  double inv = 1.0 / det;
  double sx = ox - v0x, sy = oy - v0y, sz = oz - v0z;
  double uu = (sx * px + sy * py + sz * pz) * inv;
  double qx = sy * e1z - sz * e1y, qy = sz * e1x - sx * e1z, qz = sx * e1y - sy * e1x;
  double vv = (dx * qx + dy * qy + dz * qz) * inv;
  double tt = (e2x * qx + e2y * qy + e2z * qz) * inv;
  if (!(tt == tt) || !(uu == uu) || !(vv == vv)) return false;
  t = (float)tt;
  u = (float)uu;
  v = (float)vv;
  return true;
}

// world -> object ray with the float32 instance map (no renormalisation, so
// t is shared between the two spaces)
// (r holds the world ray on entry; tmin and tmax carry over unchanged)
__device__ __forceinline__ void to_object_od(const rt_inst_rec& I, float wox, float woy, float woz, float wdx,
                                             float wdy, float wdz, RayState& r) {
  r.ox = I.r0[0] * wox + I.r0[1] * woy + I.r0[2] * woz + I.r0[3];
  r.oy = I.r1[0] * wox + I.r1[1] * woy + I.r1[2] * woz + I.r1[3];
  r.oz = I.r2[0] * wox + I.r2[1] * woy + I.r2[2] * woz + I.r2[3];
  r.dx = I.r0[0] * wdx + I.r0[1] * wdy + I.r0[2] * wdz;
  r.dy = I.r1[0] * wdx + I.r1[1] * wdy + I.r1[2] * wdz;
  r.dz = I.r2[0] * wdx + I.r2[1] * wdy + I.r2[2] * wdz;
}

__device__ __forceinline__ void to_object(const rt_inst_rec& I, RayState& r) {
  to_object_od(I, r.ox, r.oy, r.oz, r.dx, r.dy, r.dz, r);
  ray_setup(r);
}

__device__ __forceinline__ void world_state(const rt_ray& w, RayState& r) {
  r.ox = w.ox; r.oy = w.oy; r.oz = w.oz;
  r.dx = w.dx; r.dy = w.dy; r.dz = w.dz;
  r.tmin = w.tmin; r.tmax = w.tmax;
  ray_setup(r);
}

__device__ __forceinline__ bool is_internal(uint32_t ref) { return (ref & RT_LEAF_BIT) == 0u; }
__device__ __forceinline__ bool is_inst(uint32_t ref) {
  return (ref & (RT_LEAF_BIT | RT_INST_BIT)) == (RT_LEAF_BIT | RT_INST_BIT) && ref != RT_CHILD_EMPTY;
}
__device__ __forceinline__ bool is_tri_leaf(uint32_t ref) {
  return (ref & (RT_LEAF_BIT | RT_INST_BIT)) == RT_LEAF_BIT;
}

// Inserts the hit (t, inst, prim) into a lane's list of the `cap` nearest
// hits, kept sorted by (t, inst, prim) in its output records (t, prim, inst
// bits, triangle record bits); `found` hits were seen before this one.
__device__ __forceinline__ void list_insert(float4* L, uint32_t found, uint32_t cap, float t,
                                            uint32_t inst, uint32_t prim, uint32_t rec) {
  uint32_t pos = min(found, cap);
  while (pos > 0) {
    float4 e = L[pos - 1];
    uint32_t ei = __float_as_uint(e.z), ep = __float_as_uint(e.y);
    bool greater = (e.x > t) || (e.x == t && (ei > inst || (ei == inst && ep > prim)));
    if (!greater) break;
    if (pos < cap) L[pos] = e;
    --pos;
  }
  if (pos < cap) L[pos] = make_float4(t, __uint_as_float(prim), __uint_as_float(inst), __uint_as_float(rec));
}

// ---------------------------------------------------------------------------
// the persistent traversal kernel
// ---------------------------------------------------------------------------
// MODE 0: one accel (uniform geometry); MODE 1: batched (geometry per lane
// from the batch descriptor of the lane's ray); MODE 2: one accel with the
// query options (ray masks against instance masks, a skipped triangle per
// ray); MODE 3: as MODE 2, enumerating all hits within [tmin, tmax] (no
// culling by the nearest hit) into per-ray lists of the `cap` nearest.
// Two-level kernels of width <= 4 are asked to fit six waves per SIMD (80
// VGPRs): on the 1,024-instance workload 4 -> 6 waves measured +12%, with no
// spills (8-wide nodes, the counting variants and the batched mode, which
// keeps per-lane geometry pointers, would spill, so they keep the compiler's
// choice).
// float64 finalize of ray `local`'s closest hit: the traversal left float32
// t, the winner's triangle record and (two-level) its instance in hits[local];
// (t, u, v) are recomputed in float64 from the record and the record's prim
// id replaces it.  Misses keep t = +inf and the invalid id.
template <bool INST>
__device__ __forceinline__ void finalize_ray(const rt_ray* rays, rt_hit* hits, const float4* tris,
                                             const rt_inst_rec64* insts64, uint32_t* inst_ids,
                                             uint32_t local) {
  float4* hp = reinterpret_cast<float4*>(hits + local);
  float4 h = *hp;
  uint32_t rec = __float_as_uint(h.y);
  if (rec == RT_INVALID_ID) {
    if (inst_ids) inst_ids[local] = RT_INVALID_ID;
    return;
  }
  uint32_t inst = __float_as_uint(h.z);
  rt_ray q = load_ray(rays, local);
  double ox = q.ox, oy = q.oy, oz = q.oz, dx = q.dx, dy = q.dy, dz = q.dz;
  if constexpr (INST) {
    const rt_inst_rec64& M = insts64[inst];
    double a = M.m[0] * ox + M.m[1] * oy + M.m[2] * oz + M.m[3];
    double b = M.m[4] * ox + M.m[5] * oy + M.m[6] * oz + M.m[7];
    double c = M.m[8] * ox + M.m[9] * oy + M.m[10] * oz + M.m[11];
    double e = M.m[0] * dx + M.m[1] * dy + M.m[2] * dz;
    double f = M.m[4] * dx + M.m[5] * dy + M.m[6] * dz;
    double gg = M.m[8] * dx + M.m[9] * dy + M.m[10] * dz;
    ox = a; oy = b; oz = c; dx = e; dy = f; dz = gg;
  }
  float t, u, v;
  float prim = tris[3 * (size_t)rec].w;
  if (finalize64(tris, rec, ox, oy, oz, dx, dy, dz, t, u, v)) {
    *hp = make_float4(t, prim, u, v);
  } else {
    *hp = make_float4(h.x, prim, 0.0f, 0.0f);
  }
  if (inst_ids) inst_ids[local] = INST ? inst : 0u;
}

// finalize of ray i of a launch: one accel (MODE 0), or the batch whose ray
// range holds i (MODE 1, offsets have batch_count + 1 entries)
template <bool INST, int MODE>
__device__ __forceinline__ void finalize_index(const TraceParams& P, uint32_t i) {
  const rt_ray* rays = P.rays;
  rt_hit* hits = P.hits;
  const float4* tris = reinterpret_cast<const float4*>(P.tris);
  const rt_inst_rec64* insts64 = P.insts64;
  uint32_t* inst_ids = P.inst_ids;
  uint32_t local = i;
  if constexpr (MODE == 1) {
    uint32_t lo = 0, hi = P.batch_count;
    while (hi - lo > 1) {
      uint32_t mid = (lo + hi) >> 1;
      if (P.batch_offsets[mid] <= i) lo = mid; else hi = mid;
    }
    const BatchDesc& bd = P.batches[lo];
    local = i - P.batch_offsets[lo];
    rays = bd.rays;
    hits = bd.hits;
    tris = reinterpret_cast<const float4*>(bd.tris);
    insts64 = bd.insts64;
    inst_ids = bd.inst_ids;
  }
  finalize_ray<INST>(rays, hits, tris, insts64, inst_ids, local);
}

template <int W, bool INST, bool COUNT, int MODE>
constexpr int trace_min_waves() { return (INST && W <= 4 && !COUNT && MODE != 1) ? 5 : 1; }
template <int W, int S, int WG, bool ANY, bool INST, int MODE, bool COUNT = false>
__global__ __launch_bounds__(WG, (trace_min_waves<W, INST, COUNT, MODE>())) void trace_kernel(TraceParams P) {
  __shared__ uint32_t lds_stack[S * WG];
  // two-level: the world ray's origin and direction, restored on leaving an
  // instance (kept out of registers)
  __shared__ float lds_world[INST ? 6 * WG : 1];
  const uint32_t tid = threadIdx.x;
  const uint32_t lane = tid & 63u;
  const uint32_t gtid = blockIdx.x * WG + tid;
  // closest queries on one accel finalize their own hits (see TraceParams)
  constexpr bool FUSED = !ANY && MODE == 0 && !COUNT;
  uint32_t* my_ranges = FUSED ? P.ranges + (size_t)(gtid >> 6) * (2 * kRtRangesPerWave) : nullptr;
  uint32_t n_ranges = 0;
  const uint64_t lanemask_lt = (lane == 0) ? 0ull : (~0ull >> (64u - lane));

  Geo g;
  g.nodes = P.nodes;
  g.tris = reinterpret_cast<const float4*>(P.tris);
  g.insts = P.insts;
  g.insts64 = P.insts64;
  g.meshes = P.meshes;
  g.root = P.root;
  g.max_stack = P.max_stack;

  Stack<S, WG, COUNT> st;
  st.lds = lds_stack + tid;
  st.glob = P.gstack + gtid;
  st.gstride = P.gstride;
  st.cap = P.max_stack;
  st.sp = 0;
  st.peak = 0;
  st.over = false;

  RayState r;
  uint32_t ray_id = 0;
  uint32_t cur = RT_CHILD_EMPTY;
  // postponed triangle leaves, oldest first: up to three for closest hits
  // and six for any-hit on one accel, two on two-level accels (the counts
  // measured fastest)
  constexpr int K = INST ? 2 : (ANY ? 6 : 3);
  uint32_t pq[K];
#pragma unroll
  for (int k = 0; k < K; ++k) pq[k] = RT_CHILD_EMPTY;
  float best_t = 0.0f;
  // the nearest hit so far: its triangle record (RT_INVALID_ID: none yet;
  // the prim id is read from the record where a tie needs it and by the
  // finalize) and instance
  uint32_t best_rec = RT_INVALID_ID, best_inst = RT_INVALID_ID, cur_inst = 0;
  // two-level: the instance of each postponed leaf, and whether the
  // traversal ray is in an instance's object space (cur_inst) or in world
  // space
  uint32_t pin[K];
  bool in_inst = false;
  rt_hit* hit_out = P.hits;
  uint8_t* occ_out = P.occluded;
  const rt_ray* ray_in = P.rays;
  bool live = false, retired = false;
  uint32_t batch = 0;
  uint32_t rmask = 0xFFFFFFFFu, skip_i = RT_INVALID_ID, skip_p = RT_INVALID_ID, found = 0;
  uint64_t n_nodes = 0, n_tris = 0, n_spill = 0;
  // counting variant, wave level: passes of the outer loop, refills, and
  // iterations of the node and the leaf loops (counted by the wave's first
  // active lane, so every wave iteration once)
  uint64_t w_outer = 0, w_refill = 0, w_node = 0, w_leaf = 0;
  auto first_active = [&]() -> bool {
    return lane == (uint32_t)(__ffsll((unsigned long long)__ballot(1)) - 1);
  };

  while (true) {
    if constexpr (COUNT) w_outer += lane == 0 ? 1u : 0u;
    // ---- refill finished lanes (one atomic per wave) --------------------
    bool need = !live && !retired;
    uint64_t m = __ballot(need);
    uint64_t mlive = __ballot(live);
    uint32_t n_need = __popcll(m);
    if (n_need > 0 && (mlive == 0 || n_need >= P.refill_min)) {
      if constexpr (COUNT) w_refill += lane == 0 ? 1u : 0u;
      uint32_t leader = __ffsll((unsigned long long)m) - 1;
      uint32_t base = 0;
      if (lane == leader) base = atomicAdd(P.counter, n_need);
      base = (uint32_t)__shfl((int)base, (int)leader);
      if constexpr (FUSED) {
        // remember the range [base, base + take) this wave now owns
        if (base < P.n) {
          uint32_t take = min(n_need, P.n - base);
          if (n_ranges < kRtRangesPerWave) {
            if (lane == 0) {
              my_ranges[2 * n_ranges] = base;
              my_ranges[2 * n_ranges + 1] = take;
            }
            ++n_ranges;
          } else if (lane == 0) {
            uint32_t k = atomicAdd(P.counter + 1, 1u);
            if (k < P.ovf_cap) {
              P.ovf[2 * k] = base;
              P.ovf[2 * k + 1] = take;
            }
          }
        }
      }
      if (need) {
        uint32_t my = base + __popcll(m & lanemask_lt);
        if (my < P.n) {
          ray_id = my;
          uint32_t local = my;
          if constexpr (MODE == 1) {
            // the batch whose ray range holds `my` (offsets has batch_count+1 entries)
            uint32_t lo = 0, hi = P.batch_count;
            while (hi - lo > 1) {
              uint32_t mid = (lo + hi) >> 1;
              if (P.batch_offsets[mid] <= my) lo = mid; else hi = mid;
            }
            batch = lo;
            const BatchDesc& bd = P.batches[lo];
            local = my - P.batch_offsets[lo];
            g.nodes = bd.nodes;
            g.tris = reinterpret_cast<const float4*>(bd.tris);
            g.meshes = bd.meshes;
            g.root = bd.root;
            if constexpr (INST) {
              g.insts = bd.insts;
              g.insts64 = bd.insts64;
            }
            ray_in = bd.rays;
            hit_out = bd.hits;
          }
          rt_ray wray = load_ray(ray_in, local);
          ray_id = local;
          world_state(wray, r);
          if constexpr (INST) {
            lds_world[0 * WG + tid] = wray.ox;
            lds_world[1 * WG + tid] = wray.oy;
            lds_world[2 * WG + tid] = wray.oz;
            lds_world[3 * WG + tid] = wray.dx;
            lds_world[4 * WG + tid] = wray.dy;
            lds_world[5 * WG + tid] = wray.dz;
          }
          best_t = r.tmax;
          best_rec = RT_INVALID_ID;
          best_inst = RT_INVALID_ID;
          cur_inst = 0;
          in_inst = false;
          st.sp = 0;
#pragma unroll
          for (int k = 0; k < K; ++k) pq[k] = RT_CHILD_EMPTY;
          cur = ray_void(wray) ? RT_CHILD_EMPTY : g.root;
          if constexpr (MODE >= 2) {
            rmask = P.ray_masks ? P.ray_masks[local] : 0xFFFFFFFFu;
            skip_p = P.skip_prim ? P.skip_prim[local] : RT_INVALID_ID;
            skip_i = P.skip_inst ? P.skip_inst[local] : RT_INVALID_ID;
            found = 0;
            // a single-level accel is one geometry of mask 0xFFFFFFFF
            if (!INST && rmask == 0u) cur = RT_CHILD_EMPTY;
          }
          live = true;
        } else {
          retired = true;
        }
      }
    }
    if (__ballot(live) == 0) {
      if (__ballot(!retired) == 0) break;
      continue;
    }
    if (live) {
      float tcull = fmaf(fabsf(best_t), kTieWiden, best_t);
      uint32_t linst = cur_inst;   // instance of the leaf under test
      // sets r's origin and direction to those of the world ray in instance
      // j's object space (the reciprocals stay those of the traversal frame)
      auto frame_od = [&](bool inside, uint32_t j) {
        const float wox = lds_world[0 * WG + tid], woy = lds_world[1 * WG + tid], woz = lds_world[2 * WG + tid];
        const float wdx = lds_world[3 * WG + tid], wdy = lds_world[4 * WG + tid], wdz = lds_world[5 * WG + tid];
        if (inside) {
          to_object_od(g.insts[j], wox, woy, woz, wdx, wdy, wdz, r);
        } else {
          r.ox = wox; r.oy = woy; r.oz = woz;
          r.dx = wdx; r.dy = wdy; r.dz = wdz;
        }
      };
      // Tests the triangles of one leaf; true when an any-hit query may stop.
      // Tests triangle record `rec`; true when an any-hit query may stop.
      auto test_tri = [&](uint32_t rec) -> bool {
        const float4* tp = g.tris + 3 * (size_t)rec;
        if constexpr (COUNT) n_tris++;
        float4 A = tp[0], B = tp[1], C = tp[2];
        float t;
        if (tri_test(A, B, C, r, t) && t >= r.tmin && t <= best_t) {
          uint32_t prim = __float_as_uint(A.w);
          if constexpr (MODE >= 2) {
            if (prim == skip_p && (!INST || linst == skip_i)) return false;
          }
          if constexpr (MODE == 3) {
            list_insert(reinterpret_cast<float4*>(hit_out) + (size_t)ray_id * P.cap, found, P.cap, t,
                        INST ? linst : 0u, prim, rec);
            ++found;
            return false;
          }
          if constexpr (ANY) {
            best_rec = rec;
            return true;
          } else {
            // lexicographic (t, inst, prim); t <= best_t here
            uint32_t inst = INST ? linst : 0u;
            bool better = (t < best_t) || (inst < best_inst);
            if (!better && inst == best_inst)
              better = prim < __float_as_uint(g.tris[3 * (size_t)best_rec].w);
            if (better) {
              best_t = t;
              best_inst = inst;
              best_rec = rec;
            }
          }
        }
        return false;
      };
      // Visits internal node `cur`: continues with the nearest child hit and
      // pushes the others, farthest first.
      auto step_node = [&]() {
        uint32_t refs[W];
        int nh;
        if constexpr (COUNT) n_nodes++;
        visit_node<W, ANY && !INST>(g.nodes, cur, r, tcull, refs, nh);
        if (nh == 0) {
          cur = st.pop();
        } else {
          cur = refs[0];
#pragma unroll
          for (int i = W - 1; i >= 1; --i)
            if (i < nh) {
              if constexpr (COUNT) n_spill += (st.sp >= S) ? 1 : 0;
              st.push(refs[i]);
            }
        }
      };
      // ---- internal nodes, leaves postponed ---------------------------------
      // A lane that reaches a leaf sets it aside and keeps traversing until
      // it holds K leaves and meets another, or every lane of the wave holds
      // a leaf, so that the wave enters the triangle loop together (leaf
      // postponing, Aila & Laine 2009, with more than one leaf a lane: the
      // node loop then runs with more lanes busy, the triangle loop with more
      // triangles a lane).  A postponed leaf remembers its instance, and the
      // triangle loop takes the world ray into that instance's object space
      // to test it (the float32 map of the instance entry, applied to the
      // same world ray, so the object ray is the same), so a lane holding one
      // keeps traversing across instance boundaries.
      while (cur != RT_CHILD_EMPTY) {
        if constexpr (COUNT) w_node += first_active() ? 1u : 0u;
        if constexpr (INST) {
          if (cur == RT_STACK_MARKER || is_inst(cur)) {
            if (cur == RT_STACK_MARKER) {
              r.ox = lds_world[0 * WG + tid];
              r.oy = lds_world[1 * WG + tid];
              r.oz = lds_world[2 * WG + tid];
              r.dx = lds_world[3 * WG + tid];
              r.dy = lds_world[4 * WG + tid];
              r.dz = lds_world[5 * WG + tid];
              ray_setup(r);
              in_inst = false;
              r.tmax = best_t;
              cur = st.pop();
            } else {
              uint32_t j = cur & RT_INST_INDEX_MASK;
              const rt_inst_rec& I = g.insts[j];
              bool skip = I.root == RT_CHILD_EMPTY;
              if constexpr (MODE >= 2) skip = skip || (I.mask & rmask) == 0u;
              if (skip) {
                cur = st.pop();
              } else {
                to_object(I, r);
                r.tmax = best_t;
                cur_inst = j;
                in_inst = true;
                st.push(RT_STACK_MARKER);
                cur = I.root;
              }
            }
            // a node or a leaf after the frame change is taken in the same
            // iteration; another frame change or the end waits for the next
            if (cur == RT_CHILD_EMPTY || cur == RT_STACK_MARKER || is_inst(cur)) continue;
          }
        }
        auto postpone = [&]() {
          bool placed = false;
#pragma unroll
          for (int k = 0; k < K; ++k)
            if (!placed && pq[k] == RT_CHILD_EMPTY) {
              pq[k] = cur;
              if constexpr (INST) pin[k] = cur_inst;
              placed = true;
            }
          cur = st.pop();
        };
        if constexpr (INST || (!ANY && MODE != 1)) {
          // an internal node under a postponed leaf is visited in the same
          // iteration, so that a lane's iterations are node visits (batched
          // single-level plans: -2% with it)
          bool visit = true;
          if (is_tri_leaf(cur)) {
            if (pq[K - 1] != RT_CHILD_EMPTY) break;
            postpone();
            visit = is_internal(cur);
          }
          if (visit) step_node();
        } else {
          // (single-level any-hit: the same fall-through measured -0.6% on
          // incoherent and +1.2% on shadow rays; the simpler loop stays)
          if (is_tri_leaf(cur)) {
            if (pq[K - 1] != RT_CHILD_EMPTY) break;
            postpone();
          } else {
            step_node();
          }
        }
        if (__ballot(pq[0] == RT_CHILD_EMPTY) == 0) break;
      }
      // ---- triangle leaves: the postponed ones, then those on the stack top -
      // One triangle per iteration: a lane whose leaf is done moves on to
      // its next leaf while others finish longer leaves (leaves hold 1-15
      // triangles), instead of waiting for the longest leaf of the wave.
      // The nearest-hit cull distance is updated after each leaf, as before.
      // r's origin and direction are in frame rf (RT_INVALID_ID: world)
      const uint32_t home = in_inst ? cur_inst : RT_INVALID_ID;
      uint32_t rf = home;
      auto take_postponed = [&](uint32_t& first, uint32_t& count) {
        first = pq[0] & RT_LEAF_FIRST_MASK;
        count = pq[0] != RT_CHILD_EMPTY ? (pq[0] >> RT_LEAF_COUNT_SHIFT) & RT_LEAF_COUNT_MASK : 0u;
        if constexpr (INST) {
          if (pq[0] != RT_CHILD_EMPTY) {
            linst = pin[0];
            if (rf != pin[0]) {
              frame_od(true, pin[0]);
              rf = pin[0];
            }
          }
#pragma unroll
          for (int k = 0; k + 1 < K; ++k) pin[k] = pin[k + 1];
        }
#pragma unroll
        for (int k = 0; k + 1 < K; ++k) pq[k] = pq[k + 1];
        pq[K - 1] = RT_CHILD_EMPTY;
      };
      uint32_t tnext, tleft;
      take_postponed(tnext, tleft);
      while (tleft > 0) {
        if constexpr (COUNT) w_leaf += first_active() ? 1u : 0u;
        bool stop = test_tri(tnext);
        ++tnext;
        --tleft;
        if (ANY && stop) {
          cur = RT_CHILD_EMPTY;
#pragma unroll
          for (int k = 0; k < K; ++k) pq[k] = RT_CHILD_EMPTY;
          st.sp = 0;
          break;
        }
        if (tleft == 0) {
          tcull = fmaf(fabsf(best_t), kTieWiden, best_t);
          if (pq[0] != RT_CHILD_EMPTY) {
            take_postponed(tnext, tleft);
          } else if (cur != RT_CHILD_EMPTY && is_tri_leaf(cur)) {
            if constexpr (INST) {
              // the leaves on the stack top are in the traversal frame
              if (rf != home) {
                frame_od(in_inst, cur_inst);
                rf = home;
              }
              linst = cur_inst;
            }
            tnext = cur & RT_LEAF_FIRST_MASK;
            tleft = (cur >> RT_LEAF_COUNT_SHIFT) & RT_LEAF_COUNT_MASK;
            cur = st.pop();
          }
        }
      }
      if constexpr (INST) {
        if (rf != home) frame_od(in_inst, cur_inst);   // back to the traversal frame
      }
      // ---- finished: write the result --------------------------------------
      // (the float64 (t, u, v) and the prim id of a closest hit are written
      // by the finalize: for one-accel closest queries (MODE 0) by this wave
      // once all rays of its ranges are done, below, and by
      // finalize_ovf_kernel for ranges past its list; for batched, masked
      // and counting launches by finalize_kernel, one thread per ray.  Here:
      // float32 t, the triangle record in the prim slot and the instance in
      // the u slot)
      if (cur == RT_CHILD_EMPTY && pq[0] == RT_CHILD_EMPTY) {
        if constexpr (MODE == 3) {
          P.counts[ray_id] = found;
        } else if constexpr (ANY) {
          occ_out[ray_id] = (best_rec != RT_INVALID_ID) ? 1 : 0;
        } else {
          bool hit = best_rec != RT_INVALID_ID;
          float4* hp = reinterpret_cast<float4*>(hit_out + ray_id);
          *hp = make_float4(hit ? best_t : __int_as_float(0x7f800000), __uint_as_float(best_rec),
                            __uint_as_float(hit ? (INST ? best_inst : 0u) : 0u), 0.0f);
        }
        live = false;
      }
    }
  }
  if constexpr (COUNT) {
    if (st.over) __hip_atomic_store(P.status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  if constexpr (FUSED) {
    // every ray this wave took is finished: float64 finalize of its listed
    // ranges with full waves, while other waves still trace (the wave's own
    // hit stores precede these loads)
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    for (uint32_t k = 0; k < n_ranges; ++k) {
      uint32_t b = my_ranges[2 * k], c = my_ranges[2 * k + 1];
      for (uint32_t o = 0; o < c; o += 64) {
        if (o + lane < c)
          finalize_index<INST, MODE>(P, b + o + lane);
      }
    }
  }
  if constexpr (COUNT) {
    atomicAdd(reinterpret_cast<unsigned long long*>(P.counters) + 0, (unsigned long long)n_nodes);
    atomicAdd(reinterpret_cast<unsigned long long*>(P.counters) + 1, (unsigned long long)n_tris);
    atomicAdd(reinterpret_cast<unsigned long long*>(P.counters) + 2, (unsigned long long)n_spill);
    atomicMax(reinterpret_cast<unsigned long long*>(P.counters) + 3, (unsigned long long)st.peak);
    if (P.phase_counters) {
      uint64_t w[4] = {w_outer, w_refill, w_node, w_leaf};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        for (int d = 32; d >= 1; d >>= 1) w[k] += __shfl_xor(w[k], d);
        if (lane == 0) atomicAdd(reinterpret_cast<unsigned long long*>(P.counters) + 4 + k, (unsigned long long)w[k]);
      }
    }
  }
  (void)batch;
}

// ---------------------------------------------------------------------------
// adjoint of the closest hit at fixed triangles (one ray per thread)
// ---------------------------------------------------------------------------
// The hit solves o + t d = (1-u-v) v0 + u v1 + v v2, i.e. M (t,u,v)^T = o - v0
// with M = [-d | v1-v0 | v2-v0].  For L with dL/d(t,u,v) = g the implicit
// function theorem gives lambda = M^-T g and dL/do = lambda, dL/dd = t lambda,
// dL/dv_k = -w_k lambda with w = (1-u-v, u, v).
struct Adjoint64 {
  double t, u, v;
  double lx, ly, lz;     // lambda
  double p[3][3];        // the triangle's vertices (float32 promoted)
  uint32_t id[3];        // their indices
};

// the solve from the triangle's vertices pv (float32, vertex-major)
__device__ __forceinline__ bool adjoint64_solve(const float* pv, double ox, double oy, double oz, double dx,
                                                double dy, double dz, double gt, double gu, double gv,
                                                Adjoint64& A) {
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) A.p[k][c] = pv[3 * k + c];
  double v0x = A.p[0][0], v0y = A.p[0][1], v0z = A.p[0][2];
  double e1x = A.p[1][0] - v0x, e1y = A.p[1][1] - v0y, e1z = A.p[1][2] - v0z;
  double e2x = A.p[2][0] - v0x, e2y = A.p[2][1] - v0y, e2z = A.p[2][2] - v0z;
  // rows of M^-1 are (e1 x e2, e2 x c0, c0 x e1) / det with c0 = -d
  double c0x = -dx, c0y = -dy, c0z = -dz;
  double r0x = e1y * e2z - e1z * e2y, r0y = e1z * e2x - e1x * e2z, r0z = e1x * e2y - e1y * e2x;
  double r1x = e2y * c0z - e2z * c0y, r1y = e2z * c0x - e2x * c0z, r1z = e2x * c0y - e2y * c0x;
  double r2x = c0y * e1z - c0z * e1y, r2y = c0z * e1x - c0x * e1z, r2z = c0x * e1y - c0y * e1x;
  double det = c0x * r0x + c0y * r0y + c0z * r0z;
  if (det == 0.0) return false;
  double inv = 1.0 / det;
  double sx = ox - v0x, sy = oy - v0y, sz = oz - v0z;
  A.t = (r0x * sx + r0y * sy + r0z * sz) * inv;
  A.u = (r1x * sx + r1y * sy + r1z * sz) * inv;
  A.v = (r2x * sx + r2y * sy + r2z * sz) * inv;
  // lambda = M^-T g = sum_i g_i row_i(M^-1)
  A.lx = (gt * r0x + gu * r1x + gv * r2x) * inv;
  A.ly = (gt * r0y + gu * r1y + gv * r2y) * inv;
  A.lz = (gt * r0z + gu * r1z + gv * r2z) * inv;
  return true;
}

__device__ __forceinline__ bool adjoint64(const rt_mesh_dev& mesh, uint32_t prim, double ox,
                                          double oy, double oz, double dx, double dy, double dz,
                                          double gt, double gu, double gv, Adjoint64& A) {
  const uint32_t* ix = mesh.indices + 3 * (size_t)prim;
  const float* V = mesh.vertices;
  float pv[9];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    A.id[k] = ix[k];
#pragma unroll
    for (int c = 0; c < 3; ++c) pv[3 * k + c] = V[3 * (size_t)A.id[k] + c];
  }
  return adjoint64_solve(pv, ox, oy, oz, dx, dy, dz, gt, gu, gv, A);
}

__device__ __forceinline__ void zero3(float* a) { a[0] = a[1] = a[2] = 0.0f; }

// Bucket starts of one tile: an exclusive scan of the bucket totals over
// the workgroup (1024 threads, at most 16 buckets per thread) plus the
// tile's offsets, into pos[]; workgroup 0 also stores the starts for the
// summing kernels.  The caller synchronises before reading pos.
__device__ __forceinline__ void bucket_starts(const rta::Bucketing& B, uint32_t* pos) {
  __shared__ uint32_t wsum[16];
  constexpr uint32_t C = rta::kMaxBuckets / 1024;
  const uint32_t chunk = (B.buckets + 1023u) / 1024u;
  const uint32_t c0 = min(B.buckets, threadIdx.x * chunk), c1 = min(B.buckets, c0 + chunk);
  const uint32_t* tile_off = B.counts + (size_t)blockIdx.x * B.buckets;
  uint32_t tot[C], off[C];
  uint32_t own = 0;
#pragma unroll
  for (uint32_t k = 0; k < C; ++k) {
    const bool in = c0 + k < c1;
    tot[k] = in ? B.totals[c0 + k] : 0u;
    off[k] = in ? tile_off[c0 + k] : 0u;
    own += tot[k];
  }
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  uint32_t inc = own;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t o = (uint32_t)__shfl_up((int)inc, d);
    if (lane >= (uint32_t)d) inc += o;
  }
  if (lane == 63u) wsum[w] = inc;
  __syncthreads();
  uint32_t r = inc - own;
  for (uint32_t k = 0; k < w; ++k) r += wsum[k];
#pragma unroll
  for (uint32_t k = 0; k < C; ++k)
    if (c0 + k < c1) {
      pos[c0 + k] = r + off[k];
      if (blockIdx.x == 0) B.base[c0 + k] = r;
      r += tot[k];
    }
  if (blockIdx.x == 0 && threadIdx.x == 1023u) B.base[B.buckets] = r;
  __syncthreads();   // wsum is reused by a second call
}

// Record stores: three 16-byte stores each (record buffers are 256-byte
// aligned, records 48 bytes).
__device__ __forceinline__ float2 dwords(double x) {
  return make_float2(__int_as_float(__double2loint(x)), __int_as_float(__double2hiint(x)));
}

__device__ __forceinline__ void store_rayrec(rta::RayRec* dst, double lx, double ly, double lz, double u, double v,
                                             uint32_t prim) {
  float4* p = reinterpret_cast<float4*>(dst);
  float2 a = dwords(lx), b = dwords(ly), c = dwords(lz), d = dwords(u), e = dwords(v);
  p[0] = make_float4(a.x, a.y, b.x, b.y);
  p[1] = make_float4(c.x, c.y, d.x, d.y);
  p[2] = make_float4(e.x, e.y, __uint_as_float(prim), 0.0f);
}

__device__ __forceinline__ void store_framerec(rta::RayRec* dst, double lx, double ly, double lz, double px,
                                               double py, double pz) {
  float4* p = reinterpret_cast<float4*>(dst);
  float2 a = dwords(lx), b = dwords(ly), c = dwords(lz), d = dwords(px), e = dwords(py), f = dwords(pz);
  p[0] = make_float4(a.x, a.y, b.x, b.y);
  p[1] = make_float4(c.x, c.y, d.x, d.y);
  p[2] = make_float4(e.x, e.y, f.x, f.y);
}

// dL/do and dL/dd of the rays of one tile, and each hit ray's record
// (lambda, u, v, triangle) placed in its triangle's bucket (LDS counters
// start at the tile's offsets; see accumulate.h).  A hit whose adjoint is
// undefined (a singular M) still takes its slot, with a zero record.  Every
// thread handles kTile / 1024 rays, two at a time with all of their loads
// issued before either solve (the chain hit -> triangle vertices is what
// the kernel waits on).
__global__ __launch_bounds__(1024) void backward_kernel(BackwardParams P) {
  extern __shared__ uint32_t pos[];
  constexpr uint32_t R = rta::kTile / 1024, G = 2;
  static_assert(R % G == 0, "rays per thread");
  const rta::Bucketing& B = P.bk;
  const uint32_t base = blockIdx.x * rta::kTile;
  const uint32_t tc = P.mesh.triangle_count;
  uint32_t prim[R];
#pragma unroll
  for (uint32_t r = 0; r < R; ++r) {
    uint32_t i = base + r * 1024 + threadIdx.x;
    prim[r] = i < P.n ? P.hits[i].prim_id : RT_INVALID_ID;
  }
  bucket_starts(B, pos);
  __syncthreads();
#pragma unroll
  for (uint32_t r0 = 0; r0 < R; r0 += G) {
    float4 ra[G], rb[G];
    float gr[G][3], pv[G][9];
#pragma unroll
    for (uint32_t g = 0; g < G; ++g) {
      uint32_t i = base + (r0 + g) * 1024 + threadIdx.x;
      if (prim[r0 + g] < tc) {
        const float4* rp = reinterpret_cast<const float4*>(P.rays + i);
        ra[g] = rp[0];
        rb[g] = rp[1];
        const float* q = P.d_tuv + 3 * (size_t)i;
        gr[g][0] = q[0];
        gr[g][1] = q[1];
        gr[g][2] = q[2];
        const float* tv = P.tri_vertices + 9 * (size_t)prim[r0 + g];
#pragma unroll
        for (int k = 0; k < 9; ++k) pv[g][k] = tv[k];
      }
    }
#pragma unroll
    for (uint32_t g = 0; g < G; ++g) {
      uint32_t i = base + (r0 + g) * 1024 + threadIdx.x;
      if (i >= P.n) continue;
      const uint32_t pr = prim[r0 + g];
      float* go = P.d_origins + 3 * (size_t)i;
      float* gd = P.d_directions + 3 * (size_t)i;
      Adjoint64 A;
      const bool valid = pr < tc;
      bool ok = false;
      if (valid)
        ok = adjoint64_solve(pv[g], ra[g].x, ra[g].y, ra[g].z, rb[g].x, rb[g].y, rb[g].z, gr[g][0], gr[g][1],
                             gr[g][2], A);
      if (ok) {
        go[0] = (float)A.lx; go[1] = (float)A.ly; go[2] = (float)A.lz;
        gd[0] = (float)(A.t * A.lx); gd[1] = (float)(A.t * A.ly); gd[2] = (float)(A.t * A.lz);
      } else {
        zero3(go);
        zero3(gd);
      }
      if (valid) {
        uint32_t p = atomicAdd(&pos[pr >> B.shift], 1u);
        store_rayrec(B.rec + p, ok ? A.lx : 0.0, ok ? A.ly : 0.0, ok ? A.lz : 0.0, ok ? A.u : 0.0, ok ? A.v : 0.0,
                     pr);
      }
    }
  }
}

// Two-level hits (§6.2: the hit on an instance is the hit of the object-space
// ray x = A^-1 (w - T)).  t, u and v are invariant under the affine frame, so
// the object-space solve gives them and lambda_o; the world-space adjoint is
// lambda_w = A^-T lambda_o (A^-1 is the float64 map the finalize uses), the
// object vertices take -w_k lambda_o directly.  For the frame world = T +
// R(qh) (S x), qh = q/|q|, with the object hit point p and a = S p:
//   dL/dT = -lambda_w,   dL/dS_j = -(R^T lambda_w)_j p_j,
//   dL/dqh (through R a = a + 2 w (v x a) + 2 v x (v x a), qh = (v, w)):
//     w-part  -2 lambda.(v x a),
//     v-part  -2 [w (a x lambda) + (v x a) x lambda + a x (lambda x v)],
//   dL/dq = (dL/dqh - qh (qh . dL/dqh)) / |q|.
__device__ __forceinline__ void cross3(double ax, double ay, double az, double bx, double by,
                                       double bz, double& cx, double& cy, double& cz) {
  cx = ay * bz - az * by;
  cy = az * bx - ax * bz;
  cz = ax * by - ay * bx;
}

template <int PHASE>
__global__ __launch_bounds__(256) void backward_inst_kernel(BackwardInstParams P) {
  uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= P.n) return;
  const float4* hp = reinterpret_cast<const float4*>(P.hits + i);
  uint32_t prim = __float_as_uint(hp->y);
  uint32_t inst = P.inst_ids[i];
  float* go = P.d_origins + 3 * (size_t)i;
  float* gd = P.d_directions + 3 * (size_t)i;
  auto no_contribution = [&]() {
    if constexpr (PHASE == 0) {
      zero3(go);
      zero3(gd);
    }
  };
  if (prim == RT_INVALID_ID || inst >= P.inst_count) {
    no_contribution();
    return;
  }
  uint32_t mesh = P.insts[inst].mesh;
  const rt_mesh_dev& md = P.meshes[mesh];
  const rt_inst_rec64& M = P.insts64[inst];
  rt_ray q = load_ray(P.rays, i);
  double ox = q.ox, oy = q.oy, oz = q.oz, dx = q.dx, dy = q.dy, dz = q.dz;
  double xo = M.m[0] * ox + M.m[1] * oy + M.m[2] * oz + M.m[3];
  double yo = M.m[4] * ox + M.m[5] * oy + M.m[6] * oz + M.m[7];
  double zo = M.m[8] * ox + M.m[9] * oy + M.m[10] * oz + M.m[11];
  double xd = M.m[0] * dx + M.m[1] * dy + M.m[2] * dz;
  double yd = M.m[4] * dx + M.m[5] * dy + M.m[6] * dz;
  double zd = M.m[8] * dx + M.m[9] * dy + M.m[10] * dz;
  const float* gr = P.d_tuv + 3 * (size_t)i;
  Adjoint64 A;
  if (prim >= md.triangle_count ||
      !adjoint64(md, prim, xo, yo, zo, xd, yd, zd, gr[0], gr[1], gr[2], A)) {
    no_contribution();
    return;
  }
  // lambda_w = (A^-1)^T lambda_o
  double lx = M.m[0] * A.lx + M.m[4] * A.ly + M.m[8] * A.lz;
  double ly = M.m[1] * A.lx + M.m[5] * A.ly + M.m[9] * A.lz;
  double lz = M.m[2] * A.lx + M.m[6] * A.ly + M.m[10] * A.lz;
  if constexpr (PHASE == 0) {
    go[0] = (float)lx; go[1] = (float)ly; go[2] = (float)lz;
    gd[0] = (float)(A.t * lx); gd[1] = (float)(A.t * ly); gd[2] = (float)(A.t * lz);
  }
  double w[3] = {1.0 - A.u - A.v, A.u, A.v};
  if (P.want_vertices) {
    uint32_t base = (uint32_t)P.vertex_base[mesh];
#pragma unroll
    for (int k = 0; k < 3; ++k)
      rta::add<PHASE>(P.acc, base + A.id[k], -w[k] * A.lx, -w[k] * A.ly, -w[k] * A.lz);
  }
  if (!P.want_frames) return;
  const rt_srt f = P.srts[inst];
  double qx = f.qx, qy = f.qy, qz = f.qz, qw = f.qw;
  double qn = sqrt(qx * qx + qy * qy + qz * qz + qw * qw);
  double iq = 1.0 / qn;
  qx *= iq; qy *= iq; qz *= iq; qw *= iq;
  // object hit point and a = S p
  double px = w[0] * A.p[0][0] + w[1] * A.p[1][0] + w[2] * A.p[2][0];
  double py = w[0] * A.p[0][1] + w[1] * A.p[1][1] + w[2] * A.p[2][1];
  double pz = w[0] * A.p[0][2] + w[1] * A.p[1][2] + w[2] * A.p[2][2];
  double ax = f.sx * px, ay = f.sy * py, az = f.sz * pz;
  // R^T lambda = lambda - 2 w (v x lambda) + 2 v x (v x lambda)
  double cx, cy, cz, ex, ey, ez;
  cross3(qx, qy, qz, lx, ly, lz, cx, cy, cz);
  cross3(qx, qy, qz, cx, cy, cz, ex, ey, ez);
  double rlx = lx - 2.0 * qw * cx + 2.0 * ex;
  double rly = ly - 2.0 * qw * cy + 2.0 * ey;
  double rlz = lz - 2.0 * qw * cz + 2.0 * ez;
  // quaternion part
  double vax, vay, vaz;           // v x a
  cross3(qx, qy, qz, ax, ay, az, vax, vay, vaz);
  double gqw = -2.0 * (lx * vax + ly * vay + lz * vaz);
  double t1x, t1y, t1z, t2x, t2y, t2z, lvx, lvy, lvz, t3x, t3y, t3z;
  cross3(ax, ay, az, lx, ly, lz, t1x, t1y, t1z);        // a x lambda
  cross3(vax, vay, vaz, lx, ly, lz, t2x, t2y, t2z);     // (v x a) x lambda
  cross3(lx, ly, lz, qx, qy, qz, lvx, lvy, lvz);        // lambda x v
  cross3(ax, ay, az, lvx, lvy, lvz, t3x, t3y, t3z);     // a x (lambda x v)
  double gqx = -2.0 * (qw * t1x + t2x + t3x);
  double gqy = -2.0 * (qw * t1y + t2y + t3y);
  double gqz = -2.0 * (qw * t1z + t2z + t3z);
  double radial = qx * gqx + qy * gqy + qz * gqz + qw * gqw;
  uint32_t row = P.frame_row0 + 4u * inst;
  rta::add<PHASE>(P.acc, row + 0, -rlx * px, -rly * py, -rlz * pz);
  rta::add<PHASE>(P.acc, row + 1, (gqx - qx * radial) * iq, (gqy - qy * radial) * iq,
                  (gqz - qz * radial) * iq);
  rta::add<PHASE>(P.acc, row + 2, (gqw - qw * radial) * iq, -lx, -ly);
  rta::add<PHASE>(P.acc, row + 3, -lz, 0.0, 0.0);
}

// Two-level adjoint of one tile without global atomics: dL/do and dL/dd of
// its rays, and each hit ray's records placed in their buckets through LDS
// counters: (lambda_o, u, v, global triangle) by triangle range for the
// vertex sums, (lambda_w, object hit point) by instance for the frame sums
// (see accumulate.h).  A hit whose adjoint is undefined keeps its slots with
// zero records.  Validity is rta::ray_key's: an instance below the count and
// a triangle of its mesh.
__global__ __launch_bounds__(1024) void backward_inst_tile_kernel(BackwardInstParams P) {
  extern __shared__ uint32_t lds_pos[];
  constexpr uint32_t R = rta::kTile / 1024;
  uint32_t* vpos = lds_pos;
  uint32_t* fpos = lds_pos + (P.want_vertices ? P.vb.buckets : 0u);
  const uint32_t base = blockIdx.x * rta::kTile;
  // every ray's hit and instance, and the instance's triangle range, before
  // the bucket scans
  uint32_t prim[R], inst[R];
#pragma unroll
  for (uint32_t r = 0; r < R; ++r) {
    const uint32_t i = base + r * 1024 + threadIdx.x;
    prim[r] = i < P.n ? P.hits[i].prim_id : RT_INVALID_ID;
    inst[r] = i < P.n ? P.inst_ids[i] : RT_INVALID_ID;
  }
  uint32_t gt[R];
#pragma unroll
  for (uint32_t r = 0; r < R; ++r) {
    gt[r] = RT_INVALID_ID;
    if (inst[r] < P.inst_count) {
      const uint2 it = P.inst_tris[inst[r]];
      if (prim[r] < it.y) gt[r] = it.x + prim[r];
    }
  }
  if (P.want_vertices) bucket_starts(P.vb, vpos);
  if (P.want_frames) bucket_starts(P.fb, fpos);
  __syncthreads();
#pragma unroll 1
  for (uint32_t r = 0; r < R; ++r) {
    const uint32_t i = base + r * 1024 + threadIdx.x;
    if (i >= P.n) break;
    float* go = P.d_origins + 3 * (size_t)i;
    float* gd = P.d_directions + 3 * (size_t)i;
    const bool valid = gt[r] != RT_INVALID_ID;
    bool ok = false;
    Adjoint64 A;
    double lx = 0.0, ly = 0.0, lz = 0.0;
    if (valid) {
      // independent loads: the ray, its gradient, the frame, the triangle
      const rt_inst_rec64& M = P.insts64[inst[r]];
      rt_ray q = load_ray(P.rays, i);
      const float* gr = P.d_tuv + 3 * (size_t)i;
      const float* tv = P.tri_vertices + 9 * (size_t)gt[r];
      float pv[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) pv[k] = tv[k];
      double m[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) m[k] = M.m[k];
      const double g0 = gr[0], g1 = gr[1], g2 = gr[2];
      double ox = q.ox, oy = q.oy, oz = q.oz, dx = q.dx, dy = q.dy, dz = q.dz;
      double xo = m[0] * ox + m[1] * oy + m[2] * oz + m[3];
      double yo = m[4] * ox + m[5] * oy + m[6] * oz + m[7];
      double zo = m[8] * ox + m[9] * oy + m[10] * oz + m[11];
      double xd = m[0] * dx + m[1] * dy + m[2] * dz;
      double yd = m[4] * dx + m[5] * dy + m[6] * dz;
      double zd = m[8] * dx + m[9] * dy + m[10] * dz;
      ok = adjoint64_solve(pv, xo, yo, zo, xd, yd, zd, g0, g1, g2, A);
      if (ok) {
        // lambda_w = (A^-1)^T lambda_o
        lx = m[0] * A.lx + m[4] * A.ly + m[8] * A.lz;
        ly = m[1] * A.lx + m[5] * A.ly + m[9] * A.lz;
        lz = m[2] * A.lx + m[6] * A.ly + m[10] * A.lz;
      }
    }
    if (ok) {
      go[0] = (float)lx; go[1] = (float)ly; go[2] = (float)lz;
      gd[0] = (float)(A.t * lx); gd[1] = (float)(A.t * ly); gd[2] = (float)(A.t * lz);
    } else {
      zero3(go);
      zero3(gd);
    }
    if (!valid) continue;
    if (P.want_vertices) {
      uint32_t p = atomicAdd(&vpos[gt[r] >> P.vb.shift], 1u);
      store_rayrec(P.vb.rec + p, ok ? A.lx : 0.0, ok ? A.ly : 0.0, ok ? A.lz : 0.0, ok ? A.u : 0.0,
                   ok ? A.v : 0.0, gt[r]);
    }
    if (P.want_frames) {
      double px = 0.0, py = 0.0, pz = 0.0;
      if (ok) {
        const double w0 = 1.0 - A.u - A.v, w1 = A.u, w2 = A.v;
        px = w0 * A.p[0][0] + w1 * A.p[1][0] + w2 * A.p[2][0];
        py = w0 * A.p[0][1] + w1 * A.p[1][1] + w2 * A.p[2][1];
        pz = w0 * A.p[0][2] + w1 * A.p[1][2] + w2 * A.p[2][2];
      }
      uint32_t p = atomicAdd(&fpos[inst[r]], 1u);
      store_framerec(P.fb.rec + p, lx, ly, lz, px, py, pz);
    }
  }
}

// ---------------------------------------------------------------------------
// float64 finalize of closest hits (one thread per ray, after the traversal)
// ---------------------------------------------------------------------------
// Recomputes (t, u, v) of the winning triangle in float64 from the float32
// vertices of its record (for instances, the ray is taken to object space
// with the float64 inverse frame) and writes the instance id.  Misses are
// left as written.
template <bool INST, int MODE>
__global__ __launch_bounds__(256) void finalize_kernel(TraceParams P) {
  uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= P.n) return;
  finalize_index<INST, MODE>(P, i);
}

// float64 finalize of the ranges that fused closest-hit traversal waves could
// not keep in their lists: one wave per range (a range holds at most 64 rays)
template <bool INST>
__global__ __launch_bounds__(64) void finalize_ovf_kernel(TraceParams P) {
  uint32_t count = min(P.counter[1], P.ovf_cap);
  for (uint32_t k = blockIdx.x; k < count; k += gridDim.x) {
    uint32_t b = P.ovf[2 * k], c = P.ovf[2 * k + 1];
    for (uint32_t o = threadIdx.x; o < c; o += 64)
      finalize_index<INST, 0>(P, b + o);
  }
}

// float64 finalize of all-hit lists: one thread per list entry; entries past
// a ray's stored hits become misses (t = +inf, prim and instance invalid).
template <bool INST>
__global__ __launch_bounds__(256) void finalize_all_kernel(TraceParams P) {
  uint32_t e = blockIdx.x * 256u + threadIdx.x;
  if (e >= P.n * P.cap) return;
  uint32_t ray = e / P.cap, j = e - ray * P.cap;
  float4* hp = reinterpret_cast<float4*>(P.hits + e);
  if (j >= min(P.counts[ray], P.cap)) {
    *hp = make_float4(__int_as_float(0x7f800000), __uint_as_float(RT_INVALID_ID), 0.0f, 0.0f);
    if (P.inst_ids) P.inst_ids[e] = RT_INVALID_ID;
    return;
  }
  float4 h = *hp;
  uint32_t inst = __float_as_uint(h.z);
  uint32_t rec = __float_as_uint(h.w);
  rt_ray q = load_ray(P.rays, ray);
  double ox = q.ox, oy = q.oy, oz = q.oz, dx = q.dx, dy = q.dy, dz = q.dz;
  if constexpr (INST) {
    const rt_inst_rec64& M = P.insts64[inst];
    double a = M.m[0] * ox + M.m[1] * oy + M.m[2] * oz + M.m[3];
    double b = M.m[4] * ox + M.m[5] * oy + M.m[6] * oz + M.m[7];
    double c = M.m[8] * ox + M.m[9] * oy + M.m[10] * oz + M.m[11];
    double f = M.m[0] * dx + M.m[1] * dy + M.m[2] * dz;
    double g = M.m[4] * dx + M.m[5] * dy + M.m[6] * dz;
    double k = M.m[8] * dx + M.m[9] * dy + M.m[10] * dz;
    ox = a; oy = b; oz = c; dx = f; dy = g; dz = k;
  }
  float t, u, v;
  if (finalize64(reinterpret_cast<const float4*>(P.tris), rec, ox, oy, oz, dx, dy, dz, t, u, v)) {
    *hp = make_float4(t, h.y, u, v);
  } else {
    *hp = make_float4(h.x, h.y, 0.0f, 0.0f);
  }
  if (P.inst_ids) P.inst_ids[e] = INST ? inst : 0u;
}

// ---------------------------------------------------------------------------
// refit: triangle records from new vertices, then child boxes bottom-up
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool lex_less3(float ax, float ay, float az, float bx, float by, float bz) {
  if (ax != bx) return ax < bx;
  if (ay != by) return ay < by;
  return az < bz;
}

__global__ __launch_bounds__(256) void refit_tris_kernel(rt_tri_rec* tris, uint32_t n,
                                                         rt_mesh_dev mesh) {
  uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  rt_tri_rec r = tris[i];
  const uint32_t* ix = mesh.indices + 3 * (size_t)r.prim;
  float p[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int a = 0; a < 3; ++a) p[k][a] = mesh.vertices[3 * (size_t)ix[k] + a];
  // disable the triangle (NaN record: never hit, ignored by the box fit)
  // when a vertex is not finite or its float64 normal is zero
  bool finite = true;
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int a = 0; a < 3; ++a) finite = finite && (fabsf(p[k][a]) < __int_as_float(0x7f800000));
  double e1x = (double)p[1][0] - p[0][0], e1y = (double)p[1][1] - p[0][1], e1z = (double)p[1][2] - p[0][2];
  double e2x = (double)p[2][0] - p[0][0], e2y = (double)p[2][1] - p[0][1], e2z = (double)p[2][2] - p[0][2];
  double nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
  bool ok = finite && !(nx == 0.0 && ny == 0.0 && nz == 0.0);
  // sort the vertices lexicographically (three compare-exchanges), keeping
  // the original corner of each slot
  uint32_t corner[3] = {0u, 1u, 2u};
#define RT_VSWAP(a, b)                                                              \
  if (lex_less3(p[b][0], p[b][1], p[b][2], p[a][0], p[a][1], p[a][2])) {            \
    for (int c_ = 0; c_ < 3; ++c_) { float t_ = p[a][c_]; p[a][c_] = p[b][c_]; p[b][c_] = t_; } \
    uint32_t k_ = corner[a]; corner[a] = corner[b]; corner[b] = k_;                 \
  }
  RT_VSWAP(0, 1);
  RT_VSWAP(1, 2);
  RT_VSWAP(0, 1);
#undef RT_VSWAP
  r.order = (0u << (2 * corner[0])) | (1u << (2 * corner[1])) | (2u << (2 * corner[2]));
  float nan = __int_as_float(0x7fc00000);
  r.p0x = ok ? p[0][0] : nan; r.p0y = p[0][1]; r.p0z = p[0][2];
  r.p1x = p[1][0]; r.p1y = p[1][1]; r.p1z = p[1][2];
  r.p2x = p[2][0]; r.p2y = p[2][1]; r.p2z = p[2][2];
  if (!ok) {
    r.p0y = r.p0z = r.p1x = r.p1y = r.p1z = r.p2x = r.p2y = r.p2z = nan;
  }
  tris[i] = r;
}

// One tree level: for each node, every child slot's box becomes the exact
// float32 bounds of what lies below it (a leaf's triangle records, or the
// union of an internal child's child boxes, refitted by the previous launch).
// fminf/fmaxf skip the NaN coordinates of disabled triangles.
template <int W>
__global__ __launch_bounds__(256) void refit_nodes_kernel(float* nodes, const rt_tri_rec* tris,
                                                          const uint32_t* node_ids, uint32_t count) {
  uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= count) return;
  float* nd = nodes + (size_t)node_ids[i] * (8 * W);
  const float inf = __int_as_float(0x7f800000);
  for (int c = 0; c < W; ++c) {
    uint32_t ref = __float_as_uint(nd[6 * W + c]);
    if (ref == RT_CHILD_EMPTY) continue;
    float lo[3] = {inf, inf, inf}, hi[3] = {-inf, -inf, -inf};
    if ((ref & RT_LEAF_BIT) == 0u) {
      const float* ch = nodes + (size_t)ref * (8 * W);
      for (int k = 0; k < W; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          lo[a] = fminf(lo[a], ch[(2 * a) * W + k]);
          hi[a] = fmaxf(hi[a], ch[(2 * a + 1) * W + k]);
        }
    } else {
      uint32_t first = ref & RT_LEAF_FIRST_MASK;
      uint32_t cnt = (ref >> RT_LEAF_COUNT_SHIFT) & RT_LEAF_COUNT_MASK;
      for (uint32_t k = 0; k < cnt; ++k) {
        const rt_tri_rec& t = tris[first + k];
        const float v[9] = {t.p0x, t.p0y, t.p0z, t.p1x, t.p1y, t.p1z, t.p2x, t.p2y, t.p2z};
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], v[3 * j + a]);
            hi[a] = fmaxf(hi[a], v[3 * j + a]);
          }
      }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      nd[(2 * a) * W + c] = lo[a];
      nd[(2 * a + 1) * W + c] = hi[a];
    }
  }
}

// ---------------------------------------------------------------------------
// ambient occlusion (§4): rays from closest hits, then the occluded fraction
// ---------------------------------------------------------------------------
// Sample k of ray r: shading point p = o + t d, unit geometric normal n of
// the hit triangle turned toward the incoming ray, tangent t0 = (v1 - v0)
// normalised, bi-tangent t1 = n x t0; the cosine-weighted direction of §4.1
// (phi = 2 pi xi0, rr = sqrt(xi1), (rr cos phi, sqrt(max(1 - rr^2, 0)),
// rr sin phi) in the (t0, n, t1) frame); origin p + offset n; t in
// [0, radius].  Misses give void rays (tmin = 1 > tmax = 0).  float64 math,
// rounded once to float32.
__global__ __launch_bounds__(256) void ao_rays_kernel(AoParams P) {
  uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= P.n * P.samples) return;
  uint32_t ray = i / P.samples;
  float4* out = reinterpret_cast<float4*>(P.out + i);
  float4 h = *reinterpret_cast<const float4*>(P.hits + ray);
  uint32_t prim = __float_as_uint(h.y);
  rt_mesh_dev mesh = P.mesh;
  uint32_t inst = 0;
  bool ok = prim != RT_INVALID_ID;
  if (ok && P.inst_ids) {
    inst = P.inst_ids[ray];
    ok = inst < P.inst_count;
    if (ok) mesh = P.meshes[P.insts[inst].mesh];
  }
  if (!ok || prim >= mesh.triangle_count) {
    out[0] = make_float4(0.0f, 0.0f, 0.0f, 1.0f);
    out[1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    return;
  }
  rt_ray q = load_ray(P.rays, ray);
  const uint32_t* ix = mesh.indices + 3 * (size_t)prim;
  double v[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) v[k][c] = mesh.vertices[3 * (size_t)ix[k] + c];
  if (P.inst_ids) {
    // corners to world space: T + R(qhat)(S x), with R a = a + 2w (u x a) + 2u x (u x a)
    // for the unit quaternion (u, w)
    const rt_srt f = P.srts[inst];
    double qx = f.qx, qy = f.qy, qz = f.qz, qw = f.qw;
    double iq = 1.0 / sqrt(qx * qx + qy * qy + qz * qz + qw * qw);
    qx *= iq; qy *= iq; qz *= iq; qw *= iq;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double ax = f.sx * v[k][0], ay = f.sy * v[k][1], az = f.sz * v[k][2];
      double cx, cy, cz, ex, ey, ez;
      cross3(qx, qy, qz, ax, ay, az, cx, cy, cz);
      cross3(qx, qy, qz, cx, cy, cz, ex, ey, ez);
      v[k][0] = f.tx + (ax + 2.0 * qw * cx + 2.0 * ex);
      v[k][1] = f.ty + (ay + 2.0 * qw * cy + 2.0 * ey);
      v[k][2] = f.tz + (az + 2.0 * qw * cz + 2.0 * ez);
    }
  }
  double ax = v[1][0] - v[0][0], ay = v[1][1] - v[0][1], az = v[1][2] - v[0][2];
  double bx = v[2][0] - v[0][0], by = v[2][1] - v[0][1], bz = v[2][2] - v[0][2];
  double nx = ay * bz - az * by, ny = az * bx - ax * bz, nz = ax * by - ay * bx;
  double nl = sqrt(nx * nx + ny * ny + nz * nz);
  nx /= nl; ny /= nl; nz /= nl;
  if (nx * q.dx + ny * q.dy + nz * q.dz > 0.0) {
    nx = -nx; ny = -ny; nz = -nz;
  }
  double al = sqrt(ax * ax + ay * ay + az * az);
  double t0x = ax / al, t0y = ay / al, t0z = az / al;
  double t1x = ny * t0z - nz * t0y, t1y = nz * t0x - nx * t0z, t1z = nx * t0y - ny * t0x;
  double t = h.x;
  double px = q.ox + q.dx * t, py = q.oy + q.dy * t, pz = q.oz + q.dz * t;
  const float* u = P.xi + 2 * (size_t)i;
  double phi = 6.283185307179586476925286766559 * (double)u[0];
  double rr = sqrt((double)u[1]);
  double x = rr * cos(phi), z = rr * sin(phi);
  double y = 1.0 - rr * rr;
  y = sqrt(y > 0.0 ? y : 0.0);
  double dx = t0x * x + t1x * z + nx * y;
  double dy = t0y * x + t1y * z + ny * y;
  double dz = t0z * x + t1z * z + nz * y;
  out[0] = make_float4((float)(px + nx * P.offset), (float)(py + ny * P.offset),
                       (float)(pz + nz * P.offset), 0.0f);
  out[1] = make_float4((float)dx, (float)dy, (float)dz, P.radius);
}

__global__ __launch_bounds__(256) void ao_resolve_kernel(const uint8_t* occ, uint32_t n,
                                                         uint32_t samples, float* ao) {
  uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  const uint8_t* o = occ + (size_t)i * samples;
  uint32_t c = 0;
  for (uint32_t k = 0; k < samples; ++k) c += o[k] ? 1u : 0u;
  ao[i] = (float)c / (float)samples;
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t n, uint32_t value) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

}  // namespace rtk

// ---------------------------------------------------------------------------
// launch table
// ---------------------------------------------------------------------------
namespace {

template <int W, int S, int WG, bool ANY, bool INST, int MODE>
const void* kernel_ptr() {
  return reinterpret_cast<const void*>(&rtk::trace_kernel<W, S, WG, ANY, INST, MODE>);
}

template <int W>
const void* pick_query(bool any, bool inst, int mode) {
  if (mode == 3) return inst ? kernel_ptr<W, 16, 256, false, true, 3>() : kernel_ptr<W, 16, 256, false, false, 3>();
  if (any) return inst ? kernel_ptr<W, 16, 256, true, true, 2>() : kernel_ptr<W, 16, 256, true, false, 2>();
  return inst ? kernel_ptr<W, 16, 256, false, true, 2>() : kernel_ptr<W, 16, 256, false, false, 2>();
}

template <int W, bool ANY, bool INST>
const void* kernel_ptr_c() {
  return reinterpret_cast<const void*>(&rtk::trace_kernel<W, 16, 256, ANY, INST, 0, true>);
}
template <int W>
const void* count_kernel_w(bool any, bool inst) {
  if (inst) return any ? kernel_ptr_c<W, true, true>() : kernel_ptr_c<W, false, true>();
  return any ? kernel_ptr_c<W, true, false>() : kernel_ptr_c<W, false, false>();
}

template <int W, int S, int WG>
const void* pick_mode(bool any, bool inst, int mode) {
  if (mode == 1) return inst ? kernel_ptr<W, S, WG, false, true, 1>() : kernel_ptr<W, S, WG, false, false, 1>();
  if (any) return inst ? kernel_ptr<W, S, WG, true, true, 0>() : kernel_ptr<W, S, WG, true, false, 0>();
  return inst ? kernel_ptr<W, S, WG, false, true, 0>() : kernel_ptr<W, S, WG, false, false, 0>();
}

template <int W, int S>
const void* pick_wg(int wg, bool any, bool inst, int mode) {
  switch (wg) {
    case 64: return pick_mode<W, S, 64>(any, inst, mode);
    case 128: return pick_mode<W, S, 128>(any, inst, mode);
    case 256: return pick_mode<W, S, 256>(any, inst, mode);
    default: return nullptr;
  }
}

template <int W>
const void* pick_s(int s, int wg, bool any, bool inst, int mode) {
  switch (s) {
    case 8: return pick_wg<W, 8>(wg, any, inst, mode);
    case 16: return pick_wg<W, 16>(wg, any, inst, mode);
    case 32: return pick_wg<W, 32>(wg, any, inst, mode);
    default: return nullptr;
  }
}

}  // namespace

// Counting variants (node visits, triangle tests, stack spills per launch):
// stack 16, workgroup 256; two-level variants count the nodes of both levels.
const void* rtk_count_kernel(int width, bool any, bool inst) {
  switch (width) {
    case 2: return count_kernel_w<2>(any, inst);
    case 4: return count_kernel_w<4>(any, inst);
    case 8: return count_kernel_w<8>(any, inst);
    default: return nullptr;
  }
}

const void* rtk_trace_kernel(int width, int stack, int wg, bool any, bool inst, int mode) {
  if (mode >= 2) {
    if (stack != 16 || wg != 256 || (mode == 3 && any)) return nullptr;
    switch (width) {
      case 2: return pick_query<2>(any, inst, mode);
      case 4: return pick_query<4>(any, inst, mode);
      case 8: return pick_query<8>(any, inst, mode);
      default: return nullptr;
    }
  }
  switch (width) {
    case 2: return pick_s<2>(stack, wg, any, inst, mode);
    case 4: return pick_s<4>(stack, wg, any, inst, mode);
    case 8: return pick_s<8>(stack, wg, any, inst, mode);
    default: return nullptr;
  }
}

hipError_t rtk_launch_trace(const void* kern, uint32_t grid, uint32_t wg, const TraceParams& p,
                            hipStream_t stream) {
  TraceParams q = p;
  void* args[] = {&q};
  return hipLaunchKernel(kern, dim3(grid), dim3(wg), args, 0, stream);
}

hipError_t rtk_launch_backward(const BackwardParams& p, hipStream_t stream) {
  if (p.n == 0) return hipSuccess;
  BackwardParams q = p;
  void* args[] = {&q};
  return hipLaunchKernel(reinterpret_cast<const void*>(&rtk::backward_kernel), dim3(p.bk.tiles), dim3(1024),
                         args, p.bk.buckets * sizeof(uint32_t), stream);
}

hipError_t rtk_launch_backward_inst_tiles(const BackwardInstParams& p, hipStream_t stream) {
  if (p.n == 0) return hipSuccess;
  BackwardInstParams q = p;
  void* args[] = {&q};
  uint32_t tiles = (p.n + rta::kTile - 1) / rta::kTile;
  size_t lds = ((p.want_vertices ? p.vb.buckets : 0u) + (p.want_frames ? p.fb.buckets : 0u)) * sizeof(uint32_t);
  return hipLaunchKernel(reinterpret_cast<const void*>(&rtk::backward_inst_tile_kernel), dim3(tiles), dim3(1024),
                         args, lds, stream);
}

hipError_t rtk_launch_backward_inst(const BackwardInstParams& p, int phase, hipStream_t stream) {
  if (p.n == 0) return hipSuccess;
  BackwardInstParams q = p;
  void* args[] = {&q};
  const void* k = phase == 0 ? reinterpret_cast<const void*>(&rtk::backward_inst_kernel<0>)
                             : reinterpret_cast<const void*>(&rtk::backward_inst_kernel<1>);
  return hipLaunchKernel(k, dim3((p.n + 255) / 256), dim3(256), args, 0, stream);
}

hipError_t rtk_launch_finalize(bool inst, int mode, const TraceParams& p, hipStream_t stream) {
  if (p.n == 0) return hipSuccess;
  const void* k = mode == 1 ? (inst ? reinterpret_cast<const void*>(&rtk::finalize_kernel<true, 1>)
                                   : reinterpret_cast<const void*>(&rtk::finalize_kernel<false, 1>))
                  : inst    ? reinterpret_cast<const void*>(&rtk::finalize_kernel<true, 0>)
                            : reinterpret_cast<const void*>(&rtk::finalize_kernel<false, 0>);
  TraceParams q = p;
  void* args[] = {&q};
  return hipLaunchKernel(k, dim3((p.n + 255) / 256), dim3(256), args, 0, stream);
}

bool rtk_trace_fuses_finalize(bool any, bool inst, int mode) {
  (void)inst;
  return !any && mode == 0;
}

hipError_t rtk_launch_finalize_ovf(bool inst, const TraceParams& p, hipStream_t stream) {
  if (p.n == 0 || p.ovf_cap == 0) return hipSuccess;
  TraceParams q = p;
  void* args[] = {&q};
  const void* k = inst ? reinterpret_cast<const void*>(&rtk::finalize_ovf_kernel<true>)
                       : reinterpret_cast<const void*>(&rtk::finalize_ovf_kernel<false>);
  // one wave per listed range at most (the list holds no more than ovf_cap)
  return hipLaunchKernel(k, dim3(std::min<uint32_t>(2048u, p.ovf_cap)), dim3(64), args, 0, stream);
}

hipError_t rtk_launch_finalize_all(bool inst, const TraceParams& p, hipStream_t stream) {
  uint64_t total = (uint64_t)p.n * p.cap;
  if (total == 0) return hipSuccess;
  const void* k = inst ? reinterpret_cast<const void*>(&rtk::finalize_all_kernel<true>)
                       : reinterpret_cast<const void*>(&rtk::finalize_all_kernel<false>);
  TraceParams q = p;
  void* args[] = {&q};
  return hipLaunchKernel(k, dim3((uint32_t)((total + 255) / 256)), dim3(256), args, 0, stream);
}

hipError_t rtk_launch_refit_tris(rt_tri_rec* tris, uint32_t n, const rt_mesh_dev& mesh,
                                 hipStream_t stream) {
  if (n == 0) return hipSuccess;
  rt_mesh_dev m = mesh;
  void* args[] = {&tris, &n, &m};
  return hipLaunchKernel(reinterpret_cast<const void*>(&rtk::refit_tris_kernel), dim3((n + 255) / 256),
                         dim3(256), args, 0, stream);
}

hipError_t rtk_launch_refit_nodes(int width, float* nodes, const rt_tri_rec* tris,
                                  const uint32_t* node_ids, uint32_t count, hipStream_t stream) {
  if (count == 0) return hipSuccess;
  const void* k = width == 2   ? reinterpret_cast<const void*>(&rtk::refit_nodes_kernel<2>)
                  : width == 4 ? reinterpret_cast<const void*>(&rtk::refit_nodes_kernel<4>)
                               : reinterpret_cast<const void*>(&rtk::refit_nodes_kernel<8>);
  void* args[] = {&nodes, &tris, &node_ids, &count};
  return hipLaunchKernel(k, dim3((count + 255) / 256), dim3(256), args, 0, stream);
}

hipError_t rtk_launch_ao_rays(const AoParams& p, hipStream_t stream) {
  uint64_t total = (uint64_t)p.n * p.samples;
  if (total == 0) return hipSuccess;
  AoParams q = p;
  void* args[] = {&q};
  return hipLaunchKernel(reinterpret_cast<const void*>(&rtk::ao_rays_kernel),
                         dim3((uint32_t)((total + 255) / 256)), dim3(256), args, 0, stream);
}

hipError_t rtk_launch_ao_resolve(const uint8_t* occluded, uint32_t n, uint32_t samples, float* ao,
                                 hipStream_t stream) {
  if (n == 0) return hipSuccess;
  void* args[] = {&occluded, &n, &samples, &ao};
  return hipLaunchKernel(reinterpret_cast<const void*>(&rtk::ao_resolve_kernel),
                         dim3((n + 255) / 256), dim3(256), args, 0, stream);
}

hipError_t rtk_launch_fill(uint32_t* ptr, uint32_t n, uint32_t value, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  void* args[] = {&ptr, &n, &value};
  return hipLaunchKernel(reinterpret_cast<const void*>(&rtk::fill_u32_kernel),
                         dim3((n + 255) / 256), dim3(256), args, 0, stream);
}
