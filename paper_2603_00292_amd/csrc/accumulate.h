// accumulate.h -- deterministic accumulation of per-ray gradient
// contributions (librtq internal).
//
// Two forms.  The first, below, adds into rows with device atomics: it serves
// the two-level adjoint of accels with more instances than the bucketed form
// has LDS counters for.  The second, further below, groups the rays first and
// needs no global atomic; both form the same exact sums.
//
// A contribution adds three float64 values to one row (a vertex, or a part of
// an instance frame).  The sums are formed in 64-bit integers, so they do not
// depend on the order in which rays reach a row:
//   phase 0  every contribution raises expo[row] to the binary exponent of its
//            largest component (an atomic maximum, skipped when a plain load
//            already shows that exponent or a larger one: the stored value
//            only grows, so a stale load can only cost an extra atomic);
//   phase 1  every component c is rounded to the integer nearest
//            c * 2^(shift0 - e), e = expo[row], and added to the row's integer
//            sum (integer addition is associative);
//   convert  every touched row's sums are scaled back by 2^(e - shift0),
//            rounded to float32 and added to the output, and the row is reset.
// shift0 = 62 - H, where 2^H exceeds the number of contributions a row can
// receive (one per ray at most), so no sum overflows: a scaled component is
// at most 2^(63 - H) in magnitude.  Each row keeps shift0 bits below its
// largest contribution (at least 30 bits for 2^31 rays), more than the
// float32 result holds.  A non-finite contribution makes its row NaN.
//
// The phase-1 sums are kept per XCD (the chip's eight dies, each with its own
// L2): a wave adds into the copy of the die it runs on, with atomics of
// workgroup scope that complete in that die's L2 instead of travelling to the
// memory side as device-scope atomics do; no other die touches that copy
// during the launch, and the kernel boundary makes the copies visible to the
// convert, which adds the eight integer partial sums (exactly, in any order).
// Random atomics still run at about 25 G per second on this chip whatever
// their scope, which is why the grouped form exists.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace rta {

constexpr uint32_t kExpoBias = 2048;               // stored exponent = ilogb + bias; 0 = untouched
constexpr uint32_t kExpoNonFinite = 0xFFFFFFFFu;   // a row that received inf or NaN

constexpr uint32_t kCopies = 8;                     // per-die copies of the sums

// Accumulator rows in device memory (owned by an accel).
struct Rows {
  uint32_t* expo = nullptr;             // count entries
  unsigned long long* sums = nullptr;   // [kCopies][count][4] (three used), two's complement
  uint32_t count = 0;
};

// What a producing kernel needs.
struct Acc {
  uint32_t* expo;
  unsigned long long* sums;
  uint32_t rows;
  int shift0;
};

// The XCD (die) the calling wave runs on: bits 3:0 of the XCC_ID hardware
// register (s_getreg of register 20, four bits from offset 0).
__device__ __forceinline__ uint32_t die_id() {
  return (uint32_t)__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & (kCopies - 1u);
}

// 62 - H for launches of n rays (2^H > n).
inline int shift0_for(uint64_t n) {
  int h = 0;
  while (h < 63 && (1ull << h) <= n) ++h;
  return 62 - h;
}

// Allocates `count` rows (not cleared: clear() them before use).
hipError_t alloc(Rows& r, uint32_t count);
void release(Rows& r);

// Resets every row (stream-ordered fill kernels; after an interrupted call).
hipError_t clear(const Rows& r, hipStream_t stream);

// Converts rows [first, first + count) and adds them to `out`, resetting them.
// layout 0: out[3 i + c] for row first + i (vertex rows);
// layout 1: rows 4 j + part hold instance j's frame parameters
//           3 part + c < 10 (S xyz, q xyz, q w, T xyz): out[10 j + 3 part + c].
hipError_t convert(const Rows& r, uint32_t first, uint32_t count, int layout, int shift0, float* out,
                   hipStream_t stream);

template <int PHASE>
__device__ __forceinline__ void add(const Acc& a, uint32_t row, double x, double y, double z) {
  bool finite = isfinite(x) && isfinite(y) && isfinite(z);
  double m = fmax(fabs(x), fmax(fabs(y), fabs(z)));
  if (finite && m == 0.0) return;
  if constexpr (PHASE == 0) {
    uint32_t e = finite ? (uint32_t)(ilogb(m) + (int)kExpoBias) : kExpoNonFinite;
    if (a.expo[row] < e) atomicMax(a.expo + row, e);
  } else {
    uint32_t e = a.expo[row];
    if (e == kExpoNonFinite) return;
    int sh = a.shift0 - ((int)e - (int)kExpoBias);
    unsigned long long* s = a.sums + 4 * ((size_t)die_id() * a.rows + row);
    long long vx = __double2ll_rn(ldexp(x, sh));
    long long vy = __double2ll_rn(ldexp(y, sh));
    long long vz = __double2ll_rn(ldexp(z, sh));
    if (vx) __hip_atomic_fetch_add(s + 0, (unsigned long long)vx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (vy) __hip_atomic_fetch_add(s + 1, (unsigned long long)vy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (vz) __hip_atomic_fetch_add(s + 2, (unsigned long long)vz, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

}  // namespace rta

// ---------------------------------------------------------------------------
// Gradients without global atomics: rays grouped by what they add to
// ---------------------------------------------------------------------------
//   bucket   the hit rays are grouped by key (a triangle range: buckets of
//            2^shift triangles, the smallest shift that keeps the bucket
//            count within kMaxBuckets; or an instance): per-tile LDS
//            histograms of the keys, then one launch that scans every
//            bucket's column of tile counts; then the adjoint kernel scans
//            the bucket totals in LDS and writes each hit ray's 48-byte
//            record straight into its bucket through LDS counters (the
//            order inside a bucket is not fixed, and does not need to be);
//   corner   one workgroup per triangle bucket sums -w_k lambda of its rays
//            per (triangle, corner) in LDS, exactly, as 64-bit integers at
//            the row's binary scale (an LDS maximum of the exponents first),
//            and writes each row's float64 value;
//   vertex   every vertex adds its corners' values in ascending (triangle,
//            corner) order through a vertex -> (triangle, corner) list,
//            rounds once to float32 and adds to the output;
//   frame    (two-level) one workgroup per instance forms each ray's ten
//            frame derivatives from its record and sums them exactly per
//            row as in the atomic rows above (a workgroup maximum of the
//            exponents, then 64-bit integer sums reduced over the
//            workgroup), and adds the rounded sums to the output.
// Two-level accels number the triangles and vertices of all meshes one
// after another in build order (global ids).  The integer sums keep
// shift0 = 62 - H bits below each row's largest contribution (2^H > n), so
// the result is independent of the schedule and of the order of the rays:
// repeated calls and permuted rays give bit-identical gradients.
namespace rta {

constexpr uint32_t kMaxBuckets = 16384;     // LDS counters
constexpr uint32_t kTile = 4096;            // rays per workgroup of the histogram and the adjoint
constexpr uint32_t kNoKey = 0xFFFFFFFFu;

// per hit ray: float64 lambda (object space for two-level hits), u, v and
// the (global) triangle
struct RayRec {
  double lx, ly, lz, u, v;
  uint32_t prim, pad;
};

// per two-level hit ray: float64 world-space lambda and object hit point
struct FrameRec {
  double lx, ly, lz, px, py, pz;
};
static_assert(sizeof(FrameRec) == sizeof(RayRec), "one record buffer type");

// log2 of the bucket size for `triangles` triangles, at least min_shift
// (0: too many triangles)
inline uint32_t bucket_shift(uint32_t triangles, uint32_t min_shift = 8) {
  for (uint32_t sh = min_shift; sh <= 10; ++sh)
    if (((uint64_t)triangles + (1u << sh) - 1) >> sh <= kMaxBuckets) return sh;
  return 0;
}

// Per accel: the vertex -> (triangle << 2 | corner) lists, the corner values
// and a copy of every triangle's three vertices (so the adjoint reads one
// 36-byte record per hit instead of an index triple and three vertices).
// Two-level: global triangle and vertex ids, plus each instance's mesh as
// (first global triangle, triangle count).
struct Gather {
  uint32_t* csr_off = nullptr;   // vertices + 1
  uint32_t* csr_ent = nullptr;   // 3 * triangles
  double* corner = nullptr;      // 9 per triangle: corner k's 3 components
  float* tri_vertices = nullptr; // 9 per triangle: vertex k's x, y, z
  uint2* inst_tris = nullptr;    // two-level: one per instance
  bool tri_vertices_valid = false;
  uint32_t vertices = 0, triangles = 0, shift = 0, buckets = 0;
};

// Where a ray's key comes from: kind 0, its triangle (single level); 1, its
// global triangle; 2, its instance.  Rays without a valid hit have no key.
struct KeySource {
  const uint32_t* hit_words;     // prim id at hit_words[4 i + 1]
  const uint32_t* inst_ids;      // two-level
  const uint2* inst_tris;        // two-level
  uint32_t inst_count;
  uint32_t triangles;            // single level
  uint32_t kind;
};

__device__ __forceinline__ uint32_t ray_key(const KeySource& k, uint32_t i) {
  const uint32_t prim = k.hit_words[4 * (size_t)i + 1];
  if (k.kind == 0) return prim < k.triangles ? prim : kNoKey;
  const uint32_t inst = k.inst_ids[i];
  if (inst >= k.inst_count) return kNoKey;
  const uint2 it = k.inst_tris[inst];
  if (prim >= it.y) return kNoKey;
  return k.kind == 1 ? it.x + prim : inst;
}

// Per context: buffers sized by the ray count (grown stream-ordered).
struct SortBuf {
  RayRec* rec = nullptr;         // cap: records grouped by bucket
  uint32_t* counts = nullptr;    // tiles x buckets histogram (tile-major), scanned per bucket in place
  uint32_t* scan = nullptr;      // bucket totals (buckets), bucket starts (buckets + 1)
  size_t cap = 0, count_cap = 0, scan_cap = 0;
};

// What the adjoint kernel needs to place its records: tile t's first slot
// in bucket b is base[b] + counts[t * buckets + b], base the exclusive scan
// of the totals (which the adjoint kernel's workgroup 0 stores).
struct Bucketing {
  const uint32_t* counts;
  const uint32_t* totals;        // rays per bucket
  uint32_t* base;                // buckets + 1 bucket starts (the last one: the hit count)
  uint32_t tiles, buckets, shift;
  RayRec* rec;
};

// Builds g from the mesh's indices (host copy): counting sort by vertex,
// entries in ascending (triangle, corner) order.
hipError_t gather_build(Gather& g, const uint32_t* host_indices, uint32_t vertices, uint32_t triangles);
// The same over several meshes (two-level): host indices of mesh m at
// indices[m], global ids in mesh order; inst_mesh: host, one per instance.
hipError_t gather_build_multi(Gather& g, const uint32_t* const* host_indices, const uint32_t* vertex_counts,
                              const uint32_t* triangle_counts, uint32_t meshes, const uint32_t* inst_mesh,
                              uint32_t instances, uint32_t min_shift);
void gather_release(Gather& g);
// Refreshes g.tri_vertices of mesh m (first global triangle `first`) from its
// device indices and vertices; mark_valid after the last mesh.
hipError_t gather_tri_vertices(Gather& g, const uint32_t* indices, const float* vertices, uint32_t triangles,
                               uint32_t first, hipStream_t s);
// Makes b hold n rays in `buckets` buckets; a larger n or bucket count
// frees and allocates stream-ordered on s (no device-wide synchronisation).
hipError_t sort_reserve(SortBuf& b, uint32_t buckets, size_t n, hipStream_t s);
void sort_release(SortBuf& b);
// Histogram of the rays' keys (buckets of 2^shift keys) and its scans;
// returns the adjoint kernel's placement.
hipError_t bucket_rays(const KeySource& keys, uint32_t buckets, uint32_t shift, SortBuf& b, uint32_t n,
                       hipStream_t s, Bucketing* out);
// After the adjoint kernel placed the records: sum per corner and per
// vertex, out[3 v + c] += the vertex sums.
hipError_t gather_vertices(Gather& g, SortBuf& b, uint32_t n, float* out, hipStream_t s);
// After the adjoint kernel placed the frame records (one bucket per
// instance): out[10 j + k] += instance j's frame gradients; srt: 10 floats
// per instance (sx sy sz qx qy qz qw tx ty tz).
hipError_t frame_sums(SortBuf& b, uint32_t instances, const float* srt, uint32_t n, float* out, hipStream_t s);

}  // namespace rta
