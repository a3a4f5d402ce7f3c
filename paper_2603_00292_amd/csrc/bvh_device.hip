// bvh_device.hip -- device-side BVH construction of one mesh (see bvh_device.h).
//
// Steps, each a kernel (or a hipCUB primitive) on the caller's stream:
//   1. compact float3 / uint3 copies of the strided mesh, index range check;
//   2. per triangle: validity (finite vertices, non-zero float64 normal) and
//      the centre of its box;
//   3. compaction of the valid triangle ids (hipCUB select);
//   4. bounds of the centres (block reduction + order-preserving atomics);
//   5. 30-bit Morton code of each centre, made unique by the position in the
//      compacted list, and a radix sort of (code, id) pairs (hipCUB);
//   6. bottom-up clustering (§6.2 construction paragraph: every triangle
//      starts as a cluster and clusters are merged until one is left) by
//      PLOC (Meister & Bittner 2018): the clusters stay in Morton order; each
//      finds, among the kPlocRadius clusters on either side, the one whose
//      merged box has the least surface area; mutual nearest neighbours are
//      merged into a new node; the list is compacted; repeat.  One pass is
//      four launches (neighbours, merge flags, an exclusive scan that
//      numbers the new nodes, merge + compaction), so the tree is the same
//      on every run;
//   7. the binary tree collapsed into W-wide nodes level by level (the
//      widest-child expansion of the host builder), leaves holding subtrees
//      of at most max_leaf triangles; each subtree gets a contiguous range of
//      triangle records, handed down from its parent;
//   8. triangle records in that order (vertices sorted, corner order kept).
#include "bvh_device.h"
#include "rt_alloc.h"

#include <hipcub/hipcub.hpp>

#include <algorithm>

namespace rtd {
namespace {


// order-preserving map of a float to an unsigned int (for atomic min / max)
__device__ __forceinline__ uint32_t ord(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unord(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u);
}

__global__ void copy_vertices_kernel(const uint8_t* src, uint32_t stride, uint32_t n, float* dst) {
  uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  const float* p = reinterpret_cast<const float*>(src + (size_t)i * stride);
  dst[3 * (size_t)i + 0] = p[0];
  dst[3 * (size_t)i + 1] = p[1];
  dst[3 * (size_t)i + 2] = p[2];
}

__global__ void copy_indices_kernel(const uint8_t* src, uint32_t stride, uint32_t n,
                                    uint32_t vertex_count, uint32_t* dst, uint32_t* error) {
  uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  const uint32_t* p = reinterpret_cast<const uint32_t*>(src + (size_t)i * stride);
  uint32_t a = p[0], b = p[1], c = p[2];
  if (a >= vertex_count || b >= vertex_count || c >= vertex_count) atomicOr(error, 1u);
  dst[3 * (size_t)i + 0] = a;
  dst[3 * (size_t)i + 1] = b;
  dst[3 * (size_t)i + 2] = c;
}

__device__ __forceinline__ void load_tri(const float* V, const uint32_t* I, uint32_t t, float p[3][3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    uint32_t v = I[3 * (size_t)t + k];
#pragma unroll
    for (int a = 0; a < 3; ++a) p[k][a] = V[3 * (size_t)v + a];
  }
}

// validity (finite vertices, non-zero float64 normal) and box centre
__global__ void prep_kernel(const float* V, const uint32_t* I, uint32_t n, uint8_t* valid,
                            float4* centre) {
  uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  float p[3][3];
  load_tri(V, I, i, p);
  bool finite = true;
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int a = 0; a < 3; ++a) finite = finite && (fabsf(p[k][a]) < __int_as_float(0x7f800000));
  double e1x = (double)p[1][0] - p[0][0], e1y = (double)p[1][1] - p[0][1], e1z = (double)p[1][2] - p[0][2];
  double e2x = (double)p[2][0] - p[0][0], e2y = (double)p[2][1] - p[0][1], e2z = (double)p[2][2] - p[0][2];
  double nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
  valid[i] = (finite && !(nx == 0.0 && ny == 0.0 && nz == 0.0)) ? 1 : 0;
  float c[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float lo = fminf(fminf(p[0][a], p[1][a]), p[2][a]);
    float hi = fmaxf(fmaxf(p[0][a], p[1][a]), p[2][a]);
    c[a] = 0.5f * lo + 0.5f * hi;
  }
  centre[i] = make_float4(c[0], c[1], c[2], 0.0f);
}

// bounds of the centres of the valid triangles: ord-encoded (min x,y,z, max x,y,z)
__global__ __launch_bounds__(256) void centre_bounds_kernel(const float4* centre, const uint32_t* ids,
                                                            uint32_t m, uint32_t* bounds) {
  __shared__ uint32_t s[6][256];
  uint32_t i = blockIdx.x * 256u + threadIdx.x;
  uint32_t v[6] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u, 0u};
  if (i < m) {
    float4 c = centre[ids[i]];
    v[0] = v[3] = ord(c.x);
    v[1] = v[4] = ord(c.y);
    v[2] = v[5] = ord(c.z);
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) s[k][threadIdx.x] = v[k];
  __syncthreads();
  for (uint32_t off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
#pragma unroll
      for (int k = 0; k < 3; ++k) s[k][threadIdx.x] = min(s[k][threadIdx.x], s[k][threadIdx.x + off]);
#pragma unroll
      for (int k = 3; k < 6; ++k) s[k][threadIdx.x] = max(s[k][threadIdx.x], s[k][threadIdx.x + off]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int k = 0; k < 3; ++k) atomicMin(bounds + k, s[k][0]);
    for (int k = 3; k < 6; ++k) atomicMax(bounds + k, s[k][0]);
  }
}

__device__ __forceinline__ uint32_t spread10(uint32_t x) {
  x &= 0x3FFu;
  x = (x | (x << 16)) & 0x030000FFu;
  x = (x | (x << 8)) & 0x0300F00Fu;
  x = (x | (x << 4)) & 0x030C30C3u;
  x = (x | (x << 2)) & 0x09249249u;
  return x;
}

// key = (30-bit Morton code of the centre) << 32 | position; value = triangle id
__global__ void morton_kernel(const float4* centre, const uint32_t* ids, uint32_t m,
                              const uint32_t* bounds, uint64_t* keys) {
  uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= m) return;
  float4 c = centre[ids[i]];
  float cc[3] = {c.x, c.y, c.z};
  uint32_t q[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float lo = unord(bounds[a]), hi = unord(bounds[3 + a]);
    float ext = hi - lo;
    float x = ext > 0.0f ? (cc[a] - lo) / ext * 1024.0f : 0.0f;
    x = fminf(fmaxf(x, 0.0f), 1023.0f);
    q[a] = (uint32_t)x;
  }
  uint32_t code = spread10(q[0]) | (spread10(q[1]) << 1) | (spread10(q[2]) << 2);
  keys[i] = ((uint64_t)code << 32) | i;
}

// ---------------------------------------------------------------------------
// PLOC.  Binary node ids: leaf k (k-th triangle in Morton order) is m - 1 + k;
// internal nodes take ids m - 2, m - 3, ... in the order they are made, so
// the last merge makes the root, node 0.
// ---------------------------------------------------------------------------
// Search radius: on the 1.3M-triangle icosphere, radii 8 / 16 / 32 / 64 gave
// 20.6 / 21.3 / 20.4 / 20.8 node visits per incoherent ray; 32 is kept.
constexpr int kPlocRadius = 32;

__global__ void leaf_boxes_kernel(const float* V, const uint32_t* I, const uint32_t* sorted_ids, uint32_t m,
                                  float* box, uint32_t* count, uint32_t* clusters) {
  uint32_t k = blockIdx.x * 256u + threadIdx.x;
  if (k >= m) return;
  float p[3][3];
  load_tri(V, I, sorted_ids[k], p);
  uint32_t id = m - 1u + k;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    box[6 * (size_t)id + a] = fminf(fminf(p[0][a], p[1][a]), p[2][a]);
    box[6 * (size_t)id + 3 + a] = fmaxf(fmaxf(p[0][a], p[1][a]), p[2][a]);
  }
  count[id] = 1u;
  clusters[k] = id;
}

// symmetric 32-bit hash of a pair of positions (a < b): breaks ties between
// equal merged areas so that duplicate boxes still pair up (multiplicative
// mixing followed by the MurmurHash3 finaliser)
__device__ __forceinline__ uint32_t pair_hash(uint32_t a, uint32_t b) {
  uint32_t h = a * 0x9E3779B1u + b * 0x85EBCA77u + 0x165667B1u;
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}

// nn[i] = the cluster among positions [i - r, i + r] whose merged box with i
// has the least half surface area (ties: the pair hash).  A pair's key is
// the same computed from either side, so mutual neighbours are well defined.
__global__ __launch_bounds__(256) void ploc_nn_kernel(const uint32_t* clusters, uint32_t n, const float* box,
                                                     uint32_t* nn) {
  constexpr int T = 256 + 2 * kPlocRadius;
  __shared__ float sb[6][T];
  const int base = (int)(blockIdx.x * 256u) - kPlocRadius;
  for (int t = threadIdx.x; t < T; t += 256) {
    int i = base + t;
    if (i >= 0 && i < (int)n) {
      const float* q = box + 6 * (size_t)clusters[i];
#pragma unroll
      for (int a = 0; a < 6; ++a) sb[a][t] = q[a];
    }
  }
  __syncthreads();
  const int i = (int)(blockIdx.x * 256u + threadIdx.x);
  if (i >= (int)n) return;
  const int li = i - base;
  const float lx = sb[0][li], ly = sb[1][li], lz = sb[2][li];
  const float hx = sb[3][li], hy = sb[4][li], hz = sb[5][li];
  uint64_t best = ~0ull;
  uint32_t arg = (uint32_t)i;
  const int jlo = max(i - kPlocRadius, 0), jhi = min(i + kPlocRadius, (int)n - 1);
  for (int j = jlo; j <= jhi; ++j) {
    if (j == i) continue;
    const int lj = j - base;
    float dx = fmaxf(hx, sb[3][lj]) - fminf(lx, sb[0][lj]);
    float dy = fmaxf(hy, sb[4][lj]) - fminf(ly, sb[1][lj]);
    float dz = fmaxf(hz, sb[5][lj]) - fminf(lz, sb[2][lj]);
    float area = dx * dy + dy * dz + dz * dx;  // >= 0: boxes are finite and not inverted
    uint32_t lo = (uint32_t)min(i, j), hi = (uint32_t)max(i, j);
    uint64_t key = ((uint64_t)__float_as_uint(area) << 32) | pair_hash(lo, hi);
    if (key < best) {
      best = key;
      arg = (uint32_t)j;
    }
  }
  nn[i] = arg;
}

// The partner of position i in this pass: its nearest neighbour when the
// relation is mutual (or, in a pass forced to pair (2k, 2k+1) because the
// previous pass found no mutual pair, its even/odd partner); n if none.
__device__ __forceinline__ uint32_t ploc_partner(const uint32_t* nn, uint32_t n, int force, uint32_t i) {
  if (force) {
    uint32_t j = i ^ 1u;
    return j < n ? j : n;
  }
  uint32_t j = nn[i];
  return (j < n && j != i && nn[j] == i) ? j : n;
}

__global__ void ploc_flag_kernel(const uint32_t* nn, uint32_t n, int force, uint32_t* flag) {
  uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  uint32_t j = ploc_partner(nn, n, force, i);
  flag[i] = (j < n && i < j) ? 1u : 0u;
}

// The lower position of a merged pair makes node top - off[i] and keeps its
// place in the list; the higher one is dropped (keep = 0).
__global__ void ploc_merge_kernel(const uint32_t* clusters, const uint32_t* nn, uint32_t n, int force,
                                  const uint32_t* off, uint32_t top, uint32_t* left, uint32_t* right,
                                  uint32_t* count, float* box, uint32_t* out, uint8_t* keep) {
  uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  uint32_t j = ploc_partner(nn, n, force, i);
  uint32_t ci = clusters[i];
  if (j >= n) {
    out[i] = ci;
    keep[i] = 1;
    return;
  }
  if (j < i) {
    keep[i] = 0;
    return;
  }
  uint32_t cj = clusters[j];
  uint32_t id = top - off[i];
  left[id] = ci;
  right[id] = cj;
  count[id] = count[ci] + count[cj];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    box[6 * (size_t)id + a] = fminf(box[6 * (size_t)ci + a], box[6 * (size_t)cj + a]);
    box[6 * (size_t)id + 3 + a] = fmaxf(box[6 * (size_t)ci + 3 + a], box[6 * (size_t)cj + 3 + a]);
  }
  out[i] = id;
  keep[i] = 1;
}

struct Item {
  uint32_t bnode;   // binary node id
  uint32_t wnode;   // wide node index
  uint32_t stack;   // stack entries above this node
  uint32_t first;   // first triangle record of the subtree
};

struct CollapseParams {
  const uint32_t* left;
  const uint32_t* right;
  const uint32_t* count;   // triangles below each binary node
  uint32_t* perm;          // record position -> Morton position
  const float* box;
  int m;
  int width;
  int max_leaf;
  const Item* in;
  uint32_t n_in;
  Item* out;
  uint32_t* n_out;
  uint32_t* node_counter;
  uint32_t* leaf_counter;
  uint32_t* max_stack;
  double* area_sum;
  float* nodes;
};

__device__ __forceinline__ bool is_leaf(const CollapseParams& P, uint32_t b) { return b >= (uint32_t)(P.m - 1); }
__device__ __forceinline__ uint32_t count_of(const CollapseParams& P, uint32_t b) { return P.count[b]; }
__device__ __forceinline__ double area_of(const float* box, uint32_t b) {
  const float* q = box + 6 * (size_t)b;
  double dx = (double)q[3] - q[0], dy = (double)q[4] - q[1], dz = (double)q[5] - q[2];
  return 2.0 * (dx * dy + dy * dz + dz * dx);
}
__device__ __forceinline__ bool is_big(const CollapseParams& P, uint32_t b) {
  return !is_leaf(P, b) && count_of(P, b) > (uint32_t)P.max_leaf;
}

// One wide node per thread: widest-child expansion of binary node `bnode`.
__global__ void collapse_kernel(CollapseParams P) {
  uint32_t t = blockIdx.x * 256u + threadIdx.x;
  if (t >= P.n_in) return;
  Item it = P.in[t];
  const int W = P.width;
  uint32_t kids[8];
  int nk = 0;
  if (!is_big(P, it.bnode)) {
    kids[nk++] = it.bnode;
  } else {
    kids[nk++] = P.left[it.bnode];
    kids[nk++] = P.right[it.bnode];
    while (nk < W) {
      int pick = -1;
      double best = -1.0;
      for (int i = 0; i < nk; ++i)
        if (is_big(P, kids[i]) && area_of(P.box, kids[i]) > best) {
          best = area_of(P.box, kids[i]);
          pick = i;
        }
      if (pick < 0) break;
      uint32_t b = kids[pick];
      for (int i = nk; i > pick + 1; --i) kids[i] = kids[i - 1];
      kids[pick] = P.left[b];
      kids[pick + 1] = P.right[b];
      ++nk;
    }
  }
  uint32_t stack_here = it.stack + (uint32_t)nk - 1u;
  atomicMax(P.max_stack, stack_here + 1u);
  atomicAdd(P.area_sum, area_of(P.box, it.bnode));
  float* nd = P.nodes + (size_t)it.wnode * 8 * W;
  uint32_t first = it.first;  // the children split the parent's record range in order
  for (int i = 0; i < W; ++i) {
    float lo[3] = {__int_as_float(0x7f800000), __int_as_float(0x7f800000), __int_as_float(0x7f800000)};
    float hi[3] = {__int_as_float(0xff800000), __int_as_float(0xff800000), __int_as_float(0xff800000)};
    uint32_t ref = RT_CHILD_EMPTY;
    if (i < nk) {
      uint32_t b = kids[i];
      const float* q = P.box + 6 * (size_t)b;
      for (int a = 0; a < 3; ++a) {
        lo[a] = q[a];
        hi[a] = q[3 + a];
      }
      if (is_big(P, b)) {
        uint32_t w = atomicAdd(P.node_counter, 1u);
        uint32_t slot = atomicAdd(P.n_out, 1u);
        P.out[slot] = Item{b, w, stack_here, first};
        ref = w;
      } else {
        // a leaf: its (at most max_leaf <= 15) triangles, depth first
        ref = RT_LEAF_BIT | (count_of(P, b) << RT_LEAF_COUNT_SHIFT) | first;
        atomicAdd(P.leaf_counter, 1u);
        uint32_t stk[16];
        int sp = 0;
        uint32_t pos = first;
        stk[sp++] = b;
        while (sp > 0) {
          uint32_t x = stk[--sp];
          if (is_leaf(P, x)) {
            P.perm[pos++] = x - (uint32_t)(P.m - 1);
          } else {
            stk[sp++] = P.right[x];
            stk[sp++] = P.left[x];
          }
        }
      }
      first += count_of(P, b);
    }
    nd[0 * W + i] = lo[0];
    nd[1 * W + i] = hi[0];
    nd[2 * W + i] = lo[1];
    nd[3 * W + i] = hi[1];
    nd[4 * W + i] = lo[2];
    nd[5 * W + i] = hi[2];
    nd[6 * W + i] = __uint_as_float(ref);
    nd[7 * W + i] = 0.0f;
  }
}

__device__ __forceinline__ bool lex_less(const float* a, const float* b) {
  if (a[0] != b[0]) return a[0] < b[0];
  if (a[1] != b[1]) return a[1] < b[1];
  return a[2] < b[2];
}

// triangle record k = the triangle at Morton position perm[k]
__global__ void records_kernel(const float* V, const uint32_t* I, const uint32_t* sorted_ids,
                               const uint32_t* perm, uint32_t m, rt_tri_rec* out) {
  uint32_t k = blockIdx.x * 256u + threadIdx.x;
  if (k >= m) return;
  uint32_t prim = sorted_ids[perm[k]];
  float p[3][3];
  load_tri(V, I, prim, p);
  uint32_t corner[3] = {0u, 1u, 2u};
  auto cswap = [&](int a, int b) {
    if (lex_less(p[b], p[a])) {
      for (int c = 0; c < 3; ++c) {
        float t = p[a][c];
        p[a][c] = p[b][c];
        p[b][c] = t;
      }
      uint32_t t = corner[a];
      corner[a] = corner[b];
      corner[b] = t;
    }
  };
  cswap(0, 1);
  cswap(1, 2);
  cswap(0, 1);
  rt_tri_rec r;
  r.p0x = p[0][0]; r.p0y = p[0][1]; r.p0z = p[0][2];
  r.prim = prim;
  r.p1x = p[1][0]; r.p1y = p[1][1]; r.p1z = p[1][2];
  r.order = (0u << (2 * corner[0])) | (1u << (2 * corner[1])) | (2u << (2 * corner[2]));
  r.p2x = p[2][0]; r.p2y = p[2][1]; r.p2z = p[2][2];
  r.pad2 = 0;
  out[k] = r;
}

__global__ void relocate_kernel(float* nodes, uint32_t count, int W, uint32_t nb, uint32_t tb) {
  uint32_t t = blockIdx.x * 256u + threadIdx.x;
  if (t >= count * (uint32_t)W) return;
  uint32_t i = t / (uint32_t)W, c = t % (uint32_t)W;
  float* slot = nodes + (size_t)i * 8 * W + 6 * W + c;
  uint32_t ref = __float_as_uint(*slot);
  if (ref == RT_CHILD_EMPTY) return;
  if ((ref & RT_LEAF_BIT) == 0u) ref += nb;
  else if ((ref & RT_INST_BIT) == 0u) ref += tb;  // the first record is the low bits
  *slot = __uint_as_float(ref);
}

__global__ void fill_kernel(uint32_t* p, uint32_t n, uint32_t v) {
  uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void iota_kernel(uint32_t* p, uint32_t begin, uint32_t n) {
  uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i < n) p[i] = begin + i;
}

uint32_t blocks(uint64_t n) { return (uint32_t)((n + 255) / 256); }

// temporaries freed on every exit
struct Temps {
  std::vector<void*> p;
  ~Temps() {
    for (void* q : p) (void)hipFree(q);
  }
  template <typename T>
  hipError_t alloc(T** out, size_t count) {
    *out = nullptr;
    if (count == 0) count = 1;
    hipError_t e = rt_malloc(reinterpret_cast<void**>(out), count * sizeof(T));
    if (e == hipSuccess) p.push_back(*out);
    return e;
  }
};

template <typename T>
hipError_t keep(Output& out, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = rt_malloc(reinterpret_cast<void**>(p), count * sizeof(T));
  if (e == hipSuccess) {
    out.owned.push_back(*p);
    out.owned_bytes += count * sizeof(T);
  }
  return e;
}

#define RTD_TRY(x)                     \
  do {                                 \
    hipError_t e_ = (x);               \
    if (e_ != hipSuccess) return e_;   \
  } while (0)

}  // namespace

hipError_t build(const Input& in, Output& out, bool& index_error, hipStream_t s) {
  index_error = false;
  const uint32_t nv = in.vertex_count, nt = in.triangle_count;
  const int W = in.width;
  Temps tmp;
  // 1. compact copies and the index check
  RTD_TRY(keep(out, &out.vertices, (size_t)nv * 3));
  RTD_TRY(keep(out, &out.indices, (size_t)nt * 3));
  uint32_t* err = nullptr;
  RTD_TRY(tmp.alloc(&err, 1));
  hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(256), 0, s, err, 1u, 0u);
  if (nv) hipLaunchKernelGGL(copy_vertices_kernel, dim3(blocks(nv)), dim3(256), 0, s,
                             reinterpret_cast<const uint8_t*>(in.vertices), in.vertex_stride, nv, out.vertices);
  if (nt) hipLaunchKernelGGL(copy_indices_kernel, dim3(blocks(nt)), dim3(256), 0, s,
                             reinterpret_cast<const uint8_t*>(in.indices), in.index_stride, nt, nv, out.indices, err);
  RTD_TRY(hipGetLastError());
  uint32_t h_err = 0;
  RTD_TRY(hipMemcpyAsync(&h_err, err, 4, hipMemcpyDeviceToHost, s));
  RTD_TRY(hipStreamSynchronize(s));
  if (h_err) {
    index_error = true;
    return hipSuccess;
  }
  out.refit_levels.assign(1, 0);
  if (nt == 0) return hipSuccess;
  // 2. validity and centres
  uint8_t* valid = nullptr;
  float4* centre = nullptr;
  RTD_TRY(tmp.alloc(&valid, nt));
  RTD_TRY(tmp.alloc(&centre, nt));
  hipLaunchKernelGGL(prep_kernel, dim3(blocks(nt)), dim3(256), 0, s, out.vertices, out.indices, nt, valid, centre);
  // 3. valid ids
  uint32_t *ids = nullptr, *n_sel = nullptr;
  RTD_TRY(tmp.alloc(&ids, nt));
  RTD_TRY(tmp.alloc(&n_sel, 1));
  hipcub::CountingInputIterator<uint32_t> counting(0);
  size_t bytes = 0;
  RTD_TRY(hipcub::DeviceSelect::Flagged(nullptr, bytes, counting, valid, ids, n_sel, (int)nt, s));
  void* scratch = nullptr;
  RTD_TRY(tmp.alloc(reinterpret_cast<uint8_t**>(&scratch), bytes));
  RTD_TRY(hipcub::DeviceSelect::Flagged(scratch, bytes, counting, valid, ids, n_sel, (int)nt, s));
  uint32_t m = 0;
  RTD_TRY(hipMemcpyAsync(&m, n_sel, 4, hipMemcpyDeviceToHost, s));
  RTD_TRY(hipStreamSynchronize(s));
  out.tri_count = m;
  if (m == 0) return hipSuccess;
  // 4. centre bounds
  uint32_t* bounds = nullptr;
  RTD_TRY(tmp.alloc(&bounds, 6));
  uint32_t init[6] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u, 0u};
  RTD_TRY(hipMemcpyAsync(bounds, init, sizeof(init), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(centre_bounds_kernel, dim3(blocks(m)), dim3(256), 0, s, centre, ids, m, bounds);
  // 5. Morton keys and the sort
  uint64_t *keys = nullptr, *keys_sorted = nullptr;
  uint32_t* ids_sorted = nullptr;
  RTD_TRY(tmp.alloc(&keys, m));
  RTD_TRY(tmp.alloc(&keys_sorted, m));
  RTD_TRY(tmp.alloc(&ids_sorted, m));
  hipLaunchKernelGGL(morton_kernel, dim3(blocks(m)), dim3(256), 0, s, centre, ids, m, bounds, keys);
  bytes = 0;
  RTD_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, keys, keys_sorted, ids, ids_sorted, (int)m, 0, 62, s));
  void* sort_tmp = nullptr;
  RTD_TRY(tmp.alloc(reinterpret_cast<uint8_t**>(&sort_tmp), bytes));
  RTD_TRY(hipcub::DeviceRadixSort::SortPairs(sort_tmp, bytes, keys, keys_sorted, ids, ids_sorted, (int)m, 0, 62, s));
  // 6. PLOC
  const uint32_t nb = 2 * m - 1;
  uint32_t *left = nullptr, *right = nullptr, *count = nullptr, *perm = nullptr;
  uint32_t *cl_a = nullptr, *cl_b = nullptr, *nn = nullptr, *flag = nullptr, *off = nullptr, *n_keep = nullptr;
  uint8_t* keep_flag = nullptr;
  float* box = nullptr;
  RTD_TRY(tmp.alloc(&left, m));
  RTD_TRY(tmp.alloc(&right, m));
  RTD_TRY(tmp.alloc(&count, nb));
  RTD_TRY(tmp.alloc(&perm, m));
  RTD_TRY(tmp.alloc(&cl_a, m));
  RTD_TRY(tmp.alloc(&cl_b, m));
  RTD_TRY(tmp.alloc(&nn, m));
  RTD_TRY(tmp.alloc(&flag, m));
  RTD_TRY(tmp.alloc(&off, m));
  RTD_TRY(tmp.alloc(&n_keep, 1));
  RTD_TRY(tmp.alloc(&keep_flag, m));
  RTD_TRY(tmp.alloc(&box, (size_t)nb * 6));
  hipLaunchKernelGGL(leaf_boxes_kernel, dim3(blocks(m)), dim3(256), 0, s, out.vertices, out.indices, ids_sorted, m,
                     box, count, cl_a);
  RTD_TRY(hipGetLastError());
  size_t scan_bytes = 0, sel_bytes = 0;
  RTD_TRY(hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, flag, off, (int)m, s));
  RTD_TRY(hipcub::DeviceSelect::Flagged(nullptr, sel_bytes, cl_b, keep_flag, cl_a, n_keep, (int)m, s));
  const size_t ploc_bytes = std::max(scan_bytes, sel_bytes);
  void* ploc_tmp = nullptr;
  RTD_TRY(tmp.alloc(reinterpret_cast<uint8_t**>(&ploc_tmp), ploc_bytes));
  // the n clusters are cl_a[0, n); internal ids below `top` + 1 are still free
  uint32_t n = m, made = 0;
  int force = 0;
  while (n > 1) {
    const uint32_t top = m - 2 - made;  // id of this pass's first new node
    if (!force) hipLaunchKernelGGL(ploc_nn_kernel, dim3(blocks(n)), dim3(256), 0, s, cl_a, n, box, nn);
    hipLaunchKernelGGL(ploc_flag_kernel, dim3(blocks(n)), dim3(256), 0, s, nn, n, force, flag);
    size_t b1 = ploc_bytes;
    RTD_TRY(hipcub::DeviceScan::ExclusiveSum(ploc_tmp, b1, flag, off, (int)n, s));
    hipLaunchKernelGGL(ploc_merge_kernel, dim3(blocks(n)), dim3(256), 0, s, cl_a, nn, n, force, off, top, left,
                       right, count, box, cl_b, keep_flag);
    size_t b2 = ploc_bytes;
    RTD_TRY(hipcub::DeviceSelect::Flagged(ploc_tmp, b2, cl_b, keep_flag, cl_a, n_keep, (int)n, s));
    RTD_TRY(hipGetLastError());
    uint32_t n_new = n;
    RTD_TRY(hipMemcpyAsync(&n_new, n_keep, 4, hipMemcpyDeviceToHost, s));
    RTD_TRY(hipStreamSynchronize(s));
    if (n_new > n) return hipErrorUnknown;  // cannot happen
    made += n - n_new;
    // a pass without a mutual pair (possible only through exact ties of both
    // area and hash) is followed by one that pairs (2k, 2k + 1)
    force = (n_new == n) ? 1 : 0;
    n = n_new;
  }
  if (made != m - 1) return hipErrorUnknown;  // m - 1 merges made ids m - 2 .. 0
  // 7. collapse, level by level; wide nodes of one level are numbered
  // consecutively, so the levels are index ranges
  const size_t fpn = 8 * (size_t)W;
  float* nodes_tmp = nullptr;
  RTD_TRY(tmp.alloc(&nodes_tmp, (size_t)m * fpn));  // at most m wide nodes
  Item *items_a = nullptr, *items_b = nullptr;
  uint32_t* counters = nullptr;  // node counter, n_out, leaf counter, max stack
  double* area_sum = nullptr;
  RTD_TRY(tmp.alloc(&items_a, m));
  RTD_TRY(tmp.alloc(&items_b, m));
  RTD_TRY(tmp.alloc(&counters, 4));
  RTD_TRY(tmp.alloc(&area_sum, 1));
  uint32_t cinit[4] = {1u, 0u, 0u, 0u};
  double zero = 0.0;
  Item root{0u, 0u, 0u, 0u};  // the binary root is internal node 0, or the only leaf when m == 1
  RTD_TRY(hipMemcpyAsync(counters, cinit, sizeof(cinit), hipMemcpyHostToDevice, s));
  RTD_TRY(hipMemcpyAsync(area_sum, &zero, sizeof(zero), hipMemcpyHostToDevice, s));
  RTD_TRY(hipMemcpyAsync(items_a, &root, sizeof(root), hipMemcpyHostToDevice, s));
  std::vector<uint32_t> level_begin{0u};
  uint32_t n_in = 1, node_count = 1;
  while (n_in > 0) {
    CollapseParams P{};
    P.left = left;
    P.right = right;
    P.count = count;
    P.perm = perm;
    P.box = box;
    P.m = (int)m;
    P.width = W;
    P.max_leaf = in.max_leaf;
    P.in = items_a;
    P.n_in = n_in;
    P.out = items_b;
    P.n_out = counters + 1;
    P.node_counter = counters;
    P.leaf_counter = counters + 2;
    P.max_stack = counters + 3;
    P.area_sum = area_sum;
    P.nodes = nodes_tmp;
    hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(256), 0, s, counters + 1, 1u, 0u);
    hipLaunchKernelGGL(collapse_kernel, dim3(blocks(n_in)), dim3(256), 0, s, P);
    RTD_TRY(hipGetLastError());
    uint32_t c[2];
    RTD_TRY(hipMemcpyAsync(c, counters, sizeof(c), hipMemcpyDeviceToHost, s));
    RTD_TRY(hipStreamSynchronize(s));
    level_begin.push_back(node_count);
    node_count = c[0];
    n_in = c[1];
    std::swap(items_a, items_b);
  }
  // 8. triangle records in the order the collapse gave them
  RTD_TRY(keep(out, &out.tris, m));
  hipLaunchKernelGGL(records_kernel, dim3(blocks(m)), dim3(256), 0, s, out.vertices, out.indices, ids_sorted, perm, m,
                     out.tris);
  RTD_TRY(hipGetLastError());
  // level_begin[l] .. level_begin[l+1] are the wide nodes of depth l+1
  uint32_t c[4];
  double area = 0.0;
  RTD_TRY(hipMemcpyAsync(c, counters, sizeof(c), hipMemcpyDeviceToHost, s));
  RTD_TRY(hipMemcpyAsync(&area, area_sum, sizeof(area), hipMemcpyDeviceToHost, s));
  float root_box[6];
  RTD_TRY(hipMemcpyAsync(root_box, box, sizeof(root_box), hipMemcpyDeviceToHost, s));
  RTD_TRY(hipStreamSynchronize(s));
  out.node_count = node_count;
  for (int a = 0; a < 6; ++a) out.bounds[a] = root_box[a];
  out.leaf_count = c[2];
  out.max_stack = std::max(c[3], 1u);
  out.max_depth = (uint32_t)level_begin.size() - 1;
  out.root = 0;
  double dx = (double)root_box[3] - root_box[0], dy = (double)root_box[4] - root_box[1],
         dz = (double)root_box[5] - root_box[2];
  double ra = 2.0 * (dx * dy + dy * dz + dz * dx);
  out.sah_cost = ra > 0.0 ? area / ra : 0.0;
  RTD_TRY(keep(out, &out.nodes, (size_t)node_count * fpn));
  RTD_TRY(hipMemcpyAsync(out.nodes, nodes_tmp, (size_t)node_count * fpn * sizeof(float), hipMemcpyDeviceToDevice, s));
  // refit order: deepest level first
  RTD_TRY(keep(out, &out.refit_nodes, node_count));
  uint32_t pos = 0;
  for (size_t l = level_begin.size() - 1; l-- > 0;) {
    uint32_t b = level_begin[l], e = level_begin[l + 1];
    if (e > b)
      hipLaunchKernelGGL(iota_kernel, dim3(blocks(e - b)), dim3(256), 0, s, out.refit_nodes + pos, b, e - b);
    pos += e - b;
    out.refit_levels.push_back(pos);
  }
  RTD_TRY(hipGetLastError());
  RTD_TRY(hipStreamSynchronize(s));
  return hipSuccess;
}

hipError_t relocate(float* nodes, uint32_t node_count, int width, uint32_t node_base, uint32_t tri_base,
                    hipStream_t s) {
  if (node_count == 0) return hipSuccess;
  hipLaunchKernelGGL(relocate_kernel, dim3(blocks((uint64_t)node_count * width)), dim3(256), 0, s, nodes, node_count,
                     width, node_base, tri_base);
  return hipGetLastError();
}

}  // namespace rtd
