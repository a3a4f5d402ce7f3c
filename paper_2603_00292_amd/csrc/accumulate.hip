// accumulate.hip -- conversion and reset of the integer accumulator rows
// (see accumulate.h).
#include "accumulate.h"

namespace rta {
namespace {

__global__ __launch_bounds__(256) void convert_kernel(uint32_t* expo, unsigned long long* sums,
                                                      uint32_t rows, uint32_t first, uint32_t count,
                                                      int layout, int shift0, float* out) {
  uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= count) return;
  uint32_t row = first + i;
  uint32_t e = expo[row];
  if (e == 0u) return;
  // the per-die partial sums, added exactly (two's complement addition is
  // associative, and the total fits)
  unsigned long long t[3] = {0ull, 0ull, 0ull};
#pragma unroll
  for (uint32_t k = 0; k < kCopies; ++k) {
    unsigned long long* s = sums + 4 * ((size_t)k * rows + row);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      t[c] += s[c];
      s[c] = 0ull;
    }
  }
  float v[3];
  if (e == kExpoNonFinite) {
    v[0] = v[1] = v[2] = __int_as_float(0x7fc00000);
  } else {
    int sh = shift0 - ((int)e - (int)kExpoBias);
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = (float)ldexp((double)(long long)t[c], -sh);
  }
  if (layout == 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c) out[3 * (size_t)i + c] += v[c];
  } else {
    uint32_t j = i >> 2, part = i & 3u;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      uint32_t k = 3 * part + c;
      if (k < 10) out[10 * (size_t)j + k] += v[c];
    }
  }
  expo[row] = 0u;
}

__global__ __launch_bounds__(256) void clear_kernel(uint32_t* expo, unsigned long long* sums, uint32_t count) {
  uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= count) return;
  expo[i] = 0u;
  for (uint32_t k = 0; k < kCopies; ++k) {
    unsigned long long* s = sums + 4 * ((size_t)k * count + i);
    s[0] = s[1] = s[2] = s[3] = 0ull;
  }
}

}  // namespace

hipError_t alloc(Rows& r, uint32_t count) {
  release(r);
  if (count == 0) return hipSuccess;
  const size_t nsum = (size_t)kCopies * 4 * count;
  hipError_t e = hipMalloc(&r.expo, count * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(&r.sums, nsum * sizeof(unsigned long long));
  if (e != hipSuccess) {
    release(r);
    return e;
  }
  r.count = count;
  return hipSuccess;
}

void release(Rows& r) {
  if (r.expo) (void)hipFree(r.expo);
  if (r.sums) (void)hipFree(r.sums);
  r = Rows();
}

hipError_t clear(const Rows& r, hipStream_t stream) {
  if (r.count == 0) return hipSuccess;
  uint32_t* expo = r.expo;
  unsigned long long* sums = r.sums;
  uint32_t count = r.count;
  void* args[] = {&expo, &sums, &count};
  return hipLaunchKernel(reinterpret_cast<const void*>(&clear_kernel), dim3((count + 255) / 256),
                         dim3(256), args, 0, stream);
}

hipError_t convert(const Rows& r, uint32_t first, uint32_t count, int layout, int shift0, float* out,
                   hipStream_t stream) {
  if (count == 0) return hipSuccess;
  if ((uint64_t)first + count > r.count) return hipErrorInvalidValue;
  uint32_t* expo = r.expo;
  unsigned long long* sums = r.sums;
  uint32_t rows = r.count;
  void* args[] = {&expo, &sums, &rows, &first, &count, &layout, &shift0, &out};
  return hipLaunchKernel(reinterpret_cast<const void*>(&convert_kernel), dim3((count + 255) / 256),
                         dim3(256), args, 0, stream);
}

}  // namespace rta

// ---------------------------------------------------------------------------
// vertex gradients without global atomics (see accumulate.h)
// ---------------------------------------------------------------------------
#include <algorithm>
#include <cfloat>
#include <climits>
#include <vector>

namespace rta {
namespace {

constexpr uint32_t kScanChunk = 2048;   // elements per workgroup of the scan

// per-tile histogram of the rays' buckets: counts[bucket * tiles + tile];
// counts the rays whose prim id is a triangle of the mesh
__global__ __launch_bounds__(1024) void hist_kernel(const uint32_t* hit_words, uint32_t n, uint32_t triangles,
                                                    uint32_t shift, uint32_t buckets, uint32_t tiles,
                                                    uint32_t* counts) {
  extern __shared__ uint32_t h[];
  for (uint32_t b = threadIdx.x; b < buckets; b += 1024) h[b] = 0u;
  __syncthreads();
  uint32_t base = blockIdx.x * kTile;
  uint32_t end = min(n, base + kTile);
  for (uint32_t i = base + threadIdx.x; i < end; i += 1024) {
    uint32_t k = hit_words[4 * (size_t)i + 1];
    if (k < triangles) atomicAdd(&h[k >> shift], 1u);
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < buckets; b += 1024) counts[(size_t)b * tiles + blockIdx.x] = h[b];
}

// exclusive scan of m elements in three launches: chunk sums, a scan of the
// sums (one workgroup), then each chunk scanned from its offset
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t o = (uint32_t)__shfl_up((int)v, d);
    if (lane >= (uint32_t)d) v += o;
  }
  return v;
}

// exclusive scan of one value per thread over a 256-thread workgroup; *total
// receives the sum
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* wsum, uint32_t* total) {
  uint32_t inc = wave_incl_scan(v);
  uint32_t w = threadIdx.x >> 6;
  if ((threadIdx.x & 63u) == 63u) wsum[w] = inc;
  __syncthreads();
  uint32_t off = 0, all = 0;
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k) {
    uint32_t x = wsum[k];
    off += (k < w) ? x : 0u;
    all += x;
  }
  __syncthreads();
  *total = all;
  return off + inc - v;
}

__global__ __launch_bounds__(256) void scan_reduce_kernel(const uint32_t* x, uint32_t m, uint32_t* partial) {
  __shared__ uint32_t wsum[4];
  uint32_t base = blockIdx.x * kScanChunk;
  uint32_t s = 0;
  for (uint32_t i = base + threadIdx.x; i < min(m, base + kScanChunk); i += 256) s += x[i];
  uint32_t total;
  (void)block_excl_scan(s, wsum, &total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void scan_partials_kernel(uint32_t* partial, uint32_t parts) {
  __shared__ uint32_t wsum[4];
  uint32_t carry = 0;
  for (uint32_t base = 0; base < parts; base += 256) {
    uint32_t i = base + threadIdx.x;
    uint32_t v = i < parts ? partial[i] : 0u;
    uint32_t total;
    uint32_t ex = block_excl_scan(v, wsum, &total);
    if (i < parts) partial[i] = carry + ex;
    carry += total;
  }
}

// scans chunk blockIdx.x in place from its offset (8 elements per thread);
// element m receives the grand total
__global__ __launch_bounds__(256) void scan_down_kernel(uint32_t* x, uint32_t m, const uint32_t* partial,
                                                        uint32_t parts) {
  __shared__ uint32_t wsum[4];
  uint32_t base = blockIdx.x * kScanChunk + threadIdx.x * 8;
  uint32_t v[8];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    v[k] = (base + k < m) ? x[base + k] : 0u;
    s += v[k];
  }
  uint32_t total;
  uint32_t run = partial[blockIdx.x] + block_excl_scan(s, wsum, &total);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (base + k < m) x[base + k] = run;
    run += v[k];
  }
  if (blockIdx.x + 1 == parts && threadIdx.x == 0) x[m] = partial[blockIdx.x] + total;
}

// one workgroup per bucket: exact corner sums of its rays (TB triangles)
template <uint32_t TB>
__global__ __launch_bounds__(512) void corner_kernel(const RayRec* rec, const uint32_t* offsets, uint32_t tiles,
                                                     uint32_t triangles, int shift0, double* corner) {
  constexpr uint32_t R = 3 * TB;   // rows (triangle, corner)
  __shared__ unsigned long long sum[3 * R];
  __shared__ int expo[R];
  const uint32_t b = blockIdx.x;
  for (uint32_t r = threadIdx.x; r < R; r += 512) {
    expo[r] = INT_MIN;
    sum[3 * r] = sum[3 * r + 1] = sum[3 * r + 2] = 0ull;
  }
  __syncthreads();
  const uint32_t lo = offsets[(size_t)b * tiles], hi = offsets[(size_t)(b + 1) * tiles];
  const uint32_t t0 = b * TB;
  // pass 1: each row's largest binary exponent
  for (uint32_t j = lo + threadIdx.x; j < hi; j += 512) {
    RayRec q = rec[j];
    uint32_t tl = q.prim - t0;
    double w[3] = {1.0 - q.u - q.v, q.u, q.v};
    // bounds every component of -w_k lambda; a NaN or inf makes the row NaN
    double m = fabs(q.lx) + fabs(q.ly) + fabs(q.lz);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double a = fabs(w[k]) * m;
      if (a != 0.0) atomicMax(&expo[3 * tl + k], a <= DBL_MAX ? ilogb(a) : INT_MAX);
    }
  }
  __syncthreads();
  // pass 2: integer sums at each row's scale
  for (uint32_t j = lo + threadIdx.x; j < hi; j += 512) {
    RayRec q = rec[j];
    uint32_t tl = q.prim - t0;
    double w[3] = {1.0 - q.u - q.v, q.u, q.v};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      int e = expo[3 * tl + k];
      if (e == INT_MIN || e == INT_MAX) continue;
      int sh = shift0 - e;
      double c[3] = {-w[k] * q.lx, -w[k] * q.ly, -w[k] * q.lz};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        long long v = __double2ll_rn(ldexp(c[d], sh));
        if (v) atomicAdd(&sum[3 * (3 * tl + k) + d], (unsigned long long)v);
      }
    }
  }
  __syncthreads();
  for (uint32_t r = threadIdx.x; r < R; r += 512) {
    uint32_t t = t0 + r / 3;
    if (t >= triangles) continue;
    int e = expo[r];
    double* o = corner + 9 * (size_t)t + 3 * (r % 3);
    for (int d = 0; d < 3; ++d) {
      double v = 0.0;
      if (e == INT_MAX) v = __longlong_as_double(0x7ff8000000000000ll);
      else if (e != INT_MIN) v = ldexp((double)(long long)sum[3 * r + d], e - shift0);
      o[d] = v;
    }
  }
}

__global__ __launch_bounds__(256) void vertex_kernel(const uint32_t* csr_off, const uint32_t* csr_ent,
                                                     const double* corner, uint32_t vertices, float* out) {
  uint32_t v = blockIdx.x * 256u + threadIdx.x;
  if (v >= vertices) return;
  double x = 0.0, y = 0.0, z = 0.0;
  for (uint32_t j = csr_off[v]; j < csr_off[v + 1]; ++j) {
    uint32_t e = csr_ent[j];
    const double* c = corner + 9 * (size_t)(e >> 2) + 3 * (e & 3u);
    x += c[0];
    y += c[1];
    z += c[2];
  }
  if (x == 0.0 && y == 0.0 && z == 0.0) return;
  out[3 * (size_t)v + 0] += (float)x;
  out[3 * (size_t)v + 1] += (float)y;
  out[3 * (size_t)v + 2] += (float)z;
}

template <typename T>
hipError_t grow(T** p, size_t* cap, size_t n, hipStream_t s) {
  if (n <= *cap && *p) return hipSuccess;
  size_t c = std::max<size_t>(std::max(n, 2 * *cap), 4096);
  if (*p) (void)hipFreeAsync(*p, s);
  *p = nullptr;
  *cap = 0;
  hipError_t e = hipMallocAsync(reinterpret_cast<void**>(p), c * sizeof(T), s);
  if (e == hipSuccess) *cap = c;
  return e;
}

}  // namespace

hipError_t gather_build(Gather& g, const uint32_t* I, uint32_t vertices, uint32_t triangles) {
  gather_release(g);
  uint32_t shift = bucket_shift(triangles);
  if (shift == 0) return hipErrorInvalidValue;
  std::vector<uint32_t> off((size_t)vertices + 1, 0u), ent(3 * (size_t)triangles);
  for (size_t t = 0; t < triangles; ++t)
    for (int k = 0; k < 3; ++k) off[I[3 * t + k] + 1]++;
  for (size_t v = 0; v < vertices; ++v) off[v + 1] += off[v];
  std::vector<uint32_t> fill(off.begin(), off.end() - 1);
  for (size_t t = 0; t < triangles; ++t)
    for (uint32_t k = 0; k < 3; ++k) ent[fill[I[3 * t + k]]++] = (uint32_t)(t << 2) | k;
  hipError_t e = hipMalloc(&g.csr_off, off.size() * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(&g.csr_ent, std::max<size_t>(ent.size(), 1) * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(&g.corner, std::max<size_t>(9 * (size_t)triangles, 1) * sizeof(double));
  if (e == hipSuccess) e = hipMemcpy(g.csr_off, off.data(), off.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && !ent.empty())
    e = hipMemcpy(g.csr_ent, ent.data(), ent.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    gather_release(g);
    return e;
  }
  g.vertices = vertices;
  g.triangles = triangles;
  g.shift = shift;
  g.buckets = (uint32_t)(((uint64_t)triangles + (1u << shift) - 1) >> shift);
  return hipSuccess;
}

void gather_release(Gather& g) {
  void* ps[] = {g.csr_off, g.csr_ent, g.corner};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  g = Gather();
}

hipError_t sort_reserve(SortBuf& b, const Gather& g, size_t n, hipStream_t s) {
  size_t tiles = (n + kTile - 1) / kTile;
  size_t m = (size_t)g.buckets * tiles;
  size_t parts = (m + kScanChunk - 1) / kScanChunk;
  hipError_t e = grow(&b.rec, &b.cap, n, s);
  if (e == hipSuccess) e = grow(&b.counts, &b.count_cap, m + 1, s);
  if (e == hipSuccess) e = grow(&b.partial, &b.partial_cap, std::max<size_t>(parts, 1), s);
  return e;
}

void sort_release(SortBuf& b) {
  void* ps[] = {b.rec, b.counts, b.partial};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  b = SortBuf();
}

hipError_t bucket_rays(const Gather& g, SortBuf& b, const uint32_t* hit_words, uint32_t n, hipStream_t s,
                       Bucketing* out) {
  uint32_t buckets = g.buckets, shift = g.shift, tris = g.triangles;
  uint32_t tiles = (n + kTile - 1) / kTile;
  uint32_t m = buckets * tiles;
  uint32_t parts = (m + kScanChunk - 1) / kScanChunk;
  uint32_t* counts = b.counts;
  uint32_t* partial = b.partial;
  *out = Bucketing{counts, tiles, buckets, shift, b.rec};
  if (m == 0) return hipSuccess;   // no triangles: no ray has a bucket
  void* a1[] = {&hit_words, &n, &tris, &shift, &buckets, &tiles, &counts};
  hipError_t e = hipLaunchKernel(reinterpret_cast<const void*>(&hist_kernel), dim3(tiles), dim3(1024), a1,
                                 buckets * sizeof(uint32_t), s);
  if (e != hipSuccess) return e;
  void* a2[] = {&counts, &m, &partial};
  e = hipLaunchKernel(reinterpret_cast<const void*>(&scan_reduce_kernel), dim3(parts), dim3(256), a2, 0, s);
  if (e != hipSuccess) return e;
  void* a3[] = {&partial, &parts};
  e = hipLaunchKernel(reinterpret_cast<const void*>(&scan_partials_kernel), dim3(1), dim3(256), a3, 0, s);
  if (e != hipSuccess) return e;
  void* a4[] = {&counts, &m, &partial, &parts};
  return hipLaunchKernel(reinterpret_cast<const void*>(&scan_down_kernel), dim3(parts), dim3(256), a4, 0, s);
}

hipError_t gather_vertices(Gather& g, SortBuf& b, uint32_t n, float* out, hipStream_t s) {
  if (n == 0 || g.buckets == 0 || g.vertices == 0) return hipSuccess;
  uint32_t tiles = (n + kTile - 1) / kTile;
  RayRec* rec = b.rec;
  uint32_t* counts = b.counts;
  uint32_t tris = g.triangles;
  int shift0 = shift0_for(n);
  double* corner = g.corner;
  void* a6[] = {&rec, &counts, &tiles, &tris, &shift0, &corner};
  const void* k = g.shift == 8   ? reinterpret_cast<const void*>(&corner_kernel<256>)
                  : g.shift == 9 ? reinterpret_cast<const void*>(&corner_kernel<512>)
                                 : reinterpret_cast<const void*>(&corner_kernel<1024>);
  hipError_t e = hipLaunchKernel(k, dim3(g.buckets), dim3(512), a6, 0, s);
  if (e != hipSuccess) return e;
  uint32_t* off = g.csr_off;
  uint32_t* ent = g.csr_ent;
  uint32_t verts = g.vertices;
  void* a7[] = {&off, &ent, &corner, &verts, &out};
  return hipLaunchKernel(reinterpret_cast<const void*>(&vertex_kernel), dim3((verts + 255) / 256), dim3(256), a7, 0, s);
}

}  // namespace rta
