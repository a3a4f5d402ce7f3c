// accumulate.hip -- conversion and reset of the integer accumulator rows
// (see accumulate.h).
#include "accumulate.h"
#include "rt_alloc.h"

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
  hipError_t e = rt_malloc(&r.expo, count * sizeof(uint32_t));
  if (e == hipSuccess) e = rt_malloc(&r.sums, nsum * sizeof(unsigned long long));
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

// per-tile histogram of the rays' buckets: counts[tile * buckets + bucket]
// (bucket = key >> shift); rays without a key are not counted
__global__ __launch_bounds__(1024) void hist_kernel(KeySource keys, uint32_t n, uint32_t shift, uint32_t buckets,
                                                    uint32_t* counts) {
  extern __shared__ uint32_t h[];
  for (uint32_t b = threadIdx.x; b < buckets; b += 1024) h[b] = 0u;
  __syncthreads();
  uint32_t base = blockIdx.x * kTile;
  uint32_t end = min(n, base + kTile);
  for (uint32_t i = base + threadIdx.x; i < end; i += 1024) {
    uint32_t k = ray_key(keys, i);
    if (k != kNoKey) atomicAdd(&h[k >> shift], 1u);
  }
  __syncthreads();
  uint32_t* row = counts + (size_t)blockIdx.x * buckets;
  for (uint32_t b = threadIdx.x; b < buckets; b += 1024) row[b] = h[b];
}

// Column scan: workgroup g owns buckets 64 g .. 64 g + 63 (one per lane) and
// splits the tiles over its 16 waves; each bucket's tile counts become the
// offsets of the tiles inside the bucket, and its total goes to totals[]
// (the adjoint kernel scans the totals into bucket starts).
__global__ __launch_bounds__(1024) void colscan_kernel(uint32_t* counts, uint32_t tiles, uint32_t buckets,
                                                       uint32_t* totals) {
  __shared__ uint32_t part[16][64];
  const uint32_t l = threadIdx.x & 63u, w = threadIdx.x >> 6;
  const uint32_t b = blockIdx.x * 64u + l;
  const uint32_t per = (tiles + 15u) / 16u;
  const uint32_t t0 = min(tiles, w * per), t1 = min(tiles, t0 + per);
  // the loads of a block of kU tiles are issued together; the first block
  // stays in registers for the second pass (all of it when tiles <= 16 kU)
  constexpr uint32_t kU = 16;
  uint32_t first[kU];
  uint32_t s = 0;
#pragma unroll
  for (uint32_t k = 0; k < kU; ++k) {
    first[k] = (b < buckets && t0 + k < t1) ? counts[(size_t)(t0 + k) * buckets + b] : 0u;
    s += first[k];
  }
  if (b < buckets)
    for (uint32_t t = t0 + kU; t < t1; t += kU) {
      uint32_t v[kU];
#pragma unroll
      for (uint32_t k = 0; k < kU; ++k) v[k] = t + k < t1 ? counts[(size_t)(t + k) * buckets + b] : 0u;
#pragma unroll
      for (uint32_t k = 0; k < kU; ++k) s += v[k];
    }
  part[w][l] = s;
  __syncthreads();
  uint32_t run = 0, total = 0;
#pragma unroll
  for (uint32_t k = 0; k < 16; ++k) {
    uint32_t x = part[k][l];
    run += k < w ? x : 0u;
    total += x;
  }
  if (b < buckets) {
#pragma unroll
    for (uint32_t k = 0; k < kU; ++k)
      if (t0 + k < t1) {
        counts[(size_t)(t0 + k) * buckets + b] = run;
        run += first[k];
      }
    for (uint32_t t = t0 + kU; t < t1; t += kU) {
      uint32_t v[kU];
#pragma unroll
      for (uint32_t k = 0; k < kU; ++k) v[k] = t + k < t1 ? counts[(size_t)(t + k) * buckets + b] : 0u;
#pragma unroll
      for (uint32_t k = 0; k < kU; ++k)
        if (t + k < t1) {
          counts[(size_t)(t + k) * buckets + b] = run;
          run += v[k];
        }
    }
    if (w == 0) totals[b] = total;
  }
}

// one workgroup per bucket: exact corner sums of its rays (TB triangles).
// A thread's first kCache records stay in registers between the two passes.
template <uint32_t TB>
__global__ __launch_bounds__(512) void corner_kernel(const RayRec* rec, const uint32_t* bucket_base,
                                                     uint32_t triangles, int shift0, double* corner) {
  constexpr uint32_t R = 3 * TB;   // rows (triangle, corner)
  constexpr uint32_t kCache = 4;
  __shared__ unsigned long long sum[3 * R];
  __shared__ int expo[R];
  const uint32_t b = blockIdx.x;
  for (uint32_t r = threadIdx.x; r < R; r += 512) {
    expo[r] = INT_MIN;
    sum[3 * r] = sum[3 * r + 1] = sum[3 * r + 2] = 0ull;
  }
  const uint32_t lo = bucket_base[b], hi = bucket_base[b + 1];
  const uint32_t t0 = b * TB;
  RayRec cache[kCache];
#pragma unroll
  for (uint32_t k = 0; k < kCache; ++k) {
    uint32_t j = lo + threadIdx.x + k * 512;
    if (j < hi) cache[k] = rec[j];
  }
  __syncthreads();
  // pass 1: each row's largest binary exponent
  auto bound = [&](const RayRec& q) {
    uint32_t tl = q.prim - t0;
    double w[3] = {1.0 - q.u - q.v, q.u, q.v};
    // bounds every component of -w_k lambda; a NaN or inf makes the row NaN
    double m = fabs(q.lx) + fabs(q.ly) + fabs(q.lz);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double a = fabs(w[k]) * m;
      if (a != 0.0) atomicMax(&expo[3 * tl + k], a <= DBL_MAX ? ilogb(a) : INT_MAX);
    }
  };
#pragma unroll
  for (uint32_t k = 0; k < kCache; ++k)
    if (lo + threadIdx.x + k * 512 < hi) bound(cache[k]);
  for (uint32_t j = lo + threadIdx.x + kCache * 512; j < hi; j += 512) bound(rec[j]);
  __syncthreads();
  // pass 2: integer sums at each row's scale
  auto add = [&](const RayRec& q) {
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
  };
#pragma unroll
  for (uint32_t k = 0; k < kCache; ++k)
    if (lo + threadIdx.x + k * 512 < hi) add(cache[k]);
  for (uint32_t j = lo + threadIdx.x + kCache * 512; j < hi; j += 512) add(rec[j]);
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

// every triangle's vertices, in index order, 9 floats per triangle
__global__ __launch_bounds__(256) void tri_vertices_kernel(const uint32_t* I, const float* V, uint32_t triangles,
                                                           float* out) {
  uint32_t t = blockIdx.x * 256u + threadIdx.x;
  if (t >= triangles) return;
  float* o = out + 9 * (size_t)t;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float* v = V + 3 * (size_t)I[3 * (size_t)t + k];
    o[3 * k] = v[0];
    o[3 * k + 1] = v[1];
    o[3 * k + 2] = v[2];
  }
}

// each vertex: its corner values added in list order (the loads of up to
// eight entries issued together; the sum order is the list order)
__global__ __launch_bounds__(256) void vertex_kernel(const uint32_t* csr_off, const uint32_t* csr_ent,
                                                     const double* corner, uint32_t vertices, float* out) {
  uint32_t v = blockIdx.x * 256u + threadIdx.x;
  if (v >= vertices) return;
  constexpr uint32_t U = 8;
  double x = 0.0, y = 0.0, z = 0.0;
  const uint32_t j1 = csr_off[v + 1];
  for (uint32_t j = csr_off[v]; j < j1; j += U) {
    uint32_t e[U];
#pragma unroll
    for (uint32_t k = 0; k < U; ++k) e[k] = j + k < j1 ? csr_ent[j + k] : 0u;
    double c[U][3];
#pragma unroll
    for (uint32_t k = 0; k < U; ++k)
      if (j + k < j1) {
        const double* p = corner + 9 * (size_t)(e[k] >> 2) + 3 * (e[k] & 3u);
        c[k][0] = p[0];
        c[k][1] = p[1];
        c[k][2] = p[2];
      }
#pragma unroll
    for (uint32_t k = 0; k < U; ++k)
      if (j + k < j1) {
        x += c[k][0];
        y += c[k][1];
        z += c[k][2];
      }
  }
  if (x == 0.0 && y == 0.0 && z == 0.0) return;
  out[3 * (size_t)v + 0] += (float)x;
  out[3 * (size_t)v + 1] += (float)y;
  out[3 * (size_t)v + 2] += (float)z;
}

// one workgroup per instance: the exact row sums of its rays' frame
// derivatives (rows: S xyz; q xyz; q w, T x, T y; T z), as the atomic rows
// form them: per row the largest binary exponent of a contribution's
// largest component (a non-finite component makes the row NaN), then the
// components rounded to integers at that scale and summed in 64 bits.
// For the frame world = T + R(qh) (S x), qh = q / |q| = (v, w), with the
// object hit point p, a = S p and the world-space lambda:
//   dL/dT = -lambda,   dL/dS_j = -(R^T lambda)_j p_j,
//   dL/dqh: w-part -2 lambda.(v x a),
//           v-part -2 [w (a x lambda) + (v x a) x lambda + a x (lambda x v)],
//   dL/dq = (dL/dqh - qh (qh . dL/dqh)) / |q|.
__device__ __forceinline__ void cross3d(double ax, double ay, double az, double bx, double by, double bz,
                                        double& cx, double& cy, double& cz) {
  cx = ay * bz - az * by;
  cy = az * bx - ax * bz;
  cz = ax * by - ay * bx;
}

__global__ __launch_bounds__(256) void frame_kernel(const FrameRec* rec, const uint32_t* bucket_base,
                                                    const float* srt, int shift0, float* out) {
  const uint32_t j = blockIdx.x;
  const uint32_t lo = bucket_base[j], hi = bucket_base[j + 1];
  if (lo == hi) return;
  const float* f = srt + 10 * (size_t)j;
  const double sx = f[0], sy = f[1], sz = f[2];
  double qx = f[3], qy = f[4], qz = f[5], qw = f[6];
  const double qn = sqrt(qx * qx + qy * qy + qz * qz + qw * qw);
  const double iq = 1.0 / qn;
  qx *= iq;
  qy *= iq;
  qz *= iq;
  qw *= iq;
  auto rows = [&](const FrameRec& q, double (&c)[4][3]) {
    const double lx = q.lx, ly = q.ly, lz = q.lz, px = q.px, py = q.py, pz = q.pz;
    const double ax = sx * px, ay = sy * py, az = sz * pz;
    double cx, cy, cz, ex, ey, ez;
    cross3d(qx, qy, qz, lx, ly, lz, cx, cy, cz);
    cross3d(qx, qy, qz, cx, cy, cz, ex, ey, ez);
    const double rlx = lx - 2.0 * qw * cx + 2.0 * ex;
    const double rly = ly - 2.0 * qw * cy + 2.0 * ey;
    const double rlz = lz - 2.0 * qw * cz + 2.0 * ez;
    double vax, vay, vaz;
    cross3d(qx, qy, qz, ax, ay, az, vax, vay, vaz);
    const double gqw = -2.0 * (lx * vax + ly * vay + lz * vaz);
    double t1x, t1y, t1z, t2x, t2y, t2z, lvx, lvy, lvz, t3x, t3y, t3z;
    cross3d(ax, ay, az, lx, ly, lz, t1x, t1y, t1z);
    cross3d(vax, vay, vaz, lx, ly, lz, t2x, t2y, t2z);
    cross3d(lx, ly, lz, qx, qy, qz, lvx, lvy, lvz);
    cross3d(ax, ay, az, lvx, lvy, lvz, t3x, t3y, t3z);
    const double gqx = -2.0 * (qw * t1x + t2x + t3x);
    const double gqy = -2.0 * (qw * t1y + t2y + t3y);
    const double gqz = -2.0 * (qw * t1z + t2z + t3z);
    const double radial = qx * gqx + qy * gqy + qz * gqz + qw * gqw;
    c[0][0] = -rlx * px;
    c[0][1] = -rly * py;
    c[0][2] = -rlz * pz;
    c[1][0] = (gqx - qx * radial) * iq;
    c[1][1] = (gqy - qy * radial) * iq;
    c[1][2] = (gqz - qz * radial) * iq;
    c[2][0] = (gqw - qw * radial) * iq;
    c[2][1] = -lx;
    c[2][2] = -ly;
    c[3][0] = -lz;
    c[3][1] = 0.0;
    c[3][2] = 0.0;
  };
  __shared__ int se[4][4];
  __shared__ unsigned long long ss[4][12];
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  // pass 1: each row's exponent (INT_MIN: nothing added, INT_MAX: not finite)
  int e[4] = {INT_MIN, INT_MIN, INT_MIN, INT_MIN};
  for (uint32_t k = lo + threadIdx.x; k < hi; k += 256) {
    double c[4][3];
    rows(rec[k], c);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      bool finite = isfinite(c[r][0]) && isfinite(c[r][1]) && isfinite(c[r][2]);
      double m = fmax(fabs(c[r][0]), fmax(fabs(c[r][1]), fabs(c[r][2])));
      if (!finite) e[r] = INT_MAX;
      else if (m != 0.0) e[r] = max(e[r], ilogb(m));
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    for (int d = 32; d >= 1; d >>= 1) e[r] = max(e[r], __shfl_xor(e[r], d));
    if (lane == 0) se[w][r] = e[r];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r) e[r] = max(max(se[0][r], se[1][r]), max(se[2][r], se[3][r]));
  // pass 2: integer sums at each row's scale
  unsigned long long acc[4][3] = {};
  for (uint32_t k = lo + threadIdx.x; k < hi; k += 256) {
    double c[4][3];
    rows(rec[k], c);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (e[r] == INT_MIN || e[r] == INT_MAX) continue;
      const int sh = shift0 - e[r];
#pragma unroll
      for (int d = 0; d < 3; ++d) acc[r][d] += (unsigned long long)__double2ll_rn(ldexp(c[r][d], sh));
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      unsigned long long v = acc[r][d];
      for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
      if (lane == 0) ss[w][3 * r + d] = v;
    }
  __syncthreads();
  if (threadIdx.x < 10) {
    const int k = (int)threadIdx.x, r = k / 3;
    if (e[r] == INT_MIN) return;
    float v = __int_as_float(0x7fc00000);
    if (e[r] != INT_MAX) {
      unsigned long long t = ss[0][k] + ss[1][k] + ss[2][k] + ss[3][k];
      v = (float)ldexp((double)(long long)t, e[r] - shift0);
    }
    out[10 * (size_t)j + k] += v;
  }
}

template <typename T>
hipError_t grow(T** p, size_t* cap, size_t n, hipStream_t s) {
  if (n <= *cap && *p) return hipSuccess;
  size_t c = std::max<size_t>(std::max(n, 2 * *cap), 4096);
  if (*p) (void)hipFreeAsync(*p, s);
  *p = nullptr;
  *cap = 0;
  hipError_t e = rt_malloc_async(reinterpret_cast<void**>(p), c * sizeof(T), s);
  if (e == hipSuccess) *cap = c;
  return e;
}

}  // namespace

hipError_t gather_build_multi(Gather& g, const uint32_t* const* I, const uint32_t* vertex_counts,
                              const uint32_t* triangle_counts, uint32_t meshes, const uint32_t* inst_mesh,
                              uint32_t instances, uint32_t min_shift) {
  gather_release(g);
  uint64_t nv = 0, nt = 0;
  std::vector<uint32_t> vbase(meshes), tbase((size_t)meshes + 1);
  for (uint32_t m = 0; m < meshes; ++m) {
    vbase[m] = (uint32_t)nv;
    tbase[m] = (uint32_t)nt;
    nv += vertex_counts[m];
    nt += triangle_counts[m];
  }
  if (nv >= 0xFFFFFFFFull || nt >= (1ull << 30)) return hipErrorInvalidValue;
  tbase[meshes] = (uint32_t)nt;
  const uint32_t vertices = (uint32_t)nv, triangles = (uint32_t)nt;
  uint32_t shift = bucket_shift(triangles, min_shift);
  if (shift == 0) return hipErrorInvalidValue;
  // counting sort of the (triangle, corner) entries by global vertex
  std::vector<uint32_t> off((size_t)vertices + 1, 0u), ent(3 * (size_t)triangles);
  for (uint32_t m = 0; m < meshes; ++m)
    for (size_t t = 0; t < triangle_counts[m]; ++t)
      for (int k = 0; k < 3; ++k) off[vbase[m] + I[m][3 * t + k] + 1]++;
  for (size_t v = 0; v < vertices; ++v) off[v + 1] += off[v];
  std::vector<uint32_t> fill(off.begin(), off.end() - 1);
  for (uint32_t m = 0; m < meshes; ++m)
    for (size_t t = 0; t < triangle_counts[m]; ++t)
      for (uint32_t k = 0; k < 3; ++k)
        ent[fill[vbase[m] + I[m][3 * t + k]]++] = (uint32_t)((tbase[m] + t) << 2) | k;
  hipError_t e = rt_malloc(&g.csr_off, off.size() * sizeof(uint32_t));
  if (e == hipSuccess) e = rt_malloc(&g.csr_ent, std::max<size_t>(ent.size(), 1) * sizeof(uint32_t));
  if (e == hipSuccess) e = rt_malloc(&g.corner, std::max<size_t>(9 * (size_t)triangles, 1) * sizeof(double));
  if (e == hipSuccess) e = rt_malloc(&g.tri_vertices, std::max<size_t>(9 * (size_t)triangles, 1) * sizeof(float));
  std::vector<uint2> it(instances);
  for (uint32_t j = 0; j < instances; ++j) {
    uint32_t m = inst_mesh[j] < meshes ? inst_mesh[j] : 0u;
    it[j] = make_uint2(tbase[m], inst_mesh[j] < meshes ? triangle_counts[m] : 0u);
  }
  if (e == hipSuccess && instances > 0) e = rt_malloc(&g.inst_tris, (size_t)instances * sizeof(uint2));
  if (e == hipSuccess) e = hipMemcpy(g.csr_off, off.data(), off.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && !ent.empty())
    e = hipMemcpy(g.csr_ent, ent.data(), ent.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && instances > 0)
    e = hipMemcpy(g.inst_tris, it.data(), (size_t)instances * sizeof(uint2), hipMemcpyHostToDevice);
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

hipError_t gather_build(Gather& g, const uint32_t* I, uint32_t vertices, uint32_t triangles) {
  return gather_build_multi(g, &I, &vertices, &triangles, 1, nullptr, 0, 8);
}

hipError_t gather_tri_vertices(Gather& g, const uint32_t* indices, const float* vertices, uint32_t triangles,
                               uint32_t first, hipStream_t s) {
  if (triangles == 0) return hipSuccess;
  if ((uint64_t)first + triangles > g.triangles) return hipErrorInvalidValue;
  float* out = g.tri_vertices + 9 * (size_t)first;
  void* a[] = {&indices, &vertices, &triangles, &out};
  return hipLaunchKernel(reinterpret_cast<const void*>(&tri_vertices_kernel), dim3((triangles + 255) / 256),
                         dim3(256), a, 0, s);
}

void gather_release(Gather& g) {
  void* ps[] = {g.csr_off, g.csr_ent, g.corner, g.tri_vertices, g.inst_tris};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  g = Gather();
}

hipError_t sort_reserve(SortBuf& b, uint32_t buckets, size_t n, hipStream_t s) {
  size_t tiles = (n + kTile - 1) / kTile;
  size_t m = (size_t)buckets * tiles;
  hipError_t e = grow(&b.rec, &b.cap, n, s);
  if (e == hipSuccess) e = grow(&b.counts, &b.count_cap, std::max<size_t>(m, 1), s);
  if (e == hipSuccess) e = grow(&b.scan, &b.scan_cap, 2 * (size_t)buckets + 1, s);
  return e;
}

void sort_release(SortBuf& b) {
  void* ps[] = {b.rec, b.counts, b.scan};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  b = SortBuf();
}

hipError_t bucket_rays(const KeySource& keys, uint32_t buckets, uint32_t shift, SortBuf& b, uint32_t n,
                       hipStream_t s, Bucketing* out) {
  uint32_t tiles = (n + kTile - 1) / kTile;
  uint32_t* counts = b.counts;
  uint32_t* totals = b.scan;
  uint32_t* base = b.scan + buckets;
  *out = Bucketing{counts, totals, base, tiles, buckets, shift, b.rec};
  if (buckets == 0 || tiles == 0) return hipSuccess;   // no keys or no rays: no ray has a bucket
  KeySource k = keys;
  void* a1[] = {&k, &n, &shift, &buckets, &counts};
  hipError_t e = hipLaunchKernel(reinterpret_cast<const void*>(&hist_kernel), dim3(tiles), dim3(1024), a1,
                                 buckets * sizeof(uint32_t), s);
  if (e != hipSuccess) return e;
  void* a2[] = {&counts, &tiles, &buckets, &totals};
  return hipLaunchKernel(reinterpret_cast<const void*>(&colscan_kernel), dim3((buckets + 63) / 64), dim3(1024),
                         a2, 0, s);
}

hipError_t gather_vertices(Gather& g, SortBuf& b, uint32_t n, float* out, hipStream_t s) {
  if (n == 0 || g.buckets == 0 || g.vertices == 0) return hipSuccess;
  RayRec* rec = b.rec;
  uint32_t* base = b.scan + g.buckets;
  uint32_t tris = g.triangles;
  int shift0 = shift0_for(n);
  double* corner = g.corner;
  void* a6[] = {&rec, &base, &tris, &shift0, &corner};
  const void* k = g.shift == 6   ? reinterpret_cast<const void*>(&corner_kernel<64>)
                  : g.shift == 7 ? reinterpret_cast<const void*>(&corner_kernel<128>)
                  : g.shift == 8 ? reinterpret_cast<const void*>(&corner_kernel<256>)
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

hipError_t frame_sums(SortBuf& b, uint32_t instances, const float* srt, uint32_t n, float* out, hipStream_t s) {
  if (n == 0 || instances == 0) return hipSuccess;
  const FrameRec* rec = reinterpret_cast<const FrameRec*>(b.rec);
  const uint32_t* base = b.scan + instances;
  int shift0 = shift0_for(n);
  void* a[] = {&rec, &base, &srt, &shift0, &out};
  return hipLaunchKernel(reinterpret_cast<const void*>(&frame_kernel), dim3(instances), dim3(256), a, 0, s);
}

}  // namespace rta
