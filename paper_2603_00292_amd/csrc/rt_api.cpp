// rt_api.cpp -- host runtime behind the C ABI of include/rt.h.
//
// Owns contexts (device, trace variant, scratch: ray-queue counters and the
// global spill stack), acceleration structures (device copies of the BVH
// nodes, triangle records, instance maps and the original vertices and
// indices) and batch plans.  All argument checks happen here, before any
// work is enqueued; no C++ exception leaves this file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/rt.h"
#include "bvh_build.h"
#include "bvh_device.h"
#include "rt_kernels.h"
#include "rt_alloc.h"
#include "rt_layout.h"

namespace {

thread_local std::string g_last_error;

rt_status fail(rt_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

rt_status ok() {
  g_last_error.clear();
  return RT_SUCCESS;
}

// As RT_HIP, inside a function that owns a partly built object and a
// `bail` that releases it.
#define RT_HIP_BAIL(call)                                                                 \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return bail(fail(e_ == hipErrorOutOfMemory ? RT_ERROR_OUT_OF_MEMORY : RT_ERROR_HIP, \
                       "%s: %s", #call, hipGetErrorString(e_)));                          \
  } while (0)

#define RT_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) {                                                               \
      if (e_ == hipErrorOutOfMemory)                                                      \
        return fail(RT_ERROR_OUT_OF_MEMORY, "%s: %s", #call, hipGetErrorString(e_));      \
      return fail(RT_ERROR_HIP, "%s: %s", #call, hipGetErrorString(e_));                  \
    }                                                                                     \
  } while (0)

int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  if (!v || !*v) return dflt;
  return std::atoi(v);
}

const uint32_t kStackChoices[] = {8, 16, 32};
const uint32_t kWorkgroupChoices[] = {64, 128, 256};
const uint32_t kWidthChoices[] = {2, 4, 8};

bool valid_variant(const rt_variant& v) {
  bool s_ok = false, wg_ok = false;
  for (uint32_t x : kStackChoices) s_ok = s_ok || v.stack_entries == x;
  for (uint32_t x : kWorkgroupChoices) wg_ok = wg_ok || v.workgroup == x;
  return s_ok && wg_ok;
}

// device scratch of one launch: queue counter + global spill stack
struct Scratch {
  uint32_t* counter = nullptr;   // [0] ray queue head, [1] overflow ranges
  uint32_t* gstack = nullptr;
  size_t gstack_entries = 0;
  uint32_t* ranges = nullptr;    // fused finalize: per-wave range lists + overflow list
  size_t ranges_entries = 0;
};

void free_scratch(Scratch& s) {
  if (s.counter) (void)hipFree(s.counter);
  if (s.gstack) (void)hipFree(s.gstack);
  if (s.ranges) (void)hipFree(s.ranges);
  s = Scratch();
}

}  // namespace

struct rt_context_s {
  int device = 0;
  int cu_count = 0;
  rt_variant variant{16, 256};
  uint32_t refill_min = 32;
  uint32_t blocks_per_cu = 0;  // 0 = the occupancy API's resident count
  uint32_t stack_limit = 0;    // RT_STACK_LIMIT: caps every lane's stack below the
                               // accel's bound (exercises the overflow report); 0 = off
  uint32_t* status = nullptr;  // host-mapped word: set by a lane whose stack overflows
  bool backward_atomic = false;  // RT_BACKWARD_ATOMIC: two-level backward through the atomic rows
  std::mutex mu;
  Scratch scratch;
  rta::SortBuf sortbuf;                      // backward: rays grouped by triangle range
  rta::SortBuf sortbuf2;                     // two-level backward: rays grouped by instance
  hipEvent_t last_event = nullptr;
  hipStream_t last_stream = nullptr;
  bool has_last = false;
  std::vector<std::pair<const void*, uint32_t>> occupancy;  // kernel -> resident blocks
  // traversal-kernel timing (rt_context_set_timing): event pairs used
  // round-robin, and the launches recorded since the last read
  std::vector<hipEvent_t> tbeg, tend;
  uint64_t trecorded = 0;
};

struct rt_accel_s {
  rt_context ctx = nullptr;                  // context it was built with (variant, scratch)
  int device = 0;
  int width = 4;
  bool two_level = false;
  uint32_t root = RT_CHILD_EMPTY;
  uint32_t max_stack = 1;
  float* nodes = nullptr;
  rt_tri_rec* tris = nullptr;
  rt_inst_rec* insts = nullptr;
  rt_inst_rec64* insts64 = nullptr;
  rt_mesh_dev* meshes = nullptr;             // device array of mesh records
  rt_srt* srts = nullptr;                    // two-level: frames as given to the build
  uint64_t* vertex_base = nullptr;           // two-level: first gradient row per mesh
  uint32_t instance_count = 0;
  uint64_t vertex_rows = 0;                  // two-level: sum of the meshes' vertex counts
  rta::Gather gather;                         // single-level backward: vertex lists, triangle sums
  rta::Rows grad_rows;                       // two-level backward: integer accumulator rows (vertex rows,
                                             // then 4 frame rows per instance), allocated by the
                                             // accel's first backward call
  bool grad_dirty = false;                   // a backward call stopped between its launches
  std::vector<void*> owned;                  // every device allocation
  std::vector<rt_mesh_dev> host_meshes;      // device pointers, host copy
  std::vector<rt_inst_rec> host_insts;       // two-level: host copy of the instance records
  uint32_t* refit_nodes = nullptr;           // node ids, deepest level first (single level)
  std::vector<uint32_t> refit_levels;        // level boundaries in refit_nodes
  // two-level, for rt_update_instances: the top-level nodes (host copy,
  // nodes [0, count) of the node array), their depths, the frames and mesh
  // of every instance and each mesh's bounds
  std::vector<float> tlas_nodes;
  std::vector<uint32_t> tlas_depth;
  std::vector<uint32_t> host_inst_mesh;
  std::vector<rt_srt> host_srts;             // the current frames
  std::vector<rtb::Box> mesh_bounds;
  std::vector<uint32_t> mesh_root;           // root node of each mesh's tree (RT_CHILD_EMPTY: none)
  std::vector<uint32_t> mesh_tri_base;       // first triangle record of each mesh
  rt_accel_info info{};
};

struct rt_batch_plan_s {
  rt_context ctx = nullptr;
  int width = 4;
  bool two_level = false;                    // all accels two-level (else all single level)
  uint32_t batch_count = 0;
  uint32_t total = 0;
  uint32_t max_stack = 1;
  BatchDesc* descs = nullptr;
  uint32_t* offsets = nullptr;
  Scratch scratch;
  uint32_t grid = 0;
  uint32_t workgroup = 256;                  // of `kernel` (the variant at creation)
  uint32_t stack_entries = 16;               // of `kernel`
  const void* kernel = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
};

namespace {

template <typename T>
rt_status dev_alloc(rt_accel_s* a, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return RT_SUCCESS;
  void* q = nullptr;
  RT_HIP(rt_malloc(&q, count * sizeof(T)));
  a->owned.push_back(q);
  a->info.device_bytes += count * sizeof(T);
  *p = static_cast<T*>(q);
  return RT_SUCCESS;
}

void destroy_accel(rt_accel_s* a) {
  for (void* p : a->owned) (void)hipFree(p);
  rta::release(a->grad_rows);
  rta::gather_release(a->gather);
  delete a;
}

// Resident workgroups of a kernel on the whole device.
uint32_t resident_blocks(const void* kern, int wg, int cu_count) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, wg, 0) != hipSuccess ||
      per_cu <= 0)
    per_cu = 1;
  return (uint32_t)per_cu * (uint32_t)std::max(cu_count, 1);
}

// Makes sure scratch holds a counter and a spill stack of `entries` entries.
rt_status ensure_scratch(Scratch& s, size_t entries) {
  if (!s.counter) RT_HIP(rt_malloc(&s.counter, 256));
  if (entries > s.gstack_entries) {
    if (s.gstack) {
      RT_HIP(hipDeviceSynchronize());
      RT_HIP(hipFree(s.gstack));
      s.gstack = nullptr;
      s.gstack_entries = 0;
    }
    RT_HIP(rt_malloc(&s.gstack, entries * sizeof(uint32_t)));
    s.gstack_entries = entries;
  }
  return RT_SUCCESS;
}

// Range lists of a fused closest-hit launch of `gstride` threads over n rays:
// kRtRangesPerWave pairs per wave, then the overflow list.  Every range a
// wave takes holds at least min(refill_min, 64) rays except the one that
// reaches the end of the queue, so n / min(refill_min, 64) + 1 overflow
// pairs always suffice.
rt_status ensure_ranges(Scratch& s, uint32_t gstride, uint32_t n, uint32_t refill_min,
                        uint32_t** ranges, uint32_t** ovf, uint32_t* ovf_cap) {
  size_t waves = gstride / 64u;
  size_t per_wave = 2 * (size_t)kRtRangesPerWave;
  size_t cap = (size_t)n / std::max<uint32_t>(1u, std::min<uint32_t>(refill_min, 64u)) + 1;
  size_t entries = waves * per_wave + 2 * cap;
  if (entries > s.ranges_entries) {
    if (s.ranges) {
      RT_HIP(hipDeviceSynchronize());
      RT_HIP(hipFree(s.ranges));
      s.ranges = nullptr;
      s.ranges_entries = 0;
    }
    RT_HIP(rt_malloc(&s.ranges, entries * sizeof(uint32_t)));
    s.ranges_entries = entries;
  }
  *ranges = s.ranges;
  *ovf = s.ranges + waves * per_wave;
  *ovf_cap = (uint32_t)cap;
  return RT_SUCCESS;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

rt_status check_device(int dev) {
  int cur = -1;
  RT_HIP(hipGetDevice(&cur));
  if (cur != dev) RT_HIP(hipSetDevice(dev));
  return RT_SUCCESS;
}

// Scratch of rt_trace_closest_noalloc.  Every GPU the library runs on holds
// its own copy of this array until the process ends; host code reaches a
// GPU's copy only through the address hipGetSymbolAddress returns with that
// GPU current (noalloc_setup), never through the array's name.
constexpr size_t kNoAllocWords = RT_NOALLOC_SCRATCH_BYTES / sizeof(uint32_t);
constexpr int kNoAllocMaxDevices = 64;
std::mutex g_noalloc_mu;
uint32_t* g_noalloc_ptr[kNoAllocMaxDevices] = {};

}  // namespace

static __device__ __align__(256) uint32_t scratch[kNoAllocWords];

namespace {

// With device `dev` current: finds the address of that device's copy of the
// no-alloc scratch (once per device; called by rt_context_create).
rt_status noalloc_setup(int dev) {
  if (dev < 0 || dev >= kNoAllocMaxDevices)
    return fail(RT_ERROR_UNSUPPORTED, "rt_context_create: device id %d >= %d", dev, kNoAllocMaxDevices);
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (g_noalloc_ptr[dev]) return RT_SUCCESS;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(RT_ERROR_HIP, "rt_context_create: hipGetSymbolAddress of the no-alloc scratch: %s",
                hipGetErrorString(e));
  g_noalloc_ptr[dev] = static_cast<uint32_t*>(ptr);
  return RT_SUCCESS;
}

uint32_t* noalloc_ptr(int dev) {
  if (dev < 0 || dev >= kNoAllocMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  return g_noalloc_ptr[dev];
}

// Reports (and clears) a stack overflow flagged by an earlier traversal on
// this context.  The flag is written by the device into host-mapped memory;
// a launch still running when this is read is reported by a later call.
rt_status take_overflow(rt_context ctx, const char* who) {
  volatile uint32_t* f = reinterpret_cast<volatile uint32_t*>(ctx->status);
  if (*f == 0u) return RT_SUCCESS;
  *f = 0u;
  return fail(RT_ERROR_STACK_OVERFLOW,
              "%s: an earlier traversal on this context exceeded its accel's stack bound; "
              "that query's results may lack hits", who);
}

}  // namespace

// allocations left until the injected failure (0: none armed; see rt_alloc.h)
static std::atomic<int64_t> g_fault_alloc{0};

bool rt_alloc_fault() {
  int64_t v = g_fault_alloc.load(std::memory_order_relaxed);
  while (v > 0)
    if (g_fault_alloc.compare_exchange_weak(v, v - 1, std::memory_order_relaxed)) return v == 1;
  return false;
}

extern "C" {

const char* rt_status_string(rt_status s) {
  switch (s) {
    case RT_SUCCESS: return "RT_SUCCESS";
    case RT_ERROR_INVALID_VALUE: return "RT_ERROR_INVALID_VALUE";
    case RT_ERROR_OUT_OF_MEMORY: return "RT_ERROR_OUT_OF_MEMORY";
    case RT_ERROR_NO_DEVICE: return "RT_ERROR_NO_DEVICE";
    case RT_ERROR_HIP: return "RT_ERROR_HIP";
    case RT_ERROR_UNSUPPORTED: return "RT_ERROR_UNSUPPORTED";
    case RT_ERROR_INDEX_OUT_OF_RANGE: return "RT_ERROR_INDEX_OUT_OF_RANGE";
    case RT_ERROR_STACK_OVERFLOW: return "RT_ERROR_STACK_OVERFLOW";
  }
  return "RT_ERROR_UNKNOWN";
}

const char* rt_last_error_message(void) { return g_last_error.c_str(); }

uint32_t rt_version(void) { return 100; }

rt_status rt_context_create(int hip_device, rt_context* out) {
  if (!out) return fail(RT_ERROR_INVALID_VALUE, "rt_context_create: out is NULL");
  *out = nullptr;
  g_fault_alloc.store(std::max<int64_t>(0, env_int("RT_FAULT_ALLOC", 0)), std::memory_order_relaxed);
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0)
    return fail(RT_ERROR_NO_DEVICE, "rt_context_create: no HIP device (%s)", hipGetErrorString(e));
  if (hip_device < 0 || hip_device >= n)
    return fail(RT_ERROR_NO_DEVICE, "rt_context_create: device %d out of range (%d devices)",
                hip_device, n);
  RT_HIP(hipSetDevice(hip_device));
  rt_context_s* c = new (std::nothrow) rt_context_s();
  if (!c) return fail(RT_ERROR_OUT_OF_MEMORY, "rt_context_create: host allocation");
  c->device = hip_device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) {
    delete c;
    return fail(RT_ERROR_HIP, "rt_context_create: hipGetDeviceProperties failed");
  }
  c->cu_count = prop.multiProcessorCount;
  rt_variant v{(uint32_t)env_int("RT_STACK", 16), (uint32_t)env_int("RT_WG", 256)};
  if (valid_variant(v)) c->variant = v;
  c->refill_min = (uint32_t)std::min(64, std::max(1, env_int("RT_REFILL", 32)));
  c->blocks_per_cu = (uint32_t)std::min(64, std::max(0, env_int("RT_BLOCKS_PER_CU", 0)));
  c->stack_limit = (uint32_t)std::max(0, env_int("RT_STACK_LIMIT", 0));
  c->backward_atomic = env_int("RT_BACKWARD_ATOMIC", 0) != 0;
  if (hipEventCreateWithFlags(&c->last_event, hipEventDisableTiming) != hipSuccess) {
    delete c;
    return fail(RT_ERROR_HIP, "rt_context_create: hipEventCreate failed");
  }
  if (rt_host_malloc(reinterpret_cast<void**>(&c->status), sizeof(uint32_t), hipHostMallocDefault) !=
      hipSuccess) {
    (void)hipEventDestroy(c->last_event);
    delete c;
    return fail(RT_ERROR_OUT_OF_MEMORY, "rt_context_create: hipHostMalloc of the status word failed");
  }
  *reinterpret_cast<volatile uint32_t*>(c->status) = 0u;
  rt_status ns = noalloc_setup(hip_device);
  if (ns != RT_SUCCESS) {
    (void)hipHostFree(c->status);
    (void)hipEventDestroy(c->last_event);
    delete c;
    return ns;
  }
  *out = c;
  return ok();
}

rt_status rt_context_destroy(rt_context ctx) {
  if (!ctx) return fail(RT_ERROR_INVALID_VALUE, "rt_context_destroy: NULL context");
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  free_scratch(ctx->scratch);
  rta::sort_release(ctx->sortbuf);
  rta::sort_release(ctx->sortbuf2);
  if (ctx->last_event) (void)hipEventDestroy(ctx->last_event);
  for (hipEvent_t e : ctx->tbeg) (void)hipEventDestroy(e);
  for (hipEvent_t e : ctx->tend) (void)hipEventDestroy(e);
  if (ctx->status) (void)hipHostFree(ctx->status);
  delete ctx;
  return ok();
}

static void drop_timing(rt_context ctx) {
  for (hipEvent_t e : ctx->tbeg) (void)hipEventDestroy(e);
  for (hipEvent_t e : ctx->tend) (void)hipEventDestroy(e);
  ctx->tbeg.clear();
  ctx->tend.clear();
  ctx->trecorded = 0;
}

rt_status rt_context_set_timing(rt_context ctx, uint32_t slots) {
  if (!ctx) return fail(RT_ERROR_INVALID_VALUE, "rt_context_set_timing: NULL context");
  if (slots > RT_TIMING_MAX_SLOTS)
    return fail(RT_ERROR_INVALID_VALUE, "rt_context_set_timing: more than 4096 slots");
  rt_status st = check_device(ctx->device);
  if (st != RT_SUCCESS) return st;
  std::lock_guard<std::mutex> lk(ctx->mu);
  for (hipEvent_t e : ctx->tend) (void)hipEventSynchronize(e);
  drop_timing(ctx);
  for (uint32_t i = 0; i < slots; ++i) {
    hipEvent_t b = nullptr, e = nullptr;
    hipError_t eb = hipEventCreate(&b);
    hipError_t ee = eb == hipSuccess ? hipEventCreate(&e) : eb;
    if (ee != hipSuccess) {
      if (b) (void)hipEventDestroy(b);
      drop_timing(ctx);
      return fail(RT_ERROR_HIP, "rt_context_set_timing: %s", hipGetErrorString(ee));
    }
    ctx->tbeg.push_back(b);
    ctx->tend.push_back(e);
  }
  return ok();
}

rt_status rt_context_read_timing(rt_context ctx, float* ms, uint32_t capacity, uint32_t* count) {
  if (!ctx || !count || (capacity && !ms))
    return fail(RT_ERROR_INVALID_VALUE, "rt_context_read_timing: NULL argument");
  rt_status st = check_device(ctx->device);
  if (st != RT_SUCCESS) return st;
  std::lock_guard<std::mutex> lk(ctx->mu);
  *count = 0;
  size_t slots = ctx->tend.size();
  if (slots == 0) return ok();
  uint64_t avail = std::min<uint64_t>(ctx->trecorded, slots);
  uint64_t k = std::min<uint64_t>(avail, capacity);
  // the k most recent launches, oldest first
  for (uint64_t j = 0; j < k; ++j) {
    size_t slot = (size_t)((ctx->trecorded - k + j) % slots);
    RT_HIP(hipEventSynchronize(ctx->tend[slot]));
    float t = 0.0f;
    RT_HIP(hipEventElapsedTime(&t, ctx->tbeg[slot], ctx->tend[slot]));
    ms[j] = t;
  }
  *count = (uint32_t)k;
  ctx->trecorded = 0;
  return ok();
}

rt_status rt_context_set_variant(rt_context ctx, const rt_variant* v) {
  if (!ctx || !v) return fail(RT_ERROR_INVALID_VALUE, "rt_context_set_variant: NULL argument");
  if (!valid_variant(*v))
    return fail(RT_ERROR_INVALID_VALUE,
                "rt_context_set_variant: stack_entries must be 8/16/32 and workgroup "
                "64/128/256");
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->variant = *v;
  return ok();
}

rt_status rt_context_get_variant(rt_context ctx, rt_variant* out) {
  if (!ctx || !out) return fail(RT_ERROR_INVALID_VALUE, "rt_context_get_variant: NULL argument");
  *out = ctx->variant;
  return ok();
}

// ---------------------------------------------------------------------------
// build
// ---------------------------------------------------------------------------

static rt_status read_mesh(const rt_mesh_desc& m, hipStream_t s, std::vector<float>& V,
                           std::vector<uint32_t>& I) {
  V.assign((size_t)m.vertex_count * 3, 0.0f);
  I.assign((size_t)m.triangle_count * 3, 0u);
  if (m.vertex_count) {
    if (m.vertex_stride == 12) {
      RT_HIP(hipMemcpyAsync(V.data(), m.vertices, V.size() * 4, hipMemcpyDefault, s));
    } else {
      std::vector<uint8_t> raw((size_t)(m.vertex_count - 1) * m.vertex_stride + 12);
      RT_HIP(hipMemcpyAsync(raw.data(), m.vertices, raw.size(), hipMemcpyDefault, s));
      RT_HIP(hipStreamSynchronize(s));
      for (uint32_t i = 0; i < m.vertex_count; ++i)
        std::memcpy(&V[3 * (size_t)i], raw.data() + (size_t)i * m.vertex_stride, 12);
    }
  }
  if (m.triangle_count) {
    if (m.index_stride == 12) {
      RT_HIP(hipMemcpyAsync(I.data(), m.indices, I.size() * 4, hipMemcpyDefault, s));
    } else {
      std::vector<uint8_t> raw((size_t)(m.triangle_count - 1) * m.index_stride + 12);
      RT_HIP(hipMemcpyAsync(raw.data(), m.indices, raw.size(), hipMemcpyDefault, s));
      RT_HIP(hipStreamSynchronize(s));
      for (uint32_t i = 0; i < m.triangle_count; ++i)
        std::memcpy(&I[3 * (size_t)i], raw.data() + (size_t)i * m.index_stride, 12);
    }
  }
  RT_HIP(hipStreamSynchronize(s));
  return RT_SUCCESS;
}

// world = T + R(q/|q|)(S x); returns the world->object map in float64 rows
static void srt_inverse(const rt_srt& f, double m[12]) {
  double qx = f.qx, qy = f.qy, qz = f.qz, qw = f.qw;
  double nq = std::sqrt(qx * qx + qy * qy + qz * qz + qw * qw);
  qx /= nq; qy /= nq; qz /= nq; qw /= nq;
  double R[3][3] = {{1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qz * qw), 2 * (qx * qz + qy * qw)},
                    {2 * (qx * qy + qz * qw), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qx * qw)},
                    {2 * (qx * qz - qy * qw), 2 * (qy * qz + qx * qw), 1 - 2 * (qx * qx + qy * qy)}};
  double S[3] = {f.sx, f.sy, f.sz}, T[3] = {f.tx, f.ty, f.tz};
  for (int i = 0; i < 3; ++i) {
    // row i of S^-1 R^T is column i of R divided by S_i
    double a = R[0][i] / S[i], b = R[1][i] / S[i], c = R[2][i] / S[i];
    m[4 * i + 0] = a;
    m[4 * i + 1] = b;
    m[4 * i + 2] = c;
    m[4 * i + 3] = -(a * T[0] + b * T[1] + c * T[2]);
  }
}

static rtb::Box world_box(const rtb::Box& b, const rt_srt& f) {
  double qx = f.qx, qy = f.qy, qz = f.qz, qw = f.qw;
  double nq = std::sqrt(qx * qx + qy * qy + qz * qz + qw * qw);
  qx /= nq; qy /= nq; qz /= nq; qw /= nq;
  double R[3][3] = {{1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qz * qw), 2 * (qx * qz + qy * qw)},
                    {2 * (qx * qy + qz * qw), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qx * qw)},
                    {2 * (qx * qz - qy * qw), 2 * (qy * qz + qx * qw), 1 - 2 * (qx * qx + qy * qy)}};
  double S[3] = {f.sx, f.sy, f.sz}, T[3] = {f.tx, f.ty, f.tz};
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int c = 0; c < 8; ++c) {
    double x[3] = {(c & 1) ? b.hi[0] : b.lo[0], (c & 2) ? b.hi[1] : b.lo[1],
                   (c & 4) ? b.hi[2] : b.lo[2]};
    for (int i = 0; i < 3; ++i) {
      double w = T[i] + R[i][0] * S[0] * x[0] + R[i][1] * S[1] * x[1] + R[i][2] * S[2] * x[2];
      lo[i] = std::min(lo[i], w);
      hi[i] = std::max(hi[i], w);
    }
  }
  rtb::Box out;
  for (int i = 0; i < 3; ++i) {
    // round outward, with a relative margin for the float64 arithmetic above
    double pad = 1e-12 * (std::fabs(lo[i]) + std::fabs(hi[i]) + 1.0);
    out.lo[i] = std::nextafter((float)(lo[i] - pad), -INFINITY);
    out.hi[i] = std::nextafter((float)(hi[i] + pad), INFINITY);
  }
  return out;
}

// Single-level accel built on the device (RT_BUILD_DEVICE).
// Frames must be finite, with non-zero scales and a non-zero quaternion.
static rt_status check_frames(const rt_srt* srt, uint32_t count, const char* who) {
  for (uint32_t j = 0; j < count; ++j) {
    const rt_srt& f = srt[j];
    const float all[10] = {f.sx, f.sy, f.sz, f.qx, f.qy, f.qz, f.qw, f.tx, f.ty, f.tz};
    for (float x : all)
      if (!std::isfinite(x)) return fail(RT_ERROR_INVALID_VALUE, "%s: instance %u frame is not finite", who, j);
    if (f.sx == 0.0f || f.sy == 0.0f || f.sz == 0.0f)
      return fail(RT_ERROR_INVALID_VALUE, "%s: instance %u has a zero scale", who, j);
    if (f.qx == 0.0f && f.qy == 0.0f && f.qz == 0.0f && f.qw == 0.0f)
      return fail(RT_ERROR_INVALID_VALUE, "%s: instance %u has a zero quaternion", who, j);
  }
  return RT_SUCCESS;
}

// Instance records (float32 and float64 world->object maps, bottom-level
// roots, masks), the frames as given and the per-mesh gradient row offsets of
// a two-level accel.  blas_root[m] is the root reference of mesh m's tree in
// the accel's node array (RT_CHILD_EMPTY for a mesh without triangles).
static rt_status setup_instances(rt_accel_s* a, const rt_mesh_desc* meshes, uint32_t mesh_count,
                                 const uint32_t* instance_mesh, const rt_srt* instance_srt,
                                 uint32_t instance_count, const std::vector<uint32_t>& blas_root,
                                 hipStream_t s) {
  rt_status st;
  std::vector<rt_inst_rec> ir(instance_count);
  std::vector<rt_inst_rec64> ir64(instance_count);
  for (uint32_t j = 0; j < instance_count; ++j) {
    double m[12];
    srt_inverse(instance_srt[j], m);
    std::memcpy(ir64[j].m, m, sizeof(m));
    for (int k = 0; k < 4; ++k) {
      ir[j].r0[k] = (float)m[k];
      ir[j].r1[k] = (float)m[4 + k];
      ir[j].r2[k] = (float)m[8 + k];
    }
    uint32_t mm = instance_mesh[j];
    ir[j].root = blas_root[mm];
    ir[j].mesh = mm;
    ir[j].mask = 0xFFFFFFFFu;
    ir[j].pad = 0;
  }
  st = dev_alloc(a, &a->insts, ir.size());
  if (st != RT_SUCCESS) return st;
  st = dev_alloc(a, &a->insts64, ir64.size());
  if (st != RT_SUCCESS) return st;
  RT_HIP(hipMemcpyAsync(a->insts, ir.data(), ir.size() * sizeof(rt_inst_rec), hipMemcpyHostToDevice, s));
  a->host_insts = ir;
  RT_HIP(hipMemcpyAsync(a->insts64, ir64.data(), ir64.size() * sizeof(rt_inst_rec64), hipMemcpyHostToDevice, s));
  // frames and per-mesh gradient rows for the two-level adjoint
  std::vector<uint64_t> base(mesh_count);
  uint64_t acc = 0;
  for (uint32_t m = 0; m < mesh_count; ++m) {
    base[m] = acc;
    acc += meshes[m].vertex_count;
  }
  st = dev_alloc(a, &a->srts, instance_count);
  if (st != RT_SUCCESS) return st;
  a->vertex_rows = acc;
  st = dev_alloc(a, &a->vertex_base, mesh_count);
  if (st != RT_SUCCESS) return st;
  RT_HIP(hipMemcpyAsync(a->srts, instance_srt, instance_count * sizeof(rt_srt), hipMemcpyHostToDevice, s));
  RT_HIP(hipMemcpyAsync(a->vertex_base, base.data(), mesh_count * sizeof(uint64_t), hipMemcpyHostToDevice, s));
  a->instance_count = instance_count;
  a->host_inst_mesh.assign(instance_mesh, instance_mesh + instance_count);
  a->host_srts.assign(instance_srt, instance_srt + instance_count);
  a->mesh_root = blas_root;
  return RT_SUCCESS;
}

static rt_status build_on_device(rt_context ctx, const rt_mesh_desc& mesh, int width, int max_leaf,
                                 hipStream_t s, rt_accel* out) {
  rt_accel_s* a = new (std::nothrow) rt_accel_s();
  if (!a) return fail(RT_ERROR_OUT_OF_MEMORY, "rt_build: host allocation");
  a->ctx = ctx;
  a->device = ctx->device;
  a->width = width;
  a->two_level = false;
  a->info.node_width = (uint32_t)width;
  rtd::Input in{static_cast<const float*>(mesh.vertices), mesh.vertex_count, mesh.vertex_stride,
                static_cast<const uint32_t*>(mesh.indices), mesh.triangle_count, mesh.index_stride,
                width, max_leaf};
  rtd::Output o;
  bool index_error = false;
  hipError_t e;
  try {
    e = rtd::build(in, o, index_error, s);
  } catch (const std::bad_alloc&) {
    e = hipErrorOutOfMemory;
  }
  for (void* p : o.owned) a->owned.push_back(p);
  a->info.device_bytes += o.owned_bytes;
  if (e != hipSuccess) {
    destroy_accel(a);
    return fail(e == hipErrorOutOfMemory ? RT_ERROR_OUT_OF_MEMORY : RT_ERROR_HIP,
                "rt_build (device): %s", hipGetErrorString(e));
  }
  if (index_error) {
    destroy_accel(a);
    return fail(RT_ERROR_INDEX_OUT_OF_RANGE, "rt_build: a vertex index is >= vertex_count");
  }
  a->nodes = o.nodes;
  a->tris = o.tris;
  a->root = o.tri_count ? o.root : RT_CHILD_EMPTY;
  a->max_stack = std::max(o.max_stack, 1u);
  a->refit_nodes = o.tri_count ? o.refit_nodes : nullptr;
  a->refit_levels = o.tri_count ? o.refit_levels : std::vector<uint32_t>();
  a->info.node_count = o.tri_count ? o.node_count : 0;
  a->info.triangle_count = o.tri_count;
  a->info.input_triangles = mesh.triangle_count;
  a->info.max_depth = o.tri_count ? o.max_depth : 0;
  a->info.max_stack = a->max_stack;
  a->info.leaf_count = o.leaf_count;
  a->info.sah_cost = o.sah_cost;
  a->host_meshes.assign(1, rt_mesh_dev{o.vertices, o.indices, mesh.vertex_count, mesh.triangle_count});
  rt_status st = dev_alloc(a, &a->meshes, 1);
  if (st != RT_SUCCESS) {
    destroy_accel(a);
    return st;
  }
  hipError_t ce = hipMemcpyAsync(a->meshes, a->host_meshes.data(), sizeof(rt_mesh_dev), hipMemcpyHostToDevice, s);
  if (ce == hipSuccess) ce = hipStreamSynchronize(s);
  if (ce != hipSuccess) {
    destroy_accel(a);
    return fail(RT_ERROR_HIP, "rt_build (device): %s", hipGetErrorString(ce));
  }
  *out = a;
  return ok();
}

// Two-level build with every bottom-level tree built on the GPU (one device
// build per mesh) and the top-level tree over the instances' world boxes
// built on the host (one box per instance: milliseconds for thousands).  The
// parts are placed on the device in the layout of the host build -- nodes
// [top][mesh 0][mesh 1]..., records [mesh 0][mesh 1]... -- with their
// references relocated there.
static rt_status build_two_level_on_device(rt_context ctx, const rt_mesh_desc* meshes, uint32_t mesh_count,
                                           const uint32_t* instance_mesh, const rt_srt* instance_srt,
                                           uint32_t instance_count, int width, int max_leaf, hipStream_t s,
                                           rt_accel* out) {
  rt_accel_s* a = new (std::nothrow) rt_accel_s();
  if (!a) return fail(RT_ERROR_OUT_OF_MEMORY, "rt_build: host allocation");
  a->ctx = ctx;
  a->device = ctx->device;
  a->width = width;
  a->two_level = true;
  a->info.node_width = (uint32_t)width;
  a->info.instance_count = instance_count;
  std::vector<rtd::Output> parts;
  auto free_parts = [&]() {
    for (rtd::Output& o : parts)
      for (void* q : o.owned) (void)hipFree(q);
    parts.clear();
  };
  auto bail = [&](rt_status e) {
    (void)hipStreamSynchronize(s);
    free_parts();
    destroy_accel(a);
    return e;
  };
  auto hip_fail = [&](hipError_t e, const char* what) {
    return bail(fail(e == hipErrorOutOfMemory ? RT_ERROR_OUT_OF_MEMORY : RT_ERROR_HIP, "rt_build (device): %s: %s",
                     what, hipGetErrorString(e)));
  };
  try {
    parts.resize(mesh_count);
    uint64_t input_tris = 0;
    for (uint32_t m = 0; m < mesh_count; ++m) {
      const rt_mesh_desc& d = meshes[m];
      rtd::Input in{static_cast<const float*>(d.vertices), d.vertex_count, d.vertex_stride,
                    static_cast<const uint32_t*>(d.indices), d.triangle_count, d.index_stride, width, max_leaf};
      bool index_error = false;
      hipError_t e = rtd::build(in, parts[m], index_error, s);
      if (e != hipSuccess) return hip_fail(e, "bottom-level build");
      if (index_error)
        return bail(fail(RT_ERROR_INDEX_OUT_OF_RANGE, "rt_build: mesh %u: a vertex index is >= vertex_count", m));
      input_tris += d.triangle_count;
    }
    // top level over the instances' world boxes
    std::vector<rtb::Box> boxes(instance_count);
    for (uint32_t j = 0; j < instance_count; ++j) {
      const rtd::Output& o = parts[instance_mesh[j]];
      if (o.tri_count == 0) {
        for (int k = 0; k < 3; ++k) {
          boxes[j].lo[k] = INFINITY;
          boxes[j].hi[k] = -INFINITY;
        }
      } else {
        rtb::Box b;
        for (int k = 0; k < 3; ++k) {
          b.lo[k] = o.bounds[k];
          b.hi[k] = o.bounds[3 + k];
        }
        boxes[j] = world_box(b, instance_srt[j]);
      }
    }
    int threads = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    rtb::WideTree tlas;
    rtb::build_instances(boxes, width, tlas, threads);
    // placement
    const uint32_t fpn = 8u * (uint32_t)width;
    uint64_t node_total = tlas.node_count, tri_total = 0;
    std::vector<uint32_t> node_base(mesh_count), tri_base(mesh_count), blas_root(mesh_count);
    for (uint32_t m = 0; m < mesh_count; ++m) {
      const rtd::Output& o = parts[m];
      node_base[m] = (uint32_t)node_total;
      tri_base[m] = (uint32_t)tri_total;
      blas_root[m] = o.tri_count ? node_base[m] : RT_CHILD_EMPTY;
      node_total += o.tri_count ? o.node_count : 0u;
      tri_total += o.tri_count;
    }
    if (node_total >= 0x7FFFFFFFull || tri_total > RT_MAX_TRI_RECORDS)
      return bail(fail(RT_ERROR_INVALID_VALUE, "rt_build: scene too large for one accel"));
    rt_status st = dev_alloc(a, &a->nodes, (size_t)node_total * fpn);
    if (st != RT_SUCCESS) return bail(st);
    st = dev_alloc(a, &a->tris, (size_t)tri_total);
    if (st != RT_SUCCESS) return bail(st);
    hipError_t e = hipSuccess;
    if (tlas.node_count)
      e = hipMemcpyAsync(a->nodes, tlas.nodes.data(), (size_t)tlas.node_count * fpn * 4, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "top-level copy");
    uint32_t max_blas_stack = 0, max_blas_depth = 0;
    a->host_meshes.resize(mesh_count);
    for (uint32_t m = 0; m < mesh_count; ++m) {
      rtd::Output& o = parts[m];
      if (o.tri_count) {
        float* dst = a->nodes + (size_t)node_base[m] * fpn;
        e = hipMemcpyAsync(dst, o.nodes, (size_t)o.node_count * fpn * 4, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = rtd::relocate(dst, o.node_count, width, node_base[m], tri_base[m], s);
        if (e == hipSuccess)
          e = hipMemcpyAsync(a->tris + tri_base[m], o.tris, (size_t)o.tri_count * sizeof(rt_tri_rec),
                             hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "bottom-level placement");
        max_blas_stack = std::max(max_blas_stack, o.max_stack);
        max_blas_depth = std::max(max_blas_depth, o.max_depth);
        a->info.leaf_count += o.leaf_count;
      }
      // the compact mesh copies stay with the accel (finalize and adjoint)
      std::vector<void*>& ow = o.owned;
      ow.erase(std::remove_if(ow.begin(), ow.end(),
                              [&](void* q) { return q == (void*)o.vertices || q == (void*)o.indices; }),
               ow.end());
      a->owned.push_back(o.vertices);
      a->owned.push_back(o.indices);
      a->info.device_bytes += 12ull * (std::max(meshes[m].vertex_count, 1u) + std::max(meshes[m].triangle_count, 1u));
      a->host_meshes[m] = rt_mesh_dev{o.vertices, o.indices, meshes[m].vertex_count, meshes[m].triangle_count};
    }
    st = dev_alloc(a, &a->meshes, mesh_count);
    if (st != RT_SUCCESS) return bail(st);
    e = hipMemcpyAsync(a->meshes, a->host_meshes.data(), mesh_count * sizeof(rt_mesh_dev), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "mesh records");
    // refit order: a device build numbers the wide nodes of one depth
    // consecutively, depth 1 first, and lists the level sizes deepest first
    std::vector<std::vector<std::pair<uint32_t, uint32_t>>> ranges(mesh_count);  // per depth - 1: [begin, end)
    uint32_t maxd = 0;
    for (uint32_t m = 0; m < mesh_count; ++m) {
      const rtd::Output& o = parts[m];
      if (!o.tri_count) continue;
      const std::vector<uint32_t>& lv = o.refit_levels;
      const uint32_t L = lv.empty() ? 0u : (uint32_t)lv.size() - 1;
      std::vector<std::pair<uint32_t, uint32_t>> r(L);
      uint32_t begin = 0;
      for (uint32_t d = 1; d <= L; ++d) {
        uint32_t k = L - d;  // position of depth d in the deepest-first list
        uint32_t size = lv[k + 1] - lv[k];
        r[d - 1] = {node_base[m] + begin, node_base[m] + begin + size};
        begin += size;
      }
      ranges[m] = r;
      maxd = std::max(maxd, L);
    }
    std::vector<uint32_t> order;
    a->refit_levels.assign(1, 0);
    for (uint32_t d = maxd; d >= 1; --d) {
      for (uint32_t m = 0; m < mesh_count; ++m)
        if (d <= ranges[m].size())
          for (uint32_t i = ranges[m][d - 1].first; i < ranges[m][d - 1].second; ++i) order.push_back(i);
      a->refit_levels.push_back((uint32_t)order.size());
    }
    a->mesh_tri_base = tri_base;
    if (!order.empty()) {
      st = dev_alloc(a, &a->refit_nodes, order.size());
      if (st != RT_SUCCESS) return bail(st);
      e = hipMemcpyAsync(a->refit_nodes, order.data(), order.size() * 4, hipMemcpyHostToDevice, s);
      if (e != hipSuccess) return hip_fail(e, "refit order");
    }
    st = setup_instances(a, meshes, mesh_count, instance_mesh, instance_srt, instance_count, blas_root, s);
    if (st != RT_SUCCESS) return bail(st);
    a->tlas_nodes = tlas.nodes;
    a->tlas_nodes.resize((size_t)tlas.node_count * fpn);
    a->tlas_depth = tlas.node_depth;
    a->tlas_depth.resize(tlas.node_count);
    a->mesh_bounds.resize(mesh_count);
    for (uint32_t m = 0; m < mesh_count; ++m)
      for (int k = 0; k < 3; ++k) {
        a->mesh_bounds[m].lo[k] = parts[m].tri_count ? parts[m].bounds[k] : INFINITY;
        a->mesh_bounds[m].hi[k] = parts[m].tri_count ? parts[m].bounds[3 + k] : -INFINITY;
      }
    a->root = tlas.root;
    a->max_stack = std::max(tlas.max_stack + 1 + max_blas_stack, 1u);
    a->info.node_count = (uint32_t)node_total;
    a->info.triangle_count = (uint32_t)tri_total;
    a->info.input_triangles = (uint32_t)std::min<uint64_t>(input_tris, 0xFFFFFFFFull);
    a->info.max_depth = tlas.max_depth + max_blas_depth;
    a->info.max_stack = a->max_stack;
    a->info.leaf_count += tlas.leaf_count;
    a->info.sah_cost = tlas.sah_cost;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "synchronize");
    free_parts();  // the per-mesh node and record arrays, now copied
  } catch (const std::bad_alloc&) {
    return bail(fail(RT_ERROR_OUT_OF_MEMORY, "rt_build: host allocation failed"));
  } catch (const std::exception& ex) {
    return bail(fail(RT_ERROR_INVALID_VALUE, "rt_build: %s", ex.what()));
  }
  *out = a;
  return ok();
}

rt_status rt_build(rt_context ctx, const rt_mesh_desc* meshes, uint32_t mesh_count,
                   const uint32_t* instance_mesh, const rt_srt* instance_srt,
                   uint32_t instance_count, const rt_build_options* options, void* stream,
                   rt_accel* out) {
  if (!out) return fail(RT_ERROR_INVALID_VALUE, "rt_build: out is NULL");
  *out = nullptr;
  if (!ctx) return fail(RT_ERROR_INVALID_VALUE, "rt_build: NULL context");
  if (!meshes || mesh_count == 0) return fail(RT_ERROR_INVALID_VALUE, "rt_build: no meshes");
  if (instance_count == 0 && mesh_count != 1)
    return fail(RT_ERROR_INVALID_VALUE, "rt_build: a single-level build takes exactly one mesh");
  if (instance_count == 0 && (instance_mesh || instance_srt))
    return fail(RT_ERROR_INVALID_VALUE, "rt_build: instance arrays given with instance_count 0");
  if (instance_count > 0 && (!instance_mesh || !instance_srt))
    return fail(RT_ERROR_INVALID_VALUE, "rt_build: instance arrays are NULL");
  if (instance_count > RT_INST_INDEX_MASK)
    return fail(RT_ERROR_INVALID_VALUE, "rt_build: too many instances");
  int width = 4, max_leaf = 4;
  bool on_device = false;
  if (options) {
    if ((options->flags & ~RT_BUILD_DEVICE) != 0)
      return fail(RT_ERROR_INVALID_VALUE, "rt_build: unknown flags");
    on_device = (options->flags & RT_BUILD_DEVICE) != 0;
    if (options->node_width != 0) width = (int)options->node_width;
    if (options->max_leaf_size != 0) max_leaf = (int)options->max_leaf_size;
  }
  if (width != 2 && width != 4 && width != 8)
    return fail(RT_ERROR_INVALID_VALUE, "rt_build: node_width must be 0, 2, 4 or 8");
  if (max_leaf < 1 || max_leaf > (int)RT_MAX_LEAF_SIZE)
    return fail(RT_ERROR_INVALID_VALUE, "rt_build: max_leaf_size must be 1..15");
  for (uint32_t m = 0; m < mesh_count; ++m) {
    const rt_mesh_desc& d = meshes[m];
    if ((d.vertex_count > 0 && !d.vertices) || (d.triangle_count > 0 && !d.indices))
      return fail(RT_ERROR_INVALID_VALUE, "rt_build: mesh %u has a NULL buffer", m);
    if (d.vertex_stride < 12 || d.index_stride < 12)
      return fail(RT_ERROR_INVALID_VALUE, "rt_build: mesh %u stride < 12", m);
  }
  for (uint32_t j = 0; j < instance_count; ++j)
    if (instance_mesh[j] >= mesh_count)
      return fail(RT_ERROR_INDEX_OUT_OF_RANGE, "rt_build: instance %u refers to mesh %u of %u", j,
                  instance_mesh[j], mesh_count);
  if (instance_count > 0) {
    rt_status fs = check_frames(instance_srt, instance_count, "rt_build");
    if (fs != RT_SUCCESS) return fs;
  }
  if (on_device) {
    for (uint32_t m = 0; m < mesh_count; ++m) {
      const rt_mesh_desc& d = meshes[m];
      if (((uintptr_t)d.vertices | (uintptr_t)d.indices | d.vertex_stride | d.index_stride) & 3u)
        return fail(RT_ERROR_INVALID_VALUE, "rt_build: the device build needs 4-byte aligned pointers and strides");
      if (d.triangle_count > RT_MAX_TRI_RECORDS)
        return fail(RT_ERROR_INVALID_VALUE, "rt_build: mesh too large for one accel");
    }
  }
  rt_status st = check_device(ctx->device);
  if (st != RT_SUCCESS) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (on_device)
    return instance_count > 0 ? build_two_level_on_device(ctx, meshes, mesh_count, instance_mesh, instance_srt,
                                                          instance_count, width, max_leaf, s, out)
                              : build_on_device(ctx, meshes[0], width, max_leaf, s, out);
  int threads = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));

  rt_accel_s* a = new (std::nothrow) rt_accel_s();
  if (!a) return fail(RT_ERROR_OUT_OF_MEMORY, "rt_build: host allocation");
  a->ctx = ctx;
  a->device = ctx->device;
  a->width = width;
  a->two_level = instance_count > 0;
  a->info.node_width = (uint32_t)width;
  a->info.instance_count = instance_count;

  auto bail = [&](rt_status e) {
    destroy_accel(a);
    return e;
  };

  try {
    std::vector<rtb::WideTree> blas(mesh_count);
    std::vector<std::vector<float>> hv(mesh_count);
    std::vector<std::vector<uint32_t>> hi(mesh_count);
    uint64_t input_tris = 0;
    for (uint32_t m = 0; m < mesh_count; ++m) {
      st = read_mesh(meshes[m], s, hv[m], hi[m]);
      if (st != RT_SUCCESS) return bail(st);
      rtb::BuildInput in{hv[m].data(), hi[m].data(), meshes[m].vertex_count, meshes[m].triangle_count};
      std::string err;
      if (!rtb::build_mesh(in, width, max_leaf, blas[m], err, threads)) {
        rt_status code = err.find("vertex index") != std::string::npos ? RT_ERROR_INDEX_OUT_OF_RANGE
                                                                        : RT_ERROR_INVALID_VALUE;
        return bail(fail(code, "rt_build: mesh %u: %s", m, err.c_str()));
      }
      input_tris += meshes[m].triangle_count;
    }
    rtb::WideTree tlas;
    if (a->two_level) {
      std::vector<rtb::Box> boxes(instance_count);
      for (uint32_t j = 0; j < instance_count; ++j) {
        const rtb::WideTree& b = blas[instance_mesh[j]];
        if (b.root == RT_CHILD_EMPTY) {
          for (int k = 0; k < 3; ++k) {
            boxes[j].lo[k] = INFINITY;
            boxes[j].hi[k] = -INFINITY;
          }
        } else {
          boxes[j] = world_box(b.bounds, instance_srt[j]);
        }
      }
      rtb::build_instances(boxes, width, tlas, threads);
    }
    // concatenate node and triangle arrays: [tlas][blas 0][blas 1]...
    const uint32_t fpn = 8u * (uint32_t)width;
    uint64_t node_total = tlas.node_count, tri_total = 0;
    std::vector<uint32_t> node_base(mesh_count), tri_base(mesh_count);
    for (uint32_t m = 0; m < mesh_count; ++m) {
      node_base[m] = (uint32_t)node_total;
      tri_base[m] = (uint32_t)tri_total;
      node_total += blas[m].node_count;
      tri_total += blas[m].tris.size();
    }
    if (node_total >= 0x7FFFFFFFull || tri_total > RT_MAX_TRI_RECORDS)
      return bail(fail(RT_ERROR_INVALID_VALUE, "rt_build: scene too large for one accel"));
    std::vector<float> nodes((size_t)node_total * fpn);
    std::vector<rt_tri_rec> tris((size_t)tri_total);
    auto relocate = [&](const rtb::WideTree& t, uint32_t nb, uint32_t tb, float* dst) {
      std::memcpy(dst, t.nodes.data(), t.nodes.size() * 4);
      for (uint32_t i = 0; i < t.node_count; ++i)
        for (int c = 0; c < width; ++c) {
          uint32_t ref;
          float* slot = dst + (size_t)i * fpn + 6 * width + c;
          std::memcpy(&ref, slot, 4);
          if (ref == RT_CHILD_EMPTY) continue;
          if ((ref & RT_LEAF_BIT) == 0) ref += nb;
          else if ((ref & RT_INST_BIT) == 0) ref += tb;  // first-record field is the low bits
          std::memcpy(slot, &ref, 4);
        }
    };
    if (tlas.node_count) relocate(tlas, 0, 0, nodes.data());
    uint32_t max_blas_stack = 0, max_blas_depth = 0;
    for (uint32_t m = 0; m < mesh_count; ++m) {
      if (blas[m].node_count) relocate(blas[m], node_base[m], tri_base[m], nodes.data() + (size_t)node_base[m] * fpn);
      std::copy(blas[m].tris.begin(), blas[m].tris.end(), tris.begin() + tri_base[m]);
      max_blas_stack = std::max(max_blas_stack, blas[m].max_stack);
      max_blas_depth = std::max(max_blas_depth, blas[m].max_depth);
      a->info.leaf_count += blas[m].leaf_count;
    }
    double sah = 0.0;
    if (a->two_level) {
      a->root = tlas.root;  // node 0 or empty
      a->max_stack = tlas.max_stack + 1 + max_blas_stack;
      a->info.max_depth = tlas.max_depth + max_blas_depth;
      a->info.leaf_count += tlas.leaf_count;
      sah = tlas.sah_cost;
    } else {
      a->root = blas[0].root == RT_CHILD_EMPTY ? RT_CHILD_EMPTY : node_base[0];
      a->max_stack = blas[0].max_stack;
      a->info.max_depth = blas[0].max_depth;
      sah = blas[0].sah_cost;
    }
    a->max_stack = std::max(a->max_stack, 1u);
    a->info.node_count = (uint32_t)node_total;
    a->info.triangle_count = (uint32_t)tri_total;
    a->info.input_triangles = (uint32_t)std::min<uint64_t>(input_tris, 0xFFFFFFFFull);
    a->info.max_stack = a->max_stack;
    a->info.sah_cost = sah;

    // device copies
    st = dev_alloc(a, &a->nodes, nodes.size());
    if (st != RT_SUCCESS) return bail(st);
    st = dev_alloc(a, &a->tris, tris.size());
    if (st != RT_SUCCESS) return bail(st);
    if (!nodes.empty()) RT_HIP_BAIL(hipMemcpyAsync(a->nodes, nodes.data(), nodes.size() * 4, hipMemcpyHostToDevice, s));
    if (!tris.empty())
      RT_HIP_BAIL(hipMemcpyAsync(a->tris, tris.data(), tris.size() * sizeof(rt_tri_rec), hipMemcpyHostToDevice, s));
    a->host_meshes.resize(mesh_count);
    for (uint32_t m = 0; m < mesh_count; ++m) {
      float* dv = nullptr;
      uint32_t* di = nullptr;
      st = dev_alloc(a, &dv, hv[m].size());
      if (st != RT_SUCCESS) return bail(st);
      st = dev_alloc(a, &di, hi[m].size());
      if (st != RT_SUCCESS) return bail(st);
      if (!hv[m].empty()) RT_HIP_BAIL(hipMemcpyAsync(dv, hv[m].data(), hv[m].size() * 4, hipMemcpyHostToDevice, s));
      if (!hi[m].empty()) RT_HIP_BAIL(hipMemcpyAsync(di, hi[m].data(), hi[m].size() * 4, hipMemcpyHostToDevice, s));
      a->host_meshes[m] = rt_mesh_dev{dv, di, meshes[m].vertex_count, meshes[m].triangle_count};
    }
    st = dev_alloc(a, &a->meshes, mesh_count);
    if (st != RT_SUCCESS) return bail(st);
    RT_HIP_BAIL(hipMemcpyAsync(a->meshes, a->host_meshes.data(), mesh_count * sizeof(rt_mesh_dev), hipMemcpyHostToDevice, s));
    {
      // the meshes' node ids grouped by depth in their own tree, deepest
      // first, for the bottom-up refit (a node's children are one deeper)
      uint32_t maxd = 0;
      for (uint32_t m = 0; m < mesh_count; ++m)
        for (uint32_t i = 0; i < blas[m].node_count && i < blas[m].node_depth.size(); ++i)
          maxd = std::max(maxd, blas[m].node_depth[i]);
      std::vector<uint32_t> order;
      a->refit_levels.assign(1, 0);
      for (uint32_t d = maxd; d >= 1; --d) {
        for (uint32_t m = 0; m < mesh_count; ++m) {
          const std::vector<uint32_t>& dep = blas[m].node_depth;
          for (uint32_t i = 0; i < blas[m].node_count && i < dep.size(); ++i)
            if (dep[i] == d) order.push_back(i + node_base[m]);
        }
        a->refit_levels.push_back((uint32_t)order.size());
      }
      a->mesh_tri_base = tri_base;
      if (!order.empty()) {
        st = dev_alloc(a, &a->refit_nodes, order.size());
        if (st != RT_SUCCESS) return bail(st);
        RT_HIP_BAIL(hipMemcpyAsync(a->refit_nodes, order.data(), order.size() * 4, hipMemcpyHostToDevice, s));
      }
    }
    if (a->two_level) {
      std::vector<uint32_t> blas_root(mesh_count);
      for (uint32_t m = 0; m < mesh_count; ++m)
        blas_root[m] = blas[m].root == RT_CHILD_EMPTY ? RT_CHILD_EMPTY : node_base[m];
      st = setup_instances(a, meshes, mesh_count, instance_mesh, instance_srt, instance_count, blas_root, s);
      if (st != RT_SUCCESS) return bail(st);
      a->tlas_nodes = tlas.nodes;
      a->tlas_nodes.resize((size_t)tlas.node_count * fpn);
      a->tlas_depth = tlas.node_depth;
      a->tlas_depth.resize(tlas.node_count);
      a->mesh_bounds.resize(mesh_count);
      for (uint32_t m = 0; m < mesh_count; ++m) {
        if (blas[m].root == RT_CHILD_EMPTY) {
          for (int k = 0; k < 3; ++k) {
            a->mesh_bounds[m].lo[k] = INFINITY;
            a->mesh_bounds[m].hi[k] = -INFINITY;
          }
        } else {
          a->mesh_bounds[m] = blas[m].bounds;
        }
      }
    }
    RT_HIP_BAIL(hipStreamSynchronize(s));
  } catch (const std::bad_alloc&) {
    return bail(fail(RT_ERROR_OUT_OF_MEMORY, "rt_build: host allocation failed"));
  } catch (const std::exception& ex) {
    return bail(fail(RT_ERROR_INVALID_VALUE, "rt_build: %s", ex.what()));
  }
  *out = a;
  return ok();
}

rt_status rt_accel_destroy(rt_accel accel) {
  if (!accel) return fail(RT_ERROR_INVALID_VALUE, "rt_accel_destroy: NULL accel");
  (void)hipSetDevice(accel->device);
  (void)hipDeviceSynchronize();
  destroy_accel(accel);
  return ok();
}

rt_status rt_accel_get_info(rt_accel accel, rt_accel_info* out) {
  if (!accel || !out) return fail(RT_ERROR_INVALID_VALUE, "rt_accel_get_info: NULL argument");
  *out = accel->info;
  return ok();
}

// ---------------------------------------------------------------------------
// queries
// ---------------------------------------------------------------------------

static uint32_t cached_resident(rt_context ctx, const void* kern, int wg) {
  if (ctx->blocks_per_cu) return ctx->blocks_per_cu * (uint32_t)std::max(ctx->cu_count, 1);
  for (auto& e : ctx->occupancy)
    if (e.first == kern) return e.second;
  uint32_t b = resident_blocks(kern, wg, ctx->cu_count);
  ctx->occupancy.emplace_back(kern, b);
  return b;
}

// The backward's accumulator rows of an accel: one per vertex (two-level: of
// every mesh), then four per instance frame.  Allocated by the first backward
// call (sized by the accel, not by the call, so later calls allocate
// nothing) and cleared on `s`; a call that stopped between its launches left
// them dirty, and the next call clears them first.
static rt_status prepare_grad_rows(rt_accel a, hipStream_t s) {
  if (!a->grad_rows.expo) {
    uint64_t rows = a->two_level ? a->vertex_rows + 4ull * a->instance_count
                                 : (uint64_t)a->host_meshes[0].vertex_count;
    if (rows >= 0xFFFFFFFFull) return fail(RT_ERROR_UNSUPPORTED, "backward: more than 2^32 - 2 gradient rows");
    if (rows == 0) return RT_SUCCESS;
    hipError_t e = rta::alloc(a->grad_rows, (uint32_t)rows);
    if (e != hipSuccess)
      return fail(e == hipErrorOutOfMemory ? RT_ERROR_OUT_OF_MEMORY : RT_ERROR_HIP,
                  "backward: gradient rows (%llu): %s", (unsigned long long)rows, hipGetErrorString(e));
    a->info.device_bytes += rows * (sizeof(uint32_t) + rta::kCopies * 4 * sizeof(unsigned long long));
    a->grad_dirty = true;
  }
  if (a->grad_dirty) RT_HIP(rta::clear(a->grad_rows, s));
  a->grad_dirty = true;
  return RT_SUCCESS;
}

// As cached_resident, without adding to the cache (no host allocation).
static uint32_t peek_resident(rt_context ctx, const void* kern, int wg) {
  if (ctx->blocks_per_cu) return ctx->blocks_per_cu * (uint32_t)std::max(ctx->cu_count, 1);
  for (auto& e : ctx->occupancy)
    if (e.first == kern) return e.second;
  return resident_blocks(kern, wg, ctx->cu_count);
}

// mode 0: plain query; 2: with query options; 3: all hits (options, lists of
// `cap` entries and per-ray counts)
static rt_status launch_trace(rt_accel a, const rt_ray* rays, uint32_t n, rt_hit* hits,
                              uint32_t* inst_ids, uint8_t* occ, bool any, hipStream_t s,
                              uint64_t* counters = nullptr, int mode = 0,
                              const rt_query_options* opts = nullptr, uint32_t* counts = nullptr,
                              uint32_t cap = 0, bool noalloc = false, bool phases = false) {
  rt_context ctx = a->ctx;
  rt_status st = check_device(a->device);
  if (st != RT_SUCCESS) return st;
  std::lock_guard<std::mutex> lk(ctx->mu);
  st = take_overflow(ctx, "trace");
  if (st != RT_SUCCESS) return st;
  rt_variant v = ctx->variant;
  if (counters || mode >= 2) v = rt_variant{16, 256};
  const void* kern = counters ? rtk_count_kernel(a->width, any, a->two_level)
                              : rtk_trace_kernel(a->width, (int)v.stack_entries, (int)v.workgroup,
                                                 any, a->two_level, mode);
  if (!kern) return fail(RT_ERROR_UNSUPPORTED, "trace: variant not compiled");
  uint32_t wg = v.workgroup;
  uint32_t resident = noalloc ? peek_resident(ctx, kern, (int)wg) : cached_resident(ctx, kern, (int)wg);
  uint32_t blocks = std::max(std::min<uint32_t>((n + wg - 1) / wg, resident), 1u);
  size_t spill = a->max_stack > v.stack_entries ? (size_t)(a->max_stack - v.stack_entries) : 1;
  const bool fused = !counters && rtk_trace_fuses_finalize(any, a->two_level, mode);
  uint32_t* counter = nullptr;
  uint32_t* gstack = nullptr;
  uint32_t* ranges = nullptr;
  uint32_t* ovf = nullptr;
  uint32_t ovf_cap = 0;
  if (noalloc) {
    // the fixed array: 64 counter words, then (fused finalize) the per-wave
    // range lists and the overflow list, then the spill stack; the grid is
    // narrowed until they fit
    uint32_t* base = noalloc_ptr(a->device);
    if (!base) return fail(RT_ERROR_HIP, "rt_trace_closest_noalloc: no scratch on device %d", a->device);
    size_t cap_pairs = (size_t)n / std::max<uint32_t>(1u, std::min<uint32_t>(ctx->refill_min, 64u)) + 1;
    size_t fixed = 64 + (fused ? 2 * cap_pairs : 0);
    size_t per_block = (fused ? (size_t)(wg / 64u) * 2 * kRtRangesPerWave : 0) + spill * wg;
    if (fixed + per_block > kNoAllocWords)
      return fail(RT_ERROR_INVALID_VALUE,
                  "rt_trace_closest_noalloc: %u rays with a stack bound of %u need more than the %u-byte "
                  "scratch", n, a->max_stack, (unsigned)RT_NOALLOC_SCRATCH_BYTES);
    blocks = (uint32_t)std::min<size_t>(blocks, (kNoAllocWords - fixed) / per_block);
    counter = base;
    if (fused) {
      ranges = base + 64;
      ovf = ranges + (size_t)blocks * (wg / 64u) * 2 * kRtRangesPerWave;
      ovf_cap = (uint32_t)cap_pairs;
      gstack = ovf + 2 * cap_pairs;
    } else {
      gstack = base + 64;
    }
  } else {
    st = ensure_scratch(ctx->scratch, spill * (size_t)blocks * wg);
    if (st != RT_SUCCESS) return st;
    counter = ctx->scratch.counter;
    gstack = ctx->scratch.gstack;
    if (fused) {
      st = ensure_ranges(ctx->scratch, blocks * wg, n, ctx->refill_min, &ranges, &ovf, &ovf_cap);
      if (st != RT_SUCCESS) return st;
    }
  }
  uint32_t gstride = blocks * wg;
  if (ctx->has_last && ctx->last_stream != s) RT_HIP(hipStreamWaitEvent(s, ctx->last_event, 0));
  TraceParams p{};
  p.nodes = a->nodes;
  p.tris = a->tris;
  p.insts = a->insts;
  p.insts64 = a->insts64;
  p.meshes = a->meshes;
  p.rays = rays;
  p.hits = hits;
  p.inst_ids = inst_ids;
  p.occluded = occ;
  p.counter = counter;
  p.gstack = gstack;
  p.root = a->root;
  p.n = n;
  // the kernels take a bound of at least their LDS entries
  p.max_stack = ctx->stack_limit ? std::max(std::min(a->max_stack, ctx->stack_limit), v.stack_entries)
                                 : a->max_stack;
  p.gstride = gstride;
  p.refill_min = ctx->refill_min;
  p.counters = counters;
  p.phase_counters = (counters && phases) ? 1u : 0u;
  p.status = ctx->status;
  if (opts) {
    p.ray_masks = opts->ray_masks;
    p.skip_inst = opts->skip_inst;
    p.skip_prim = opts->skip_prim;
  }
  p.counts = counts;
  p.cap = cap;
  p.ranges = ranges;
  p.ovf = ovf;
  p.ovf_cap = ovf_cap;
  RT_HIP(rtk_launch_fill(counter, 2, 0u, s));
  size_t tslot = ctx->tbeg.empty() ? 0 : (size_t)(ctx->trecorded % ctx->tbeg.size());
  if (!ctx->tbeg.empty()) RT_HIP(hipEventRecord(ctx->tbeg[tslot], s));
  RT_HIP(rtk_launch_trace(kern, blocks, wg, p, s));
  if (!ctx->tbeg.empty()) {
    RT_HIP(hipEventRecord(ctx->tend[tslot], s));
    ctx->trecorded++;
  }
  if (mode == 3) {
    RT_HIP(rtk_launch_finalize_all(a->two_level, p, s));
  } else if (fused) {
    RT_HIP(rtk_launch_finalize_ovf(a->two_level, p, s));
  } else if (!any) {
    RT_HIP(rtk_launch_finalize(a->two_level, 0, p, s));
  }
  RT_HIP(hipEventRecord(ctx->last_event, s));
  ctx->last_stream = s;
  ctx->has_last = true;
  return ok();
}

rt_status rt_trace_closest(rt_accel accel, const rt_ray* rays, uint32_t n, rt_hit* hits,
                           uint32_t* inst_ids, void* stream) {
  if (!accel) return fail(RT_ERROR_INVALID_VALUE, "rt_trace_closest: NULL accel");
  if (n == 0) return ok();
  if (!rays || !hits) return fail(RT_ERROR_INVALID_VALUE, "rt_trace_closest: NULL buffer with n > 0");
  if (n > 0x7FFFFFFFu) return fail(RT_ERROR_INVALID_VALUE, "rt_trace_closest: n >= 2^31");
  if (!aligned16(rays) || !aligned16(hits))
    return fail(RT_ERROR_INVALID_VALUE, "rt_trace_closest: rays and hits must be 16-byte aligned");
  return launch_trace(accel, rays, n, hits, inst_ids, nullptr, false, static_cast<hipStream_t>(stream));
}

rt_status rt_trace_closest_noalloc(rt_accel accel, const rt_ray* rays, uint32_t n, rt_hit* hits,
                                   uint32_t* inst_ids, void* stream) {
  if (!accel) return fail(RT_ERROR_INVALID_VALUE, "rt_trace_closest_noalloc: NULL accel");
  if (n == 0) return ok();
  if (!rays || !hits) return fail(RT_ERROR_INVALID_VALUE, "rt_trace_closest_noalloc: NULL buffer with n > 0");
  if (n > 0x7FFFFFFFu) return fail(RT_ERROR_INVALID_VALUE, "rt_trace_closest_noalloc: n >= 2^31");
  if (!aligned16(rays) || !aligned16(hits))
    return fail(RT_ERROR_INVALID_VALUE, "rt_trace_closest_noalloc: rays and hits must be 16-byte aligned");
  return launch_trace(accel, rays, n, hits, inst_ids, nullptr, false, static_cast<hipStream_t>(stream),
                      nullptr, 0, nullptr, nullptr, 0, true);
}

rt_status rt_trace_any(rt_accel accel, const rt_ray* rays, uint32_t n, uint8_t* occluded,
                       void* stream) {
  if (!accel) return fail(RT_ERROR_INVALID_VALUE, "rt_trace_any: NULL accel");
  if (n == 0) return ok();
  if (!rays || !occluded) return fail(RT_ERROR_INVALID_VALUE, "rt_trace_any: NULL buffer with n > 0");
  if (n > 0x7FFFFFFFu) return fail(RT_ERROR_INVALID_VALUE, "rt_trace_any: n >= 2^31");
  if (!aligned16(rays)) return fail(RT_ERROR_INVALID_VALUE, "rt_trace_any: rays must be 16-byte aligned");
  return launch_trace(accel, rays, n, nullptr, nullptr, occluded, true, static_cast<hipStream_t>(stream));
}

static bool options_ok(rt_accel a, const rt_query_options* o) {
  return !(o && a->two_level && o->skip_prim && !o->skip_inst);
}

rt_status rt_trace_closest_ex(rt_accel accel, const rt_ray* rays, uint32_t n,
                              const rt_query_options* options, rt_hit* hits, uint32_t* inst_ids,
                              void* stream) {
  if (!accel) return fail(RT_ERROR_INVALID_VALUE, "rt_trace_closest_ex: NULL accel");
  if (!options_ok(accel, options))
    return fail(RT_ERROR_INVALID_VALUE, "rt_trace_closest_ex: skip_prim without skip_inst on a two-level accel");
  if (n == 0) return ok();
  if (!rays || !hits) return fail(RT_ERROR_INVALID_VALUE, "rt_trace_closest_ex: NULL buffer with n > 0");
  if (n > 0x7FFFFFFFu) return fail(RT_ERROR_INVALID_VALUE, "rt_trace_closest_ex: n >= 2^31");
  if (!aligned16(rays) || !aligned16(hits))
    return fail(RT_ERROR_INVALID_VALUE, "rt_trace_closest_ex: rays and hits must be 16-byte aligned");
  return launch_trace(accel, rays, n, hits, inst_ids, nullptr, false, static_cast<hipStream_t>(stream),
                      nullptr, 2, options);
}

rt_status rt_trace_any_ex(rt_accel accel, const rt_ray* rays, uint32_t n,
                          const rt_query_options* options, uint8_t* occluded, void* stream) {
  if (!accel) return fail(RT_ERROR_INVALID_VALUE, "rt_trace_any_ex: NULL accel");
  if (!options_ok(accel, options))
    return fail(RT_ERROR_INVALID_VALUE, "rt_trace_any_ex: skip_prim without skip_inst on a two-level accel");
  if (n == 0) return ok();
  if (!rays || !occluded) return fail(RT_ERROR_INVALID_VALUE, "rt_trace_any_ex: NULL buffer with n > 0");
  if (n > 0x7FFFFFFFu) return fail(RT_ERROR_INVALID_VALUE, "rt_trace_any_ex: n >= 2^31");
  if (!aligned16(rays)) return fail(RT_ERROR_INVALID_VALUE, "rt_trace_any_ex: rays must be 16-byte aligned");
  return launch_trace(accel, rays, n, nullptr, nullptr, occluded, true, static_cast<hipStream_t>(stream),
                      nullptr, 2, options);
}

rt_status rt_trace_all(rt_accel accel, const rt_ray* rays, uint32_t n,
                       const rt_query_options* options, uint32_t capacity, rt_hit* hits,
                       uint32_t* inst_ids, uint32_t* counts, void* stream) {
  if (!accel) return fail(RT_ERROR_INVALID_VALUE, "rt_trace_all: NULL accel");
  if (!options_ok(accel, options))
    return fail(RT_ERROR_INVALID_VALUE, "rt_trace_all: skip_prim without skip_inst on a two-level accel");
  if (capacity < 1 || capacity > RT_MAX_HIT_CAPACITY)
    return fail(RT_ERROR_INVALID_VALUE, "rt_trace_all: capacity %u outside [1, %u]", capacity,
                (unsigned)RT_MAX_HIT_CAPACITY);
  if (n == 0) return ok();
  if (!rays || !hits || !counts) return fail(RT_ERROR_INVALID_VALUE, "rt_trace_all: NULL buffer with n > 0");
  if ((uint64_t)n * capacity > 0x7FFFFFFFull)
    return fail(RT_ERROR_INVALID_VALUE, "rt_trace_all: n * capacity >= 2^31");
  if (!aligned16(rays) || !aligned16(hits))
    return fail(RT_ERROR_INVALID_VALUE, "rt_trace_all: rays and hits must be 16-byte aligned");
  return launch_trace(accel, rays, n, hits, inst_ids, nullptr, false, static_cast<hipStream_t>(stream),
                      nullptr, 3, options, counts, capacity);
}

rt_status rt_accel_set_instance_masks(rt_accel accel, const uint32_t* masks, void* stream) {
  if (!accel) return fail(RT_ERROR_INVALID_VALUE, "rt_accel_set_instance_masks: NULL accel");
  if (!accel->two_level)
    return fail(RT_ERROR_UNSUPPORTED, "rt_accel_set_instance_masks: single-level accel (no instances)");
  if (!masks) return fail(RT_ERROR_INVALID_VALUE, "rt_accel_set_instance_masks: masks is NULL");
  rt_status st = check_device(accel->device);
  if (st != RT_SUCCESS) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (uint32_t j = 0; j < accel->instance_count; ++j) accel->host_insts[j].mask = masks[j];
  RT_HIP(hipMemcpyAsync(accel->insts, accel->host_insts.data(),
                        accel->host_insts.size() * sizeof(rt_inst_rec), hipMemcpyHostToDevice, s));
  RT_HIP(hipStreamSynchronize(s));
  return ok();
}

// Refits the boxes of a two-level accel's top-level tree, bottom-up over
// its kept topology, to the world boxes of the instances (the current frames
// applied to the meshes' bounds), and enqueues the upload of its nodes.
static rt_status refit_top_level(rt_accel_s* a, hipStream_t s) {
  const uint32_t n = a->instance_count;
  const int W = a->width;
  const uint32_t fpn = 8u * (uint32_t)W;
  std::vector<rtb::Box> wb(n);
  for (uint32_t j = 0; j < n; ++j) {
    const rtb::Box& b = a->mesh_bounds[a->host_inst_mesh[j]];
    if (b.lo[0] <= b.hi[0] && b.lo[1] <= b.hi[1] && b.lo[2] <= b.hi[2]) {
      wb[j] = world_box(b, a->host_srts[j]);
    } else {
      for (int k = 0; k < 3; ++k) {
        wb[j].lo[k] = INFINITY;
        wb[j].hi[k] = -INFINITY;
      }
    }
  }
  // deepest nodes first; each child slot from its instance's world box or
  // from the union of its node's slots
  std::vector<float>& T = a->tlas_nodes;
  const uint32_t tn = (uint32_t)a->tlas_depth.size();
  uint32_t maxd = 0;
  for (uint32_t d : a->tlas_depth) maxd = std::max(maxd, d);
  double area_sum = 0.0;
  rtb::Box root{};
  for (uint32_t d = maxd; d >= 1; --d) {
    for (uint32_t i = 0; i < tn; ++i) {
      if (a->tlas_depth[i] != d) continue;
      float* nd = T.data() + (size_t)i * fpn;
      rtb::Box nb;
      for (int k = 0; k < 3; ++k) {
        nb.lo[k] = INFINITY;
        nb.hi[k] = -INFINITY;
      }
      for (int c = 0; c < W; ++c) {
        uint32_t ref;
        std::memcpy(&ref, &nd[6 * W + c], 4);
        if (ref == RT_CHILD_EMPTY) continue;
        rtb::Box cb;
        if ((ref & RT_LEAF_BIT) == 0u) {
          const float* ch = T.data() + (size_t)ref * fpn;  // top-level refs are node indices
          for (int k = 0; k < 3; ++k) {
            cb.lo[k] = INFINITY;
            cb.hi[k] = -INFINITY;
          }
          for (int q = 0; q < W; ++q)
            for (int k = 0; k < 3; ++k) {
              cb.lo[k] = std::min(cb.lo[k], ch[(2 * k) * W + q]);
              cb.hi[k] = std::max(cb.hi[k], ch[(2 * k + 1) * W + q]);
            }
        } else {
          cb = wb[ref & RT_INST_INDEX_MASK];
        }
        for (int k = 0; k < 3; ++k) {
          nd[(2 * k) * W + c] = cb.lo[k];
          nd[(2 * k + 1) * W + c] = cb.hi[k];
          nb.lo[k] = std::min(nb.lo[k], cb.lo[k]);
          nb.hi[k] = std::max(nb.hi[k], cb.hi[k]);
        }
      }
      double dx = (double)nb.hi[0] - nb.lo[0], dy = (double)nb.hi[1] - nb.lo[1], dz = (double)nb.hi[2] - nb.lo[2];
      if (dx >= 0 && dy >= 0 && dz >= 0) area_sum += 2.0 * (dx * dy + dy * dz + dz * dx);
      if (i == 0) root = nb;
    }
    if (d == 1) break;
  }
  if (tn > 0) {
    double dx = (double)root.hi[0] - root.lo[0], dy = (double)root.hi[1] - root.lo[1],
           dz = (double)root.hi[2] - root.lo[2];
    double ra = 2.0 * (dx * dy + dy * dz + dz * dx);
    a->info.sah_cost = ra > 0.0 ? area_sum / ra : 0.0;
    RT_HIP(hipMemcpyAsync(a->nodes, T.data(), (size_t)tn * fpn * 4, hipMemcpyHostToDevice, s));
  }
  return RT_SUCCESS;
}

rt_status rt_update_instances(rt_accel accel, const rt_srt* instance_srt, void* stream) {
  if (!accel) return fail(RT_ERROR_INVALID_VALUE, "rt_update_instances: NULL accel");
  if (!accel->two_level)
    return fail(RT_ERROR_UNSUPPORTED, "rt_update_instances: single-level accel (no instances)");
  if (!instance_srt) return fail(RT_ERROR_INVALID_VALUE, "rt_update_instances: instance_srt is NULL");
  const uint32_t n = accel->instance_count;
  rt_status st = check_frames(instance_srt, n, "rt_update_instances");
  if (st != RT_SUCCESS) return st;
  st = check_device(accel->device);
  if (st != RT_SUCCESS) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    // instance records: new maps, same roots, meshes and masks
    std::vector<rt_inst_rec64> ir64(n);
    for (uint32_t j = 0; j < n; ++j) {
      double m[12];
      srt_inverse(instance_srt[j], m);
      std::memcpy(ir64[j].m, m, sizeof(m));
      rt_inst_rec& r = accel->host_insts[j];
      for (int k = 0; k < 4; ++k) {
        r.r0[k] = (float)m[k];
        r.r1[k] = (float)m[4 + k];
        r.r2[k] = (float)m[8 + k];
      }
    }
    accel->host_srts.assign(instance_srt, instance_srt + n);
    st = refit_top_level(accel, s);
    if (st != RT_SUCCESS) return st;
    RT_HIP(hipMemcpyAsync(accel->insts, accel->host_insts.data(), n * sizeof(rt_inst_rec), hipMemcpyHostToDevice, s));
    RT_HIP(hipMemcpyAsync(accel->insts64, ir64.data(), n * sizeof(rt_inst_rec64), hipMemcpyHostToDevice, s));
    RT_HIP(hipMemcpyAsync(accel->srts, instance_srt, n * sizeof(rt_srt), hipMemcpyHostToDevice, s));
    RT_HIP(hipStreamSynchronize(s));
  } catch (const std::bad_alloc&) {
    return fail(RT_ERROR_OUT_OF_MEMORY, "rt_update_instances: host allocation failed");
  }
  return ok();
}

rt_status rt_trace_counters(rt_accel accel, const rt_ray* rays, uint32_t n, int any, rt_hit* hits,
                            uint8_t* occluded, uint64_t* counters, void* stream) {
  return rt_trace_counters_ex(accel, rays, n, any, hits, occluded, counters, 4, stream);
}

rt_status rt_trace_counters_ex(rt_accel accel, const rt_ray* rays, uint32_t n, int any, rt_hit* hits,
                               uint8_t* occluded, uint64_t* counters, uint32_t n_counters, void* stream) {
  if (n_counters != 4 && n_counters != 8)
    return fail(RT_ERROR_INVALID_VALUE, "rt_trace_counters: n_counters must be 4 or 8, got %u", n_counters);
  if (!accel) return fail(RT_ERROR_INVALID_VALUE, "rt_trace_counters: NULL accel");
  if (n == 0) return ok();
  if (!rays || !counters || (any ? !occluded : !hits))
    return fail(RT_ERROR_INVALID_VALUE, "rt_trace_counters: NULL buffer with n > 0");
  if (n > 0x7FFFFFFFu) return fail(RT_ERROR_INVALID_VALUE, "rt_trace_counters: n >= 2^31");
  if (!aligned16(rays) || (!any && !aligned16(hits)))
    return fail(RT_ERROR_INVALID_VALUE, "rt_trace_counters: rays and hits must be 16-byte aligned");
  return launch_trace(accel, rays, n, any ? nullptr : hits, nullptr, any ? occluded : nullptr,
                      any != 0, static_cast<hipStream_t>(stream), counters, 0, nullptr, nullptr, 0, false,
                      n_counters == 8);
}

rt_status rt_trace_backward(rt_accel accel, const rt_ray* rays, const rt_hit* hits,
                            const float* d_tuv, uint32_t n, float* d_vertices, float* d_origins,
                            float* d_directions, void* stream) {
  if (!accel) return fail(RT_ERROR_INVALID_VALUE, "rt_trace_backward: NULL accel");
  if (accel->two_level)
    return fail(RT_ERROR_UNSUPPORTED, "rt_trace_backward: two-level accel (use rt_trace_backward_instances)");
  if (n == 0) return ok();
  if (!rays || !hits || !d_tuv || !d_vertices || !d_origins || !d_directions)
    return fail(RT_ERROR_INVALID_VALUE, "rt_trace_backward: NULL buffer with n > 0");
  if (!aligned16(rays) || !aligned16(hits))
    return fail(RT_ERROR_INVALID_VALUE, "rt_trace_backward: rays and hits must be 16-byte aligned");
  rt_status st = check_device(accel->device);
  if (st != RT_SUCCESS) return st;
  rt_context ctx = accel->ctx;
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (ctx->has_last && ctx->last_stream != s) RT_HIP(hipStreamWaitEvent(s, ctx->last_event, 0));
  const rt_mesh_dev& mesh = accel->host_meshes[0];
  if (!accel->gather.csr_off) {
    // the vertex -> (triangle, corner) lists, built once from the accel's
    // copy of the indices
    std::vector<uint32_t> idx;
    try {
      idx.resize(3 * (size_t)mesh.triangle_count);
    } catch (const std::bad_alloc&) {
      return fail(RT_ERROR_OUT_OF_MEMORY, "rt_trace_backward: host allocation");
    }
    if (!idx.empty())
      RT_HIP(hipMemcpy(idx.data(), mesh.indices, idx.size() * sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (rta::bucket_shift(mesh.triangle_count) == 0)
      return fail(RT_ERROR_UNSUPPORTED, "rt_trace_backward: more than %u triangles", rta::kMaxBuckets << 10);
    RT_HIP(rta::gather_build(accel->gather, idx.data(), mesh.vertex_count, mesh.triangle_count));
    accel->info.device_bytes += 4ull * (mesh.vertex_count + 1) + 120ull * mesh.triangle_count;
  }
  if (!accel->gather.tri_vertices_valid) {
    RT_HIP(rta::gather_tri_vertices(accel->gather, mesh.indices, mesh.vertices, mesh.triangle_count, 0, s));
    accel->gather.tri_vertices_valid = true;
  }
  RT_HIP(rta::sort_reserve(ctx->sortbuf, accel->gather.buckets, n, s));
  BackwardParams p{};
  p.mesh = mesh;
  p.tri_vertices = accel->gather.tri_vertices;
  p.rays = rays;
  p.hits = hits;
  p.d_tuv = d_tuv;
  p.n = n;
  p.d_origins = d_origins;
  p.d_directions = d_directions;
  rta::KeySource keys{reinterpret_cast<const uint32_t*>(hits), nullptr, nullptr, 0, mesh.triangle_count, 0};
  RT_HIP(rta::bucket_rays(keys, accel->gather.buckets, accel->gather.shift, ctx->sortbuf, n, s, &p.bk));
  RT_HIP(rtk_launch_backward(p, s));
  RT_HIP(rta::gather_vertices(accel->gather, ctx->sortbuf, n, d_vertices, s));
  RT_HIP(hipEventRecord(ctx->last_event, s));
  ctx->last_stream = s;
  ctx->has_last = true;
  return ok();
}

rt_status rt_trace_backward_instances(rt_accel accel, const rt_ray* rays, const rt_hit* hits,
                                      const uint32_t* inst_ids, const float* d_tuv, uint32_t n,
                                      float* d_vertices, float* d_srt, float* d_origins,
                                      float* d_directions, void* stream) {
  if (!accel) return fail(RT_ERROR_INVALID_VALUE, "rt_trace_backward_instances: NULL accel");
  if (!accel->two_level)
    return fail(RT_ERROR_UNSUPPORTED,
                "rt_trace_backward_instances: single-level accel (use rt_trace_backward)");
  if (n == 0) return ok();
  if (!rays || !hits || !inst_ids || !d_tuv || !d_origins || !d_directions)
    return fail(RT_ERROR_INVALID_VALUE, "rt_trace_backward_instances: NULL buffer with n > 0");
  if (!aligned16(rays) || !aligned16(hits))
    return fail(RT_ERROR_INVALID_VALUE,
                "rt_trace_backward_instances: rays and hits must be 16-byte aligned");
  if (d_vertices && accel->vertex_rows >= 0xFFFFFFFFull)
    return fail(RT_ERROR_UNSUPPORTED, "rt_trace_backward_instances: more than 2^32 - 2 vertex rows");
  rt_status st = check_device(accel->device);
  if (st != RT_SUCCESS) return st;
  rt_context ctx = accel->ctx;
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (ctx->has_last && ctx->last_stream != s) RT_HIP(hipStreamWaitEvent(s, ctx->last_event, 0));
  BackwardInstParams p{};
  p.meshes = accel->meshes;
  p.vertex_base = accel->vertex_base;
  p.insts = accel->insts;
  p.insts64 = accel->insts64;
  p.srts = accel->srts;
  p.inst_count = accel->instance_count;
  p.rays = rays;
  p.hits = hits;
  p.inst_ids = inst_ids;
  p.d_tuv = d_tuv;
  p.n = n;
  p.d_origins = d_origins;
  p.d_directions = d_directions;
  p.want_vertices = (d_vertices && accel->vertex_rows > 0) ? 1u : 0u;
  p.want_frames = d_srt ? 1u : 0u;
  const uint32_t nm = (uint32_t)accel->host_meshes.size();
  uint64_t total_tris = 0;
  for (const rt_mesh_dev& md : accel->host_meshes) total_tris += md.triangle_count;
  if (!ctx->backward_atomic && accel->instance_count <= rta::kMaxBuckets && total_tris < (1ull << 30) &&
      rta::bucket_shift((uint32_t)total_tris, 6) != 0) {
    // rays grouped by triangle range and by instance, exact sums per group
    rta::Gather& g = accel->gather;
    if (!g.csr_off) {
      std::vector<std::vector<uint32_t>> idx(nm);
      std::vector<const uint32_t*> ip(nm);
      std::vector<uint32_t> vc(nm), tc(nm), im(accel->instance_count);
      try {
        for (uint32_t m = 0; m < nm; ++m) {
          const rt_mesh_dev& md = accel->host_meshes[m];
          idx[m].resize(3 * (size_t)md.triangle_count);
          vc[m] = md.vertex_count;
          tc[m] = md.triangle_count;
        }
      } catch (const std::bad_alloc&) {
        return fail(RT_ERROR_OUT_OF_MEMORY, "rt_trace_backward_instances: host allocation");
      }
      for (uint32_t m = 0; m < nm; ++m) {
        if (!idx[m].empty())
          RT_HIP(hipMemcpy(idx[m].data(), accel->host_meshes[m].indices, idx[m].size() * sizeof(uint32_t),
                           hipMemcpyDeviceToHost));
        ip[m] = idx[m].data();
      }
      for (uint32_t j = 0; j < accel->instance_count; ++j) im[j] = accel->host_insts[j].mesh;
      RT_HIP(rta::gather_build_multi(g, ip.data(), vc.data(), tc.data(), nm, im.data(), accel->instance_count, 6));
      accel->info.device_bytes += 4ull * (accel->vertex_rows + 1) + 120ull * total_tris + 8ull * accel->instance_count;
    }
    if (!g.tri_vertices_valid) {
      uint32_t first = 0;
      for (uint32_t m = 0; m < nm; ++m) {
        const rt_mesh_dev& md = accel->host_meshes[m];
        RT_HIP(rta::gather_tri_vertices(g, md.indices, md.vertices, md.triangle_count, first, s));
        first += md.triangle_count;
      }
      g.tri_vertices_valid = true;
    }
    p.tri_vertices = g.tri_vertices;
    p.inst_tris = g.inst_tris;
    rta::KeySource keys{reinterpret_cast<const uint32_t*>(hits), inst_ids, g.inst_tris, accel->instance_count, 0, 1};
    if (p.want_vertices) {
      RT_HIP(rta::sort_reserve(ctx->sortbuf, g.buckets, n, s));
      RT_HIP(rta::bucket_rays(keys, g.buckets, g.shift, ctx->sortbuf, n, s, &p.vb));
    }
    if (p.want_frames) {
      keys.kind = 2;
      RT_HIP(rta::sort_reserve(ctx->sortbuf2, accel->instance_count, n, s));
      RT_HIP(rta::bucket_rays(keys, accel->instance_count, 0, ctx->sortbuf2, n, s, &p.fb));
    }
    RT_HIP(rtk_launch_backward_inst_tiles(p, s));
    if (p.want_vertices) RT_HIP(rta::gather_vertices(g, ctx->sortbuf, n, d_vertices, s));
    if (p.want_frames)
      RT_HIP(rta::frame_sums(ctx->sortbuf2, accel->instance_count, reinterpret_cast<const float*>(accel->srts), n,
                             d_srt, s));
    RT_HIP(hipEventRecord(ctx->last_event, s));
    ctx->last_stream = s;
    ctx->has_last = true;
    return ok();
  }
  // more instances than LDS counters: fixed-point rows with global atomics
  st = prepare_grad_rows(accel, s);
  if (st != RT_SUCCESS) return st;
  p.acc = rta::Acc{accel->grad_rows.expo, accel->grad_rows.sums, accel->grad_rows.count, rta::shift0_for(n)};
  p.frame_row0 = (uint32_t)accel->vertex_rows;
  RT_HIP(rtk_launch_backward_inst(p, 0, s));
  RT_HIP(rtk_launch_backward_inst(p, 1, s));
  if (d_vertices)
    RT_HIP(rta::convert(accel->grad_rows, 0, (uint32_t)accel->vertex_rows, 0, p.acc.shift0, d_vertices, s));
  if (d_srt)
    RT_HIP(rta::convert(accel->grad_rows, (uint32_t)accel->vertex_rows, 4u * accel->instance_count, 1,
                        p.acc.shift0, d_srt, s));
  accel->grad_dirty = false;
  RT_HIP(hipEventRecord(ctx->last_event, s));
  ctx->last_stream = s;
  ctx->has_last = true;
  return ok();
}

static rt_status ao_rays_impl(const char* who, rt_accel accel, const rt_ray* rays, const rt_hit* hits,
                              const uint32_t* inst_ids, uint32_t n, uint32_t samples, const float* xi,
                              float offset, float radius, rt_ray* ao_rays, void* stream) {
  if (samples < 1) return fail(RT_ERROR_INVALID_VALUE, "%s: samples must be >= 1", who);
  if (!(radius >= 0.0f) || !(offset >= 0.0f) || !std::isfinite(offset))
    return fail(RT_ERROR_INVALID_VALUE, "%s: offset must be finite and >= 0, radius >= 0", who);
  if (n == 0) return ok();
  if ((uint64_t)n * samples > 0x7FFFFFFFull)
    return fail(RT_ERROR_INVALID_VALUE, "%s: n * samples >= 2^31", who);
  if (!rays || !hits || !xi || !ao_rays || (accel->two_level && !inst_ids))
    return fail(RT_ERROR_INVALID_VALUE, "%s: NULL buffer with n > 0", who);
  if (!aligned16(rays) || !aligned16(hits) || !aligned16(ao_rays))
    return fail(RT_ERROR_INVALID_VALUE, "%s: rays, hits and ao_rays must be 16-byte aligned", who);
  rt_status st = check_device(accel->device);
  if (st != RT_SUCCESS) return st;
  AoParams p{};
  if (accel->two_level) {
    p.meshes = accel->meshes;
    p.insts = accel->insts;
    p.srts = accel->srts;
    p.inst_ids = inst_ids;
    p.inst_count = accel->instance_count;
  } else {
    p.mesh = accel->host_meshes[0];
  }
  p.rays = rays;
  p.hits = hits;
  p.xi = xi;
  p.out = ao_rays;
  p.n = n;
  p.samples = samples;
  p.offset = offset;
  p.radius = radius;
  RT_HIP(rtk_launch_ao_rays(p, static_cast<hipStream_t>(stream)));
  return ok();
}

rt_status rt_ao_rays(rt_accel accel, const rt_ray* rays, const rt_hit* hits, uint32_t n,
                     uint32_t samples, const float* xi, float offset, float radius,
                     rt_ray* ao_rays, void* stream) {
  if (!accel) return fail(RT_ERROR_INVALID_VALUE, "rt_ao_rays: NULL accel");
  if (accel->two_level)
    return fail(RT_ERROR_UNSUPPORTED, "rt_ao_rays: two-level accel (use rt_ao_rays_instances)");
  return ao_rays_impl("rt_ao_rays", accel, rays, hits, nullptr, n, samples, xi, offset, radius, ao_rays, stream);
}

rt_status rt_ao_rays_instances(rt_accel accel, const rt_ray* rays, const rt_hit* hits, const uint32_t* inst_ids,
                               uint32_t n, uint32_t samples, const float* xi, float offset, float radius,
                               rt_ray* ao_rays, void* stream) {
  if (!accel) return fail(RT_ERROR_INVALID_VALUE, "rt_ao_rays_instances: NULL accel");
  if (!accel->two_level)
    return fail(RT_ERROR_UNSUPPORTED, "rt_ao_rays_instances: single-level accel (use rt_ao_rays)");
  return ao_rays_impl("rt_ao_rays_instances", accel, rays, hits, inst_ids, n, samples, xi, offset, radius, ao_rays,
                      stream);
}

rt_status rt_ao_resolve(const uint8_t* occluded, uint32_t n, uint32_t samples, float* ao,
                        void* stream) {
  if (samples < 1) return fail(RT_ERROR_INVALID_VALUE, "rt_ao_resolve: samples must be >= 1");
  if (n == 0) return ok();
  if ((uint64_t)n * samples > 0x7FFFFFFFull)
    return fail(RT_ERROR_INVALID_VALUE, "rt_ao_resolve: n * samples >= 2^31");
  if (!occluded || !ao) return fail(RT_ERROR_INVALID_VALUE, "rt_ao_resolve: NULL buffer with n > 0");
  RT_HIP(rtk_launch_ao_resolve(occluded, n, samples, ao, static_cast<hipStream_t>(stream)));
  return ok();
}

// Two-level refit: every mesh's vertex rows (one after another in build
// order), records and nodes, then the meshes' bounds and the top level.
static rt_status refit_two_level(rt_accel_s* a, const float* vertices, hipStream_t s) {
  const uint32_t nm = (uint32_t)a->host_meshes.size();
  a->gather.tri_vertices_valid = false;   // the backward's per-triangle vertex copy
  const uint32_t fpn = 8u * (uint32_t)a->width;
  uint64_t row = 0;
  for (uint32_t m = 0; m < nm; ++m) {
    const rt_mesh_dev& md = a->host_meshes[m];
    if (md.vertex_count > 0)
      RT_HIP(hipMemcpyAsync(const_cast<float*>(md.vertices), vertices + 3 * row, (size_t)md.vertex_count * 12,
                            hipMemcpyDefault, s));
    row += md.vertex_count;
  }
  for (uint32_t m = 0; m < nm; ++m) {
    uint32_t b = a->mesh_tri_base[m];
    uint32_t e = m + 1 < nm ? a->mesh_tri_base[m + 1] : a->info.triangle_count;
    if (e > b) RT_HIP(rtk_launch_refit_tris(a->tris + b, e - b, a->host_meshes[m], s));
  }
  for (size_t l = 0; l + 1 < a->refit_levels.size(); ++l) {
    uint32_t b = a->refit_levels[l], e = a->refit_levels[l + 1];
    RT_HIP(rtk_launch_refit_nodes(a->width, a->nodes, a->tris, a->refit_nodes + b, e - b, s));
  }
  // each mesh's bounds: the union of its root node's slots
  std::vector<float> roots((size_t)nm * fpn, 0.0f);
  for (uint32_t m = 0; m < nm; ++m)
    if (a->mesh_root[m] != RT_CHILD_EMPTY)
      RT_HIP(hipMemcpyAsync(roots.data() + (size_t)m * fpn, a->nodes + (size_t)a->mesh_root[m] * fpn, fpn * 4,
                            hipMemcpyDeviceToHost, s));
  RT_HIP(hipStreamSynchronize(s));
  const int W = a->width;
  for (uint32_t m = 0; m < nm; ++m) {
    rtb::Box& bb = a->mesh_bounds[m];
    for (int k = 0; k < 3; ++k) {
      bb.lo[k] = INFINITY;
      bb.hi[k] = -INFINITY;
    }
    if (a->mesh_root[m] == RT_CHILD_EMPTY) continue;
    const float* nd = roots.data() + (size_t)m * fpn;
    for (int c = 0; c < W; ++c)
      for (int k = 0; k < 3; ++k) {
        bb.lo[k] = std::min(bb.lo[k], nd[(2 * k) * W + c]);
        bb.hi[k] = std::max(bb.hi[k], nd[(2 * k + 1) * W + c]);
      }
  }
  rt_status st = refit_top_level(a, s);
  if (st != RT_SUCCESS) return st;
  RT_HIP(hipStreamSynchronize(s));
  return RT_SUCCESS;
}

rt_status rt_refit(rt_accel accel, const float* vertices, void* stream) {
  if (!accel) return fail(RT_ERROR_INVALID_VALUE, "rt_refit: NULL accel");
  if (accel->two_level) {
    if (accel->vertex_rows > 0 && !vertices) return fail(RT_ERROR_INVALID_VALUE, "rt_refit: vertices is NULL");
    rt_status st = check_device(accel->device);
    if (st != RT_SUCCESS) return st;
    try {
      st = refit_two_level(accel, vertices, static_cast<hipStream_t>(stream));
    } catch (const std::bad_alloc&) {
      return fail(RT_ERROR_OUT_OF_MEMORY, "rt_refit: host allocation failed");
    }
    return st == RT_SUCCESS ? ok() : st;
  }
  const rt_mesh_dev& m = accel->host_meshes[0];
  if (m.vertex_count > 0 && !vertices) return fail(RT_ERROR_INVALID_VALUE, "rt_refit: vertices is NULL");
  rt_status st = check_device(accel->device);
  if (st != RT_SUCCESS) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (m.vertex_count > 0)
    RT_HIP(hipMemcpyAsync(const_cast<float*>(m.vertices), vertices, (size_t)m.vertex_count * 12,
                          hipMemcpyDefault, s));
  accel->gather.tri_vertices_valid = false;   // the backward's per-triangle vertex copy
  RT_HIP(rtk_launch_refit_tris(accel->tris, accel->info.triangle_count, m, s));
  for (size_t l = 0; l + 1 < accel->refit_levels.size(); ++l) {
    uint32_t b = accel->refit_levels[l], e = accel->refit_levels[l + 1];
    RT_HIP(rtk_launch_refit_nodes(accel->width, accel->nodes, accel->tris, accel->refit_nodes + b, e - b, s));
  }
  return ok();
}

// ---------------------------------------------------------------------------
// autotuning
// ---------------------------------------------------------------------------

rt_status rt_autotune(rt_context ctx, const rt_mesh_desc* mesh, const rt_ray* probe_rays,
                      uint32_t n_probe, uint32_t repeats, void* stream, rt_tune_entry* best,
                      rt_tune_entry* table, uint32_t table_cap, uint32_t* table_len) {
  if (!ctx || !mesh || !best) return fail(RT_ERROR_INVALID_VALUE, "rt_autotune: NULL argument");
  if (n_probe == 0 || !probe_rays)
    return fail(RT_ERROR_INVALID_VALUE, "rt_autotune: no probe rays");
  if (table_cap > 0 && !table) return fail(RT_ERROR_INVALID_VALUE, "rt_autotune: NULL table");
  if (repeats == 0) repeats = 3;
  hipStream_t s = static_cast<hipStream_t>(stream);
  rt_status st = check_device(ctx->device);
  if (st != RT_SUCCESS) return st;
  rt_hit* hits = nullptr;
  RT_HIP(rt_malloc(&hits, (size_t)n_probe * sizeof(rt_hit)));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(hits);
    return fail(RT_ERROR_HIP, "rt_autotune: hipEventCreate failed");
  }
  rt_variant saved = ctx->variant;
  rt_tune_entry win{0, 0, 0, INFINITY};
  rt_tune_entry dflt{0, 0, 0, INFINITY};  // width 4, stack 16, workgroup 256
  uint32_t count = 0;
  st = RT_SUCCESS;
  for (uint32_t w : kWidthChoices) {
    rt_build_options opt{w, 0, 0};
    rt_accel a = nullptr;
    st = rt_build(ctx, mesh, 1, nullptr, nullptr, 0, &opt, stream, &a);
    if (st != RT_SUCCESS) break;
    for (uint32_t sn : kStackChoices) {
      for (uint32_t wg : kWorkgroupChoices) {
        {
          std::lock_guard<std::mutex> lk(ctx->mu);
          ctx->variant = rt_variant{sn, wg};
        }
        std::vector<float> ms;
        for (uint32_t r = 0; r <= repeats && st == RT_SUCCESS; ++r) {
          if (hipEventRecord(e0, s) != hipSuccess) st = fail(RT_ERROR_HIP, "rt_autotune: event");
          if (st == RT_SUCCESS) st = launch_trace(a, probe_rays, n_probe, hits, nullptr, nullptr, false, s);
          if (st == RT_SUCCESS && hipEventRecord(e1, s) != hipSuccess) st = fail(RT_ERROR_HIP, "rt_autotune: event");
          if (st == RT_SUCCESS && hipEventSynchronize(e1) != hipSuccess) st = fail(RT_ERROR_HIP, "rt_autotune: sync");
          float t = 0.0f;
          if (st == RT_SUCCESS && hipEventElapsedTime(&t, e0, e1) != hipSuccess) st = fail(RT_ERROR_HIP, "rt_autotune: timing");
          if (st == RT_SUCCESS && r > 0) ms.push_back(t);  // the first launch warms up
        }
        if (st != RT_SUCCESS) break;
        std::sort(ms.begin(), ms.end());
        rt_tune_entry e{w, sn, wg, ms[ms.size() / 2]};
        if (count < table_cap) table[count] = e;
        ++count;
        if (e.ms < win.ms) win = e;
        if (w == 4 && sn == 16 && wg == 256) dflt = e;
      }
      if (st != RT_SUCCESS) break;
    }
    rt_accel_destroy(a);
    if (st != RT_SUCCESS) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(hits);
  if (table_len) *table_len = count;
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (st != RT_SUCCESS) {
    ctx->variant = saved;
    return st;
  }
  // another configuration replaces the default only when it is faster by
  // more than the launch-to-launch spread (1%), so that repeated tuning on
  // the same workload settles on the same choice
  if (dflt.ms <= win.ms * 1.01f) win = dflt;
  ctx->variant = rt_variant{win.stack_entries, win.workgroup};
  *best = win;
  return ok();
}

// ---------------------------------------------------------------------------
// batched plans
// ---------------------------------------------------------------------------

static rt_status plan_create(rt_context ctx, const rt_accel* accels, const rt_ray* const* rays,
                             rt_hit* const* hits, uint32_t* const* inst_ids, const uint32_t* counts,
                             uint32_t batch_count, rt_batch_plan* out) {
  if (!out) return fail(RT_ERROR_INVALID_VALUE, "rt_batch_plan_create: out is NULL");
  *out = nullptr;
  if (!ctx || !accels || !rays || !hits || !counts || batch_count == 0)
    return fail(RT_ERROR_INVALID_VALUE, "rt_batch_plan_create: NULL argument or empty batch");
  int width = -1;
  uint64_t total = 0;
  uint32_t max_stack = 1;
  const bool two_level = accels[0] && accels[0]->two_level;
  for (uint32_t b = 0; b < batch_count; ++b) {
    rt_accel a = accels[b];
    if (!a) return fail(RT_ERROR_INVALID_VALUE, "rt_batch_plan_create: accel %u is NULL", b);
    if (a->two_level != two_level)
      return fail(RT_ERROR_INVALID_VALUE, "rt_batch_plan_create: accel %u: a plan's accels are all single-level "
                  "or all two-level", b);
    if (inst_ids && inst_ids[b] && !two_level)
      return fail(RT_ERROR_INVALID_VALUE, "rt_batch_plan_create: instance ids for single-level accel %u", b);
    if (a->device != ctx->device)
      return fail(RT_ERROR_INVALID_VALUE, "rt_batch_plan_create: accel %u is on another device", b);
    if (width < 0) width = a->width;
    if (a->width != width)
      return fail(RT_ERROR_UNSUPPORTED, "rt_batch_plan_create: accels must share one node width");
    if (counts[b] > 0 && (!rays[b] || !hits[b]))
      return fail(RT_ERROR_INVALID_VALUE, "rt_batch_plan_create: batch %u has a NULL buffer", b);
    if (counts[b] > 0 && (!aligned16(rays[b]) || !aligned16(hits[b])))
      return fail(RT_ERROR_INVALID_VALUE, "rt_batch_plan_create: batch %u buffers not 16-byte aligned", b);
    total += counts[b];
    max_stack = std::max(max_stack, a->max_stack);
  }
  if (total > 0x7FFFFFFFull) return fail(RT_ERROR_INVALID_VALUE, "rt_batch_plan_create: >= 2^31 rays");
  rt_status st = check_device(ctx->device);
  if (st != RT_SUCCESS) return st;
  rt_batch_plan_s* p = new (std::nothrow) rt_batch_plan_s();
  if (!p) return fail(RT_ERROR_OUT_OF_MEMORY, "rt_batch_plan_create: host allocation");
  p->ctx = ctx;
  p->width = width;
  p->two_level = two_level;
  p->batch_count = batch_count;
  p->total = (uint32_t)total;
  p->max_stack = max_stack;
  auto bail = [&](rt_status e) {
    free_scratch(p->scratch);
    if (p->descs) (void)hipFree(p->descs);
    if (p->offsets) (void)hipFree(p->offsets);
    delete p;
    return e;
  };
  std::vector<BatchDesc> d(batch_count);
  std::vector<uint32_t> off(batch_count + 1, 0);
  for (uint32_t b = 0; b < batch_count; ++b) {
    rt_accel a = accels[b];
    d[b] = BatchDesc{a->nodes,   a->tris,    a->meshes, rays[b], hits[b], a->root, counts[b],
                     a->insts,    a->insts64, inst_ids ? inst_ids[b] : nullptr};
    off[b + 1] = off[b] + counts[b];
  }
  rt_variant v = ctx->variant;
  p->kernel = rtk_trace_kernel(width, (int)v.stack_entries, (int)v.workgroup, false, two_level, 1);
  if (!p->kernel) return bail(fail(RT_ERROR_UNSUPPORTED, "rt_batch_plan_create: variant not compiled"));
  uint32_t wg = v.workgroup;
  uint32_t resident;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    resident = cached_resident(ctx, p->kernel, (int)wg);
  }
  p->grid = std::max(1u, std::min<uint32_t>((p->total + wg - 1) / wg, resident));
  p->workgroup = wg;
  p->stack_entries = v.stack_entries;
  size_t spill = max_stack > v.stack_entries ? (size_t)(max_stack - v.stack_entries) : 1;
  hipError_t e1 = rt_malloc(&p->descs, d.size() * sizeof(BatchDesc));
  hipError_t e2 = rt_malloc(&p->offsets, off.size() * sizeof(uint32_t));
  if (e1 != hipSuccess || e2 != hipSuccess)
    return bail(fail(RT_ERROR_OUT_OF_MEMORY, "rt_batch_plan_create: device allocation failed"));
  st = ensure_scratch(p->scratch, spill * p->grid * wg);
  if (st != RT_SUCCESS) return bail(st);
  if (hipMemcpy(p->descs, d.data(), d.size() * sizeof(BatchDesc), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->offsets, off.data(), off.size() * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(RT_ERROR_HIP, "rt_batch_plan_create: descriptor upload failed"));
  *out = p;
  return ok();
}

rt_status rt_batch_plan_create(rt_context ctx, const rt_accel* accels, const rt_ray* const* rays,
                               rt_hit* const* hits, const uint32_t* counts, uint32_t batch_count,
                               rt_batch_plan* out) {
  return plan_create(ctx, accels, rays, hits, nullptr, counts, batch_count, out);
}

rt_status rt_batch_plan_create_instances(rt_context ctx, const rt_accel* accels, const rt_ray* const* rays,
                                         rt_hit* const* hits, uint32_t* const* inst_ids, const uint32_t* counts,
                                         uint32_t batch_count, rt_batch_plan* out) {
  return plan_create(ctx, accels, rays, hits, inst_ids, counts, batch_count, out);
}

static rt_status enqueue_plan(rt_batch_plan p, hipStream_t s) {
  // the kernel, grid and scratch were chosen with the context's variant at
  // creation; a later rt_context_set_variant does not change the plan
  TraceParams q{};
  q.counter = p->scratch.counter;
  q.gstack = p->scratch.gstack;
  q.batches = p->descs;
  q.batch_offsets = p->offsets;
  q.batch_count = p->batch_count;
  q.n = p->total;
  q.max_stack = p->ctx->stack_limit ? std::max(std::min(p->max_stack, p->ctx->stack_limit), p->stack_entries)
                                    : p->max_stack;
  q.gstride = p->grid * p->workgroup;
  q.refill_min = p->ctx->refill_min;
  q.status = p->ctx->status;
  q.root = RT_CHILD_EMPTY;
  RT_HIP(rtk_launch_fill(p->scratch.counter, 1, 0u, s));
  RT_HIP(rtk_launch_trace(p->kernel, p->grid, p->workgroup, q, s));
  RT_HIP(rtk_launch_finalize(p->two_level, 1, q, s));
  return RT_SUCCESS;
}

rt_status rt_batch_plan_launch(rt_batch_plan plan, void* stream) {
  if (!plan) return fail(RT_ERROR_INVALID_VALUE, "rt_batch_plan_launch: NULL plan");
  if (plan->total == 0) return ok();
  rt_status st = check_device(plan->ctx->device);
  if (st != RT_SUCCESS) return st;
  {
    std::lock_guard<std::mutex> lk(plan->ctx->mu);
    st = take_overflow(plan->ctx, "rt_batch_plan_launch");
  }
  if (st != RT_SUCCESS) return st;
  st = enqueue_plan(plan, static_cast<hipStream_t>(stream));
  if (st != RT_SUCCESS) return st;
  return ok();
}

rt_status rt_batch_plan_graph(rt_batch_plan plan, void* stream, void** out_graph_exec) {
  if (!plan || !out_graph_exec) return fail(RT_ERROR_INVALID_VALUE, "rt_batch_plan_graph: NULL argument");
  *out_graph_exec = nullptr;
  if (!stream) return fail(RT_ERROR_INVALID_VALUE, "rt_batch_plan_graph: capture needs a non-null stream");
  rt_status st = check_device(plan->ctx->device);
  if (st != RT_SUCCESS) return st;
  if (!plan->graph_exec) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    RT_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    rt_status e = (plan->total > 0) ? enqueue_plan(plan, s) : RT_SUCCESS;
    hipGraph_t g = nullptr;
    hipError_t ee = hipStreamEndCapture(s, &g);
    if (e != RT_SUCCESS) {
      if (g) (void)hipGraphDestroy(g);
      return e;
    }
    if (ee != hipSuccess) return fail(RT_ERROR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(ee));
    hipGraphExec_t x = nullptr;
    hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      (void)hipGraphDestroy(g);
      return fail(RT_ERROR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
    }
    plan->graph = g;
    plan->graph_exec = x;
  }
  *out_graph_exec = plan->graph_exec;
  return ok();
}

rt_status rt_batch_plan_destroy(rt_batch_plan plan) {
  if (!plan) return fail(RT_ERROR_INVALID_VALUE, "rt_batch_plan_destroy: NULL plan");
  (void)hipSetDevice(plan->ctx->device);
  (void)hipDeviceSynchronize();
  if (plan->graph_exec) (void)hipGraphExecDestroy(plan->graph_exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  free_scratch(plan->scratch);
  if (plan->descs) (void)hipFree(plan->descs);
  if (plan->offsets) (void)hipFree(plan->offsets);
  delete plan;
  return ok();
}

}  // extern "C"
