// bvh_build.cpp -- host BVH construction for librtq (see bvh_build.h).
#include "bvh_build.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <limits>
#include <thread>

namespace rtb {
namespace {

constexpr int kBins = 32;
constexpr float kInf = std::numeric_limits<float>::infinity();
// relative costs of one node visit and one triangle test in the SAH; the
// node cost can be changed with RT_SAH_TRAVERSAL_COST (read at each build)
constexpr float kTriangleCost = 1.0f;
float traversal_cost_from_env() {
  const char* v = std::getenv("RT_SAH_TRAVERSAL_COST");
  float x = v ? (float)std::atof(v) : 1.0f;
  return (x > 0.0f && x < 1000.0f) ? x : 1.0f;
}

Box empty_box() {
  Box b;
  for (int a = 0; a < 3; ++a) {
    b.lo[a] = kInf;
    b.hi[a] = -kInf;
  }
  return b;
}
void grow(Box& b, const Box& o) {
  for (int a = 0; a < 3; ++a) {
    b.lo[a] = std::min(b.lo[a], o.lo[a]);
    b.hi[a] = std::max(b.hi[a], o.hi[a]);
  }
}
double area(const Box& b) {
  double dx = (double)b.hi[0] - b.lo[0], dy = (double)b.hi[1] - b.lo[1],
         dz = (double)b.hi[2] - b.lo[2];
  if (!(dx >= 0) || !(dy >= 0) || !(dz >= 0)) return 0.0;
  return 2.0 * (dx * dy + dy * dz + dz * dx);
}

struct Prim {
  Box b;
  float c[3];  // box centre
  uint32_t id; // triangle id (mesh build) or instance id (instance build)
};

struct BNode {
  Box b;
  uint32_t left = 0;   // children at left, left + 1 when count == 0
  uint32_t first = 0;  // leaf range when count > 0
  uint32_t count = 0;
};

struct Binary {
  std::vector<BNode> nodes;
  std::atomic<uint32_t> used{1};
  std::vector<Prim>* prims = nullptr;
  int max_leaf = 4;
  int spawn_depth = 0;
  float traversal_cost = 1.0f;
};

// Binned SAH split of prims[lo, hi) in node `ni` (Wald 2007).
void build_node(Binary& B, uint32_t ni, uint32_t lo, uint32_t hi, int depth) {
  std::vector<Prim>& P = *B.prims;
  Box bb = empty_box(), cb = empty_box();
  for (uint32_t i = lo; i < hi; ++i) {
    grow(bb, P[i].b);
    for (int a = 0; a < 3; ++a) {
      cb.lo[a] = std::min(cb.lo[a], P[i].c[a]);
      cb.hi[a] = std::max(cb.hi[a], P[i].c[a]);
    }
  }
  BNode& node = B.nodes[ni];
  node.b = bb;
  uint32_t n = hi - lo;
  auto make_leaf = [&]() {
    node.first = lo;
    node.count = n;
  };
  if (n <= 1) {
    make_leaf();
    return;
  }
  // best split over the three axes
  double best_cost = std::numeric_limits<double>::infinity();
  int best_axis = -1, best_split = -1;
  for (int a = 0; a < 3; ++a) {
    float ext = cb.hi[a] - cb.lo[a];
    if (!(ext > 0.0f)) continue;
    float k = (float)kBins / ext;
    Box bin_box[kBins];
    uint32_t bin_n[kBins];
    for (int i = 0; i < kBins; ++i) {
      bin_box[i] = empty_box();
      bin_n[i] = 0;
    }
    for (uint32_t i = lo; i < hi; ++i) {
      int bi = (int)((P[i].c[a] - cb.lo[a]) * k);
      bi = std::min(std::max(bi, 0), kBins - 1);
      grow(bin_box[bi], P[i].b);
      bin_n[bi]++;
    }
    double right_area[kBins];
    uint32_t right_n[kBins];
    Box acc = empty_box();
    uint32_t cnt = 0;
    for (int i = kBins - 1; i > 0; --i) {
      grow(acc, bin_box[i]);
      cnt += bin_n[i];
      right_area[i] = area(acc);
      right_n[i] = cnt;
    }
    acc = empty_box();
    cnt = 0;
    for (int i = 0; i < kBins - 1; ++i) {
      grow(acc, bin_box[i]);
      cnt += bin_n[i];
      if (cnt == 0 || right_n[i + 1] == 0) continue;
      double cost = area(acc) * cnt + right_area[i + 1] * right_n[i + 1];
      if (cost < best_cost) {
        best_cost = cost;
        best_axis = a;
        best_split = i;
      }
    }
  }
  double node_area = area(bb);
  double leaf_cost = kTriangleCost * (double)n;
  double split_cost =
      (best_axis >= 0 && node_area > 0.0)
          ? B.traversal_cost + kTriangleCost * best_cost / node_area
          : std::numeric_limits<double>::infinity();
  if ((int)n <= B.max_leaf && leaf_cost <= split_cost) {
    make_leaf();
    return;
  }
  uint32_t mid;
  if (best_axis >= 0) {
    float ext = cb.hi[best_axis] - cb.lo[best_axis];
    float k = (float)kBins / ext;
    int a = best_axis;
    auto it = std::partition(P.begin() + lo, P.begin() + hi, [&](const Prim& p) {
      int bi = (int)((p.c[a] - cb.lo[a]) * k);
      bi = std::min(std::max(bi, 0), kBins - 1);
      return bi <= best_split;
    });
    mid = (uint32_t)(it - P.begin());
    if (mid == lo || mid == hi) mid = lo + n / 2;
  } else {
    // all centres coincide: split the range in half
    mid = lo + n / 2;
  }
  uint32_t left = B.used.fetch_add(2);
  node.left = left;
  node.count = 0;
  if (depth < B.spawn_depth && n > 65536) {
    std::thread th([&B, left, lo, mid, depth]() { build_node(B, left, lo, mid, depth + 1); });
    build_node(B, left + 1, mid, hi, depth + 1);
    th.join();
  } else {
    build_node(B, left, lo, mid, depth + 1);
    build_node(B, left + 1, mid, hi, depth + 1);
  }
}

struct Collapse {
  const Binary* B;
  int W;
  WideTree* out;
  std::function<uint32_t(const BNode&)> leaf_ref;  // emits a leaf, returns its ref
  double internal_area = 0.0;
};

// Writes wide node `wi` for binary node `bi` and recurses.
void collapse(Collapse& C, uint32_t bi, uint32_t wi, uint32_t depth, uint32_t stack_above) {
  const std::vector<BNode>& N = C.B->nodes;
  const int W = C.W;
  std::vector<uint32_t> kids;
  const BNode& root = N[bi];
  if (root.count > 0) {
    kids.push_back(bi);
  } else {
    kids.push_back(root.left);
    kids.push_back(root.left + 1);
    while ((int)kids.size() < W) {
      int pick = -1;
      double best = -1.0;
      for (size_t i = 0; i < kids.size(); ++i) {
        const BNode& k = N[kids[i]];
        if (k.count == 0 && area(k.b) > best) {
          best = area(k.b);
          pick = (int)i;
        }
      }
      if (pick < 0) break;
      uint32_t l = N[kids[pick]].left;
      kids[pick] = l;
      kids.insert(kids.begin() + pick + 1, l + 1);
    }
  }
  C.internal_area += area(root.b);
  WideTree& T = *C.out;
  uint32_t stack_here = stack_above + (uint32_t)kids.size() - 1;
  T.max_stack = std::max(T.max_stack, stack_here + 1);
  T.max_depth = std::max(T.max_depth, depth);
  if (T.node_depth.size() <= wi) T.node_depth.resize((size_t)wi + 1, 0);
  T.node_depth[wi] = depth;
  // allocate the internal children consecutively, then fill this node
  std::vector<uint32_t> child_node(kids.size(), RT_CHILD_EMPTY);
  for (size_t i = 0; i < kids.size(); ++i)
    if (N[kids[i]].count == 0) child_node[i] = T.node_count++;
  if ((size_t)T.node_count * 8 * W > T.nodes.size()) T.nodes.resize((size_t)T.node_count * 8 * W * 2);
  float* nd = T.nodes.data() + (size_t)wi * 8 * W;
  for (int i = 0; i < W; ++i) {
    Box b = empty_box();
    uint32_t ref = RT_CHILD_EMPTY;
    if (i < (int)kids.size()) {
      const BNode& k = N[kids[i]];
      b = k.b;
      ref = (k.count > 0) ? C.leaf_ref(k) : child_node[i];
    }
    // the vector may have grown: take the pointer again
    nd = T.nodes.data() + (size_t)wi * 8 * W;
    nd[0 * W + i] = b.lo[0];
    nd[1 * W + i] = b.hi[0];
    nd[2 * W + i] = b.lo[1];
    nd[3 * W + i] = b.hi[1];
    nd[4 * W + i] = b.lo[2];
    nd[5 * W + i] = b.hi[2];
    std::memcpy(&nd[6 * W + i], &ref, 4);
    uint32_t zero = 0;
    std::memcpy(&nd[7 * W + i], &zero, 4);
  }
  for (size_t i = 0; i < kids.size(); ++i)
    if (child_node[i] != RT_CHILD_EMPTY) collapse(C, kids[i], child_node[i], depth + 1, stack_here);
}

bool lex_less(const float* a, const float* b) {
  if (a[0] != b[0]) return a[0] < b[0];
  if (a[1] != b[1]) return a[1] < b[1];
  return a[2] < b[2];
}

void finish_tree(Binary& B, int width, WideTree& out, const std::function<uint32_t(const BNode&)>& leaf) {
  out.width = width;
  out.nodes.clear();
  out.node_count = 0;
  out.max_depth = 0;
  out.max_stack = 0;
  out.node_depth.clear();
  if (B.prims->empty()) {
    out.root = RT_CHILD_EMPTY;
    out.sah_cost = 0.0;
    out.bounds = empty_box();
    return;
  }
  out.nodes.resize((size_t)8 * width * 64);
  out.node_count = 1;
  Collapse C;
  C.B = &B;
  C.W = width;
  C.out = &out;
  C.leaf_ref = leaf;
  collapse(C, 0, 0, 1, 0);
  out.nodes.resize((size_t)out.node_count * 8 * width);
  out.root = 0;
  out.bounds = B.nodes[0].b;
  double ra = area(out.bounds);
  out.sah_cost = ra > 0.0 ? C.internal_area / ra : 0.0;
}

int spawn_depth_for(int threads) {
  int d = 0;
  while ((1 << d) < threads) ++d;
  return d;
}

}  // namespace

bool build_mesh(const BuildInput& in, int width, int max_leaf, WideTree& out, std::string& err,
                int threads) {
  std::vector<Prim> prims;
  prims.reserve(in.triangle_count);
  for (uint32_t k = 0; k < in.triangle_count; ++k) {
    const uint32_t* ix = in.indices + 3 * (size_t)k;
    if (ix[0] >= in.vertex_count || ix[1] >= in.vertex_count || ix[2] >= in.vertex_count) {
      err = "triangle " + std::to_string(k) + " has a vertex index >= vertex_count";
      return false;
    }
    const float* v[3] = {in.vertices + 3 * (size_t)ix[0], in.vertices + 3 * (size_t)ix[1],
                         in.vertices + 3 * (size_t)ix[2]};
    bool finite = true;
    for (int j = 0; j < 3; ++j)
      for (int a = 0; a < 3; ++a) finite = finite && std::isfinite(v[j][a]);
    if (!finite) continue;
    // float64 normal of the float32 vertices (exact: differences and products
    // of float32 values are exact in float64)
    double e1[3], e2[3];
    for (int a = 0; a < 3; ++a) {
      e1[a] = (double)v[1][a] - v[0][a];
      e2[a] = (double)v[2][a] - v[0][a];
    }
    double nx = e1[1] * e2[2] - e1[2] * e2[1];
    double ny = e1[2] * e2[0] - e1[0] * e2[2];
    double nz = e1[0] * e2[1] - e1[1] * e2[0];
    if (nx == 0.0 && ny == 0.0 && nz == 0.0) continue;
    Prim p;
    p.b = empty_box();
    for (int j = 0; j < 3; ++j)
      for (int a = 0; a < 3; ++a) {
        p.b.lo[a] = std::min(p.b.lo[a], v[j][a]);
        p.b.hi[a] = std::max(p.b.hi[a], v[j][a]);
      }
    for (int a = 0; a < 3; ++a) p.c[a] = 0.5f * (p.b.lo[a] + p.b.hi[a]);
    p.id = k;
    prims.push_back(p);
  }
  if (prims.size() > RT_MAX_TRI_RECORDS) {
    err = "too many triangles for one mesh (limit 67108864)";
    return false;
  }
  Binary B;
  B.prims = &prims;
  B.max_leaf = max_leaf;
  B.spawn_depth = spawn_depth_for(threads);
  B.traversal_cost = traversal_cost_from_env();
  if (!prims.empty()) {
    B.nodes.resize(2 * prims.size());
    build_node(B, 0, 0, (uint32_t)prims.size(), 0);
  }
  out.tris.clear();
  out.tris.reserve(prims.size());
  out.leaf_count = 0;
  auto leaf = [&](const BNode& k) -> uint32_t {
    uint32_t first = (uint32_t)out.tris.size();
    for (uint32_t i = k.first; i < k.first + k.count; ++i) {
      uint32_t id = prims[i].id;
      const uint32_t* ix = in.indices + 3 * (size_t)id;
      const float* corner[3] = {in.vertices + 3 * (size_t)ix[0], in.vertices + 3 * (size_t)ix[1],
                                in.vertices + 3 * (size_t)ix[2]};
      const float* p[3] = {corner[0], corner[1], corner[2]};
      std::sort(p, p + 3, [](const float* a, const float* b) { return lex_less(a, b); });
      rt_tri_rec r;
      r.order = 0;
      for (uint32_t c = 0; c < 3; ++c)
        for (uint32_t slot = 0; slot < 3; ++slot)
          if (p[slot] == corner[c]) {
            r.order |= slot << (2 * c);
            break;
          }
      r.p0x = p[0][0]; r.p0y = p[0][1]; r.p0z = p[0][2];
      r.p1x = p[1][0]; r.p1y = p[1][1]; r.p1z = p[1][2];
      r.p2x = p[2][0]; r.p2y = p[2][1]; r.p2z = p[2][2];
      r.prim = id;
      r.pad2 = 0;
      out.tris.push_back(r);
    }
    out.leaf_count++;
    return rt_make_leaf(first, k.count);
  };
  finish_tree(B, width, out, leaf);
  out.stored_triangles = (uint32_t)out.tris.size();
  return true;
}

void build_instances(const std::vector<Box>& boxes, int width, WideTree& out, int threads) {
  std::vector<Prim> prims;
  prims.reserve(boxes.size());
  for (size_t j = 0; j < boxes.size(); ++j) {
    const Box& b = boxes[j];
    bool ok = true;
    for (int a = 0; a < 3; ++a) ok = ok && (b.lo[a] <= b.hi[a]);
    if (!ok) continue;  // an instance of an empty mesh
    Prim p;
    p.b = b;
    for (int a = 0; a < 3; ++a) p.c[a] = 0.5f * (b.lo[a] + b.hi[a]);
    p.id = (uint32_t)j;
    prims.push_back(p);
  }
  Binary B;
  B.prims = &prims;
  B.max_leaf = 1;
  B.spawn_depth = spawn_depth_for(threads);
  if (!prims.empty()) {
    B.nodes.resize(2 * prims.size());
    build_node(B, 0, 0, (uint32_t)prims.size(), 0);
  }
  out.tris.clear();
  out.leaf_count = 0;
  auto leaf = [&](const BNode& k) -> uint32_t {
    out.leaf_count++;
    return rt_make_inst(prims[k.first].id);
  };
  finish_tree(B, width, out, leaf);
  out.stored_triangles = 0;
}

}  // namespace rtb
