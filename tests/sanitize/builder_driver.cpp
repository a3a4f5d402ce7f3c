// Host driver of the BVH builder (bvh_build.cpp) for sanitizer builds: builds
// seeded random meshes (soups with degenerate, repeated and non-finite
// triangles, a grid) at widths 2, 4 and 8, leaf sizes 1..15 and 1 or 4
// threads, and instance trees; walks every tree and checks its structure:
// each kept triangle in exactly one leaf, child boxes equal to the float32
// min/max of what lies below, empty slots inverted, max_stack and max_depth
// consistent with the walk.  Exit status 0 when every check passes.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "bvh_build.h"

namespace {

uint64_t rng_state = 0x9E3779B97F4A7C15ull;
uint64_t next_u64() {  // splitmix64
  uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
float uni(float lo, float hi) { return lo + (hi - lo) * (float)((next_u64() >> 40) * (1.0 / 16777216.0)); }

int failures = 0;
void fail(const char* what, const char* label) {
  std::fprintf(stderr, "FAIL %s: %s\n", label, what);
  ++failures;
}

struct Walk {
  std::vector<int> seen;     // per stored record: times reached
  uint32_t deepest = 0;
};

// returns the box of `ref` (min/max over what lies below)
rtb::Box walk(const rtb::WideTree& t, uint32_t ref, uint32_t depth, Walk& w, const char* label) {
  rtb::Box b{{INFINITY, INFINITY, INFINITY}, {-INFINITY, -INFINITY, -INFINITY}};
  auto grow = [&](float x, float y, float z) {
    float p[3] = {x, y, z};
    for (int c = 0; c < 3; ++c) {
      b.lo[c] = std::fmin(b.lo[c], p[c]);
      b.hi[c] = std::fmax(b.hi[c], p[c]);
    }
  };
  if (ref & RT_LEAF_BIT) {
    if (ref & RT_INST_BIT) {
      fail("instance leaf in a mesh tree", label);
      return b;
    }
    uint32_t first = ref & RT_LEAF_FIRST_MASK, cnt = (ref >> RT_LEAF_COUNT_SHIFT) & RT_LEAF_COUNT_MASK;
    if (cnt == 0 || first + cnt > t.tris.size()) {
      fail("leaf range", label);
      return b;
    }
    for (uint32_t k = first; k < first + cnt; ++k) {
      w.seen[k]++;
      const rt_tri_rec& r = t.tris[k];
      grow(r.p0x, r.p0y, r.p0z);
      grow(r.p1x, r.p1y, r.p1z);
      grow(r.p2x, r.p2y, r.p2z);
    }
    return b;
  }
  if (ref >= t.node_count) {
    fail("node index", label);
    return b;
  }
  if (depth > w.deepest) w.deepest = depth;
  const int W = t.width;
  const float* n = t.nodes.data() + (size_t)ref * 8 * W;
  const uint32_t* child = reinterpret_cast<const uint32_t*>(n + 6 * W);
  for (int i = 0; i < W; ++i) {
    float lo[3] = {n[0 * W + i], n[2 * W + i], n[4 * W + i]};
    float hi[3] = {n[1 * W + i], n[3 * W + i], n[5 * W + i]};
    if (child[i] == RT_CHILD_EMPTY) {
      for (int c = 0; c < 3; ++c)
        if (!(lo[c] == INFINITY && hi[c] == -INFINITY)) fail("empty slot box not inverted", label);
      continue;
    }
    rtb::Box cb = walk(t, child[i], depth + 1, w, label);
    for (int c = 0; c < 3; ++c) {
      if (cb.lo[c] != lo[c] || cb.hi[c] != hi[c]) fail("child box is not the exact min/max", label);
      b.lo[c] = std::fmin(b.lo[c], cb.lo[c]);
      b.hi[c] = std::fmax(b.hi[c], cb.hi[c]);
    }
  }
  return b;
}

bool degenerate(const float* V, const uint32_t* I) {
  double p[3][3];
  for (int k = 0; k < 3; ++k)
    for (int c = 0; c < 3; ++c) {
      p[k][c] = V[3 * I[k] + c];
      if (!std::isfinite(p[k][c])) return true;
    }
  double e1[3], e2[3];
  for (int c = 0; c < 3; ++c) {
    e1[c] = p[1][c] - p[0][c];
    e2[c] = p[2][c] - p[0][c];
  }
  double nx = e1[1] * e2[2] - e1[2] * e2[1], ny = e1[2] * e2[0] - e1[0] * e2[2], nz = e1[0] * e2[1] - e1[1] * e2[0];
  return nx == 0.0 && ny == 0.0 && nz == 0.0;
}

void check_mesh(const std::vector<float>& V, const std::vector<uint32_t>& I, int width, int leaf, int threads,
                const char* label) {
  rtb::BuildInput in{V.data(), I.data(), (uint32_t)(V.size() / 3), (uint32_t)(I.size() / 3)};
  rtb::WideTree t;
  std::string err;
  if (!rtb::build_mesh(in, width, leaf, t, err, threads)) {
    fail(err.c_str(), label);
    return;
  }
  uint32_t kept = 0;
  for (uint32_t k = 0; k < in.triangle_count; ++k) kept += degenerate(V.data(), I.data() + 3 * k) ? 0u : 1u;
  if (t.stored_triangles != kept || t.tris.size() != kept) fail("stored triangle count", label);
  std::vector<int> prim_seen(in.triangle_count, 0);
  for (const rt_tri_rec& r : t.tris) {
    if (r.prim >= in.triangle_count) {
      fail("prim id out of range", label);
      continue;
    }
    prim_seen[r.prim]++;
    // sorted vertex order and the corner map
    float p[3][3] = {{r.p0x, r.p0y, r.p0z}, {r.p1x, r.p1y, r.p1z}, {r.p2x, r.p2y, r.p2z}};
    for (int k = 0; k < 2; ++k) {
      bool le = p[k][0] < p[k + 1][0] || (p[k][0] == p[k + 1][0] &&
                (p[k][1] < p[k + 1][1] || (p[k][1] == p[k + 1][1] && p[k][2] <= p[k + 1][2])));
      if (!le) fail("record vertices not sorted", label);
    }
    for (int c = 0; c < 3; ++c) {
      uint32_t slot = (r.order >> (2 * c)) & 3u;
      if (slot > 2) {
        fail("corner map", label);
        continue;
      }
      for (int d = 0; d < 3; ++d)
        if (p[slot][d] != V[3 * I[3 * r.prim + c] + d]) fail("corner map does not give the vertex", label);
    }
  }
  for (uint32_t k = 0; k < in.triangle_count; ++k)
    if (prim_seen[k] != (degenerate(V.data(), I.data() + 3 * k) ? 0 : 1)) fail("triangle kept twice or lost", label);
  if (kept == 0) {
    if (t.root != RT_CHILD_EMPTY) fail("empty tree has a root", label);
    return;
  }
  Walk w;
  w.seen.assign(t.tris.size(), 0);
  walk(t, t.root, 1, w, label);
  for (int s : w.seen)
    if (s != 1) fail("record reached other than once", label);
  if (!(t.root & RT_LEAF_BIT) && w.deepest != t.max_depth) fail("max_depth", label);
  // a depth-first traversal holds at most (W - 1) entries per level above
  if (t.max_stack < 1 || (uint64_t)t.max_stack > (uint64_t)(width - 1) * t.max_depth + 1)
    fail("max_stack bound", label);
}

}  // namespace

int main() {
  const int widths[3] = {2, 4, 8};
  for (int round = 0; round < 6; ++round) {
    // a soup with degenerate, repeated and non-finite triangles
    uint32_t nt = 1 + (uint32_t)(next_u64() % 700);
    std::vector<float> V;
    std::vector<uint32_t> I;
    for (uint32_t k = 0; k < nt; ++k) {
      float cx = uni(0, 1), cy = uni(0, 1), cz = uni(0, 1);
      uint32_t b = (uint32_t)(V.size() / 3);
      for (int j = 0; j < 3; ++j) {
        V.push_back(cx + uni(-0.03f, 0.03f));
        V.push_back(cy + uni(-0.03f, 0.03f));
        V.push_back(cz + uni(-0.03f, 0.03f));
      }
      uint64_t kind = next_u64() % 16;
      if (kind == 0) {
        I.insert(I.end(), {b, b, b + 1});                     // repeated vertex
      } else if (kind == 1) {
        V[3 * (b + 2) + 1] = NAN;                             // non-finite vertex
        I.insert(I.end(), {b, b + 1, b + 2});
      } else if (kind == 2 && k > 0) {
        I.insert(I.end(), {I[0], I[1], I[2]});                // duplicate of triangle 0
      } else if (kind == 3) {
        for (int c = 0; c < 3; ++c) V[3 * (b + 2) + c] = 2 * V[3 * (b + 1) + c] - V[3 * b + c];  // collinear
        I.insert(I.end(), {b, b + 1, b + 2});
      } else {
        I.insert(I.end(), {b, b + 1, b + 2});
      }
    }
    for (int w : widths)
      for (int leaf : {1, 4, 15})
        for (int th : {1, 4}) {
          char label[96];
          std::snprintf(label, sizeof label, "soup round %d: %u triangles, W=%d leaf=%d threads=%d", round, nt, w,
                        leaf, th);
          check_mesh(V, I, w, leaf, th, label);
        }
  }
  {
    // a 40 x 30 grid (shared vertices)
    std::vector<float> V;
    std::vector<uint32_t> I;
    const uint32_t nx = 40, nz = 30;
    for (uint32_t z = 0; z <= nz; ++z)
      for (uint32_t x = 0; x <= nx; ++x) {
        V.push_back((float)x);
        V.push_back(uni(-0.1f, 0.1f));
        V.push_back((float)z);
      }
    for (uint32_t z = 0; z < nz; ++z)
      for (uint32_t x = 0; x < nx; ++x) {
        uint32_t a = z * (nx + 1) + x;
        I.insert(I.end(), {a, a + 1, a + nx + 1, a + 1, a + nx + 2, a + nx + 1});
      }
    for (int w : widths) check_mesh(V, I, w, 4, 4, "grid");
  }
  {
    // an index out of range is refused
    std::vector<float> V = {0, 0, 0, 1, 0, 0, 0, 1, 0};
    std::vector<uint32_t> I = {0, 1, 3};
    rtb::BuildInput in{V.data(), I.data(), 3, 1};
    rtb::WideTree t;
    std::string err;
    if (rtb::build_mesh(in, 4, 4, t, err, 1) || err.empty()) fail("index out of range accepted", "bad index");
  }
  {
    // an empty mesh
    std::vector<float> V;
    std::vector<uint32_t> I;
    check_mesh(V, I, 4, 4, 1, "empty mesh");
  }
  for (int w : widths) {
    // instance trees: every instance in exactly one leaf
    uint32_t ni = 1 + (uint32_t)(next_u64() % 300);
    std::vector<rtb::Box> boxes(ni);
    for (auto& b : boxes)
      for (int c = 0; c < 3; ++c) {
        float a = uni(-10, 10), e = uni(0, 2);
        b.lo[c] = a;
        b.hi[c] = a + e;
      }
    rtb::WideTree t;
    rtb::build_instances(boxes, w, t, 4);
    std::vector<int> seen(ni, 0);
    std::vector<uint32_t> todo = {t.root};
    while (!todo.empty()) {
      uint32_t ref = todo.back();
      todo.pop_back();
      if (ref & RT_LEAF_BIT) {
        if (!(ref & RT_INST_BIT) || (ref & RT_INST_INDEX_MASK) >= ni) {
          fail("instance leaf", "instances");
          continue;
        }
        seen[ref & RT_INST_INDEX_MASK]++;
        continue;
      }
      if (ref >= t.node_count) {
        fail("instance node index", "instances");
        continue;
      }
      const uint32_t* child = reinterpret_cast<const uint32_t*>(t.nodes.data() + (size_t)ref * 8 * w + 6 * w);
      for (int i = 0; i < w; ++i)
        if (child[i] != RT_CHILD_EMPTY) todo.push_back(child[i]);
    }
    for (int s : seen)
      if (s != 1) fail("instance reached other than once", "instances");
  }
  std::printf("builder checks done, %d failures\n", failures);
  return failures == 0 ? 0 : 1;
}
