/* Host driver of the oracle (rt_oracle.c) for sanitizer builds: seeded small
 * scenes (a soup with degenerate and non-finite triangles, a grid, a
 * two-mesh instanced scene with masks and filters) and rays (random, void,
 * zero direction components, NaN), run through every oracle entry point;
 * the BVH-driven queries must equal the linear search exactly.  Exit status
 * 0 when every check passes. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "rt_oracle.h"

static uint64_t rng_state = 0x2545F4914F6CDD1Dull;
static uint64_t next_u64(void) { /* splitmix64 */
  uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static float uni(float lo, float hi) { return lo + (hi - lo) * (float)((next_u64() >> 40) * (1.0 / 16777216.0)); }

static int failures = 0;
static void check(int ok, const char* what, const char* label) {
  if (!ok) {
    fprintf(stderr, "FAIL %s: %s\n", label, what);
    ++failures;
  }
}

static void make_rays(float* R, int64_t n, float lo, float hi) {
  for (int64_t r = 0; r < n; ++r) {
    float* q = R + 8 * r;
    double d[3], l = 0;
    for (int c = 0; c < 3; ++c) {
      q[c] = uni(lo, hi);
      d[c] = uni(-1, 1);
      l += d[c] * d[c];
    }
    l = sqrt(l);
    for (int c = 0; c < 3; ++c) q[4 + c] = (float)(d[c] / l);
    q[3] = 0.0f;
    q[7] = INFINITY;
    switch (r % 23) {
      case 1: q[4] = 0.0f; break;                        /* zero direction component */
      case 2: q[4] = q[5] = q[6] = 0.0f; break;          /* void: zero direction */
      case 3: q[3] = 2.0f; q[7] = 1.0f; break;           /* void: tmin > tmax */
      case 4: q[1] = NAN; break;                         /* void: NaN origin */
      case 5: q[7] = 0.3f; break;                        /* short ray */
      default: break;
    }
  }
}

static void queries(const orc_scene* lin, const orc_scene* acc, const float* R, int64_t n, const orc_opts* o,
                    int single, int64_t nv_total, const char* label) {
  uint32_t *i1 = malloc(n * 4), *i2 = malloc(n * 4), *p1 = malloc(n * 4), *p2 = malloc(n * 4);
  double *t1 = malloc(n * 24), *t2 = malloc(n * 24);
  uint8_t *o1 = malloc(n), *o2 = malloc(n);
  check(orc_closest_ex(lin, R, n, o, i1, p1, t1) == 0, "closest (linear)", label);
  check(orc_closest_ex(acc, R, n, o, i2, p2, t2) == 0, "closest (bvh)", label);
  check(!memcmp(i1, i2, n * 4) && !memcmp(p1, p2, n * 4) && !memcmp(t1, t2, n * 24), "closest bvh == linear", label);
  check(orc_any_ex(lin, R, n, o, o1) == 0 && orc_any_ex(acc, R, n, o, o2) == 0, "any", label);
  check(!memcmp(o1, o2, n), "any bvh == linear", label);
  for (int64_t r = 0; r < n; ++r) check(o1[r] == (p1[r] != ORC_NONE), "any == closest found", label);
  const int32_t K = 4;
  int64_t *c1 = malloc(n * 8), *c2 = malloc(n * 8);
  uint32_t *ai1 = malloc(n * K * 4), *ai2 = malloc(n * K * 4), *ap1 = malloc(n * K * 4), *ap2 = malloc(n * K * 4);
  double *at1 = malloc(n * K * 24), *at2 = malloc(n * K * 24);
  check(orc_all(lin, R, n, o, K, c1, ai1, ap1, at1) == 0 && orc_all(acc, R, n, o, K, c2, ai2, ap2, at2) == 0, "all",
        label);
  check(!memcmp(c1, c2, n * 8) && !memcmp(ap1, ap2, n * K * 4) && !memcmp(at1, at2, n * K * 24),
        "all bvh == linear", label);
  uint8_t *m1 = malloc(n), *m2 = malloc(n), *a1 = malloc(n), *a2 = malloc(n);
  int32_t *k1 = malloc(n * 4), *k2 = malloc(n * 4);
  double *s1 = malloc(n * K * 8), *s2 = malloc(n * K * 8);
  check(orc_accept_ex(lin, R, n, o, 1e-5, K, m1, k1, ai1, ap1, at1, s1, a1) == 0, "accept (linear)", label);
  check(orc_accept_ex(acc, R, n, o, 1e-5, K, m2, k2, ai2, ap2, at2, s2, a2) == 0, "accept (bvh)", label);
  check(!memcmp(m1, m2, n) && !memcmp(k1, k2, n * 4) && !memcmp(ap1, ap2, n * K * 4) && !memcmp(a1, a2, n),
        "accept bvh == linear", label);
  for (int64_t r = 0; r < n; ++r)
    if (p1[r] != ORC_NONE && k1[r] > 0) {
      int in = 0;
      for (int32_t j = 0; j < (k1[r] < K ? k1[r] : K); ++j) in |= ap1[r * K + j] == p1[r] && ai1[r * K + j] == i1[r];
      check(in || k1[r] > K, "the exact closest hit is acceptable", label);
    }
  int32_t* ns = malloc(n * 4);
  double *lo = malloc(n * K * 8), *hi = malloc(n * K * 8);
  uint8_t* sure = malloc(n * K);
  check(orc_classify_all(acc, R, n, o, 1e-5, K, k1, ns, ai1, ap1, at1, s1, lo, hi, sure) == 0, "classify_all", label);
  double* g = malloc(n * 24);
  for (int64_t j = 0; j < 3 * n; ++j) g[j] = uni(-1, 1);
  double *dor = malloc(n * 24), *ddi = malloc(n * 24);
  if (single) {
    double* dv = calloc(nv_total * 3, 8);
    double* fd = malloc(n * 15 * 8);
    check(orc_adjoint(lin, R, p1, n, g, dv, dor, ddi) == 0, "adjoint", label);
    check(orc_fd(lin, R, p1, n, g, 1e-6, fd) == 0, "fd", label);
    check(orc_fixed_tuv(lin, R, p1, n, t2) == 0, "fixed_tuv", label);
    const int32_t N = 2;
    float* xi = malloc(n * N * 2 * 4);
    float* ao = malloc(n * N * 8 * 4);
    for (int64_t j = 0; j < n * N * 2; ++j) xi[j] = uni(0, 1);
    check(orc_ao_rays(lin, R, p1, t1, n, N, xi, 1e-4, 1.0, ao) == 0, "ao_rays", label);
    free(dv); free(fd); free(xi); free(ao);
  } else {
    double* dv = calloc(nv_total * 3, 8);
    double* dvp[2] = {dv, dv + 3 * 60};
    double* dsrt = calloc(lin->n_inst * 10, 8);
    double* fd = malloc(n * 25 * 8);
    check(orc_adjoint_inst(lin, R, i1, p1, n, g, dvp, dsrt, dor, ddi) == 0, "adjoint_inst", label);
    check(orc_fd_inst(lin, R, i1, p1, n, g, 1e-6, fd) == 0, "fd_inst", label);
    const int32_t N = 2;
    float* xi = malloc(n * N * 2 * 4);
    float* ao = malloc(n * N * 8 * 4);
    for (int64_t j = 0; j < n * N * 2; ++j) xi[j] = uni(0, 1);
    check(orc_ao_rays_inst(lin, R, i1, p1, t1, n, N, xi, 1e-4, 1.0, ao) == 0, "ao_rays_inst", label);
    free(dv); free(dsrt); free(fd); free(xi); free(ao);
  }
  int64_t st[4], chk[2];
  check(orc_bvh_stats(acc->bvh, st) == 0, "bvh_stats", label);
  check(orc_bvh_check(acc, R, n, 1, 1e-5, chk) == 0 && chk[1] == 0, "bvh culling invariant", label);
  free(i1); free(i2); free(p1); free(p2); free(t1); free(t2); free(o1); free(o2); free(c1); free(c2);
  free(ai1); free(ai2); free(ap1); free(ap2); free(at1); free(at2); free(m1); free(m2); free(a1); free(a2);
  free(k1); free(k2); free(s1); free(s2); free(ns); free(lo); free(hi); free(sure); free(g); free(dor); free(ddi);
}

int main(void) {
  orc_set_num_threads(1);
  /* single mesh: a soup with degenerate and non-finite triangles */
  {
    const int64_t nt = 300, nv = 3 * nt, n = 1500;
    float* V = malloc(nv * 12);
    uint32_t* I = malloc(nt * 12);
    for (int64_t k = 0; k < nt; ++k) {
      float cx = uni(0, 1), cy = uni(0, 1), cz = uni(0, 1);
      for (int j = 0; j < 3; ++j) {
        V[9 * k + 3 * j] = cx + uni(-0.08f, 0.08f);
        V[9 * k + 3 * j + 1] = cy + uni(-0.08f, 0.08f);
        V[9 * k + 3 * j + 2] = cz + uni(-0.08f, 0.08f);
        I[3 * k + j] = (uint32_t)(3 * k + j);
      }
      if (k % 29 == 0) I[3 * k + 2] = I[3 * k];          /* repeated vertex */
      if (k % 31 == 0) V[9 * k + 4] = NAN;               /* non-finite vertex */
    }
    const float* vp[1] = {V};
    const uint32_t* ip[1] = {I};
    int64_t nvs[1] = {nv}, nts[1] = {nt};
    orc_scene lin = {1, vp, nvs, ip, nts, 0, NULL, NULL, NULL};
    orc_bvh* b = NULL;
    check(orc_bvh_create(&lin, &b) == 0, "bvh_create", "soup");
    orc_scene acc = lin;
    acc.bvh = b;
    float* R = malloc(n * 32);
    make_rays(R, n, -0.2f, 1.2f);
    uint32_t* skip = malloc(n * 4);
    for (int64_t r = 0; r < n; ++r) skip[r] = (r % 3 == 0) ? (uint32_t)(next_u64() % nt) : ORC_NONE;
    orc_opts none = {NULL, NULL, NULL, NULL};
    orc_opts filt = {NULL, NULL, NULL, skip};
    queries(&lin, &acc, R, n, &none, 1, nv, "soup");
    queries(&lin, &acc, R, n, &filt, 1, nv, "soup, filtered");
    orc_bvh_destroy(b);
    free(V); free(I); free(R); free(skip);
  }
  /* two meshes (a soup of 20 and a 5x4 grid of 40 triangles), 9 instances */
  {
    const int64_t n = 1200, ni = 9;
    float V0[60 * 3], V1[30 * 3];
    uint32_t I0[20 * 3], I1[40 * 3];
    for (int k = 0; k < 60 * 3; ++k) V0[k] = uni(-1, 1);
    for (int k = 0; k < 60; ++k) I0[k] = (uint32_t)k;
    for (int z = 0, v = 0; z < 5; ++z)
      for (int x = 0; x < 6; ++x, ++v) {
        V1[3 * v] = (float)x - 2.5f;
        V1[3 * v + 1] = uni(-0.2f, 0.2f);
        V1[3 * v + 2] = (float)z - 2.0f;
      }
    for (int z = 0; z < 4; ++z)
      for (int x = 0; x < 5; ++x) {
        uint32_t a = (uint32_t)(z * 6 + x);
        uint32_t q[6] = {a, a + 1, a + 6, a + 1, a + 7, a + 6};
        for (int j = 0; j < 6; ++j) I1[6 * (z * 5 + x) + j] = q[j];
      }
    const float* vp[2] = {V0, V1};
    const uint32_t* ip[2] = {I0, I1};
    int64_t nvs[2] = {60, 30}, nts[2] = {20, 40};
    uint32_t im[9];
    float srt[9 * 10];
    for (int j = 0; j < ni; ++j) {
      im[j] = (uint32_t)(j % 2);
      float* f = srt + 10 * j;
      for (int c = 0; c < 3; ++c) f[c] = uni(0.5f, 2.0f) * ((next_u64() & 1) ? 1.0f : -1.0f);
      for (int c = 3; c < 7; ++c) f[c] = uni(-1, 1);
      for (int c = 7; c < 10; ++c) f[c] = uni(-4, 4);
    }
    orc_scene lin = {2, vp, nvs, ip, nts, ni, im, srt, NULL};
    orc_bvh* b = NULL;
    check(orc_bvh_create(&lin, &b) == 0, "bvh_create", "instances");
    orc_scene acc = lin;
    acc.bvh = b;
    float* R = malloc(n * 32);
    make_rays(R, n, -6.0f, 6.0f);
    uint32_t imask[9], rmask[1200], si[1200], sp[1200];
    for (int j = 0; j < ni; ++j) imask[j] = 1u << (j % 3);
    for (int64_t r = 0; r < n; ++r) {
      rmask[r] = (uint32_t)(next_u64() & 7);
      si[r] = (uint32_t)(next_u64() % ni);
      sp[r] = (r % 4 == 0) ? (uint32_t)(next_u64() % 20) : ORC_NONE;
    }
    orc_opts none = {NULL, NULL, NULL, NULL};
    orc_opts all = {imask, rmask, si, sp};
    queries(&lin, &acc, R, n, &none, 0, 90, "instances");
    queries(&lin, &acc, R, n, &all, 0, 90, "instances, masks and filter");
    orc_bvh_destroy(b);
    free(R);
  }
  printf("oracle checks done, %d failures\n", failures);
  return failures == 0 ? 0 : 1;
}
