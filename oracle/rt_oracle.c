/* rt_oracle.c -- FP64 CPU reference for ray/triangle queries.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product library.  It shares no
 * code, header or table with the HIP path.
 *
 * What it follows (arxiv 2603.00292, "Ray Tracing using HIP"):
 *   - the ray R(t) = o + t d (§3.1, ray equation);
 *   - the plane parameter t = n.(v0 - o) / n.d with n = (v1-v0) x (v2-v1)
 *     (§3.1, plane equation and its solution for t);
 *   - the three inclusive edge tests 0 <= n.((v_{i+1}-v_i) x (R(t)-v_i))
 *     (§3.1, edge-test inequalities);
 *   - the accepted range MIN_T <= t <= MAX_T (§3.1 listing), read as the
 *     per-ray [tmin, tmax], both ends inclusive;
 *   - the closest hit as the linear search with a strict "t < minT" update in
 *     ascending triangle order, so the lowest index wins at equal t (§3.3);
 *   - any hit as "some triangle is hit within the ray's length" (§4.2);
 *   - two-level scenes: the ray is taken to object space with the inverse of
 *     the instance transform (§6.2, two-level hierarchy) whose frame is given
 *     as scale, rotation, translation (§7.3).
 * Readings where the paper is silent (all documented with the design):
 *   degenerate triangles (n = 0) and rays parallel to the plane (n.d = 0)
 *   never hit; t must be finite; rays with a NaN, a zero direction or
 *   tmin > tmax are misses; faces are two-sided; (u,v) are the barycentric
 *   weights of v1 and v2, so the hit point is (1-u-v) v0 + u v1 + v v2; a miss
 *   reports t = +inf, u = v = 0, prim = 0xFFFFFFFF.
 * The acceptable-set classification, the adjoint and the finite differences
 * are test machinery derived from those definitions (see each function). */
#include "rt_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double x, y, z; } vec3;

static vec3 mk(double x, double y, double z) { vec3 r = {x, y, z}; return r; }
static vec3 sub(vec3 a, vec3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static vec3 add(vec3 a, vec3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static vec3 scl(vec3 a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
static double dot(vec3 a, vec3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static vec3 cross(vec3 a, vec3 b) {
  return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static double amax(vec3 a) {
  double m = fabs(a.x);
  if (fabs(a.y) > m) m = fabs(a.y);
  if (fabs(a.z) > m) m = fabs(a.z);
  return m;
}

/* ------------------------------------------------------------------------- */
/* rays and frames                                                            */
/* ------------------------------------------------------------------------- */

typedef struct {
  vec3 o, d;
  double tmin, tmax;
} ray64;

static ray64 load_ray(const float* r) {
  ray64 q;
  q.o = mk(r[0], r[1], r[2]);
  q.tmin = r[3];
  q.d = mk(r[4], r[5], r[6]);
  q.tmax = r[7];
  return q;
}

/* Rays that can never hit (reading of the paper's silence): any NaN, a zero
 * direction, or an empty range tmin > tmax. */
static int ray_is_void(const ray64* q) {
  if (isnan(q->o.x) || isnan(q->o.y) || isnan(q->o.z)) return 1;
  if (isnan(q->d.x) || isnan(q->d.y) || isnan(q->d.z)) return 1;
  if (isnan(q->tmin) || isnan(q->tmax)) return 1;
  if (q->d.x == 0.0 && q->d.y == 0.0 && q->d.z == 0.0) return 1;
  if (q->tmin > q->tmax) return 1;
  return 0;
}

/* Frame world = T + R(qhat)(S*x) and its inverse x = S^-1 R^T (world - T). */
typedef struct {
  double R[3][3];
  vec3 S, T;
} frame64;

/* The frame of ten float64 parameters (sx,sy,sz, qx,qy,qz,qw, tx,ty,tz). */
static frame64 frame_from(const double* f) {
  frame64 F;
  double qx = f[3], qy = f[4], qz = f[5], qw = f[6];
  double nq = sqrt(qx * qx + qy * qy + qz * qz + qw * qw);
  qx /= nq; qy /= nq; qz /= nq; qw /= nq;
  F.R[0][0] = 1 - 2 * (qy * qy + qz * qz);
  F.R[0][1] = 2 * (qx * qy - qz * qw);
  F.R[0][2] = 2 * (qx * qz + qy * qw);
  F.R[1][0] = 2 * (qx * qy + qz * qw);
  F.R[1][1] = 1 - 2 * (qx * qx + qz * qz);
  F.R[1][2] = 2 * (qy * qz - qx * qw);
  F.R[2][0] = 2 * (qx * qz - qy * qw);
  F.R[2][1] = 2 * (qy * qz + qx * qw);
  F.R[2][2] = 1 - 2 * (qx * qx + qy * qy);
  F.S = mk(f[0], f[1], f[2]);
  F.T = mk(f[7], f[8], f[9]);
  return F;
}

static frame64 load_frame(const float* f) {
  double p[10];
  for (int i = 0; i < 10; ++i) p[i] = f[i];
  return frame_from(p);
}

/* world = T + R (S*x) */
static vec3 to_world(const frame64* F, vec3 x) {
  vec3 a = mk(F->S.x * x.x, F->S.y * x.y, F->S.z * x.z);
  return mk(F->T.x + F->R[0][0] * a.x + F->R[0][1] * a.y + F->R[0][2] * a.z,
            F->T.y + F->R[1][0] * a.x + F->R[1][1] * a.y + F->R[1][2] * a.z,
            F->T.z + F->R[2][0] * a.x + F->R[2][1] * a.y + F->R[2][2] * a.z);
}

/* R^T a, then divide by the per-axis scale. */
static vec3 to_object_dir(const frame64* F, vec3 a) {
  vec3 r = mk(F->R[0][0] * a.x + F->R[1][0] * a.y + F->R[2][0] * a.z,
              F->R[0][1] * a.x + F->R[1][1] * a.y + F->R[2][1] * a.z,
              F->R[0][2] * a.x + F->R[1][2] * a.y + F->R[2][2] * a.z);
  return mk(r.x / F->S.x, r.y / F->S.y, r.z / F->S.z);
}

/* Infinity norm of the inverse linear part S^-1 R^T (used for slack only). */
static double inv_linear_norm(const frame64* F) {
  double m = 0.0;
  for (int i = 0; i < 3; ++i) {
    double s = (i == 0 ? F->S.x : (i == 1 ? F->S.y : F->S.z));
    double row = (fabs(F->R[0][i]) + fabs(F->R[1][i]) + fabs(F->R[2][i])) / fabs(s);
    if (row > m) m = row;
  }
  return m;
}

/* ------------------------------------------------------------------------- */
/* scene access                                                               */
/* ------------------------------------------------------------------------- */

static int scene_valid(const orc_scene* s) {
  if (!s || s->n_mesh < 1 || !s->vertices || !s->indices || !s->n_vertices || !s->n_triangles)
    return 0;
  for (int m = 0; m < s->n_mesh; ++m) {
    if (s->n_triangles[m] > 0 && (!s->vertices[m] || !s->indices[m])) return 0;
    for (int64_t k = 0; k < 3 * s->n_triangles[m]; ++k)
      if ((int64_t)s->indices[m][k] >= s->n_vertices[m]) return 0;
  }
  if (s->n_inst > 0) {
    if (!s->inst_mesh || !s->inst_srt) return 0;
    for (int64_t j = 0; j < s->n_inst; ++j)
      if ((int32_t)s->inst_mesh[j] >= s->n_mesh) return 0;
  }
  return 1;
}

static vec3 vtx(const orc_scene* s, int m, uint32_t i) {
  const float* p = s->vertices[m] + 3 * (int64_t)i;
  return mk(p[0], p[1], p[2]);
}

static void tri(const orc_scene* s, int m, int64_t k, vec3* v0, vec3* v1, vec3* v2) {
  const uint32_t* ix = s->indices[m] + 3 * k;
  *v0 = vtx(s, m, ix[0]);
  *v1 = vtx(s, m, ix[1]);
  *v2 = vtx(s, m, ix[2]);
}

/* The object-space ray of instance j (or the world ray when there are no
 * instances); also the mesh id and an extra slack scale (the magnitude of the
 * rounding a float32 transform of the origin would carry, in object units). */
static void object_ray(const orc_scene* s, const ray64* w, int64_t j, ray64* q, int* mesh,
                       double* extra_scale, double* extra_dir) {
  if (s->n_inst == 0) {
    *q = *w;
    *mesh = 0;
    *extra_scale = 0.0;
    *extra_dir = 0.0;
    return;
  }
  frame64 F = load_frame(s->inst_srt + 10 * j);
  q->o = to_object_dir(&F, sub(w->o, F.T));
  q->d = to_object_dir(&F, w->d);
  q->tmin = w->tmin;
  q->tmax = w->tmax;
  *mesh = (int)s->inst_mesh[j];
  *extra_scale = inv_linear_norm(&F) * (amax(w->o) + amax(F.T));
  *extra_dir = inv_linear_norm(&F) * amax(w->d);
}

/* ------------------------------------------------------------------------- */
/* §3.1: plane-then-edge ray/triangle test                                    */
/* ------------------------------------------------------------------------- */

static int intersect_paper(const ray64* q, vec3 v0, vec3 v1, vec3 v2, double* t_out, double* u_out,
                           double* v_out) {
  vec3 e0 = sub(v1, v0), e1 = sub(v2, v1), e2 = sub(v0, v2);
  vec3 n = cross(e0, e1);
  double nn = dot(n, n);
  if (!(nn > 0.0) || !isfinite(nn)) return 0; /* degenerate triangle */
  double den = dot(n, q->d);
  if (den == 0.0) return 0;                   /* parallel or in-plane ray */
  double t = dot(sub(v0, q->o), n) / den;
  if (!isfinite(t)) return 0;
  if (!(q->tmin <= t && t <= q->tmax)) return 0;
  vec3 p = add(q->o, scl(q->d, t));
  double a = dot(n, cross(e0, sub(p, v0)));
  double b = dot(n, cross(e1, sub(p, v1)));
  double c = dot(n, cross(e2, sub(p, v2)));
  if (a < 0.0 || b < 0.0 || c < 0.0) return 0;
  /* a, b, c are (2 area)*(sub-triangle doubled areas); the sub-triangle
   * opposite a vertex gives that vertex's weight: c -> v1, a -> v2. */
  *t_out = t;
  *u_out = c / nn;
  *v_out = a / nn;
  (void)b;
  return 1;
}

/* Plane formula at a fixed triangle with no range or inside test; used by the
 * finite differences, so that perturbations across an edge stay smooth. */
static void plane_tuv(vec3 o, vec3 d, vec3 v0, vec3 v1, vec3 v2, double* t_out, double* u_out,
                      double* v_out) {
  vec3 e0 = sub(v1, v0), e1 = sub(v2, v1), e2 = sub(v0, v2);
  vec3 n = cross(e0, e1);
  double nn = dot(n, n);
  double t = dot(sub(v0, o), n) / dot(n, d);
  vec3 p = add(o, scl(d, t));
  *t_out = t;
  *u_out = dot(n, cross(e2, sub(p, v2))) / nn;
  *v_out = dot(n, cross(e0, sub(p, v0))) / nn;
}

/* ------------------------------------------------------------------------- */
/* closest and any                                                            */
/* ------------------------------------------------------------------------- */

static int64_t n_units(const orc_scene* s) { return s->n_inst > 0 ? s->n_inst : 1; }

/* Query options (masks and the self-intersection filter); see the header. */
static int unit_enabled(const orc_scene* s, const orc_opts* o, int64_t r, int64_t j) {
  if (!o || !o->ray_mask) return 1;
  uint32_t m = (s->n_inst > 0 && o->inst_mask) ? o->inst_mask[j] : 0xFFFFFFFFu;
  return (m & o->ray_mask[r]) != 0u;
}

static int skipped(const orc_scene* s, const orc_opts* o, int64_t r, int64_t j, int64_t k) {
  if (!o || !o->skip_prim || o->skip_prim[r] == ORC_NONE) return 0;
  if ((uint32_t)k != o->skip_prim[r]) return 0;
  if (s->n_inst > 0 && o->skip_inst && (uint32_t)j != o->skip_inst[r]) return 0;
  return 1;
}

/* ------------------------------------------------------------------------- */
/* acceptable sets                                                            */
/* ------------------------------------------------------------------------- */
/* A float32 implementation decides hit or miss from rounded quantities, so at
 * edges, silhouettes, ties and range ends several answers are correct.  The
 * model: the float32 evaluation is exact for inputs moved by a small relative
 * amount delta; near the triangle this moves the ray line relative to the
 * triangle by at most
 *     eta = 2 delta s + 2 tilt L,
 * s = largest coordinate magnitude involved (origin, vertices and, for
 * instances, the rounding of the object-space transform of the origin),
 * L = largest distance from the origin to a vertex, tilt = delta (times the
 * transform's amplification of the direction for instances).  Then a pair is
 *   a sure miss when the ray's line stays farther than eta from the triangle,
 *               or the triangle's extent along the line, widened by eta,
 *               lies outside [tmin, tmax];
 *               or (when the plane crossing is well defined) the crossing t
 *               lies outside [tmin, tmax] by more than rho_t = 2 eta/(cos |d|)
 *               (cos = |n.d| / (|n||d|): the line and the plane each move by
 *               at most eta near the triangle);
 *   a sure hit  when the line crosses the triangle's plane inside the
 *               triangle at distance at least eta/cos + eta from each edge
 *               (a shift eta of the line moves the crossing by eta/cos in the
 *               plane) and t is inside [tmin, tmax] by at least rho_t;
 *   a maybe     otherwise.
 * The acceptable closest answers of a ray are the sure and maybe pairs whose
 * lowest possible t (t - rho_t for a sure hit, the widened extent's start for
 * a maybe) does not exceed t* = min over sure hits of t + rho_t, plus "miss"
 * when there is no sure hit. */

typedef struct {
  double t, u, v, lo, hi, scale;
  uint32_t inst, prim;
  int sure;
} cand;

/* (t, inst, prim) order; a candidate whose t is undefined (a degenerate
 * triangle's plane formula gives 0/0) sorts after every defined t, so the
 * order is total and the same whatever order the pairs were found in. */
static int cand_less(const cand* a, const cand* b) {
  int an = isnan(a->t), bn = isnan(b->t);
  if (an != bn) return bn;
  if (!an && a->t != b->t) return a->t < b->t;
  if (a->inst != b->inst) return a->inst < b->inst;
  return a->prim < b->prim;
}

static double norm(vec3 a) { return sqrt(dot(a, a)); }

/* distance between the segment [A,B] and the line o + t d */
static double seg_line_dist(vec3 A, vec3 B, vec3 o, vec3 d) {
  vec3 w = cross(sub(A, o), d), z = cross(sub(B, A), d);
  double zz = dot(z, z), u = 0.0;
  if (zz > 0.0) {
    u = -dot(w, z) / zz;
    if (u < 0.0) u = 0.0;
    if (u > 1.0) u = 1.0;
  }
  return norm(add(w, scl(z, u))) / norm(d);
}

/* distance from the point p to the line through A and B */
static double point_line_dist(vec3 p, vec3 A, vec3 B) {
  vec3 e = sub(B, A);
  return norm(cross(sub(p, A), e)) / norm(e);
}

/* classification: 0 sure miss, 1 maybe, 2 sure hit; c->t = t* contribution */
static int classify(const ray64* q, vec3 v0, vec3 v1, vec3 v2, double delta, double extra_scale,
                    double extra_dir, cand* c, double* hi) {
  vec3 a0 = sub(v0, q->o), a1 = sub(v1, q->o), a2 = sub(v2, q->o);
  double s = amax(q->o);
  if (amax(v0) > s) s = amax(v0);
  if (amax(v1) > s) s = amax(v1);
  if (amax(v2) > s) s = amax(v2);
  if (extra_scale > s) s = extra_scale;
  double L = norm(a0);
  if (norm(a1) > L) L = norm(a1);
  if (norm(a2) > L) L = norm(a2);
  double dm = amax(q->d), tilt = delta;
  if (extra_dir > dm) tilt = delta * extra_dir / dm;
  double eta = 2.0 * delta * s + 2.0 * tilt * L;
  double dn = norm(q->d);

  /* does the line cross the triangle (edge functions of one sign)? */
  double E0 = dot(q->d, cross(a1, a2)), E1 = dot(q->d, cross(a2, a0)), E2 = dot(q->d, cross(a0, a1));
  int crosses = (E0 + E1 + E2 != 0.0) &&
                ((E0 >= 0.0 && E1 >= 0.0 && E2 >= 0.0) || (E0 <= 0.0 && E1 <= 0.0 && E2 <= 0.0));
  double dist = 0.0;
  if (!crosses) {
    dist = seg_line_dist(v0, v1, q->o, q->d);
    double d1 = seg_line_dist(v1, v2, q->o, q->d), d2 = seg_line_dist(v2, v0, q->o, q->d);
    if (d1 < dist) dist = d1;
    if (d2 < dist) dist = d2;
  }
  if (!(dist <= eta)) return 0;
  /* extent of the triangle along the line, widened by eta */
  double dd = dot(q->d, q->d);
  double p0 = dot(a0, q->d) / dd, p1 = dot(a1, q->d) / dd, p2 = dot(a2, q->d) / dd;
  double tlo = p0, thi = p0;
  if (p1 < tlo) tlo = p1;
  if (p2 < tlo) tlo = p2;
  if (p1 > thi) thi = p1;
  if (p2 > thi) thi = p2;
  tlo -= eta / dn;
  thi += eta / dn;
  if (thi < q->tmin || tlo > q->tmax) return 0;

  double t, u, v;
  plane_tuv(q->o, q->d, v0, v1, v2, &t, &u, &v); /* values by the plane formula of §3.1 */
  vec3 n = cross(sub(v1, v0), sub(v2, v0));
  double nl = norm(n);
  double cs = (nl > 0.0) ? fabs(dot(n, q->d)) / (nl * dn) : 0.0;
  /* where the plane crossing is well defined, the line and the plane near the
   * triangle each move by at most eta, so the crossing moves along the ray
   * by at most rt */
  double rt = (cs > 0.0 && isfinite(t)) ? 2.0 * eta / (cs * dn) : INFINITY;
  if (isfinite(rt)) {
    if (t - rt > tlo) tlo = t - rt;
    if (t + rt < thi) thi = t + rt;
    if (thi < q->tmin || tlo > q->tmax) return 0;
  }
  c->t = t;
  c->u = u;
  c->v = v;
  c->scale = s;
  c->lo = tlo;
  *hi = thi;
  if (crosses && isfinite(rt)) {
    double need = eta / cs + eta;
    vec3 p = add(q->o, scl(q->d, t));
    double cl = point_line_dist(p, v0, v1);
    double c1 = point_line_dist(p, v1, v2), c2 = point_line_dist(p, v2, v0);
    if (c1 < cl) cl = c1;
    if (c2 < cl) cl = c2;
    if (cl >= need && t - rt >= q->tmin && t + rt <= q->tmax) {
      c->lo = t - rt;
      *hi = t + rt;
      return 2;
    }
  }
  return 1;
}

/* ------------------------------------------------------------------------- */
/* the work of one (ray, triangle) pair, for every query                      */
/* ------------------------------------------------------------------------- */
/* Both searches below, the linear one and the one through the BVH, hand every
 * (ray, instance, triangle) pair they do not skip to on_pair, which does what
 * the query asks of a pair; only the order of the pairs differs.  Each query's
 * result is a function of the set of pairs, not of their order:
 *   closest: the lexicographic minimum of (t, inst, prim) -- visited in
 *            ascending (inst, prim) order, as the linear search of §3.3 does,
 *            this is the listing's strict "t < minT" update;
 *   any:     whether some pair is a hit;
 *   all:     the hits, sorted by (t, inst, prim) afterwards;
 *   classify: the sure and maybe pairs, sorted afterwards, and t* (the
 *            smallest upper t of a sure hit). */

typedef struct {
  double t, u, v;
  uint32_t inst, prim;
} hit64;

static int hit_less(const hit64* a, const hit64* b) {
  if (a->t != b->t) return a->t < b->t;
  if (a->inst != b->inst) return a->inst < b->inst;
  return a->prim < b->prim;
}

enum { Q_CLOSEST = 0, Q_ANY = 1, Q_ALL = 2, Q_CAND = 3 };

typedef struct {
  int kind;
  int cull_tstar;      /* Q_CAND: only pairs that can be the closest are wanted */
  double delta;        /* Q_CAND: relative input slack */
  double minT, bu, bv; /* Q_CLOSEST */
  uint32_t bi, bp;
  int hit;             /* Q_ANY */
  hit64* hits;         /* Q_ALL */
  cand* cands;         /* Q_CAND */
  int64_t n, cap;
  int bad;             /* a list could not grow */
  double tstar;        /* Q_CAND */
  int sures;
} qstate;

static void qstate_reset(qstate* st) {
  st->minT = INFINITY;
  st->bu = st->bv = 0.0;
  st->bi = st->bp = ORC_NONE;
  st->hit = 0;
  st->n = 0;
  st->tstar = INFINITY;
  st->sures = 0;
}

static int grow(void** buf, int64_t* cap, size_t elem) {
  int64_t nc = *cap ? 2 * *cap : 64;
  void* nb = realloc(*buf, elem * (size_t)nc);
  if (!nb) return 0;
  *buf = nb;
  *cap = nc;
  return 1;
}

/* Returns 1 when the query may stop (an any-hit query found a hit). */
static int on_pair(qstate* st, const ray64* q, uint32_t inst, uint32_t prim, vec3 v0, vec3 v1,
                   vec3 v2, double xs, double xd) {
  if (st->kind == Q_CLOSEST) {
    double t, u, v;
    if (!intersect_paper(q, v0, v1, v2, &t, &u, &v)) return 0;
    if (t < st->minT || (t == st->minT && (inst < st->bi || (inst == st->bi && prim < st->bp)))) {
      st->minT = t;
      st->bu = u;
      st->bv = v;
      st->bi = inst;
      st->bp = prim;
    }
    return 0;
  }
  if (st->kind == Q_ANY) {
    double t, u, v;
    if (!intersect_paper(q, v0, v1, v2, &t, &u, &v)) return 0;
    st->hit = 1;
    return 1;
  }
  if (st->kind == Q_ALL) {
    hit64 h;
    if (!intersect_paper(q, v0, v1, v2, &h.t, &h.u, &h.v)) return 0;
    h.inst = inst;
    h.prim = prim;
    if (st->n == st->cap && !grow((void**)&st->hits, &st->cap, sizeof(hit64))) {
      st->bad = 1;
      return 0;
    }
    st->hits[st->n++] = h;
    return 0;
  }
  cand c;
  double hi;
  int cls = classify(q, v0, v1, v2, st->delta, xs, xd, &c, &hi);
  if (cls == 0) return 0;
  c.inst = inst;
  c.prim = prim;
  c.sure = (cls == 2);
  c.hi = hi;
  if (c.sure) {
    st->sures++;
    if (hi < st->tstar) st->tstar = hi;
  }
  if (st->n == st->cap && !grow((void**)&st->cands, &st->cap, sizeof(cand))) {
    st->bad = 1;
    return 0;
  }
  st->cands[st->n++] = c;
  return 0;
}

/* ------------------------------------------------------------------------- */
/* the linear search (§3.3)                                                   */
/* ------------------------------------------------------------------------- */

/* Every triangle of mesh m, in ascending order, for unit j. */
static int scan_mesh(const orc_scene* s, const orc_opts* opts, int64_t r, int64_t j, int m,
                     const ray64* q, double xs, double xd, qstate* st) {
  for (int64_t k = 0; k < s->n_triangles[m]; ++k) {
    vec3 v0, v1, v2;
    if (skipped(s, opts, r, j, k)) continue;
    tri(s, m, k, &v0, &v1, &v2);
    if (on_pair(st, q, (uint32_t)j, (uint32_t)k, v0, v1, v2, xs, xd)) return 1;
  }
  return 0;
}

static void search_linear(const orc_scene* s, const orc_opts* opts, int64_t r, const ray64* w,
                          qstate* st) {
  for (int64_t j = 0; j < n_units(s); ++j) {
    if (!unit_enabled(s, opts, r, j)) continue;
    ray64 q;
    int m;
    double xs, xd;
    object_ray(s, w, j, &q, &m, &xs, &xd);
    if (scan_mesh(s, opts, r, j, m, &q, xs, xd, st)) return;
  }
}

/* ------------------------------------------------------------------------- */
/* FP64 bounding-volume hierarchy: an exact accelerator of the linear search  */
/* ------------------------------------------------------------------------- */
/* §6.2 (traversal paragraph): a hierarchy of boxes only lets the search skip
 * triangles whose boxes the ray misses, so the answers are those of the
 * linear search.  This one is deliberately plain: a binary tree split at the
 * median box centre along the longest axis of the centres' bounds, leaves of
 * at most four items, boxes that are the exact min/max of the float32
 * vertices (exact in float64).  The walk hands the surviving pairs to the
 * same on_pair as the linear search, so every query's answer is identical
 * bit for bit.  The box tests only skip what provably holds no wanted pair:
 *   - a hit of §3.1 puts o + t d within float64 rounding of the triangle,
 *     so its t lies in the slab interval of the box widened by
 *     2^-34 (|o|_inf + |box|_inf) (far above that rounding);
 *   - a sure or maybe pair of the tolerance model has its line within eta
 *     of the triangle and the triangle's extent along the line, widened by
 *     eta/|d|, meeting [tmin, tmax]; eta is bounded over the box by the same
 *     formula with the box's largest coordinate and farthest corner;
 *   - its lowest t (lo) is at least the smallest projection of the box's
 *     corners minus max(eta, 3 D)/|d| (D = box diagonal: a sure hit needs
 *     eta/cos <= its distance to the edges <= D, so rho_t <= 2 D/|d|).
 * Triangles with a non-finite vertex, instances with a non-finite frame or
 * whose mesh holds such triangles, and rays with a non-finite origin or
 * direction take the linear search for the part concerned. */

typedef struct {
  double lo[3], hi[3];
  int64_t a, b; /* internal: children a, b; leaf: a = -1 - first item slot, b = item count */
} bnode;

typedef struct {
  bnode* node;
  int64_t n_node;
  int64_t* item;  /* item ids, leaf after leaf */
  int64_t n_item;
  int64_t* loose; /* items with no finite box: visited for every ray */
  int64_t n_loose;
  double amax_box; /* largest |coordinate| of the root box */
  int depth;
  int64_t* parent;  /* [n_node], -1 at the root (for the bound check) */
  int64_t* leaf_of; /* [n_items] the leaf holding each item, -1 if none */
  double* nb;       /* instance tree: per node, the largest ||A||, ||A^-1||,
                     * |T|, ||A|| ||A^-1|| and mesh coordinate of its instances */
} btree;

struct orc_bvh_s {
  int32_t n_mesh;
  int64_t n_inst;
  const float* const* vertices; /* the scene it was built for */
  btree* mesh;                  /* [n_mesh] over each mesh's triangles */
  btree top;                    /* instances, over their world boxes */
  frame64* frame;               /* [n_inst] */
};
enum { NB_A, NB_AINV, NB_T, NB_KAPPA, NB_V, NB_N };

#define BVH_LEAF 4
#define BVH_STACK 160

typedef struct {
  double key;
  int64_t id;
} kv;

static int kv_less(const kv* a, const kv* b) {
  return a->key < b->key || (a->key == b->key && a->id < b->id);
}

/* Rearranges a[0..n) so that a[k] is the element of rank k and no element
 * before it is larger, none after it smaller (keys are distinct: ids are). */
static void select_kth(kv* a, int64_t n, int64_t k) {
  int64_t lo = 0, hi = n - 1;
  uint64_t seed = 0x9E3779B97F4A7C15ull ^ (uint64_t)n;
  while (hi > lo) {
    seed = seed * 6364136223846793005ull + 1442695040888963407ull;
    int64_t p = lo + (int64_t)((seed >> 33) % (uint64_t)(hi - lo + 1));
    kv pivot = a[p], tmp;
    a[p] = a[hi];
    a[hi] = pivot;
    int64_t st = lo;
    for (int64_t i = lo; i < hi; ++i)
      if (kv_less(&a[i], &pivot)) {
        tmp = a[i]; a[i] = a[st]; a[st] = tmp;
        ++st;
      }
    tmp = a[st]; a[st] = a[hi]; a[hi] = tmp;
    if (st == k) return;
    if (k < st) hi = st - 1; else lo = st + 1;
  }
}

/* box: 6 doubles per item (lo xyz, hi xyz); ids: the items of this subtree,
 * reordered in place (they live in T->item) */
static int64_t bt_build(btree* T, const double* box, int64_t* ids, int64_t n, kv* tmp, int depth) {
  int64_t me = T->n_node++;
  bnode* nd = &T->node[me];
  if (depth > T->depth) T->depth = depth;
  for (int c = 0; c < 3; ++c) {
    nd->lo[c] = INFINITY;
    nd->hi[c] = -INFINITY;
  }
  double cl[3] = {INFINITY, INFINITY, INFINITY}, ch[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = 0; i < n; ++i) {
    const double* b = box + 6 * ids[i];
    for (int c = 0; c < 3; ++c) {
      if (b[c] < nd->lo[c]) nd->lo[c] = b[c];
      if (b[3 + c] > nd->hi[c]) nd->hi[c] = b[3 + c];
      double m = 0.5 * (b[c] + b[3 + c]);
      if (m < cl[c]) cl[c] = m;
      if (m > ch[c]) ch[c] = m;
    }
  }
  if (n <= BVH_LEAF) {
    nd->a = -1 - (ids - T->item);
    nd->b = n;
    return me;
  }
  int axis = 0;
  if (ch[1] - cl[1] > ch[axis] - cl[axis]) axis = 1;
  if (ch[2] - cl[2] > ch[axis] - cl[axis]) axis = 2;
  for (int64_t i = 0; i < n; ++i) {
    const double* b = box + 6 * ids[i];
    tmp[i].key = 0.5 * (b[axis] + b[3 + axis]);
    tmp[i].id = ids[i];
  }
  int64_t h = n / 2;
  select_kth(tmp, n, h);
  for (int64_t i = 0; i < n; ++i) ids[i] = tmp[i].id;
  int64_t a = bt_build(T, box, ids, h, tmp, depth + 1);
  int64_t b = bt_build(T, box, ids + h, n - h, tmp, depth + 1);
  T->node[me].a = a;
  T->node[me].b = b;
  return me;
}

static int box_finite(const double* b) {
  for (int c = 0; c < 6; ++c)
    if (!isfinite(b[c])) return 0;
  return 1;
}

static void bt_free(btree* T) {
  free(T->node);
  free(T->item);
  free(T->loose);
  free(T->parent);
  free(T->leaf_of);
  free(T->nb);
  memset(T, 0, sizeof(*T));
}

/* A tree over n items with boxes box[6n]; items with a non-finite box or
 * excluded (skip[i] != 0, may be NULL: none) are left out, and the
 * non-finite ones listed as loose.  Returns 0 on allocation failure. */
static int bt_make(btree* T, const double* box, int64_t n, const uint8_t* skip) {
  memset(T, 0, sizeof(*T));
  int64_t nf = 0, nl = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (skip && skip[i]) continue;
    if (box_finite(box + 6 * i)) ++nf; else ++nl;
  }
  T->item = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nf ? nf : 1));
  T->loose = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nl ? nl : 1));
  T->node = (bnode*)malloc(sizeof(bnode) * (size_t)(nf ? 2 * nf : 1));
  kv* tmp = (kv*)malloc(sizeof(kv) * (size_t)(nf ? nf : 1));
  if (!T->item || !T->loose || !T->node || !tmp) {
    free(tmp);
    bt_free(T);
    return 0;
  }
  for (int64_t i = 0; i < n; ++i) {
    if (skip && skip[i]) continue;
    if (box_finite(box + 6 * i)) T->item[T->n_item++] = i; else T->loose[T->n_loose++] = i;
  }
  T->parent = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nf ? 2 * nf : 1));
  T->leaf_of = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
  if (!T->parent || !T->leaf_of) {
    free(tmp);
    bt_free(T);
    return 0;
  }
  for (int64_t i = 0; i < n; ++i) T->leaf_of[i] = -1;
  if (nf > 0) {
    bt_build(T, box, T->item, nf, tmp, 0);
    T->parent[0] = -1;
    for (int64_t i = 0; i < T->n_node; ++i) {
      const bnode* nd = &T->node[i];
      if (nd->a < 0) {
        for (int64_t k = 0; k < nd->b; ++k) T->leaf_of[T->item[-1 - nd->a + k]] = i;
      } else {
        T->parent[nd->a] = i;
        T->parent[nd->b] = i;
      }
    }
    double m = 0.0;
    for (int c = 0; c < 3; ++c) {
      if (fabs(T->node[0].lo[c]) > m) m = fabs(T->node[0].lo[c]);
      if (fabs(T->node[0].hi[c]) > m) m = fabs(T->node[0].hi[c]);
    }
    T->amax_box = m;
  }
  free(tmp);
  return T->depth < BVH_STACK - 4;
}

/* infinity norm of the linear part R(q) diag(S) */
static double linear_norm(const frame64* F) {
  double S[3] = {fabs(F->S.x), fabs(F->S.y), fabs(F->S.z)}, m = 0.0;
  for (int i = 0; i < 3; ++i) {
    double row = 0.0;
    for (int k = 0; k < 3; ++k) row += fabs(F->R[i][k]) * S[k];
    if (row > m) m = row;
  }
  return m;
}

void orc_bvh_destroy(orc_bvh* B) {
  if (!B) return;
  if (B->mesh)
    for (int m = 0; m < B->n_mesh; ++m) bt_free(&B->mesh[m]);
  free(B->mesh);
  bt_free(&B->top);
  free(B->frame);
  free(B);
}

int orc_bvh_create(const orc_scene* s, orc_bvh** out) {
  if (!out) return -1;
  *out = NULL;
  if (!scene_valid(s)) return -1;
  orc_bvh* B = (orc_bvh*)calloc(1, sizeof(orc_bvh));
  if (!B) return -1;
  B->n_mesh = s->n_mesh;
  B->n_inst = s->n_inst;
  B->vertices = s->vertices;
  B->mesh = (btree*)calloc((size_t)s->n_mesh, sizeof(btree));
  if (!B->mesh) goto fail;
  for (int m = 0; m < s->n_mesh; ++m) {
    int64_t nt = s->n_triangles[m];
    double* box = (double*)malloc(sizeof(double) * 6 * (size_t)(nt ? nt : 1));
    if (!box) goto fail;
    for (int64_t k = 0; k < nt; ++k) {
      vec3 v[3];
      tri(s, m, k, &v[0], &v[1], &v[2]);
      double* b = box + 6 * k;
      b[0] = b[3] = v[0].x;
      b[1] = b[4] = v[0].y;
      b[2] = b[5] = v[0].z;
      for (int c = 1; c < 3; ++c) {
        double x[3] = {v[c].x, v[c].y, v[c].z};
        for (int a = 0; a < 3; ++a) {
          /* a NaN coordinate leaves the box non-finite (loose) */
          if (!(x[a] >= b[a])) b[a] = x[a];
          if (!(x[a] <= b[3 + a])) b[3 + a] = x[a];
        }
      }
    }
    int okm = bt_make(&B->mesh[m], box, nt, NULL);
    free(box);
    if (!okm) goto fail;
  }
  if (s->n_inst > 0) {
    int64_t ni = s->n_inst;
    B->frame = (frame64*)malloc(sizeof(frame64) * (size_t)ni);
    double* box = (double*)malloc(sizeof(double) * 6 * (size_t)ni);
    double* ib = (double*)malloc(sizeof(double) * NB_N * (size_t)ni);
    uint8_t* skip = (uint8_t*)calloc((size_t)ni, 1);
    if (!B->frame || !box || !ib || !skip) {
      free(box);
      free(ib);
      free(skip);
      goto fail;
    }
    for (int64_t j = 0; j < ni; ++j) {
      B->frame[j] = load_frame(s->inst_srt + 10 * j);
      const frame64* F = &B->frame[j];
      const btree* T = &B->mesh[s->inst_mesh[j]];
      double* b = box + 6 * j;
      if (T->n_item == 0 && T->n_loose == 0) {
        skip[j] = 1; /* an empty mesh: no pair to find */
        continue;
      }
      double A = linear_norm(F), Ai = inv_linear_norm(F);
      int fin = T->n_loose == 0 && isfinite(A) && isfinite(Ai) && A > 0.0 &&
                isfinite(F->T.x) && isfinite(F->T.y) && isfinite(F->T.z);
      for (int c = 0; c < 3; ++c) {
        b[c] = INFINITY;
        b[3 + c] = -INFINITY;
      }
      if (fin) {
        const bnode* r0 = &T->node[0];
        for (int corner = 0; corner < 8; ++corner) {
          vec3 x = mk((corner & 1) ? r0->hi[0] : r0->lo[0], (corner & 2) ? r0->hi[1] : r0->lo[1],
                      (corner & 4) ? r0->hi[2] : r0->lo[2]);
          vec3 wpt = to_world(F, x);
          double wc[3] = {wpt.x, wpt.y, wpt.z};
          for (int c = 0; c < 3; ++c) {
            if (wc[c] < b[c]) b[c] = wc[c];
            if (wc[c] > b[3 + c]) b[3 + c] = wc[c];
          }
        }
        double slack = 0x1p-40 * (amax(F->T) + A * T->amax_box);
        for (int c = 0; c < 3; ++c) {
          b[c] -= slack;
          b[3 + c] += slack;
        }
        fin = box_finite(b);
      }
      if (!fin) {
        b[0] = NAN; /* loose: searched for every ray */
        continue;
      }
      double* e = ib + NB_N * j;
      e[NB_A] = A;
      e[NB_AINV] = Ai;
      e[NB_T] = amax(F->T);
      e[NB_KAPPA] = A * Ai;
      e[NB_V] = T->amax_box;
    }
    int okt = bt_make(&B->top, box, ni, skip);
    free(box);
    btree* TT = &B->top;
    TT->nb = okt ? (double*)calloc((size_t)NB_N * (size_t)(TT->n_node ? TT->n_node : 1), sizeof(double))
                 : NULL;
    if (!TT->nb) {
      free(ib);
      free(skip);
      goto fail;
    }
    /* per-node maxima, children before parents (nodes are numbered in
     * pre-order, so every child has a larger index than its parent) */
    for (int64_t i = TT->n_node - 1; i >= 0; --i) {
      const bnode* nd = &TT->node[i];
      double* e = TT->nb + NB_N * i;
      if (nd->a < 0) {
        for (int64_t k = 0; k < nd->b; ++k)
          for (int c = 0; c < NB_N; ++c)
            e[c] = fmax(e[c], ib[NB_N * TT->item[-1 - nd->a + k] + c]);
      } else {
        for (int c = 0; c < NB_N; ++c)
          e[c] = fmax(TT->nb[NB_N * nd->a + c], TT->nb[NB_N * nd->b + c]);
      }
    }
    free(ib);
    free(skip);
  }
  *out = B;
  return 0;
fail:
  orc_bvh_destroy(B);
  return -1;
}

int orc_bvh_stats(const orc_bvh* B, int64_t* out /* 4: nodes, loose, max depth, top nodes */) {
  if (!B || !out) return -1;
  out[0] = out[1] = out[2] = 0;
  for (int m = 0; m < B->n_mesh; ++m) {
    out[0] += B->mesh[m].n_node;
    out[1] += B->mesh[m].n_loose;
    if (B->mesh[m].depth > out[2]) out[2] = B->mesh[m].depth;
  }
  out[3] = B->top.n_node;
  return 0;
}

/* ---- walking the trees -------------------------------------------------- */

static int ray_finite(const ray64* q) {
  if (!isfinite(q->o.x) || !isfinite(q->o.y) || !isfinite(q->o.z)) return 0;
  if (!isfinite(q->d.x) || !isfinite(q->d.y) || !isfinite(q->d.z)) return 0;
  double dd = dot(q->d, q->d);
  return isfinite(dd) && dd > 0.0;
}

/* Parameters where the line o + t d enters and leaves the box widened by m
 * (relatively widened beyond the rounding of the divisions); 0 when it
 * misses. */
static int slab(const double lo[3], const double hi[3], double m, vec3 o, vec3 d, double* te,
                double* tx) {
  double O[3] = {o.x, o.y, o.z}, D[3] = {d.x, d.y, d.z};
  double a = -INFINITY, b = INFINITY;
  for (int i = 0; i < 3; ++i) {
    double l = lo[i] - m, h = hi[i] + m;
    if (D[i] == 0.0) {
      if (O[i] < l || O[i] > h) return 0;
      continue;
    }
    double t1 = (l - O[i]) / D[i], t2 = (h - O[i]) / D[i];
    if (t1 > t2) {
      double x = t1; t1 = t2; t2 = x;
    }
    if (t1 > a) a = t1;
    if (t2 < b) b = t2;
  }
  if (isfinite(a)) a -= fabs(a) * 0x1p-40;
  if (isfinite(b)) b += fabs(b) * 0x1p-40;
  if (!(a <= b)) return 0;
  *te = a;
  *tx = b;
  return 1;
}

/* per (ray, unit) constants of the box tests */
typedef struct {
  const ray64* q;
  double amax_o, m_hit; /* hit queries: the box widening */
  double xs, tilt, dd, dn; /* candidate queries */
} wprep;

static void wprep_init(wprep* P, const qstate* st, const ray64* q, double xs, double xd,
                       double amax_box) {
  P->q = q;
  P->amax_o = amax(q->o);
  P->m_hit = 0x1p-34 * (P->amax_o + amax_box);
  P->xs = xs;
  P->dd = dot(q->d, q->d);
  P->dn = sqrt(P->dd);
  double dm = amax(q->d);
  P->tilt = st->delta;
  if (xd > dm) P->tilt = st->delta * xd / dm;
}

/* Whether the box may hold a wanted pair; *key orders the children (entry t)
 * and re-checks a stacked box against the current bound (entry t for the
 * closest hit, the lowest lo for the acceptable closest answers). */
static int box_test(const wprep* P, const qstate* st, const bnode* nd, double* key) {
  const ray64* q = P->q;
  double te, tx;
  if (st->kind != Q_CAND) {
    if (!slab(nd->lo, nd->hi, P->m_hit, q->o, q->d, &te, &tx)) return 0;
    double tc = q->tmax;
    if (st->kind == Q_CLOSEST && st->minT < tc) tc = st->minT;
    if (te > tc || tx < q->tmin) return 0;
    *key = te;
    return 1;
  }
  double O[3] = {q->o.x, q->o.y, q->o.z}, D[3] = {q->d.x, q->d.y, q->d.z};
  double ab = 0.0, far2 = 0.0, diag2 = 0.0, pmin = 0.0, pmax = 0.0;
  for (int i = 0; i < 3; ++i) {
    double l = nd->lo[i], h = nd->hi[i];
    if (fabs(l) > ab) ab = fabs(l);
    if (fabs(h) > ab) ab = fabs(h);
    double f = fmax(fabs(l - O[i]), fabs(h - O[i]));
    far2 += f * f;
    diag2 += (h - l) * (h - l);
    double pl = (l - O[i]) * D[i], ph = (h - O[i]) * D[i];
    pmin += fmin(pl, ph);
    pmax += fmax(pl, ph);
  }
  double s = P->amax_o;
  if (ab > s) s = ab;
  if (P->xs > s) s = P->xs;
  double L = sqrt(far2) * (1.0 + 0x1p-40);
  double eta = 2.0 * st->delta * s + 2.0 * P->tilt * L;
  double m = eta + 0x1p-34 * (P->amax_o + ab + L);
  if (!slab(nd->lo, nd->hi, m, q->o, q->d, &te, &tx)) return 0;
  pmin /= P->dd;
  pmax /= P->dd;
  double w = m / P->dn;
  double plo = pmin - w, phi = pmax + w;
  plo -= fabs(plo) * 0x1p-40;
  phi += fabs(phi) * 0x1p-40;
  if (phi < q->tmin || plo > q->tmax) return 0;
  double lb = pmin - fmax(m, 3.0 * sqrt(diag2) * (1.0 + 0x1p-40)) / P->dn;
  lb -= fabs(lb) * 0x1p-40;
  *key = lb;
  return !(st->cull_tstar && lb > st->tstar);
}

static int stale(const qstate* st, const ray64* q, double key) {
  if (st->kind == Q_CLOSEST) return key > st->minT || key > q->tmax;
  if (st->kind == Q_CAND) return st->cull_tstar && key > st->tstar;
  return 0;
}

typedef struct {
  int64_t node;
  double key;
} sentry;

/* The pairs of unit j (mesh m) that its tree does not rule out. */
static int walk_mesh(const orc_scene* s, const orc_bvh* B, const orc_opts* opts, int64_t r,
                     int64_t j, int m, const ray64* q, double xs, double xd, qstate* st) {
  const btree* T = &B->mesh[m];
  if (!ray_finite(q)) return scan_mesh(s, opts, r, j, m, q, xs, xd, st);
  vec3 v0, v1, v2;
  for (int64_t i = 0; i < T->n_loose; ++i) {
    int64_t k = T->loose[i];
    if (skipped(s, opts, r, j, k)) continue;
    tri(s, m, k, &v0, &v1, &v2);
    if (on_pair(st, q, (uint32_t)j, (uint32_t)k, v0, v1, v2, xs, xd)) return 1;
  }
  if (T->n_node == 0) return 0;
  wprep P;
  wprep_init(&P, st, q, xs, xd, T->amax_box);
  sentry stk[BVH_STACK];
  int sp = 0;
  double key;
  if (box_test(&P, st, &T->node[0], &key)) {
    stk[0].node = 0;
    stk[0].key = key;
    sp = 1;
  }
  while (sp > 0) {
    sentry e = stk[--sp];
    if (stale(st, q, e.key)) continue;
    const bnode* nd = &T->node[e.node];
    if (nd->a < 0) {
      const int64_t* it = T->item + (-1 - nd->a);
      for (int64_t i = 0; i < nd->b; ++i) {
        int64_t k = it[i];
        if (skipped(s, opts, r, j, k)) continue;
        tri(s, m, k, &v0, &v1, &v2);
        if (on_pair(st, q, (uint32_t)j, (uint32_t)k, v0, v1, v2, xs, xd)) return 1;
      }
      continue;
    }
    double ka = 0.0, kb = 0.0;
    int ha = box_test(&P, st, &T->node[nd->a], &ka);
    int hb = box_test(&P, st, &T->node[nd->b], &kb);
    /* the nearer child on top */
    if (ha && hb && ka <= kb) {
      stk[sp].node = nd->b; stk[sp++].key = kb;
      stk[sp].node = nd->a; stk[sp++].key = ka;
    } else {
      if (ha) { stk[sp].node = nd->a; stk[sp++].key = ka; }
      if (hb) { stk[sp].node = nd->b; stk[sp++].key = kb; }
    }
  }
  return 0;
}

/* object ray of an instance from its precomputed frame (the same arithmetic
 * as object_ray) */
static void instance_ray(const orc_scene* s, const orc_bvh* B, const ray64* w, int64_t j, ray64* q,
                         int* mesh, double* xs, double* xd) {
  const frame64* F = &B->frame[j];
  q->o = to_object_dir(F, sub(w->o, F->T));
  q->d = to_object_dir(F, w->d);
  q->tmin = w->tmin;
  q->tmax = w->tmax;
  *mesh = (int)s->inst_mesh[j];
  *xs = inv_linear_norm(F) * (amax(w->o) + amax(F->T));
  *xd = inv_linear_norm(F) * amax(w->d);
}

/* World-space widening of an instance-tree box: the object-space widening
 * bounded over the box's instances (largest inverse norm, translation, mesh
 * coordinate and condition number ||A|| ||A^-1||, which bounds the tilt of
 * the direction) mapped to world space by their largest linear norm, plus
 * the rounding of the world-to-object transform. */
static double top_margin(const btree* T, int64_t node, const qstate* st, const ray64* w) {
  const double* e = T->nb + NB_N * node;
  double ao = amax(w->o), amax_box = 0.0;
  for (int c = 0; c < 3; ++c) amax_box = fmax(amax_box, fmax(fabs(T->node[node].lo[c]), fabs(T->node[node].hi[c])));
  double xs_max = e[NB_AINV] * (ao + e[NB_T]) * (1.0 + 0x1p-40);
  double m_obj = 0x1p-34 * (xs_max + e[NB_V]);
  if (st->kind == Q_CAND) {
    double sm = xs_max > e[NB_V] ? xs_max : e[NB_V];
    double L = sqrt(3.0) * (xs_max + e[NB_V]);
    double tilt = st->delta * (e[NB_KAPPA] > 1.0 ? e[NB_KAPPA] : 1.0);
    double eta = 2.0 * st->delta * sm + 2.0 * tilt * L;
    m_obj = eta + 0x1p-34 * (xs_max + e[NB_V] + L);
  }
  return e[NB_A] * m_obj * (1.0 + 0x1p-30) +
         0x1p-28 * (e[NB_KAPPA] + 1.0) * (ao + e[NB_T] + amax_box + e[NB_V]);
}

/* An instance-tree box: the line within its widening of it (any t) for
 * candidate queries; for hit queries also its slab interval against
 * [tmin, tmax] and the closest hit so far (key = entry t). */
static int top_test(const btree* T, int64_t node, const qstate* st, const ray64* w, double* key) {
  const bnode* nd = &T->node[node];
  double te, tx, mw = top_margin(T, node, st, w);
  if (!slab(nd->lo, nd->hi, mw, w->o, w->d, &te, &tx)) return 0;
  if (st->kind == Q_CAND) {
    *key = -INFINITY;
    return 1;
  }
  double tc = w->tmax;
  if (st->kind == Q_CLOSEST && st->minT < tc) tc = st->minT;
  *key = te;
  return !(te > tc || tx < w->tmin);
}

static void search_bvh(const orc_scene* s, const orc_bvh* B, const orc_opts* opts, int64_t r,
                       const ray64* w, qstate* st) {
  if (!ray_finite(w)) {
    search_linear(s, opts, r, w, st);
    return;
  }
  if (s->n_inst == 0) {
    if (unit_enabled(s, opts, r, 0)) walk_mesh(s, B, opts, r, 0, 0, w, 0.0, 0.0, st);
    return;
  }
  const btree* T = &B->top;
  ray64 q;
  int m;
  double xs, xd;
  for (int64_t i = 0; i < T->n_loose; ++i) {
    int64_t j = T->loose[i];
    if (!unit_enabled(s, opts, r, j)) continue;
    instance_ray(s, B, w, j, &q, &m, &xs, &xd);
    if (walk_mesh(s, B, opts, r, j, m, &q, xs, xd, st)) return;
  }
  if (T->n_node == 0) return;
  sentry stk[BVH_STACK];
  int sp = 0;
  double key;
  if (top_test(T, 0, st, w, &key)) {
    stk[0].node = 0;
    stk[0].key = key;
    sp = 1;
  }
  while (sp > 0) {
    sentry e = stk[--sp];
    if (stale(st, w, e.key)) continue;
    const bnode* nd = &T->node[e.node];
    if (nd->a < 0) {
      const int64_t* it = T->item + (-1 - nd->a);
      for (int64_t i = 0; i < nd->b; ++i) {
        int64_t j = it[i];
        if (!unit_enabled(s, opts, r, j)) continue;
        instance_ray(s, B, w, j, &q, &m, &xs, &xd);
        if (walk_mesh(s, B, opts, r, j, m, &q, xs, xd, st)) return;
      }
      continue;
    }
    double ka = 0.0, kb = 0.0;
    int ha = top_test(T, nd->a, st, w, &ka);
    int hb = top_test(T, nd->b, st, w, &kb);
    if (ha && hb && ka <= kb) {
      stk[sp].node = nd->b; stk[sp++].key = kb;
      stk[sp].node = nd->a; stk[sp++].key = ka;
    } else {
      if (ha) { stk[sp].node = nd->a; stk[sp++].key = ka; }
      if (hb) { stk[sp].node = nd->b; stk[sp++].key = kb; }
    }
  }
}

/* The search a scene asks for: through its BVH when it has one. */
static void search(const orc_scene* s, const orc_opts* opts, int64_t r, const ray64* w,
                   qstate* st) {
  if (s->bvh) search_bvh(s, s->bvh, opts, r, w, st);
  else search_linear(s, opts, r, w, st);
}

/* A BVH belongs to the scene it was built from. */
static int bvh_matches(const orc_scene* s) {
  const orc_bvh* B = s->bvh;
  return !B || (B->n_mesh == s->n_mesh && B->n_inst == s->n_inst && B->vertices == s->vertices);
}

/* Checks the invariant the walk relies on, pair by pair: for every (ray,
 * instance, triangle) pair the linear search finds wanted (a §3.1 hit when
 * kind = 0; a sure or maybe pair of the tolerance model when kind = 1), every
 * box from the triangle's leaf up to its tree's root, and every instance box
 * above it, must pass its test with a key no larger than the pair's t (hits)
 * or its lowest possible t (candidates).  out[0] = pairs checked, out[1] =
 * violations. */
static int path_ok(const wprep* P, const qstate* st, const btree* T, int64_t item, double bound) {
  int64_t nd = T->leaf_of[item];
  if (nd < 0) return 1; /* loose: visited for every ray */
  for (; nd >= 0; nd = T->parent[nd]) {
    double key;
    if (!box_test(P, st, &T->node[nd], &key) || key > bound) return 0;
  }
  return 1;
}

int orc_bvh_check(const orc_scene* s, const float* rays, int64_t nr, int kind, double delta,
                  int64_t* out) {
  if (nr < 0 || !scene_valid(s) || !s->bvh || !bvh_matches(s) || !out || (kind != 0 && kind != 1))
    return -1;
  const orc_bvh* B = s->bvh;
  int64_t pairs = 0, bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : pairs, bad)
  for (int64_t r = 0; r < nr; ++r) {
    ray64 w = load_ray(rays + 8 * r);
    if (ray_is_void(&w) || !ray_finite(&w)) continue;
    qstate st;
    memset(&st, 0, sizeof(st));
    st.kind = kind ? Q_CAND : Q_ALL;
    st.delta = delta;
    qstate_reset(&st);
    for (int64_t j = 0; j < n_units(s); ++j) {
      ray64 q;
      int m;
      double xs, xd;
      object_ray(s, &w, j, &q, &m, &xs, &xd);
      if (!ray_finite(&q)) continue;
      const btree* T = &B->mesh[m];
      wprep P;
      wprep_init(&P, &st, &q, xs, xd, T->amax_box);
      for (int64_t k = 0; k < s->n_triangles[m]; ++k) {
        vec3 v0, v1, v2;
        tri(s, m, k, &v0, &v1, &v2);
        double bound;
        if (kind == 0) {
          double t, u, v;
          if (!intersect_paper(&q, v0, v1, v2, &t, &u, &v)) continue;
          bound = t;
        } else {
          cand c;
          double hi;
          if (classify(&q, v0, v1, v2, delta, xs, xd, &c, &hi) == 0) continue;
          bound = c.lo;
        }
        ++pairs;
        int ok = path_ok(&P, &st, T, k, bound);
        if (ok && s->n_inst > 0 && B->top.leaf_of[j] >= 0) {
          for (int64_t nd = B->top.leaf_of[j]; nd >= 0 && ok; nd = B->top.parent[nd]) {
            double key;
            ok = top_test(&B->top, nd, &st, &w, &key) && key <= bound;
          }
        }
        if (!ok) ++bad;
      }
    }
  }
  out[0] = pairs;
  out[1] = bad;
  return 0;
}

/* ------------------------------------------------------------------------- */
/* closest, any and all                                                       */
/* ------------------------------------------------------------------------- */

int orc_closest_ex(const orc_scene* s, const float* rays, int64_t nr, const orc_opts* opts,
                   uint32_t* inst_out, uint32_t* prim_out, double* tuv_out) {
  if (nr < 0 || (nr > 0 && (!rays || !prim_out || !tuv_out)) || !scene_valid(s) ||
      !bvh_matches(s))
    return -1;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t r = 0; r < nr; ++r) {
    ray64 w = load_ray(rays + 8 * r);
    qstate st;
    memset(&st, 0, sizeof(st));
    st.kind = Q_CLOSEST;
    qstate_reset(&st);
    if (!ray_is_void(&w)) search(s, opts, r, &w, &st);
    if (inst_out) inst_out[r] = st.bi;
    prim_out[r] = st.bp;
    tuv_out[3 * r + 0] = st.minT;
    tuv_out[3 * r + 1] = st.bu;
    tuv_out[3 * r + 2] = st.bv;
  }
  return 0;
}

int orc_closest(const orc_scene* s, const float* rays, int64_t nr, uint32_t* inst_out,
                uint32_t* prim_out, double* tuv_out) {
  return orc_closest_ex(s, rays, nr, NULL, inst_out, prim_out, tuv_out);
}

int orc_any_ex(const orc_scene* s, const float* rays, int64_t nr, const orc_opts* opts,
               uint8_t* occluded) {
  if (nr < 0 || (nr > 0 && (!rays || !occluded)) || !scene_valid(s) || !bvh_matches(s)) return -1;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t r = 0; r < nr; ++r) {
    ray64 w = load_ray(rays + 8 * r);
    qstate st;
    memset(&st, 0, sizeof(st));
    st.kind = Q_ANY;
    qstate_reset(&st);
    if (!ray_is_void(&w)) search(s, opts, r, &w, &st);
    occluded[r] = (uint8_t)st.hit;
  }
  return 0;
}

int orc_any(const orc_scene* s, const float* rays, int64_t nr, uint8_t* occluded) {
  return orc_any_ex(s, rays, nr, NULL, occluded);
}

/* All hits of §6.2's enumeration ("all intersections"): every pair the §3.1
 * test accepts within [tmin, tmax], sorted by (t, inst, prim). */
int orc_all(const orc_scene* s, const float* rays, int64_t nr, const orc_opts* opts, int32_t K,
            int64_t* count, uint32_t* inst_out, uint32_t* prim_out, double* tuv_out) {
  if (nr < 0 || K < 1 || !scene_valid(s) || !bvh_matches(s)) return -1;
  if (nr > 0 && (!rays || !count || !prim_out || !tuv_out)) return -1;
  int bad = 0;
#pragma omp parallel
  {
    qstate st;
    memset(&st, 0, sizeof(st));
    st.kind = Q_ALL;
#pragma omp for schedule(dynamic, 8)
    for (int64_t r = 0; r < nr; ++r) {
      qstate_reset(&st);
      ray64 w = load_ray(rays + 8 * r);
      if (!ray_is_void(&w)) search(s, opts, r, &w, &st);
      hit64* buf = st.hits;
      int64_t n = st.n;
      for (int64_t i = 1; i < n; ++i) {
        hit64 x = buf[i];
        int64_t jj = i - 1;
        while (jj >= 0 && hit_less(&x, &buf[jj])) { buf[jj + 1] = buf[jj]; --jj; }
        buf[jj + 1] = x;
      }
      count[r] = n;
      for (int64_t i = 0; i < K; ++i) {
        int64_t o = r * K + i;
        int in = i < n;
        if (inst_out) inst_out[o] = in ? buf[i].inst : ORC_NONE;
        prim_out[o] = in ? buf[i].prim : ORC_NONE;
        tuv_out[3 * o + 0] = in ? buf[i].t : INFINITY;
        tuv_out[3 * o + 1] = in ? buf[i].u : 0.0;
        tuv_out[3 * o + 2] = in ? buf[i].v : 0.0;
      }
    }
    if (st.bad) {
#pragma omp atomic write
      bad = 1;
    }
    free(st.hits);
  }
  return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------- */
/* acceptable sets of every ray                                               */
/* ------------------------------------------------------------------------- */

/* The candidates (sure and maybe pairs) of every ray, with the range
 * [lo, hi] their float32 t may take.  mode 0: the acceptable closest answers
 * (pairs whose lowest possible t does not exceed t*); mode 1: every
 * candidate (all-hit queries). */
static int accept_impl(const orc_scene* s, const float* rays, int64_t nr, const orc_opts* opts,
                       double delta, int32_t K, int mode, uint8_t* miss_ok, int32_t* count,
                       int32_t* n_sure, uint32_t* acc_inst, uint32_t* acc_prim, double* acc_tuv,
                       double* acc_scale, double* acc_lo, double* acc_hi, uint8_t* acc_sure,
                       uint8_t* any_class) {
  if (nr < 0 || K < 1 || !scene_valid(s) || !bvh_matches(s)) return -1;
  if (nr > 0 && (!rays || !miss_ok || !count || !acc_inst || !acc_prim || !acc_tuv ||
                 !acc_scale || !any_class))
    return -1;
  if (mode != 0 && mode != 1) return -1;
  int bad = 0;
#pragma omp parallel
  {
    qstate st;
    memset(&st, 0, sizeof(st));
    st.kind = Q_CAND;
    st.cull_tstar = (mode == 0);
    st.delta = delta;
#pragma omp for schedule(dynamic, 64)
    for (int64_t r = 0; r < nr; ++r) {
      qstate_reset(&st);
      ray64 w = load_ray(rays + 8 * r);
      if (!ray_is_void(&w)) search(s, opts, r, &w, &st);
      cand* buf = st.cands;
      int64_t n = st.n;
      double tstar = st.tstar;
      int any_sure = st.sures > 0;
      /* keep the candidates that can still be the closest, sorted by (t, inst, prim) */
      int64_t kept = 0;
      for (int64_t i = 0; i < n; ++i)
        if (mode == 1 || !(buf[i].lo > tstar)) buf[kept++] = buf[i];
      for (int64_t i = 1; i < kept; ++i) {
        cand x = buf[i];
        int64_t jj = i - 1;
        while (jj >= 0 && cand_less(&x, &buf[jj])) { buf[jj + 1] = buf[jj]; --jj; }
        buf[jj + 1] = x;
      }
      miss_ok[r] = (uint8_t)(!any_sure);
      count[r] = (int32_t)kept;
      if (n_sure) n_sure[r] = st.sures;
      any_class[r] = any_sure ? 1 : (n == 0 ? 0 : 2);
      for (int64_t i = 0; i < K; ++i) {
        int64_t o = r * K + i;
        if (i < kept) {
          acc_inst[o] = buf[i].inst;
          acc_prim[o] = buf[i].prim;
          acc_tuv[3 * o + 0] = buf[i].t;
          acc_tuv[3 * o + 1] = buf[i].u;
          acc_tuv[3 * o + 2] = buf[i].v;
          acc_scale[o] = buf[i].scale;
          if (acc_lo) acc_lo[o] = buf[i].lo;
          if (acc_hi) acc_hi[o] = buf[i].hi;
          if (acc_sure) acc_sure[o] = (uint8_t)buf[i].sure;
        } else {
          acc_inst[o] = ORC_NONE;
          acc_prim[o] = ORC_NONE;
          acc_tuv[3 * o + 0] = INFINITY;
          acc_tuv[3 * o + 1] = 0.0;
          acc_tuv[3 * o + 2] = 0.0;
          acc_scale[o] = 0.0;
          if (acc_lo) acc_lo[o] = INFINITY;
          if (acc_hi) acc_hi[o] = INFINITY;
          if (acc_sure) acc_sure[o] = 0;
        }
      }
    }
    if (st.bad) {
#pragma omp atomic write
      bad = 1;
    }
    free(st.cands);
  }
  return bad ? -1 : 0;
}




int orc_accept(const orc_scene* s, const float* rays, int64_t nr, double delta, int32_t K,
               uint8_t* miss_ok, int32_t* count, uint32_t* acc_inst, uint32_t* acc_prim,
               double* acc_tuv, double* acc_scale, uint8_t* any_class) {
  return accept_impl(s, rays, nr, NULL, delta, K, 0, miss_ok, count, NULL, acc_inst, acc_prim,
                     acc_tuv, acc_scale, NULL, NULL, NULL, any_class);
}

int orc_accept_ex(const orc_scene* s, const float* rays, int64_t nr, const orc_opts* opts,
                  double delta, int32_t K, uint8_t* miss_ok, int32_t* count,
                  uint32_t* acc_inst, uint32_t* acc_prim, double* acc_tuv, double* acc_scale,
                  uint8_t* any_class) {
  return accept_impl(s, rays, nr, opts, delta, K, 0, miss_ok, count, NULL, acc_inst, acc_prim,
                     acc_tuv, acc_scale, NULL, NULL, NULL, any_class);
}

int orc_classify_all(const orc_scene* s, const float* rays, int64_t nr, const orc_opts* opts,
                     double delta, int32_t K, int32_t* count, int32_t* n_sure, uint32_t* acc_inst,
                     uint32_t* acc_prim, double* acc_tuv, double* acc_scale, double* acc_lo,
                     double* acc_hi, uint8_t* acc_sure) {
  if (nr > 0 && (!n_sure || !acc_lo || !acc_hi || !acc_sure)) return -1;
  uint8_t* miss_ok = nr > 0 ? (uint8_t*)malloc((size_t)nr) : NULL;
  uint8_t* any_class = nr > 0 ? (uint8_t*)malloc((size_t)nr) : NULL;
  if (nr > 0 && (!miss_ok || !any_class)) {
    free(miss_ok);
    free(any_class);
    return -1;
  }
  int rc = accept_impl(s, rays, nr, opts, delta, K, 1, miss_ok, count, n_sure, acc_inst, acc_prim,
                       acc_tuv, acc_scale, acc_lo, acc_hi, acc_sure, any_class);
  free(miss_ok);
  free(any_class);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* adjoint and finite differences                                             */
/* ------------------------------------------------------------------------- */
/* Implicit differentiation of M x = o - v0 with M = [-d | v1-v0 | v2-v0] and
 * x = (t,u,v): for g = dL/dx, lambda = M^-T g and
 *   dL/do = lambda, dL/dd = t lambda,
 *   dL/dv0 = -(1-u-v) lambda, dL/dv1 = -u lambda, dL/dv2 = -v lambda. */

int orc_adjoint(const orc_scene* s, const float* rays, const uint32_t* prim, int64_t nr,
                const double* g, double* d_vertices, double* d_orig, double* d_dir) {
  if (nr < 0 || !scene_valid(s) || s->n_inst != 0) return -1;
  if (nr > 0 && (!rays || !prim || !g || !d_vertices || !d_orig || !d_dir)) return -1;
  for (int64_t r = 0; r < nr; ++r) {
    double* go = d_orig + 3 * r;
    double* gd = d_dir + 3 * r;
    go[0] = go[1] = go[2] = 0.0;
    gd[0] = gd[1] = gd[2] = 0.0;
    uint32_t k = prim[r];
    if (k == ORC_NONE) continue;
    if ((int64_t)k >= s->n_triangles[0]) return -1;
    ray64 q = load_ray(rays + 8 * r);
    const uint32_t* ix = s->indices[0] + 3 * (int64_t)k;
    vec3 v0 = vtx(s, 0, ix[0]), v1 = vtx(s, 0, ix[1]), v2 = vtx(s, 0, ix[2]);
    vec3 e1 = sub(v1, v0), e2 = sub(v2, v0), c0 = scl(q.d, -1.0);
    vec3 r0 = cross(e1, e2), r1 = cross(e2, c0), r2 = cross(c0, e1);
    double det = dot(c0, r0);
    if (det == 0.0) continue;
    r0 = scl(r0, 1.0 / det);
    r1 = scl(r1, 1.0 / det);
    r2 = scl(r2, 1.0 / det);
    vec3 rhs = sub(q.o, v0);
    double t = dot(r0, rhs), u = dot(r1, rhs), v = dot(r2, rhs);
    const double* gr = g + 3 * r;
    /* lambda = M^-T g = sum_i g_i row_i(M^-1) */
    vec3 lam = add(add(scl(r0, gr[0]), scl(r1, gr[1])), scl(r2, gr[2]));
    go[0] = lam.x; go[1] = lam.y; go[2] = lam.z;
    gd[0] = t * lam.x; gd[1] = t * lam.y; gd[2] = t * lam.z;
    double w[3] = {1.0 - u - v, u, v};
    for (int c = 0; c < 3; ++c) {
      double* dv = d_vertices + 3 * (int64_t)ix[c];
      dv[0] -= w[c] * lam.x;
      dv[1] -= w[c] * lam.y;
      dv[2] -= w[c] * lam.z;
    }
  }
  return 0;
}

static double coord(vec3* v, int i) { return i == 0 ? v->x : (i == 1 ? v->y : v->z); }
static void set_coord(vec3* v, int i, double x) {
  if (i == 0) v->x = x; else if (i == 1) v->y = x; else v->z = x;
}

int orc_fd(const orc_scene* s, const float* rays, const uint32_t* prim, int64_t nr,
           const double* g, double h, double* out) {
  if (nr < 0 || !scene_valid(s) || s->n_inst != 0 || !(h > 0.0)) return -1;
  if (nr > 0 && (!rays || !prim || !g || !out)) return -1;
  for (int64_t r = 0; r < nr; ++r)
    if (prim[r] != ORC_NONE && (int64_t)prim[r] >= s->n_triangles[0]) return -1;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t r = 0; r < nr; ++r) {
    double* res = out + 15 * r;
    if (prim[r] == ORC_NONE) {
      for (int i = 0; i < 15; ++i) res[i] = 0.0;
      continue;
    }
    ray64 q = load_ray(rays + 8 * r);
    vec3 p[5];
    tri(s, 0, prim[r], &p[0], &p[1], &p[2]);
    p[3] = q.o;
    p[4] = q.d;
    const double* gr = g + 3 * r;
    for (int a = 0; a < 5; ++a) {
      for (int i = 0; i < 3; ++i) {
        double x0 = coord(&p[a], i), lp, lm, t, u, v;
        set_coord(&p[a], i, x0 + h);
        plane_tuv(p[3], p[4], p[0], p[1], p[2], &t, &u, &v);
        lp = gr[0] * t + gr[1] * u + gr[2] * v;
        set_coord(&p[a], i, x0 - h);
        plane_tuv(p[3], p[4], p[0], p[1], p[2], &t, &u, &v);
        lm = gr[0] * t + gr[1] * u + gr[2] * v;
        set_coord(&p[a], i, x0);
        res[3 * a + i] = (lp - lm) / (2.0 * h);
      }
    }
  }
  return 0;
}

int orc_fixed_tuv(const orc_scene* s, const float* rays, const uint32_t* prim, int64_t nr,
                  double* tuv) {
  if (nr < 0 || !scene_valid(s) || s->n_inst != 0) return -1;
  if (nr > 0 && (!rays || !prim || !tuv)) return -1;
  for (int64_t r = 0; r < nr; ++r) {
    if (prim[r] == ORC_NONE) {
      tuv[3 * r] = INFINITY; tuv[3 * r + 1] = 0.0; tuv[3 * r + 2] = 0.0;
      continue;
    }
    if ((int64_t)prim[r] >= s->n_triangles[0]) return -1;
    ray64 q = load_ray(rays + 8 * r);
    vec3 v0, v1, v2;
    tri(s, 0, prim[r], &v0, &v1, &v2);
    plane_tuv(q.o, q.d, v0, v1, v2, &tuv[3 * r], &tuv[3 * r + 1], &tuv[3 * r + 2]);
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* two-level adjoint                                                          */
/* ------------------------------------------------------------------------- */

/* Partial derivatives of the rotation matrix R(q) of frame_from with respect
 * to the components (x, y, z, w) of a unit quaternion, read off the matrix
 * entries one by one: dR[c][i][j] = d R_ij / d q_c. */
static void rotation_partials(double x, double y, double z, double w, double dR[4][3][3]) {
  /* d/dx */
  dR[0][0][0] = 0;      dR[0][0][1] = 2 * y;  dR[0][0][2] = 2 * z;
  dR[0][1][0] = 2 * y;  dR[0][1][1] = -4 * x; dR[0][1][2] = -2 * w;
  dR[0][2][0] = 2 * z;  dR[0][2][1] = 2 * w;  dR[0][2][2] = -4 * x;
  /* d/dy */
  dR[1][0][0] = -4 * y; dR[1][0][1] = 2 * x;  dR[1][0][2] = 2 * w;
  dR[1][1][0] = 2 * x;  dR[1][1][1] = 0;      dR[1][1][2] = 2 * z;
  dR[1][2][0] = -2 * w; dR[1][2][1] = 2 * z;  dR[1][2][2] = -4 * y;
  /* d/dz */
  dR[2][0][0] = -4 * z; dR[2][0][1] = -2 * w; dR[2][0][2] = 2 * x;
  dR[2][1][0] = 2 * w;  dR[2][1][1] = -4 * z; dR[2][1][2] = 2 * y;
  dR[2][2][0] = 2 * x;  dR[2][2][1] = 2 * y;  dR[2][2][2] = 0;
  /* d/dw */
  dR[3][0][0] = 0;      dR[3][0][1] = -2 * z; dR[3][0][2] = 2 * y;
  dR[3][1][0] = 2 * z;  dR[3][1][1] = 0;      dR[3][1][2] = -2 * x;
  dR[3][2][0] = -2 * y; dR[3][2][1] = 2 * x;  dR[3][2][2] = 0;
}

/* The hit of a world ray on instance j, triangle k is the hit of the world
 * ray on the world-space triangle W_i = T + R (S*v_i) (§6.2: the instance is
 * the base mesh under an affine map; barycentrics and t do not change under
 * it).  So the adjoint is the world-space one (lambda = M_w^-T g, grad o =
 * lambda, grad d = t lambda, grad W_i = -w_i lambda), then the chain rule
 * through W_i: grad v_i = (R S)^T grad W_i, grad T = sum_i grad W_i, and with
 * G = sum_i grad W_i v_i^T: grad S_j = sum_i G_ij R_ij, grad R_ij = G_ij S_j,
 * grad qhat_c = sum_ij grad R_ij dR_ij/dqhat_c, and for the normalisation
 * qhat = q/|q|: grad q = (grad qhat - qhat (qhat . grad qhat)) / |q|. */
int orc_adjoint_inst(const orc_scene* s, const float* rays, const uint32_t* inst,
                     const uint32_t* prim, int64_t nr, const double* g,
                     double* const* d_vertices, double* d_srt, double* d_orig, double* d_dir) {
  if (nr < 0 || !scene_valid(s) || s->n_inst < 1) return -1;
  if (nr > 0 && (!rays || !inst || !prim || !g || !d_orig || !d_dir)) return -1;
  for (int64_t r = 0; r < nr; ++r) {
    if (prim[r] == ORC_NONE) continue;
    if ((int64_t)inst[r] >= s->n_inst) return -1;
    if ((int64_t)prim[r] >= s->n_triangles[s->inst_mesh[inst[r]]]) return -1;
  }
  for (int64_t r = 0; r < nr; ++r) {
    double* go = d_orig + 3 * r;
    double* gd = d_dir + 3 * r;
    go[0] = go[1] = go[2] = 0.0;
    gd[0] = gd[1] = gd[2] = 0.0;
    if (prim[r] == ORC_NONE) continue;
    int64_t j = inst[r];
    int m = (int)s->inst_mesh[j];
    const float* f = s->inst_srt + 10 * j;
    frame64 F = load_frame(f);
    ray64 q = load_ray(rays + 8 * r);
    const uint32_t* ix = s->indices[m] + 3 * (int64_t)prim[r];
    vec3 v[3], W[3];
    for (int c = 0; c < 3; ++c) {
      v[c] = vtx(s, m, ix[c]);
      W[c] = to_world(&F, v[c]);
    }
    vec3 e1 = sub(W[1], W[0]), e2 = sub(W[2], W[0]), c0 = scl(q.d, -1.0);
    vec3 r0 = cross(e1, e2), r1 = cross(e2, c0), r2 = cross(c0, e1);
    double det = dot(c0, r0);
    if (det == 0.0) continue;
    r0 = scl(r0, 1.0 / det);
    r1 = scl(r1, 1.0 / det);
    r2 = scl(r2, 1.0 / det);
    vec3 rhs = sub(q.o, W[0]);
    double t = dot(r0, rhs), u = dot(r1, rhs), vv = dot(r2, rhs);
    const double* gr = g + 3 * r;
    vec3 lam = add(add(scl(r0, gr[0]), scl(r1, gr[1])), scl(r2, gr[2]));
    go[0] = lam.x; go[1] = lam.y; go[2] = lam.z;
    gd[0] = t * lam.x; gd[1] = t * lam.y; gd[2] = t * lam.z;
    double w[3] = {1.0 - u - vv, u, vv};
    double S[3] = {F.S.x, F.S.y, F.S.z};
    double G[3][3] = {{0}}, gT[3] = {0, 0, 0};
    for (int c = 0; c < 3; ++c) {
      double gW[3] = {-w[c] * lam.x, -w[c] * lam.y, -w[c] * lam.z};
      double vc[3] = {v[c].x, v[c].y, v[c].z};
      if (d_vertices && d_vertices[m]) {
        double* dv = d_vertices[m] + 3 * (int64_t)ix[c];
        for (int b = 0; b < 3; ++b)  /* (R S)^T gW: column b of R S is S_b R[:, b] */
          dv[b] += S[b] * (F.R[0][b] * gW[0] + F.R[1][b] * gW[1] + F.R[2][b] * gW[2]);
      }
      for (int a = 0; a < 3; ++a) {
        gT[a] += gW[a];
        for (int b = 0; b < 3; ++b) G[a][b] += gW[a] * vc[b];
      }
    }
    if (!d_srt) continue;
    double qn = sqrt((double)f[3] * f[3] + (double)f[4] * f[4] + (double)f[5] * f[5] +
                     (double)f[6] * f[6]);
    double qh[4] = {f[3] / qn, f[4] / qn, f[5] / qn, f[6] / qn};
    double dR[4][3][3];
    rotation_partials(qh[0], qh[1], qh[2], qh[3], dR);
    double gS[3] = {0, 0, 0}, gqh[4] = {0, 0, 0, 0};
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        gS[b] += G[a][b] * F.R[a][b];
        double gRab = G[a][b] * S[b];
        for (int c = 0; c < 4; ++c) gqh[c] += gRab * dR[c][a][b];
      }
    double radial = qh[0] * gqh[0] + qh[1] * gqh[1] + qh[2] * gqh[2] + qh[3] * gqh[3];
    double* out = d_srt + 10 * j;
    for (int b = 0; b < 3; ++b) out[b] += gS[b];
    for (int c = 0; c < 4; ++c) out[3 + c] += (gqh[c] - qh[c] * radial) / qn;
    for (int a = 0; a < 3; ++a) out[7 + a] += gT[a];
  }
  return 0;
}

/* Central differences (step h) of l = g.(t,u,v) of the world ray against the
 * world-space triangle T + R(q/|q|)(S*v_i) by the plane formula, at the fixed
 * (inst[r], prim[r]).  Output per ray: 25 derivatives: v0, v1, v2 (object
 * space, 9), the ten frame parameters of the instance, o (3), d (3). */
int orc_fd_inst(const orc_scene* s, const float* rays, const uint32_t* inst, const uint32_t* prim,
                int64_t nr, const double* g, double h, double* out) {
  if (nr < 0 || !scene_valid(s) || s->n_inst < 1 || !(h > 0.0)) return -1;
  if (nr > 0 && (!rays || !inst || !prim || !g || !out)) return -1;
  for (int64_t r = 0; r < nr; ++r) {
    if (prim[r] == ORC_NONE) continue;
    if ((int64_t)inst[r] >= s->n_inst) return -1;
    if ((int64_t)prim[r] >= s->n_triangles[s->inst_mesh[inst[r]]]) return -1;
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t r = 0; r < nr; ++r) {
    double* res = out + 25 * r;
    if (prim[r] == ORC_NONE) {
      for (int i = 0; i < 25; ++i) res[i] = 0.0;
      continue;
    }
    int64_t j = inst[r];
    int m = (int)s->inst_mesh[j];
    ray64 q = load_ray(rays + 8 * r);
    /* x: v0, v1, v2 (9), frame (10), o (3), d (3) */
    double x[25];
    const uint32_t* ix = s->indices[m] + 3 * (int64_t)prim[r];
    for (int c = 0; c < 3; ++c) {
      vec3 p = vtx(s, m, ix[c]);
      x[3 * c] = p.x; x[3 * c + 1] = p.y; x[3 * c + 2] = p.z;
    }
    for (int i = 0; i < 10; ++i) x[9 + i] = s->inst_srt[10 * j + i];
    x[19] = q.o.x; x[20] = q.o.y; x[21] = q.o.z;
    x[22] = q.d.x; x[23] = q.d.y; x[24] = q.d.z;
    const double* gr = g + 3 * r;
    for (int i = 0; i < 25; ++i) {
      double l[2];
      for (int side = 0; side < 2; ++side) {
        double y[25];
        memcpy(y, x, sizeof y);
        y[i] += side == 0 ? h : -h;
        frame64 F = frame_from(y + 9);
        vec3 W0 = to_world(&F, mk(y[0], y[1], y[2]));
        vec3 W1 = to_world(&F, mk(y[3], y[4], y[5]));
        vec3 W2 = to_world(&F, mk(y[6], y[7], y[8]));
        double t, u, v;
        plane_tuv(mk(y[19], y[20], y[21]), mk(y[22], y[23], y[24]), W0, W1, W2, &t, &u, &v);
        l[side] = gr[0] * t + gr[1] * u + gr[2] * v;
      }
      res[i] = (l[0] - l[1]) / (2.0 * h);
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* ambient occlusion rays (§4)                                                */
/* ------------------------------------------------------------------------- */
/* For primary ray r with closest hit (prim[r], t = tuv[3r]) and sample k:
 * the shading point p = o + t d; the unit geometric normal n of the triangle,
 * turned to face the incoming ray; the tangent t0 = (v1 - v0)/|v1 - v0| and
 * bi-tangent t1 = n x t0 (§4.1: a triangle edge and the cross product of the
 * normal and the tangent); the cosine-weighted direction of §4.1 from the
 * uniforms (xi0, xi1): phi = 2 pi xi0, rr = sqrt(xi1), x = rr cos phi,
 * z = rr sin phi, y = sqrt(max(1 - rr^2, 0)), mapped as t0 x + t1 z + n y;
 * the origin p + offset n (§4.2 self-intersection offset); t in
 * [0, radius] (§4.2 limited ray length).  Misses give void rays
 * (tmin = 1, tmax = 0).  Everything in float64, rounded once to float32. */
/* Two-level scenes: the hit triangle is the one of mesh inst_mesh[j] of the
 * ray's instance j, with its corners mapped to world space by the frame
 * (world = T + R(qhat)(S*x), §7.3); everything after that as above. */
static int ao_rays_impl(const orc_scene* s, const float* rays, const uint32_t* inst, const uint32_t* prim,
                        const double* tuv, int64_t nr, int32_t N, const float* xi, double offset,
                        double radius, float* out) {
  if (nr > 0 && (!rays || !prim || !tuv || !xi || !out)) return -1;
  if (nr > 0 && s->n_inst > 0 && !inst) return -1;
  for (int64_t r = 0; r < nr; ++r) {
    if (prim[r] == ORC_NONE) continue;
    int m = 0;
    if (s->n_inst > 0) {
      if ((int64_t)inst[r] >= s->n_inst) return -1;
      m = (int)s->inst_mesh[inst[r]];
    }
    if ((int64_t)prim[r] >= s->n_triangles[m]) return -1;
  }
  const double two_pi = 6.283185307179586476925286766559;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < nr; ++r) {
    ray64 q = load_ray(rays + 8 * r);
    int hit = prim[r] != ORC_NONE;
    vec3 n = mk(0, 0, 0), t0 = mk(0, 0, 0), t1 = mk(0, 0, 0), org = mk(0, 0, 0);
    if (hit) {
      vec3 v0, v1, v2;
      if (s->n_inst > 0) {
        uint32_t j = inst[r];
        tri(s, (int)s->inst_mesh[j], prim[r], &v0, &v1, &v2);
        frame64 F = load_frame(s->inst_srt + 10 * (int64_t)j);
        v0 = to_world(&F, v0);
        v1 = to_world(&F, v1);
        v2 = to_world(&F, v2);
      } else {
        tri(s, 0, prim[r], &v0, &v1, &v2);
      }
      n = cross(sub(v1, v0), sub(v2, v0));
      n = scl(n, 1.0 / norm(n));
      if (dot(n, q.d) > 0.0) n = scl(n, -1.0);
      t0 = sub(v1, v0);
      t0 = scl(t0, 1.0 / norm(t0));
      t1 = cross(n, t0);
      vec3 p = add(q.o, scl(q.d, tuv[3 * r]));
      org = add(p, scl(n, offset));
    }
    for (int32_t k = 0; k < N; ++k) {
      float* o = out + 8 * (r * N + k);
      if (!hit) {
        o[0] = o[1] = o[2] = 0.0f;
        o[3] = 1.0f;
        o[4] = o[5] = o[6] = 0.0f;
        o[7] = 0.0f;
        continue;
      }
      const float* u = xi + 2 * (r * N + k);
      double phi = two_pi * (double)u[0], rr = sqrt((double)u[1]);
      double x = rr * cos(phi), z = rr * sin(phi);
      double y = 1.0 - rr * rr;
      y = sqrt(y > 0.0 ? y : 0.0);
      vec3 d = add(add(scl(t0, x), scl(t1, z)), scl(n, y));
      o[0] = (float)org.x; o[1] = (float)org.y; o[2] = (float)org.z;
      o[3] = 0.0f;
      o[4] = (float)d.x; o[5] = (float)d.y; o[6] = (float)d.z;
      o[7] = (float)radius;
    }
  }
  return 0;
}

int orc_ao_rays(const orc_scene* s, const float* rays, const uint32_t* prim, const double* tuv,
                int64_t nr, int32_t N, const float* xi, double offset, double radius,
                float* out) {
  if (nr < 0 || N < 1 || !scene_valid(s) || s->n_inst != 0) return -1;
  return ao_rays_impl(s, rays, NULL, prim, tuv, nr, N, xi, offset, radius, out);
}

int orc_ao_rays_inst(const orc_scene* s, const float* rays, const uint32_t* inst, const uint32_t* prim,
                     const double* tuv, int64_t nr, int32_t N, const float* xi, double offset,
                     double radius, float* out) {
  if (nr < 0 || N < 1 || !scene_valid(s) || s->n_inst < 1) return -1;
  return ao_rays_impl(s, rays, inst, prim, tuv, nr, N, xi, offset, radius, out);
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
