"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test fixes part of the oracle with something other than itself:
closed-form cases derived by hand from the paper's equations (tests/golden),
exact rational arithmetic, the textbook Moeller-Trumbore solution, scaling
and translation invariants, brute-force relations between queries, and the
consistency of the acceptable-set model with the oracle's own answers.
"""
from __future__ import annotations

import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_2603_00292_amd import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))
NONE = 0xFFFFFFFF


def _num(x):
    return float(x) if not isinstance(x, str) else float(x)


def load_cases():
    with open(os.path.join(HERE, "golden", "closed_forms.json")) as f:
        return json.load(f)["cases"]


def case_arrays(c):
    V = np.array([[_num(x) for x in v] for v in c["vertices"]], dtype=np.float32)
    I = np.array(c["indices"], dtype=np.uint32)
    R = np.array([[_num(x) for x in c["ray"]]], dtype=np.float32)
    return V, I, R


CASES = load_cases()


def dense(n_tri, n_rays, k):
    """Random soup with larger triangles and origins inside the unit cube, so
    that most rays hit something."""
    rng = wl.rng_for(k)
    V, I = wl.random_triangle_soup(rng, n_tri, 0.1)
    rays = wl.box_rays(rng, n_rays, 0.0, 1.0)
    return wl.Workload("dense", wl.Scene([wl.Mesh(V, I)]), rays)


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_closed_form_cases(orc, case):
    V, I, R = case_arrays(case)
    S = orc.OracleScene([(V, I)])
    _, prim, tuv = orc.closest(S, R)
    occ = orc.any_hit(S, R)
    e = case["expect"]
    if e["prim"] is None:
        assert prim[0] == NONE
        assert tuv[0, 0] == math.inf and tuv[0, 1] == 0.0 and tuv[0, 2] == 0.0
    else:
        assert prim[0] == e["prim"]
        assert tuv[0, 0] == e["t"] and tuv[0, 1] == e["u"] and tuv[0, 2] == e["v"]
    assert bool(occ[0]) == e["any"]


def test_empty_mesh_all_miss(orc):
    V = np.zeros((0, 3), np.float32)
    I = np.zeros((0, 3), np.uint32)
    rays = wl.box_rays(wl.rng_for(100), 64, -1, 1)
    S = orc.OracleScene([(V, I)])
    _, prim, tuv = orc.closest(S, rays)
    assert (prim == NONE).all() and np.isinf(tuv[:, 0]).all()
    assert not orc.any_hit(S, rays).any()


def test_invalid_index_rejected(orc):
    V = np.zeros((3, 3), np.float32)
    I = np.array([[0, 1, 3]], np.uint32)
    with pytest.raises(ValueError):
        orc.closest(orc.OracleScene([(V, I)]), np.zeros((1, 8), np.float32))


# ---------------------------------------------------------------------------
# exact rational arithmetic: the paper's test without rounding
# ---------------------------------------------------------------------------

def _exact_hit(o, d, tmin, tmax, v0, v1, v2):
    """Plane-then-edge test in exact rationals. Returns (t, u, v) or None."""
    F = Fraction

    def sub(a, b):
        return [a[i] - b[i] for i in range(3)]

    def cr(a, b):
        return [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]

    def dt(a, b):
        return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]

    o, d, v0, v1, v2 = ([F(float(x)) for x in a] for a in (o, d, v0, v1, v2))
    e0, e1, e2 = sub(v1, v0), sub(v2, v1), sub(v0, v2)
    n = cr(e0, e1)
    nn = dt(n, n)
    if nn == 0:
        return None
    den = dt(n, d)
    if den == 0:
        return None
    t = dt(sub(v0, o), n) / den
    if not (F(float(tmin)) <= t if math.isfinite(tmin) else tmin < 0):
        return None
    if math.isfinite(tmax) and t > F(float(tmax)):
        return None
    p = [o[i] + t * d[i] for i in range(3)]
    a = dt(n, cr(e0, sub(p, v0)))
    b = dt(n, cr(e1, sub(p, v1)))
    c = dt(n, cr(e2, sub(p, v2)))
    if a < 0 or b < 0 or c < 0:
        return None
    return t, c / nn, a / nn


def test_exact_rational_agrees(orc):
    """Small random scenes: the FP64 oracle's hit/miss decisions and values
    equal the exact-arithmetic result (closest over ascending ids)."""
    rng = wl.rng_for(101)
    for trial in range(6):
        V, I = wl.random_triangle_soup(rng, 12, 0.2)
        rays = wl.box_rays(rng, 48, 0.2, 0.8)
        S = orc.OracleScene([(V, I)])
        _, prim, tuv = orc.closest(S, rays)
        for r in range(rays.shape[0]):
            o, d = rays[r, 0:3], rays[r, 4:7]
            best = None
            for k in range(I.shape[0]):
                h = _exact_hit(o, d, float(rays[r, 3]), float(rays[r, 7]), *V[I[k]])
                if h is not None and (best is None or h[0] < best[1][0]):
                    best = (k, h)
            if best is None:
                assert prim[r] == NONE
            else:
                assert prim[r] == best[0]
                for j in range(3):
                    assert abs(tuv[r, j] - float(best[1][j])) <= 1e-12 * max(1.0, abs(float(best[1][j])))


# ---------------------------------------------------------------------------
# textbook reduction: Moeller-Trumbore in FP64
# ---------------------------------------------------------------------------

def _mt_all(o, d, V, I):
    v0 = V[I[:, 0]].astype(np.float64)
    v1 = V[I[:, 1]].astype(np.float64)
    v2 = V[I[:, 2]].astype(np.float64)
    e1, e2 = v1 - v0, v2 - v0
    p = np.cross(d, e2)
    det = np.einsum("ij,ij->i", e1, p)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / det
        s = o - v0
        u = np.einsum("ij,ij->i", s, p) * inv
        q = np.cross(s, e1)
        v = (q @ d) * inv
        t = np.einsum("ij,ij->i", e2, q) * inv
    return t, u, v


def test_moller_trumbore_agrees(orc):
    """Where a ray is not within 1e-9 of an edge or range end, the closest hit
    equals the one found with the Moeller-Trumbore solution (same (t,u,v) in
    exact arithmetic) to 1e-12."""
    W = wl.random_triangles(n_tri=256, n_rays=2048, k=102)
    V, I = W.scene.meshes[0].vertices, W.scene.meshes[0].indices
    S = orc.OracleScene([(V, I)])
    _, prim, tuv = orc.closest(S, W.rays)
    checked = 0
    for r in range(W.rays.shape[0]):
        o = W.rays[r, 0:3].astype(np.float64)
        d = W.rays[r, 4:7].astype(np.float64)
        t, u, v = _mt_all(o, d, V, I)
        margin = np.minimum(np.minimum(u, v), 1 - u - v)
        ok = np.isfinite(t) & (t >= 0)
        inside = ok & (margin >= 0)
        if (ok & (np.abs(margin) < 1e-9)).any() or (inside & (np.abs(t) < 1e-9)).any():
            continue
        checked += 1
        if not inside.any():
            assert prim[r] == NONE
            continue
        k = int(np.flatnonzero(inside)[np.argmin(t[inside])])
        assert prim[r] == k
        assert abs(tuv[r, 0] - t[k]) <= 1e-12 * max(1, abs(t[k]))
        assert abs(tuv[r, 1] - u[k]) <= 1e-12 and abs(tuv[r, 2] - v[k]) <= 1e-12
    assert checked > 1900


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------

def test_direction_scaling_halves_t(orc):
    W = dense(512, 4096, 103)
    S = orc.OracleScene.from_scene(W.scene)
    _, p1, tuv1 = orc.closest(S, W.rays)
    r2 = W.rays.copy()
    r2[:, 4:7] *= 2.0
    _, p2, tuv2 = orc.closest(S, r2)
    assert (p1 == p2).all()
    hit = p1 != NONE
    assert hit.sum() > 50
    assert np.array_equal(tuv2[hit, 0], tuv1[hit, 0] / 2)
    assert np.allclose(tuv2[hit, 1:], tuv1[hit, 1:], rtol=0, atol=1e-13)


def test_power_of_two_scaling_and_translation(orc):
    W = dense(512, 4096, 104)
    # coordinates on a 2^-12 grid, so that the float32 translation is exact
    V = (np.round(W.scene.meshes[0].vertices * 4096) / 4096).astype(np.float32)
    I = W.scene.meshes[0].indices
    W.rays[:, 0:3] = np.round(W.rays[:, 0:3] * 4096) / 4096
    S = orc.OracleScene([(V, I)])
    _, p1, tuv1 = orc.closest(S, W.rays)
    for scale, shift in ((8.0, 0.0), (0.25, 0.0), (1.0, 4.0), (1.0, -2.5)):
        V2 = (V * np.float32(scale) + np.float32(shift)).astype(np.float32)
        r2 = W.rays.copy()
        r2[:, 0:3] = r2[:, 0:3] * np.float32(scale) + np.float32(shift)
        _, p2, tuv2 = orc.closest(orc.OracleScene([(V2, I)]), r2)
        assert (p1 == p2).all()
        hit = p1 != NONE
        assert np.allclose(tuv2[hit, 0], tuv1[hit, 0] * scale, rtol=1e-12, atol=0)
        assert np.allclose(tuv2[hit, 1:], tuv1[hit, 1:], rtol=0, atol=1e-10)


def test_triangle_order_permutation(orc):
    """Reordering triangles changes only the ids (no ties in random soups)."""
    W = dense(512, 4096, 105)
    V, I = W.scene.meshes[0].vertices, W.scene.meshes[0].indices
    perm = wl.rng_for(106).permutation(I.shape[0])
    _, p1, tuv1 = orc.closest(orc.OracleScene([(V, I)]), W.rays)
    _, p2, tuv2 = orc.closest(orc.OracleScene([(V, I[perm])]), W.rays)
    hit = p1 != NONE
    assert ((p2 == NONE) == ~hit).all()
    assert (perm[p2[hit]] == p1[hit]).all()
    assert np.array_equal(tuv1, tuv2)


def test_vertex_rotation_permutes_barycentrics(orc):
    """Cycling a triangle's vertices (v0,v1,v2)->(v1,v2,v0) maps (u,v) to
    (v, 1-u-v) and keeps t: the hit point is the same convex combination."""
    W = dense(256, 4096, 107)
    V, I = W.scene.meshes[0].vertices, W.scene.meshes[0].indices
    _, p1, tuv1 = orc.closest(orc.OracleScene([(V, I)]), W.rays)
    _, p2, tuv2 = orc.closest(orc.OracleScene([(V, I[:, [1, 2, 0]])]), W.rays)
    hit = p1 != NONE
    assert hit.sum() > 20
    assert (p1 == p2).all()
    assert np.allclose(tuv2[hit, 0], tuv1[hit, 0], rtol=1e-12)
    u, v = tuv1[hit, 1], tuv1[hit, 2]
    assert np.allclose(tuv2[hit, 1], v, atol=1e-12)
    assert np.allclose(tuv2[hit, 2], 1 - u - v, atol=1e-12)


def test_hit_point_reconstruction(orc):
    """o + t d equals (1-u-v) v0 + u v1 + v v2 (the (u,v) reading)."""
    W = dense(512, 8192, 108)
    V, I = W.scene.meshes[0].vertices.astype(np.float64), W.scene.meshes[0].indices
    _, p, tuv = orc.closest(orc.OracleScene.from_scene(W.scene), W.rays)
    hit = np.flatnonzero(p != NONE)
    o, d = W.rays[hit, 0:3].astype(np.float64), W.rays[hit, 4:7].astype(np.float64)
    t, u, v = tuv[hit, 0:1], tuv[hit, 1:2], tuv[hit, 2:3]
    tri = V[I[p[hit]]]
    q = (1 - u - v) * tri[:, 0] + u * tri[:, 1] + v * tri[:, 2]
    assert np.allclose(o + t * d, q, atol=1e-12)
    assert (u >= 0).all() and (v >= 0).all() and (u + v <= 1 + 1e-15).all()


def test_any_equals_closest_hit_exists(orc):
    W = dense(1024, 8192, 109)
    S = orc.OracleScene.from_scene(W.scene)
    _, p, _ = orc.closest(S, W.rays)
    occ = orc.any_hit(S, W.rays)
    assert np.array_equal(occ.astype(bool), p != NONE)
    # shortening every ray to just below its closest t removes the hit
    r2 = W.rays.copy()
    _, _, tuv = orc.closest(S, W.rays)
    hit = p != NONE
    r2[hit, 7] = np.nextafter((tuv[hit, 0] * (1 - 1e-6)).astype(np.float32), np.float32(0))
    assert not orc.any_hit(S, r2[hit]).any()


def test_closed_mesh_containment(orc):
    """Every ray starting strictly inside a closed mesh hits it."""
    v, f = wl.icosphere(2)
    V = v.astype(np.float32)
    rng = wl.rng_for(110)
    o = rng.uniform(-0.5, 0.5, size=(2048, 3))
    rays = wl.pack_rays(o, wl.uniform_sphere_dirs(rng, 2048))
    S = orc.OracleScene([(V, f)])
    _, p, tuv = orc.closest(S, rays)
    assert (p != NONE).all()
    assert orc.any_hit(S, rays).all()


# ---------------------------------------------------------------------------
# instances
# ---------------------------------------------------------------------------

def _srt(S, q, T):
    return np.array([list(S) + list(q) + list(T)], dtype=np.float32)


def test_identity_instance_equals_single_level(orc):
    W = dense(512, 4096, 111)
    m = W.scene.meshes[0]
    _, p1, tuv1 = orc.closest(orc.OracleScene([(m.vertices, m.indices)]), W.rays)
    S2 = orc.OracleScene([(m.vertices, m.indices)], np.zeros(1, np.uint32),
                         _srt((1, 1, 1), (0, 0, 0, 1), (0, 0, 0)))
    i2, p2, tuv2 = orc.closest(S2, W.rays)
    assert np.array_equal(p1, p2) and np.array_equal(tuv1, tuv2)
    assert ((i2 == 0) == (p1 != NONE)).all()


def test_instances_equal_flattened_mesh(orc):
    """Instances with per-axis power-of-two scales, half-turn rotations and
    dyadic translations of a mesh on a 2^-10 grid are exact in float32, so the
    two-level answer equals the answer on the flattened mesh (ids mapped)."""
    W = wl.random_triangles(n_tri=256, n_rays=4096, k=112, half=0.1)
    m = W.scene.meshes[0]
    V = (np.round(m.vertices * 1024) / 1024).astype(np.float32)
    frames = [((2, 2, 2), (0, 0, 0, 1), (0.5, -1, 0.25)),
              ((1, 2, 4), (0, 0, 1, 0), (-2, 0, 1)),
              ((0.5, 0.5, 0.5), (1, 0, 0, 0), (0, 0, -0.5)),
              ((1, 1, 0.5), (0, 1, 0, 0), (1.5, 0.75, -0.25))]
    srt = np.concatenate([_srt(*f) for f in frames], 0)
    S_inst = orc.OracleScene([(V, m.indices)], np.zeros(len(frames), np.uint32), srt)
    flat_v, flat_i = [], []
    R = wl.quat_matrix(srt[:, 3:7].astype(np.float64))
    for j in range(len(frames)):
        x = V.astype(np.float64) * srt[j, 0:3].astype(np.float64)
        flat_v.append(x @ R[j].T + srt[j, 7:10].astype(np.float64))
        flat_i.append(m.indices + j * V.shape[0])
    FV = np.concatenate(flat_v).astype(np.float32)
    FI = np.concatenate(flat_i).astype(np.uint32)
    assert np.array_equal(FV.astype(np.float64), np.concatenate(flat_v))
    _, pf, tuvf = orc.closest(orc.OracleScene([(FV, FI)]), W.rays)
    ii, pi, tuvi = orc.closest(S_inst, W.rays)
    hit = pf != NONE
    assert hit.sum() > 100
    assert ((pi != NONE) == hit).all()
    n = m.indices.shape[0]
    assert (ii[hit].astype(np.int64) * n + pi[hit] == pf[hit]).all()
    assert np.allclose(tuvi[hit], tuvf[hit], rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------------------
# acceptable sets
# ---------------------------------------------------------------------------

def test_oracle_answer_in_acceptable_set(orc):
    W = wl.random_triangles(n_tri=4096, n_rays=16384, k=113)
    S = orc.OracleScene.from_scene(W.scene)
    _, p, tuv = orc.closest(S, W.rays)
    A = orc.accept(S, W.rays)
    hit = p != NONE
    in_set = np.where(hit, (A.prim == p[:, None]).any(1), A.miss_ok)
    assert in_set.all()
    assert not A.overflow.any()
    # pinned rays: the only member is the oracle's answer
    pin = A.pinned
    assert pin.mean() > 0.99
    assert np.array_equal(np.where(A.miss_ok[pin], NONE, A.prim[pin, 0]), p[pin])
    # any-hit classes agree with the any query wherever they are decided
    occ = orc.any_hit(S, W.rays)
    assert (occ[A.any_class == 1] == 1).all() and (occ[A.any_class == 0] == 0).all()


def test_acceptable_set_rejects_wrong_answers(orc):
    """A farther hit, a miss on a sure hit, and a hit on a sure miss are out."""
    W = wl.random_triangles(n_tri=4096, n_rays=16384, k=114)
    S = orc.OracleScene.from_scene(W.scene)
    A = orc.accept(S, W.rays)
    _, p, tuv = orc.closest(S, W.rays)
    sure_hit = ~A.miss_ok
    assert sure_hit.sum() > 300
    # a ray whose closest is a sure hit does not accept "miss"
    assert not A.miss_ok[sure_hit].any()
    # second-closest hits, when well separated, are not acceptable
    V, I = W.scene.meshes[0].vertices, W.scene.meshes[0].indices
    found = 0
    for r in np.flatnonzero(sure_hit & A.pinned)[:400]:
        o = W.rays[r, 0:3].astype(np.float64)
        d = W.rays[r, 4:7].astype(np.float64)
        t, u, v = _mt_all(o, d, V, I)
        inside = np.isfinite(t) & (t >= 0) & (np.minimum(np.minimum(u, v), 1 - u - v) > 1e-3)
        ks = np.flatnonzero(inside)
        if ks.size >= 2:
            order = ks[np.argsort(t[ks])]
            if t[order[1]] - t[order[0]] > 1e-3:
                assert order[1] not in A.prim[r, :A.count[r]]
                found += 1
    assert found > 5
    # a planted perturbation far beyond float32 rounding (delta = 2^-6) makes
    # sets larger; the default stays tight
    A_loose = orc.accept(S, W.rays, delta=2.0 ** -6)
    assert A_loose.pinned.mean() < A.pinned.mean()


def test_fp32_textbook_test_lands_in_set(orc):
    """A float32 Moeller-Trumbore closest hit (a different float32
    implementation of the same query) is inside the acceptable set."""
    W = wl.random_triangles(n_tri=1024, n_rays=4096, k=115)
    V, I = W.scene.meshes[0].vertices, W.scene.meshes[0].indices
    S = orc.OracleScene.from_scene(W.scene)
    A = orc.accept(S, W.rays)
    f = np.float32
    v0, v1, v2 = V[I[:, 0]], V[I[:, 1]], V[I[:, 2]]
    e1, e2 = v1 - v0, v2 - v0
    for r in range(W.rays.shape[0]):
        o, d = W.rays[r, 0:3], W.rays[r, 4:7]
        with np.errstate(divide="ignore", invalid="ignore"):
            p = np.cross(d, e2).astype(f)
            det = (e1 * p).sum(1, dtype=f)
            s = (o - v0).astype(f)
            u = (s * p).sum(1, dtype=f) / det
            q = np.cross(s, e1).astype(f)
            v = (q * d).sum(1, dtype=f) / det
            t = (e2 * q).sum(1, dtype=f) / det
        ok = (det != 0) & (u >= 0) & (v >= 0) & (u + v <= 1) & (t >= 0)
        if ok.any():
            ks = np.flatnonzero(ok)
            k = ks[np.argmin(t[ks])]
            assert k in A.prim[r, :A.count[r]]
        else:
            assert A.miss_ok[r]


# ---------------------------------------------------------------------------
# adjoint and finite differences
# ---------------------------------------------------------------------------

def test_adjoint_matches_finite_differences(orc):
    W = wl.displaced_grid(nx=32, nz=16, n_rays=2048, k=116)
    S = orc.OracleScene.from_scene(W.scene)
    _, p, tuv = orc.closest(S, W.rays)
    hit = np.flatnonzero(p != NONE)
    assert hit.size > 1500
    g = W.extra["abc"].astype(np.float64)
    rays, ph, gh = W.rays[hit], p[hit], g[hit]
    fd = orc.fd(S, rays, ph, gh, h=1e-6)
    dV, do, dd = orc.adjoint(S, rays, ph, gh)
    I = W.scene.meshes[0].indices
    # per-ray vertex gradients: recompute them one ray at a time
    for j in range(0, rays.shape[0], 97):
        dVj, _, _ = orc.adjoint(S, rays[j:j + 1], ph[j:j + 1], gh[j:j + 1])
        tri = I[ph[j]]
        an = np.concatenate([dVj[tri[0]], dVj[tri[1]], dVj[tri[2]], do[j], dd[j]])
        # a vertex shared by two corners of a triangle cannot happen here
        assert len(set(tri.tolist())) == 3
        scale = np.abs(an).max()
        assert np.abs(an - fd[j]).max() <= 1e-6 * max(scale, 1.0)


def test_adjoint_invariants(orc):
    """Translation invariance: sum of vertex gradients + origin gradient = 0.
    Homogeneity: t(s d) = t/s, u and v unchanged => d.dL/dd = -t g_t."""
    W = dense(1024, 8192, 117)
    S = orc.OracleScene.from_scene(W.scene)
    _, p, tuv = orc.closest(S, W.rays)
    hit = np.flatnonzero(p != NONE)
    g = wl.rng_for(118).standard_normal((hit.size, 3))
    for j in hit[:64]:
        jj = np.flatnonzero(hit == j)[0]
        dV, do, dd = orc.adjoint(S, W.rays[j:j + 1], p[j:j + 1], g[jj:jj + 1])
        assert np.allclose(dV.sum(0) + do[0], 0, atol=1e-9 * max(1, np.abs(do).max()))
        d = W.rays[j, 4:7].astype(np.float64)
        assert abs(d @ dd[0] + tuv[j, 0] * g[jj, 0]) <= 1e-9 * max(1, np.abs(dd).max())


def test_fixed_tuv_equals_closest_values(orc):
    W = dense(1024, 8192, 119)
    S = orc.OracleScene.from_scene(W.scene)
    _, p, tuv = orc.closest(S, W.rays)
    ft = orc.fixed_tuv(S, W.rays, p)
    hit = p != NONE
    assert np.array_equal(ft[hit], tuv[hit])
