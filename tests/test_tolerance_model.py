"""The tolerance model of the acceptable sets, checked against a float32
implementation of the ray/triangle test (CPU): every answer that a float32
watertight edge-function test with the closest-hit tie rule gives must lie
in the oracle's acceptable set, for closest and any-hit.  This is what the
relative input slack delta of the sets has to cover; the float32 test here
is written in numpy for this check (vertices sorted lexicographically so each
shared edge is evaluated identically from both sides, edge functions against
the ray, t from the plane equation), evaluated once with separate products
and sums and once with every product-sum fused into one rounding (the two
rounding orders a compiler may pick)."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2603_00292_amd import workloads as wl

NONE = 0xFFFFFFFF
f32 = np.float32


def _sorted_vertices(V, I):
    P = V[I.astype(np.int64)]                       # (T, 3, 3)
    key = np.lexsort((P[:, :, 2], P[:, :, 1], P[:, :, 0]), axis=1)
    return np.take_along_axis(P, key[:, :, None], axis=1).astype(np.float32)


def _fma(a, b, c):
    """a*b + c with one rounding (float64 product of float32 values is exact)."""
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def _cross_dot(d, e, w, fused):
    """d . (e x w) in float32."""
    cx = e[..., 1] * w[..., 2] - e[..., 2] * w[..., 1]
    cy = e[..., 2] * w[..., 0] - e[..., 0] * w[..., 2]
    cz = e[..., 0] * w[..., 1] - e[..., 1] * w[..., 0]
    if fused:
        cx = _fma(e[..., 1], w[..., 2], -(e[..., 2] * w[..., 1]))
        cy = _fma(e[..., 2], w[..., 0], -(e[..., 0] * w[..., 2]))
        cz = _fma(e[..., 0], w[..., 1], -(e[..., 1] * w[..., 0]))
        return _fma(d[..., 2], cz, _fma(d[..., 1], cy, d[..., 0] * cx))
    return d[..., 0] * cx + d[..., 1] * cy + d[..., 2] * cz


def float32_queries(P, rays, fused, chunk=64, mistake=None):
    """Closest prim and any-hit of rays (n,8) against sorted records P.
    ``mistake`` plants an error (for the check's own test): "drop_edge"
    ignores the edge function of edge 1-2, "t_sign" negates t."""
    n = rays.shape[0]
    prim = np.full(n, NONE, np.uint32)
    occ = np.zeros(n, np.uint8)
    A, B, C = P[None, :, 0], P[None, :, 1], P[None, :, 2]
    e01, e12, e02 = B - A, C - B, C - A
    nrm = np.stack([e01[..., 1] * e02[..., 2] - e01[..., 2] * e02[..., 1],
                    e01[..., 2] * e02[..., 0] - e01[..., 0] * e02[..., 2],
                    e01[..., 0] * e02[..., 1] - e01[..., 1] * e02[..., 0]], -1)
    ids = np.arange(P.shape[0], dtype=np.uint32)
    with np.errstate(all="ignore"):
        for lo in range(0, n, chunk):
            r = rays[lo:lo + chunk].astype(np.float32)
            o = r[:, None, 0:3]
            d = r[:, None, 4:7]
            w0, w1 = A - o, B - o
            g01 = _cross_dot(d, e01, w0, fused)
            g12 = _cross_dot(d, e12, w1, fused)
            g02 = _cross_dot(d, e02, w0, fused)
            F0, F1, F2 = -g12, g02, -g01
            if mistake == "drop_edge":
                F0 = np.where(F1 >= 0, np.abs(F0), -np.abs(F0))
            pos = (F0 >= 0) & (F1 >= 0) & (F2 >= 0)
            neg = (F0 <= 0) & (F1 <= 0) & (F2 <= 0)
            det = F0 + F1 + F2
            if fused:
                T = _fma(nrm[..., 2], w0[..., 2], _fma(nrm[..., 1], w0[..., 1], nrm[..., 0] * w0[..., 0]))
                nd = _fma(nrm[..., 2], d[..., 2], _fma(nrm[..., 1], d[..., 1], nrm[..., 0] * d[..., 0]))
            else:
                T = (nrm * w0).sum(-1, dtype=np.float32)
                nd = nrm[..., 0] * d[..., 0] + nrm[..., 1] * d[..., 1] + nrm[..., 2] * d[..., 2]
            t = (T / nd).astype(np.float32)
            if mistake == "t_sign":
                t = -t
            hit = (pos | neg) & (det != 0) & (nd != 0) & (t >= r[:, None, 3]) & (t <= r[:, None, 7])
            occ[lo:lo + chunk] = hit.any(1)
            tt = np.where(hit, t, np.float32(np.inf))
            best = tt.min(1)
            cand = hit & (tt == best[:, None])
            first = np.where(cand.any(1), np.argmax(cand, 1), -1)
            prim[lo:lo + chunk] = np.where(first >= 0, ids[np.maximum(first, 0)], NONE)
    return prim, occ


def _check(orc, scene, rays, label):
    V, I = scene.meshes[0].vertices, scene.meshes[0].indices
    P = _sorted_vertices(V, I)
    S = orc.OracleScene.from_scene(scene, accel=True)
    A = orc.accept(S, rays, K=32)
    assert not A.overflow.any()
    for fused in (False, True):
        prim, occ = float32_queries(P, rays, fused)
        hit = prim != NONE
        member = (A.prim == prim[:, None]) & (np.arange(A.K)[None, :] < A.count[:, None])
        ok = np.where(hit, member.any(1), A.miss_ok)
        assert ok.all(), f"{label} fused={fused}: {int((~ok).sum())} float32 answers outside the sets"
        any_ok = ~(((A.any_class == 1) & (occ == 0)) | ((A.any_class == 0) & (occ == 1)))
        assert any_ok.all(), f"{label} fused={fused}: any-hit"
    return float(A.pinned.mean())


def test_float32_test_lands_in_sets_random_soup(orc):
    W = wl.random_triangles(n_tri=4096, n_rays=4096, k=0)
    pinned = _check(orc, W.scene, W.rays, "random soup")
    assert pinned > 0.999


def test_float32_test_lands_in_sets_icosphere(orc):
    """Incoherent rays on a noisy icosphere (level 5, 20,480 triangles),
    inside and outside it, and grazing rays aimed at its silhouette."""
    rng = wl.rng_for(950)
    V, I = wl.noisy_icosphere(rng, 5, 0.02)
    scene = wl.Scene([wl.Mesh(V, I)])
    rays = wl.box_rays(rng, 1536, -1.0, 1.0)
    # camera rays from (0, 0, 3) just inside and outside the silhouette
    ang = rng.uniform(0, 2 * np.pi, 512)
    rad = rng.uniform(0.98, 1.03, 512)
    tgt = np.stack([rad * np.cos(ang), rad * np.sin(ang), np.zeros(512)], 1)
    o = np.broadcast_to(np.array([0.0, 0.0, 3.0]), tgt.shape)
    d = tgt - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays = np.concatenate([rays, wl.pack_rays(o, d)])
    pinned = _check(orc, scene, rays, "icosphere")
    assert pinned > 0.95


@pytest.mark.parametrize("mistake", ["drop_edge", "t_sign"])
def test_planted_float32_mistakes_leave_the_sets(orc, mistake):
    """The check has teeth: the same float32 test with a planted mistake (an
    edge function ignored, or t negated) answers outside the sets."""
    W = wl.random_triangles(n_tri=4096, n_rays=2048, k=952)
    V, I = W.scene.meshes[0].vertices, W.scene.meshes[0].indices
    P = _sorted_vertices(V, I)
    S = orc.OracleScene.from_scene(W.scene, accel=True)
    A = orc.accept(S, W.rays, K=32)
    prim, _ = float32_queries(P, W.rays, False, mistake=mistake)
    member = (A.prim == prim[:, None]) & (np.arange(A.K)[None, :] < A.count[:, None])
    ok = np.where(prim != NONE, member.any(1), A.miss_ok)
    assert (~ok).sum() > 20
