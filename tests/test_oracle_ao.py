"""Pins of the oracle's ambient-occlusion rays (§4).

Directions for chosen uniforms are derived by hand (the normal, the edge
tangent and the bi-tangent n x t0), every sample lies in the hemisphere of
the normal facing the incoming ray with unit length, a lone plane never
occludes itself, and between two parallel plates a distance h apart with
AO length R the occluded fraction of cosine-weighted samples is
1 - (h/R)^2 (P(cos theta >= c) = 1 - c^2 for the cosine density).
"""
from __future__ import annotations

import math

import numpy as np

from paper_2603_00292_amd import workloads as wl

NONE = 0xFFFFFFFF


def quad(y, half=10.0):
    V = np.array([[-half, y, -half], [half, y, -half], [half, y, half], [-half, y, half]], np.float32)
    I = np.array([[0, 1, 2], [0, 2, 3]], np.uint32)
    return V, I


def test_ao_directions_by_hand(orc):
    """Triangle v0=(0,0,0), v1=(1,0,0), v2=(0,0,1): (v1-v0)x(v2-v0) = (0,-1,0),
    turned to face a ray coming down: n = (0,1,0); t0 = (1,0,0);
    t1 = n x t0 = (0,0,-1).  xi=(0,0) -> n; xi=(0,1) -> t0; xi=(0.25,1) -> t1;
    xi=(0.5,1) -> -t0; xi=(0,0.25) -> (0.5, sqrt(0.75), 0)."""
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 0, 1]], np.float32)
    I = np.array([[0, 1, 2]], np.uint32)
    S = orc.OracleScene([(V, I)])
    rays = np.array([[0.25, 2, 0.25, 0, 0, -1, 0, np.inf]], np.float32)
    _, p, tuv = orc.closest(S, rays)
    assert p[0] == 0 and tuv[0, 0] == 2.0
    xi = np.array([[[0, 0], [0, 1], [0.25, 1], [0.5, 1], [0, 0.25]]], np.float32)
    ao = orc.ao_rays(S, rays, p, tuv, xi, offset=1e-4, radius=0.5)
    want = np.array([[0, 1, 0], [1, 0, 0], [0, 0, -1], [-1, 0, 0], [0.5, math.sqrt(0.75), 0]])
    assert np.allclose(ao[:, 4:7], want, atol=1e-7)
    assert np.allclose(ao[:, 0:3], [0.25, 1e-4, 0.25], atol=1e-9)
    assert (ao[:, 3] == 0).all() and (ao[:, 7] == np.float32(0.5)).all()
    # a ray from below sees the normal (0,-1,0): the hemisphere flips
    rays_up = np.array([[0.25, -2, 0.25, 0, 0, 1, 0, np.inf]], np.float32)
    _, p2, tuv2 = orc.closest(S, rays_up)
    ao2 = orc.ao_rays(S, rays_up, p2, tuv2, xi[:, :1], offset=1e-4, radius=0.5)
    assert np.allclose(ao2[0, 4:7], [0, -1, 0]) and np.allclose(ao2[0, 0:3], [0.25, -1e-4, 0.25])


def test_ao_hemisphere_and_misses(orc):
    W = wl.ao_terrain(64, 64, 8, k=160)
    S = orc.OracleScene.from_scene(W.scene)
    _, p, tuv = orc.closest(S, W.rays)
    ao = orc.ao_rays(S, W.rays, p, tuv, W.extra["xi"], W.extra["offset"], W.extra["radius"])
    ao = ao.reshape(-1, 8, 8)
    hit = p != NONE
    assert 0.3 < hit.mean() < 0.95
    d = ao[hit][:, :, 4:7].astype(np.float64)
    assert np.allclose(np.linalg.norm(d, axis=2), 1.0, atol=1e-6)
    V, I = W.scene.meshes[0].vertices.astype(np.float64), W.scene.meshes[0].indices
    tri = V[I[p[hit]]]
    n = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    dirs = W.rays[hit, 4:7].astype(np.float64)
    n[(n * dirs).sum(1) > 0] *= -1
    assert ((d * n[:, None, :]).sum(2) >= -1e-6).all()
    # misses are void rays (tmin > tmax)
    assert (ao[~hit][:, :, 3] > ao[~hit][:, :, 7]).all()
    assert not orc.any_hit(S, ao[~hit].reshape(-1, 8)).any()


def test_ao_lone_plane_never_occluded(orc):
    V, I = quad(0.0)
    S = orc.OracleScene([(V, I)])
    rng = wl.rng_for(161)
    n = 512
    o = np.stack([rng.uniform(-5, 5, n), np.full(n, 3.0), rng.uniform(-5, 5, n)], 1)
    d = np.stack([rng.uniform(-0.3, 0.3, n), -np.ones(n), rng.uniform(-0.3, 0.3, n)], 1)
    rays = wl.pack_rays(o, d / np.linalg.norm(d, axis=1, keepdims=True))
    _, p, tuv = orc.closest(S, rays)
    assert (p != NONE).all()
    xi = rng.random((n, 16, 2)).astype(np.float32)
    ao = orc.ao_rays(S, rays, p, tuv, xi, 1e-4, 2.0)
    assert not orc.any_hit(S, ao).any()


def test_ao_parallel_plates_closed_form(orc):
    """Floor at y = 0 seen from below, a second plate at y = -h: samples in
    the downward hemisphere are occluded when h / cos(theta) <= R, i.e. with
    probability 1 - (h/R)^2 under the cosine density."""
    h, R = 0.25, 0.5
    V0, I0 = quad(0.0)
    V1, I1 = quad(-h)
    V = np.concatenate([V0, V1])
    I = np.concatenate([I0, I1 + 4]).astype(np.uint32)
    S = orc.OracleScene([(V, I)])
    rng = wl.rng_for(162)
    n, N = 128, 256
    o = np.stack([rng.uniform(-3, 3, n), np.full(n, -h / 2), rng.uniform(-3, 3, n)], 1)
    rays = wl.pack_rays(o, np.tile([0.0, 1.0, 0.0], (n, 1)))
    _, p, tuv = orc.closest(S, rays)
    assert (p < 2).all()
    xi = rng.random((n, N, 2)).astype(np.float32)
    ao = orc.ao_rays(S, rays, p, tuv, xi, 1e-4, R)
    occ = orc.any_hit(S, ao)
    expect = 1 - ((h - 1e-4) / R) ** 2
    sigma = math.sqrt(expect * (1 - expect) / occ.size)
    assert abs(occ.mean() - expect) < 5 * sigma
    # per sample: occluded exactly when the cosine to the normal reaches h/R
    cos = -ao[:, 5].astype(np.float64)
    clear = np.abs(cos - (h - 1e-4) / R) > 1e-5
    assert np.array_equal(occ[clear].astype(bool), cos[clear] >= (h - 1e-4) / R)


# ---- two-level scenes ------------------------------------------------------

IDENTITY = [1, 1, 1, 0, 0, 0, 1, 0, 0, 0]


def _two_level(V, I, srt):
    from oracle import OracleScene

    return OracleScene([(V, I)], np.zeros(1, np.uint32), np.asarray([srt], np.float32))


def _ao_both(orc, S1, S2, rays1, rays2, xi, offset, radius):
    _, p1, tuv1 = orc.closest(S1, rays1)
    i2, p2, tuv2 = orc.closest(S2, rays2)
    assert np.array_equal(p1, p2)
    hit = p1 != NONE
    a1 = orc.ao_rays(S1, rays1, p1, tuv1, xi, offset, radius)
    a2 = orc.ao_rays(S2, rays2, p2, tuv2, xi, offset, radius, inst=np.where(hit, i2, 0))
    return hit, a1.reshape(len(rays1), -1, 8), a2.reshape(len(rays1), -1, 8)


def _plates():
    """Two dyadic plates (exact float32 corners) and rays coming down on them."""
    V0, I0 = quad(0.0, half=4.0)
    V1, I1 = quad(-0.5, half=4.0)
    V = np.concatenate([V0, V1])
    I = np.concatenate([I0, I1 + 4]).astype(np.uint32)
    rng = wl.rng_for(163)
    n = 256
    o = np.stack([rng.uniform(-3, 3, n), np.full(n, 2.0), rng.uniform(-3, 3, n)], 1)
    d = np.stack([rng.uniform(-0.2, 0.2, n), -np.ones(n), rng.uniform(-0.2, 0.2, n)], 1)
    return V, I, o, d / np.linalg.norm(d, axis=1, keepdims=True), rng


def test_ao_identity_instance_equals_single_level(orc):
    W = wl.random_triangles(n_tri=2048, n_rays=1024, k=164, half=0.15)
    m = W.scene.meshes[0]
    S1 = orc.OracleScene([(m.vertices, m.indices)])
    S2 = _two_level(m.vertices, m.indices, IDENTITY)
    xi = wl.rng_for(165).random((1024, 4, 2)).astype(np.float32)
    hit, a1, a2 = _ao_both(orc, S1, S2, W.rays, W.rays, xi, 1e-4, 0.5)
    assert hit.sum() > 100
    assert np.array_equal(a1.view(np.uint32), a2.view(np.uint32))


def test_ao_translated_and_scaled_instances(orc):
    """Translation by a dyadic T keeps every corner difference exact, so the
    directions are bit-equal and the origins move by T; a uniform scale 2
    (offset 0) keeps the directions and doubles the origins."""
    V, I, o, d, rng = _plates()
    xi = rng.random((o.shape[0], 8, 2)).astype(np.float32)
    S1 = orc.OracleScene([(V, I)])
    T = np.array([4.0, -2.0, 8.0])
    St = _two_level(V, I, [1, 1, 1, 0, 0, 0, 1, *T])
    hit, a1, a2 = _ao_both(orc, S1, St, wl.pack_rays(o, d), wl.pack_rays(o + T, d), xi, 1e-4, 1.0)
    assert hit.all()
    assert np.array_equal(a1[..., 4:].view(np.uint32), a2[..., 4:].view(np.uint32))
    assert np.allclose(a2[..., 0:3], a1[..., 0:3] + T, atol=4e-6, rtol=0)
    Ss = _two_level(V, I, [2, 2, 2, 0, 0, 0, 1, 0, 0, 0])
    hit, a1, a2 = _ao_both(orc, S1, Ss, wl.pack_rays(o, d), wl.pack_rays(2 * o, d), xi, 0.0, 1.0)
    assert hit.all()
    assert np.array_equal(a1[..., 4:].view(np.uint32), a2[..., 4:].view(np.uint32))
    assert np.allclose(a2[..., 0:3], 2 * a1[..., 0:3], atol=4e-6, rtol=0)


def test_ao_rotated_instance(orc):
    """A quarter turn about y, R (x, y, z) = (z, y, -x): the directions and
    origins of the rotated scene are R applied to the unrotated ones (up to
    the rounding of the float32 quaternion)."""
    V, I, o, d, rng = _plates()
    xi = rng.random((o.shape[0], 8, 2)).astype(np.float32)
    rot = lambda a: np.stack([a[..., 2], a[..., 1], -a[..., 0]], -1)
    S1 = orc.OracleScene([(V, I)])
    s = np.sqrt(0.5)
    Sr = _two_level(V, I, [1, 1, 1, 0, s, 0, s, 0, 0, 0])
    hit, a1, a2 = _ao_both(orc, S1, Sr, wl.pack_rays(o, d), wl.pack_rays(rot(o), rot(d)), xi, 1e-4, 1.0)
    assert hit.all()
    assert np.allclose(a2[..., 4:7], rot(a1[..., 4:7]), atol=1e-6, rtol=0)
    assert np.allclose(a2[..., 0:3], rot(a1[..., 0:3]), atol=1e-5, rtol=0)


def test_ao_instanced_hemisphere(orc):
    """On the instanced grids: every AO direction of a hit is a unit vector in
    the hemisphere of the hit triangle's world normal (mapped here with the
    frame written out in numpy) turned toward the incoming ray."""
    W = wl.instanced_grids(n_inst=16, n_rays=2048, k=166)
    S = orc.OracleScene.from_scene(W.scene)
    inst, prim, tuv = orc.closest(S, W.rays)
    hit = prim != NONE
    assert hit.mean() > 0.2
    xi = wl.rng_for(167).random((W.rays.shape[0], 4, 2)).astype(np.float32)
    ao = orc.ao_rays(S, W.rays, prim, tuv, xi, 1e-4, 1.0, inst=np.where(hit, inst, 0)).reshape(-1, 4, 8)
    f = W.scene.inst_srt[inst[hit]].astype(np.float64)
    q = f[:, 3:7] / np.linalg.norm(f[:, 3:7], axis=1, keepdims=True)
    R = wl.quat_matrix(q)
    corners = []
    for c in range(3):
        v = np.stack([W.scene.meshes[W.scene.inst_mesh[j]].vertices[
            W.scene.meshes[W.scene.inst_mesh[j]].indices[p, c]] for j, p in zip(inst[hit], prim[hit])]).astype(np.float64)
        corners.append(np.einsum("nij,nj->ni", R, f[:, 0:3] * v) + f[:, 7:10])
    n = np.cross(corners[1] - corners[0], corners[2] - corners[0])
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    n[(n * W.rays[hit, 4:7]).sum(1) > 0] *= -1
    dirs = ao[hit][:, :, 4:7].astype(np.float64)
    assert np.allclose(np.linalg.norm(dirs, axis=2), 1.0, atol=1e-6)
    assert ((dirs * n[:, None, :]).sum(2) >= -1e-6).all()
    assert (ao[~hit][:, :, 3] > ao[~hit][:, :, 7]).all()
