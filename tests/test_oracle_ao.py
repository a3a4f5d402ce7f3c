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
