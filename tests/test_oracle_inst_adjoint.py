"""Pins of the oracle's two-level adjoint (gradients through instance frames).

The analytic gradients are checked against central finite differences of
the plane formula evaluated on the world-space triangle, with every one of
the 25 inputs perturbed (object vertices, the ten frame parameters including
the unnormalised quaternion, ray origin and direction), and against exact
relations of the frame: a translation of the instance is a negative
translation of the ray origin, the result does not change when the
quaternion is scaled, scaling the frame's scale is scaling the object
vertices, and an identity instance reproduces the single-level adjoint.
"""
from __future__ import annotations

import numpy as np

from paper_2603_00292_amd import workloads as wl

NONE = 0xFFFFFFFF


def instanced_scene(k, n_inst=8, n_rays=4096):
    W = wl.aimed_instances(n_inst=n_inst, n_rays=n_rays, k=k)
    return W.scene, W.rays


def hits_of(orc, S, rays):
    inst, prim, tuv = orc.closest(S, rays)
    hit = np.flatnonzero(prim != NONE)
    return inst, prim, tuv, hit


def per_ray(orc, S, scene, rays, inst, prim, g, r):
    """The 25 analytic derivatives of ray r alone, in the order of fd_inst."""
    dV, dS, do, dd = orc.adjoint_inst(S, rays[r:r + 1], inst[r:r + 1], prim[r:r + 1], g[r:r + 1])
    m = int(scene.inst_mesh[inst[r]])
    tri = scene.meshes[m].indices[prim[r]]
    assert len(set(tri.tolist())) == 3
    return np.concatenate([dV[m][tri[0]], dV[m][tri[1]], dV[m][tri[2]], dS[inst[r]], do[0], dd[0]])


def test_instance_adjoint_matches_finite_differences(orc):
    scene, rays = instanced_scene(130)
    S = orc.OracleScene.from_scene(scene)
    inst, prim, _, hit = hits_of(orc, S, rays)
    assert hit.size > 2000
    assert len(set(inst[hit].tolist())) == 8
    g = wl.rng_for(131).standard_normal((rays.shape[0], 3))
    sel = hit[::23]
    fd = orc.fd_inst(S, rays[sel], inst[sel], prim[sel], g[sel], h=1e-6)
    worst = 0.0
    for i, r in enumerate(sel):
        an = per_ray(orc, S, scene, rays, inst, prim, g, r)
        scale = max(np.abs(an).max(), 1.0)
        err = np.abs(an - fd[i]).max() / scale
        worst = max(worst, err)
        assert err <= 2e-6, (r, an, fd[i])
    assert worst > 0.0  # the comparison really ran on non-trivial values


def test_instance_adjoint_accumulates_over_rays(orc):
    """One call over many rays sums the per-ray contributions."""
    scene, rays = instanced_scene(132, n_rays=512)
    S = orc.OracleScene.from_scene(scene)
    inst, prim, _, hit = hits_of(orc, S, rays)
    g = wl.rng_for(133).standard_normal((rays.shape[0], 3))
    dV, dS, do, dd = orc.adjoint_inst(S, rays, inst, prim, g)
    acc_V = [np.zeros_like(a) for a in dV]
    acc_S = np.zeros_like(dS)
    for r in range(rays.shape[0]):
        v1, s1, o1, d1 = orc.adjoint_inst(S, rays[r:r + 1], inst[r:r + 1], prim[r:r + 1], g[r:r + 1])
        for m in range(3):
            acc_V[m] += v1[m]
        acc_S += s1
        assert np.array_equal(o1[0], do[r]) and np.array_equal(d1[0], dd[r])
    for m in range(3):
        assert np.allclose(acc_V[m], dV[m], rtol=1e-12, atol=1e-12)
    assert np.allclose(acc_S, dS, rtol=1e-12, atol=1e-12)
    miss = prim == NONE
    assert miss.any() and (do[miss] == 0).all() and (dd[miss] == 0).all()


def test_instance_adjoint_frame_relations(orc):
    """Per ray: grad T = -grad o; grad q . q = 0 (normalisation);
    sum_b s_b grad s_b = sum_k v_k . grad v_k (scaling S scales the object)."""
    scene, rays = instanced_scene(134, n_rays=1024)
    S = orc.OracleScene.from_scene(scene)
    inst, prim, _, hit = hits_of(orc, S, rays)
    g = wl.rng_for(135).standard_normal((rays.shape[0], 3))
    for r in hit[:200]:
        an = per_ray(orc, S, scene, rays, inst, prim, g, r)
        gv, gs, gq, gT, go = an[0:9], an[9:12], an[12:16], an[16:19], an[19:22]
        scale = max(np.abs(an).max(), 1.0)
        assert np.abs(gT + go).max() <= 1e-12 * scale
        q = scene.inst_srt[inst[r], 3:7].astype(np.float64)
        assert abs(q @ gq) <= 1e-12 * scale * np.linalg.norm(q)
        m = int(scene.inst_mesh[inst[r]])
        tri = scene.meshes[m].indices[prim[r]]
        v = scene.meshes[m].vertices[tri].astype(np.float64).reshape(-1)
        s = scene.inst_srt[inst[r], 0:3].astype(np.float64)
        assert abs(s @ gs - v @ gv) <= 1e-11 * scale * max(1.0, np.abs(v).max())


def test_identity_instance_adjoint_equals_single_level(orc):
    W = wl.displaced_grid(nx=32, nz=16, n_rays=2048, k=136)
    m = W.scene.meshes[0]
    S1 = orc.OracleScene([(m.vertices, m.indices)])
    S2 = orc.OracleScene([(m.vertices, m.indices)], np.zeros(1, np.uint32),
                         np.array([[1, 1, 1, 0, 0, 0, 1, 0, 0, 0]], np.float32))
    _, p, _ = orc.closest(S1, W.rays)
    g = W.extra["abc"].astype(np.float64)
    dV1, do1, dd1 = orc.adjoint(S1, W.rays, p, g)
    dV2, dS2, do2, dd2 = orc.adjoint_inst(S2, W.rays, np.zeros_like(p), p, g)
    assert (p != NONE).sum() > 1500
    assert np.array_equal(do1, do2) and np.array_equal(dd1, dd2)
    assert np.array_equal(dV1, dV2[0])
    # the identity frame: grad T is minus the summed origin gradients
    assert np.allclose(dS2[0, 7:10], -do1.sum(0), rtol=1e-12, atol=1e-12)


def test_instance_adjoint_rejects_bad_ids(orc):
    scene, rays = instanced_scene(137, n_rays=16)
    S = orc.OracleScene.from_scene(scene)
    g = np.ones((16, 3))
    bad_inst = np.full(16, 8, np.uint32)
    prim = np.zeros(16, np.uint32)
    import pytest
    with pytest.raises(Exception):
        orc.adjoint_inst(S, rays, bad_inst, prim, g)
    with pytest.raises(Exception):
        orc.adjoint_inst(S, rays, np.zeros(16, np.uint32), np.full(16, 10 ** 6, np.uint32), g)
