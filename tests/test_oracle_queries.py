"""Pins of the oracle's query variants: all-hit enumeration, ray masks and
the self-intersection filter.

All-hits is pinned by a closed form (a stack of parallel triangles crossed
at known t), by its relations to the closest and any-hit queries, by
brute force over one-triangle scenes, by truncation, and by the exact
flattening of dyadic instances.  Masks are pinned by sub-scenes that hold
only the selected instances; the filter by the relation "skipping the
closest hit leaves the second of the sorted hits".
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_2603_00292_amd import workloads as wl

NONE = 0xFFFFFFFF


def dense(n_tri, n_rays, k, half=0.1):
    rng = wl.rng_for(k)
    V, I = wl.random_triangle_soup(rng, n_tri, half)
    rays = wl.box_rays(rng, n_rays, 0.0, 1.0)
    return V, I, rays


def test_all_hits_parallel_stack_closed_form(orc):
    """Seven large triangles in the planes z = 1..7, stored in a shuffled
    order; a ray up the z axis meets them at t = z exactly (u, v too)."""
    rng = np.random.default_rng(5)
    order = rng.permutation(7)
    V, I = [], []
    for slot, z in enumerate(order + 1):
        V += [[-4, -4, z], [4, -4, z], [-4, 4, z]]
        I.append([3 * slot, 3 * slot + 1, 3 * slot + 2])
    V = np.array(V, np.float32)
    I = np.array(I, np.uint32)
    S = orc.OracleScene([(V, I)])
    rays = np.array([[-1, -1, 0, 0, 0, 0, 1, np.inf],
                     [-1, -1, 0, 0, 0, 0, 1, 4.5],
                     [-1, -1, 0, 2, 0, 0, 1, np.inf],
                     [-1, -1, 0, 3, 0, 0, 1, 3.0],
                     [-1, -1, 10, 0, 0, 0, 1, np.inf]], np.float32)
    cnt, inst, prim, tuv = orc.all_hits(S, rays, K=8)
    assert cnt.tolist() == [7, 4, 6, 1, 0]
    slot_of_z = {int(z): s for s, z in enumerate(order + 1)}
    assert prim[0, :7].tolist() == [slot_of_z[z] for z in range(1, 8)]
    assert tuv[0, :7, 0].tolist() == [1, 2, 3, 4, 5, 6, 7]
    # (x, y) = (-1, -1) on each triangle: w = (1-u-v, u, v) with u = v = 3/8
    assert np.allclose(tuv[0, :7, 1:], 3 / 8, rtol=0, atol=0)
    assert (prim[0, 7:] == NONE).all() and np.isinf(tuv[0, 7:, 0]).all()
    assert tuv[2, :6, 0].tolist() == [2, 3, 4, 5, 6, 7]
    assert tuv[3, 0, 0] == 3 and (inst[:4, 0] == 0).all()
    assert (prim[4] == NONE).all()


def test_all_hits_ties_sorted_by_id(orc):
    """Coplanar overlapping triangles hit at the same t are listed by
    ascending triangle id (the lexicographic (t, inst, prim) order), and the
    first of them is the closest hit."""
    V = np.array([[-4, -4, 2], [4, -4, 2], [-4, 4, 2],
                  [-3, -5, 2], [5, -3, 2], [-5, 5, 2],
                  [-4, -4, 1], [4, -4, 1], [-4, 4, 1]], np.float32)
    for perm in ([0, 1, 2], [2, 1, 0], [1, 2, 0]):
        I = np.array([[0, 1, 2], [3, 4, 5], [6, 7, 8]], np.uint32)[perm]
        S = orc.OracleScene([(V, I)])
        rays = np.array([[-1, -1, 0, 0, 0, 0, 1, np.inf]], np.float32)
        cnt, _, prim, tuv = orc.all_hits(S, rays, K=4)
        assert cnt[0] == 3 and tuv[0, :3, 0].tolist() == [1, 2, 2]
        at2 = sorted(prim[0, 1:3].tolist())
        assert prim[0, 1:3].tolist() == at2
        _, cp, _ = orc.closest(S, rays)
        assert cp[0] == prim[0, 0]


def test_all_hits_relations(orc):
    """The first sorted hit is the closest hit (exactly), a count above zero
    is occlusion, and a smaller capacity keeps a prefix of the list."""
    V, I, rays = dense(600, 2048, 140, half=0.15)
    S = orc.OracleScene([(V, I)])
    cnt, inst, prim, tuv = orc.all_hits(S, rays, K=16)
    c3, i3, p3, t3 = orc.all_hits(S, rays, K=3)
    _, cp, ctuv = orc.closest(S, rays)
    occ = orc.any_hit(S, rays)
    assert (cnt > 3).sum() > 200
    assert np.array_equal(prim[:, 0], cp)
    hit = cp != NONE
    assert np.array_equal(tuv[hit, 0], ctuv[hit])
    assert np.array_equal(cnt > 0, occ.astype(bool))
    assert np.array_equal(c3, cnt) and np.array_equal(p3, prim[:, :3])
    assert np.array_equal(t3, tuv[:, :3])
    # sorted by (t, inst, prim), no repeated pair
    for r in range(rays.shape[0]):
        n = min(int(cnt[r]), 16)
        ts = tuv[r, :n, 0]
        assert (np.diff(ts) >= 0).all()
        assert len(set(prim[r, :n].tolist())) == n


def test_all_hits_count_by_brute_force(orc):
    """count = number of one-triangle scenes whose any-hit query reports a
    hit, for every ray."""
    V, I, rays = dense(120, 256, 141, half=0.2)
    S = orc.OracleScene([(V, I)])
    cnt, _, prim, _ = orc.all_hits(S, rays, K=120)
    per = np.zeros(rays.shape[0], np.int64)
    members = [set() for _ in range(rays.shape[0])]
    for k in range(I.shape[0]):
        occ = orc.any_hit(orc.OracleScene([(V, I[k:k + 1])]), rays)
        per += occ
        for r in np.flatnonzero(occ):
            members[r].add(k)
    assert np.array_equal(per, cnt)
    assert per.max() >= 4 and (per >= 2).sum() > 20
    for r in range(rays.shape[0]):
        assert set(prim[r, :cnt[r]].tolist()) == members[r]


def test_all_hits_instances_equal_flattened(orc):
    """Dyadic instances are exact in float32: the two-level hit lists equal
    the flattened mesh's, ids mapped."""
    W = wl.random_triangles(n_tri=128, n_rays=2048, k=142, half=0.15)
    m = W.scene.meshes[0]
    V = (np.round(m.vertices * 1024) / 1024).astype(np.float32)
    frames = np.array([[2, 2, 2, 0, 0, 0, 1, 0.5, -1, 0.25],
                       [1, 2, 4, 0, 0, 1, 0, -2, 0, 1],
                       [0.5, 0.5, 0.5, 1, 0, 0, 0, 0, 0, -0.5]], np.float32)
    S_inst = orc.OracleScene([(V, m.indices)], np.zeros(3, np.uint32), frames)
    R = wl.quat_matrix(frames[:, 3:7].astype(np.float64))
    fv = [V.astype(np.float64) * frames[j, 0:3] @ R[j].T + frames[j, 7:10] for j in range(3)]
    FV = np.concatenate(fv).astype(np.float32)
    assert np.array_equal(FV.astype(np.float64), np.concatenate(fv))
    FI = np.concatenate([m.indices + j * V.shape[0] for j in range(3)]).astype(np.uint32)
    rng = wl.rng_for(143)
    rays = wl.pack_rays(rng.uniform(-3, 3, (2048, 3)), wl.uniform_sphere_dirs(rng, 2048))
    cf, _, pf, tf = orc.all_hits(orc.OracleScene([(FV, FI)]), rays, K=12)
    ci, ii, pi, ti = orc.all_hits(S_inst, rays, K=12)
    assert np.array_equal(cf, ci) and cf.max() >= 3
    n = m.indices.shape[0]
    for r in range(rays.shape[0]):
        k = min(int(cf[r]), 12)
        got = sorted(zip(ti[r, :k, 0].tolist(), (ii[r, :k].astype(np.int64) * n + pi[r, :k]).tolist()))
        want = sorted(zip(tf[r, :k, 0].tolist(), pf[r, :k].tolist()))
        assert [g[1] for g in got] == [w[1] for w in want]
        assert np.allclose([g[0] for g in got], [w[0] for w in want], rtol=1e-12, atol=0)


def _two_level(k, n_inst=8):
    W = wl.aimed_instances(n_inst=n_inst, n_rays=4096, k=k)
    return W.scene, W.rays


def test_masks_equal_sub_scenes(orc):
    """Instance j carries mask bit (j mod 4); a ray with mask m sees exactly
    the scene made of the instances whose bit is in m."""
    scene, rays = _two_level(144)
    n = rays.shape[0]
    inst_mask = (1 << (np.arange(8) % 4)).astype(np.uint32)
    ray_mask = wl.rng_for(145).integers(0, 16, n).astype(np.uint32)
    opts = orc.Opts(inst_mask=inst_mask, ray_mask=ray_mask)
    S = orc.OracleScene.from_scene(scene)
    gi, gp, gt = orc.closest(S, rays, opts)
    occ = orc.any_hit(S, rays, opts)
    cnt, _, _, _ = orc.all_hits(S, rays, K=4, opts=opts)
    assert (gp != NONE).sum() > 500
    for m in range(16):
        sel = np.flatnonzero(ray_mask == m)
        keep = np.flatnonzero((inst_mask & m) != 0)
        if keep.size == 0:
            assert (gp[sel] == NONE).all() and not occ[sel].any() and (cnt[sel] == 0).all()
            continue
        sub = orc.OracleScene([(mm.vertices, mm.indices) for mm in scene.meshes],
                              scene.inst_mesh[keep], scene.inst_srt[keep])
        si, sp, st = orc.closest(sub, rays[sel])
        hit = sp != NONE
        assert np.array_equal(gp[sel], sp)
        assert np.array_equal(gi[sel][hit], keep[si[hit]])
        assert np.array_equal(gt[sel], st)
        assert np.array_equal(occ[sel], orc.any_hit(sub, rays[sel]))


def test_single_level_masks(orc):
    """One geometry of mask 0xFFFFFFFF: a zero ray mask misses, any other
    mask changes nothing."""
    V, I, rays = dense(300, 512, 146)
    S = orc.OracleScene([(V, I)])
    ray_mask = np.where(np.arange(512) % 3 == 0, 0, 0x80000000).astype(np.uint32)
    _, p0, t0 = orc.closest(S, rays)
    _, p1, t1 = orc.closest(S, rays, orc.Opts(ray_mask=ray_mask))
    zero = ray_mask == 0
    assert (p1[zero] == NONE).all() and np.isinf(t1[zero, 0]).all()
    assert np.array_equal(p1[~zero], p0[~zero]) and np.array_equal(t1[~zero], t0[~zero])


@pytest.mark.parametrize("two_level", [False, True])
def test_skip_filter_gives_second_hit(orc, two_level):
    """Skipping each ray's closest hit makes the second sorted hit the
    closest (exactly, ties included), and occlusion means two or more hits."""
    if two_level:
        scene, rays = _two_level(147)
        S = orc.OracleScene.from_scene(scene)
    else:
        V, I, rays = dense(600, 2048, 148, half=0.15)
        S = orc.OracleScene([(V, I)])
    cnt, ai, ap, at = orc.all_hits(S, rays, K=2)
    opts = orc.Opts(skip_inst=ai[:, 0], skip_prim=ap[:, 0])
    si, sp, st = orc.closest(S, rays, opts)
    occ = orc.any_hit(S, rays, opts)
    assert (cnt >= 2).sum() > 100
    assert np.array_equal(sp, ap[:, 1])
    two = cnt >= 2
    assert np.array_equal(st[two], at[two, 1])
    if two_level:
        assert np.array_equal(si[two], ai[two, 1])
    assert np.array_equal(occ.astype(bool), cnt >= 2)
    # a filter naming a triangle the ray does not hit changes nothing
    other = orc.Opts(skip_inst=ai[:, 0], skip_prim=np.where(ap[:, 0] == NONE, NONE, (ap[:, 0] + 1) % 7))
    _, p2, _ = orc.closest(S, rays, other)
    _, p0, _ = orc.closest(S, rays)
    moved = (p2 != p0)
    assert (ap[moved, 0] != NONE).all()
    assert (((ap[:, 0] + 1) % 7)[moved] == p0[moved]).all()


def test_classify_all_brackets_the_exact_hits(orc):
    """Every exact hit is a candidate; every sure candidate is an exact hit;
    its t lies in [lo, hi]; closest-query sets are candidates too."""
    V, I, rays = dense(600, 1024, 149, half=0.15)
    S = orc.OracleScene([(V, I)])
    K = 24
    C = orc.classify_all(S, rays, K)
    cnt, _, prim, tuv = orc.all_hits(S, rays, K)
    A = orc.accept(S, rays)
    assert (C.count <= K).all()
    assert (C.n_sure <= cnt).all() and (cnt <= C.count).all()
    assert (C.n_sure < C.count).any() and (C.n_sure == C.count).mean() > 0.9
    for r in range(rays.shape[0]):
        cands = {int(C.prim[r, i]): i for i in range(C.count[r])}
        exact = set(prim[r, :cnt[r]].tolist())
        assert exact <= set(cands)
        for p, i in cands.items():
            if C.sure[r, i]:
                assert p in exact
                assert C.lo[r, i] <= C.tuv[r, i, 0] <= C.hi[r, i]
        for j in range(A.count[r]):
            assert int(A.prim[r, j]) in cands
