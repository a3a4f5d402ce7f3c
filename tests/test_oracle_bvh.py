"""The oracle's FP64 BVH against the oracle's linear search (CPU).

The BVH is an exact accelerator of the search (§6.2: boxes only let the
traversal skip triangles the ray cannot hit), so every query through it must
return the linear search's answer bit for bit: closest hits, any-hit
occlusion, all-hit lists, the acceptable sets and the all-hit candidates.
Checked on many random small scenes (single and two-level, with masks and the
self-intersection filter, degenerate and non-finite triangles, exact ties,
rays with zero or non-finite components) and on the 4,096-triangle random soup
with its 65,536 rays in full."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2603_00292_amd import workloads as wl


def _same(a, b, what):
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    assert a.shape == b.shape, what
    assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), what


def _compare(orc, lin, acc, rays, opts=None, K=8, label=""):
    i0, p0, t0 = orc.closest(lin, rays, opts)
    i1, p1, t1 = orc.closest(acc, rays, opts)
    _same(i0, i1, f"{label} closest inst")
    _same(p0, p1, f"{label} closest prim")
    _same(t0, t1, f"{label} closest tuv")
    _same(orc.any_hit(lin, rays, opts), orc.any_hit(acc, rays, opts), f"{label} any")
    a = orc.all_hits(lin, rays, K, opts)
    b = orc.all_hits(acc, rays, K, opts)
    for x, y, n in zip(a, b, ("count", "inst", "prim", "tuv")):
        _same(x, y, f"{label} all {n}")
    A = orc.accept(lin, rays, K=K, opts=opts)
    B = orc.accept(acc, rays, K=K, opts=opts)
    for n in ("miss_ok", "count", "inst", "prim", "tuv", "scale", "any_class"):
        _same(getattr(A, n), getattr(B, n), f"{label} accept {n}")
    C = orc.classify_all(lin, rays, K, opts)
    D = orc.classify_all(acc, rays, K, opts)
    for n in ("count", "n_sure", "inst", "prim", "tuv", "scale", "lo", "hi", "sure"):
        _same(getattr(C, n), getattr(D, n), f"{label} classify_all {n}")
    return p0


def _random_scene(rng, two_level):
    n_mesh = int(rng.integers(1, 4)) if two_level else 1
    meshes = []
    for _ in range(n_mesh):
        n = int(rng.integers(0, 60)) if two_level else int(rng.integers(1, 120))
        V, I = wl.random_triangle_soup(rng, n, float(rng.choice([0.02, 0.1, 0.4])))
        V = V.copy()
        if n >= 8:
            # degenerate triangles: repeated vertex, collinear
            V[I[0, 1]] = V[I[0, 0]]
            V[I[1, 2]] = 0.5 * (V[I[1, 0]] + V[I[1, 1]])
            # an exact duplicate of another triangle (tie in t, lower id wins)
            I = I.copy()
            I[2] = I[3]
            if rng.random() < 0.3:
                V[I[4, 0], 0] = np.nan
            if rng.random() < 0.2:
                V[I[5, 2], 1] = np.inf
        meshes.append((V, I))
    if not two_level:
        return meshes, None, None
    ni = int(rng.integers(1, 40))
    inst_mesh = rng.integers(0, n_mesh, ni).astype(np.uint32)
    S = rng.uniform(0.3, 2.5, (ni, 3))
    q = wl.uniform_quaternions(rng, ni)
    T = rng.uniform(-3, 3, (ni, 3))
    srt = np.concatenate([S, q, T], 1).astype(np.float32)
    if ni > 3 and rng.random() < 0.3:
        srt[1, 0] = 0.0      # singular frame: non-finite object rays
    if ni > 3 and rng.random() < 0.2:
        srt[2, 8] = np.nan   # non-finite translation
    if ni > 4 and rng.random() < 0.5:
        srt[3] = srt[0]      # two instances with the same frame and mesh: ties
        inst_mesh[3] = inst_mesh[0]
    return meshes, inst_mesh, srt


def _random_rays(rng, n, two_level):
    lo, hi = (-5.0, 5.0) if two_level else (-0.5, 1.5)
    rays = wl.box_rays(rng, n, lo, hi)
    k = rng.random(n)
    rays[k < 0.05, 3] = rng.uniform(0, 2, int((k < 0.05).sum()))          # tmin > 0
    sel = (k >= 0.05) & (k < 0.12)
    rays[sel, 7] = rng.uniform(0, 3, int(sel.sum()))                         # finite tmax
    sel = (k >= 0.12) & (k < 0.17)
    rays[sel, 4 + rng.integers(0, 3)] = 0.0                                 # a zero component
    rays[rng.random(n) < 0.02, 4:7] = 0.0                                    # zero direction
    sel = rng.random(n) < 0.01
    rays[sel, 0] = np.inf                                                    # infinite origin
    sel = rng.random(n) < 0.01
    rays[sel, 6] = -np.inf                                                   # infinite direction
    sel = rng.random(n) < 0.01
    rays[sel, 2] = np.nan
    sel = rng.random(n) < 0.02
    rays[sel, 4:7] *= np.float32(1e-30)                                      # tiny direction
    return rays


@pytest.mark.parametrize("two_level", [False, True])
def test_bvh_equals_linear_search_random_scenes(orc, two_level):
    rng = wl.rng_for(300 + int(two_level))
    for case in range(150):
        meshes, im, srt = _random_scene(rng, two_level)
        lin = orc.OracleScene(meshes, im, srt)
        acc = orc.OracleScene(meshes, im, srt, accel=True)
        n = 300
        rays = _random_rays(rng, n, two_level)
        # rays aimed at triangle corners and edge midpoints (shared-edge ties)
        V, I = meshes[0]
        if I.shape[0] and not two_level:
            t = rng.integers(0, I.shape[0], 60)
            w = rng.choice([0.0, 0.5, 1.0], (60, 2))
            p = (V[I[t, 0]] * (1 - w[:, :1]) + V[I[t, 1]] * w[:, :1]).astype(np.float64)
            o = p + rng.normal(0, 1, (60, 3))
            rays[:60] = wl.pack_rays(o, p - o)
        opts = None
        if case % 3 == 1:
            ni = 0 if im is None else len(im)
            opts = orc.Opts(inst_mask=None if ni == 0 else rng.integers(0, 4, ni),
                            ray_mask=rng.integers(0, 4, n),
                            skip_inst=rng.integers(0, max(ni, 1), n),
                            skip_prim=np.where(rng.random(n) < 0.5, rng.integers(0, 40, n), orc.NONE))
        _compare(orc, lin, acc, rays, opts, K=int(rng.choice([1, 4, 16])), label=f"case {case}")


def test_bvh_equals_linear_search_random_soup_full(orc):
    """The 4,096-triangle soup with all 65,536 of its rays, every query."""
    W = wl.random_triangles()
    lin = orc.OracleScene.from_scene(W.scene)
    acc = orc.OracleScene.from_scene(W.scene, accel=True)
    st = acc.bvh_stats()
    assert st["loose"] == 0 and st["nodes"] > 1000
    prim = _compare(orc, lin, acc, W.rays, K=8, label="random soup")
    assert (prim != orc.NONE).sum() > 2000  # ~3.8% of the rays hit the sparse soup


def test_bvh_equals_linear_search_instanced(orc):
    """16 instances of the four displaced grids (the instanced workload's
    recipe at a size the linear search finishes), surface rays, with and
    without the self-intersection filter."""
    W = wl.instanced_grids(n_inst=16, n_rays=1024, k=302)
    lin = orc.OracleScene.from_scene(W.scene)
    acc = orc.OracleScene.from_scene(W.scene, accel=True)
    _compare(orc, lin, acc, W.rays, K=16, label="instanced")
    opts = orc.Opts(skip_inst=W.extra["src_inst"], skip_prim=W.extra["src_prim"])
    _compare(orc, lin, acc, W.rays, opts, K=16, label="instanced filtered")


def test_bvh_rejects_other_scene(orc):
    """A BVH answers only for the scene (arrays) it was built from."""
    W = wl.random_triangles(n_tri=64, n_rays=16, k=303)
    acc = orc.OracleScene.from_scene(W.scene, accel=True)
    other = orc.OracleScene.from_scene(W.scene)
    other.desc.bvh = acc.desc.bvh
    with pytest.raises(ValueError):
        orc.closest(other, W.rays)
    other.desc.bvh = None


def _edge_rays(rng, tris, n, dist, grazing):
    """Rays whose lines pass outside a random edge of a random triangle at a
    distance sweeping 1e-9 .. 1e-4 (times the scene scale), so that they land
    in every part of the tolerance model's grey band around edges; origins
    `dist` away, a fraction at grazing angles to the triangle's plane."""
    k = rng.integers(0, len(tris), n)
    e = rng.integers(0, 3, n)
    out = np.empty((n, 8), np.float32)
    for i in range(n):
        p = tris[k[i]].astype(np.float64)
        a, b, c = p[e[i]], p[(e[i] + 1) % 3], p[(e[i] + 2) % 3]
        nrm = np.cross(b - a, c - a)
        nrm /= np.linalg.norm(nrm)
        ed = (b - a) / np.linalg.norm(b - a)
        outw = np.cross(ed, nrm)
        if np.dot(outw, c - a) > 0:
            outw = -outw
        scale = np.abs(p).max() + dist
        off = 10.0 ** rng.uniform(-9, -4) * scale * rng.choice([-1.0, 1.0])
        x = a + rng.uniform(0.05, 0.95) * (b - a) + off * outw
        if grazing[i]:
            ang = 10.0 ** rng.uniform(-3, -0.5)
            dirn = np.cos(ang) * (-outw if rng.random() < 0.5 else ed) + np.sin(ang) * nrm * rng.choice([-1, 1])
        else:
            dirn = rng.normal(size=3)
        dirn /= np.linalg.norm(dirn)
        o = x - dist * rng.uniform(0.5, 1.0) * dirn
        out[i] = wl.pack_rays(o[None], dirn[None])[0]
    return out


@pytest.mark.parametrize("two_level", [False, True])
def test_bvh_equals_linear_search_margins(orc, two_level):
    """Rays in the tolerance model's bands: just outside edges (every offset
    from far inside to far outside eta), grazing rays through stacks of
    parallel triangles spaced about rho_t apart (sure hits whose t ranges
    overlap, the case that needs the box diagonal in the lowest-t bound),
    origins near and far; two-level scenes add anisotropic scales."""
    rng = wl.rng_for(310 + int(two_level))
    for case in range(24):
        # a few isolated triangles plus a stack of large parallel layers
        V, I = wl.random_triangle_soup(rng, 6, 0.3)
        V = V.astype(np.float64) * 4.0
        base = np.array([[0, 0, 0], [3, 0, 0], [0, 3, 0]], np.float64)
        ax = wl.uniform_quaternions(rng, 1)
        R = wl.quat_matrix(ax)[0]
        gap = 10.0 ** rng.uniform(-6, -3)
        layers = [(base + [0, 0, gap * j]) @ R.T + [5, 5, 5] for j in range(4)]
        V = np.concatenate([V] + layers).astype(np.float32)
        I = np.concatenate([I, np.arange(6 * 3, 6 * 3 + 12, dtype=np.uint32).reshape(4, 3)])
        tris = V[I]
        meshes = [(V, I)]
        im = srt = None
        if two_level:
            ni = 6
            im = np.zeros(ni, np.uint32)
            S = rng.uniform(0.2, 3.0, (ni, 3))
            S[0] = [0.1, 1.0, 8.0]
            q = wl.uniform_quaternions(rng, ni)
            q[1] = [0, 0, 0, 1]
            T = rng.uniform(-30, 30, (ni, 3))
            srt = np.concatenate([S, q, T], 1).astype(np.float32)
            from paper_2603_00292_amd.workloads import quat_matrix
            Rs = quat_matrix(srt[:, 3:7].astype(np.float64))
            j = rng.integers(0, ni, len(tris))
            j[-4:] = j[-1]  # the layer stack in one instance
            tris = np.einsum("nij,nkj->nki", Rs[j], srt[j, None, 0:3].astype(np.float64) * tris) + srt[j, None, 7:10]
        lin = orc.OracleScene(meshes, im, srt)
        acc = orc.OracleScene(meshes, im, srt, accel=True)
        n = 400
        grazing = rng.random(n) < 0.5
        dist = float(rng.choice([0.5, 5.0, 60.0]))
        rays = _edge_rays(rng, tris, n, dist, grazing)
        # grazing rays along the layer stack
        m = 100
        P = tris[-4:]
        c = P[:, 0] + 0.3 * (P[:, 1] - P[:, 0]) + 0.3 * (P[:, 2] - P[:, 0])
        nrm = np.cross(P[0, 1] - P[0, 0], P[0, 2] - P[0, 0])
        nrm /= np.linalg.norm(nrm)
        tang = (P[0, 1] - P[0, 0]) / np.linalg.norm(P[0, 1] - P[0, 0])
        ang = 10.0 ** rng.uniform(-4, -1, m)
        d = np.cos(ang)[:, None] * tang + np.sin(ang)[:, None] * nrm * rng.choice([-1, 1], (m, 1))
        tgt = c[rng.integers(0, 4, m)] + rng.normal(0, 0.05, (m, 3))
        o = tgt - rng.uniform(0.5, 2.0, (m, 1)) * d
        rays = np.concatenate([rays, wl.pack_rays(o, d)])
        _compare(orc, lin, acc, rays, None, K=16, label=f"margins case {case}")


def _vertex_rays(rng, tris, n, dists):
    """Lines passing an extremal vertex (of the whole scene, or of one
    triangle along a random axis) at offsets from 0 to ~1e-3 of the scale
    outside it, parallel or nearly parallel to the box face through it: the
    pairs that sit on the boxes' faces, within every fraction of eta."""
    P = tris.reshape(-1, 3)
    scale = np.abs(P).max()
    out = np.empty((n, 8), np.float32)
    for i in range(n):
        a = int(rng.integers(0, 3))
        side = rng.choice([-1.0, 1.0])
        if rng.random() < 0.5:
            v = P[np.argmax(side * P[:, a])]
        else:
            t = tris[rng.integers(0, len(tris))]
            v = t[np.argmax(side * t[:, a])]
        off = 0.0 if rng.random() < 0.2 else 10.0 ** rng.uniform(-10, -3) * (scale + 1.0)
        dist = float(rng.choice(dists)) * rng.uniform(0.5, 1.0)
        x = v.astype(np.float64).copy()
        if rng.random() < 0.6:
            x[a] += side * off
            d = rng.normal(size=3)
            d[a] = 0.0 if rng.random() < 0.5 else 10.0 ** rng.uniform(-8, -2) * rng.choice([-1, 1])
            d /= np.linalg.norm(d)
            out[i] = wl.pack_rays((x - dist * d)[None], d[None])[0]
            continue
        # nearly along the axis, from beyond the face: the range [tmin, tmax]
        # ends within every fraction of eta/|d| before the extremal vertex
        # (coming toward it) or after it (going away)
        d = np.zeros(3)
        d[a] = -side
        d += rng.normal(size=3) * 10.0 ** rng.uniform(-7, -2)
        d /= np.linalg.norm(d)
        toward = rng.random() < 0.5
        if not toward:
            d = -d
        o = x + side * dist * np.eye(3)[a] + rng.normal(size=3) * off
        f = 10.0 ** rng.uniform(-9, -3) * (scale + dist)
        tv = float(np.dot(x - o, d))
        if toward:
            out[i] = wl.pack_rays(o[None], d[None], 0.0, tv - f)[0]
        else:
            out[i] = wl.pack_rays(o[None], d[None], tv + f, np.inf)[0]
    return out


def _barely_sure_rays(rng, tris, n, delta):
    """Grazing rays that cross a triangle just farther than the tolerance
    model's sure-hit distance (eta/cos + eta) from the edge behind them: sure
    hits whose lowest t, t - rho_t, lies before every corner of the box
    (single-level scenes: eta = 2 delta (s + L))."""
    out = []
    while len(out) < n:
        p3 = tris[rng.integers(0, len(tris))].astype(np.float64)
        e = int(rng.integers(0, 3))
        a, b, c = p3[e], p3[(e + 1) % 3], p3[(e + 2) % 3]
        nrm = np.cross(b - a, c - a)
        if np.linalg.norm(nrm) == 0:
            continue
        nrm /= np.linalg.norm(nrm)
        ed = (b - a) / np.linalg.norm(b - a)
        inward = np.cross(nrm, ed)
        if np.dot(inward, c - a) < 0:
            inward = -inward
        cs = 10.0 ** rng.uniform(-3, -0.5)
        d = np.sqrt(1 - cs * cs) * inward + cs * nrm * rng.choice([-1, 1])
        m = a + rng.uniform(0.3, 0.7) * (b - a)
        dist = float(rng.choice([0.5, 5.0, 50.0]))
        o = m - dist * d
        for _ in range(3):
            s = max(np.abs(o).max(), np.abs(p3).max())
            L = np.linalg.norm(p3 - o, axis=1).max()
            eta = 2 * delta * s + 2 * delta * L
            cdist = (eta / cs + eta) * (1.0 + 10.0 ** rng.uniform(-3, 0))
            p = m + cdist * inward
            o = p - dist * d
        out.append(wl.pack_rays(o[None], d[None])[0])
    return np.array(out, np.float32)


@pytest.mark.parametrize("two_level", [False, True])
def test_bvh_culling_bounds_hold_pair_by_pair(orc, two_level):
    """The invariant behind the BVH's exactness, checked on every wanted pair
    of the linear search: each box above a hit admits it with entry t <= t,
    each box above a sure or maybe pair of the tolerance model admits it with
    its lowest-t bound <= the pair's lowest possible t.  The rays are aimed
    at the boxes' faces (lines grazing extremal vertices at every offset
    within and beyond eta) and at barely-sure grazing hits."""
    rng = wl.rng_for(320 + int(two_level))
    checked = [0, 0]
    for case in range(12):
        V, I = wl.random_triangle_soup(rng, 40, float(rng.choice([0.05, 0.3])))
        V = (V.astype(np.float64) * rng.choice([1.0, 8.0]) + rng.uniform(-3, 3, 3)).astype(np.float32)
        meshes = [(V, I)]
        im = srt = None
        tris = V[I].astype(np.float64)
        if two_level:
            ni = 8
            im = np.zeros(ni, np.uint32)
            S = rng.uniform(0.2, 3.0, (ni, 3))
            S[0] = [0.1, 1.0, 8.0]                        # anisotropic: ||A|| ||A^-1|| = 80
            S[1] = [4.0, 4.0, 4.0]
            q = np.tile([0.0, 0.0, 0.0, 1.0], (ni, 1))   # axis-aligned: the world box is tight
            q[4:] = wl.uniform_quaternions(rng, ni - 4)
            T = rng.uniform(-20, 20, (ni, 3))
            srt = np.concatenate([S, q, T], 1).astype(np.float32)
            Rs = wl.quat_matrix(srt[:, 3:7].astype(np.float64))
            tris = np.concatenate([np.einsum("ij,nkj->nki", Rs[j], srt[j, 0:3].astype(np.float64) * tris)
                                   + srt[j, 7:10] for j in range(ni)])
        acc = orc.OracleScene(meshes, im, srt, accel=True)
        rays = _vertex_rays(rng, tris, 600, (1.0, 10.0, 100.0))
        if not two_level:
            rays = np.concatenate([rays, _barely_sure_rays(rng, tris, 300, orc.DELTA)])
        for kind in (0, 1):
            pairs, bad = orc.bvh_check(acc, rays, candidates=bool(kind))
            assert bad == 0, f"case {case} kind {kind}: {bad} of {pairs} pairs culled"
            checked[kind] += pairs
        _compare(orc, orc.OracleScene(meshes, im, srt), acc, rays, None, K=16, label=f"bounds {case}")
    assert checked[0] > 1000 and checked[1] > 2000, checked
