"""GPU parity of the two-level adjoint (rt_trace_backward_instances) and of
the autograd Function over it, against the FP64 oracle's two-level adjoint
and FP64 finite differences of all 25 inputs of a hit.

Accumulated gradients (vertices, frames) are exact integer sums of the
float64-computed contributions at a per-row scale, rounded once to float32;
each entry is checked against the (looser) rounding bound of a float32 sum:
n * 2^-24 * (sum of |contributions|) for n terms, plus the float64
differences between the object-space (library) and world-space (oracle)
routes, far below that."""
from __future__ import annotations

import numpy as np
import pytest

from helpers import NONE, check_closest, to_gpu_scene
from paper_2603_00292_amd import workloads as wl

pytestmark = pytest.mark.gpu

GRAD_REL = 1e-4   # per-ray world-space ray gradients (float32 outputs of float64 math)
EPS32 = 2.0 ** -24


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def gpu():
    import torch

    from paper_2603_00292_amd import api

    torch.cuda.set_device(0)
    ctx = api.Context(0)
    yield torch, api, ctx
    torch.cuda.synchronize()


def _forward(gpu, acc, rays_np):
    torch, api, _ = gpu
    rays = torch.from_numpy(np.ascontiguousarray(rays_np)).cuda()
    hits, inst = api.trace_closest(acc, rays, want_inst=True)
    return rays, hits, inst


def _backward(gpu, acc, rays, hits, inst, g, n_vert, n_inst):
    torch, api, _ = gpu
    gt = torch.from_numpy(np.ascontiguousarray(g, dtype=np.float32)).cuda()
    dV = torch.zeros((n_vert, 3), dtype=torch.float32, device="cuda")
    dS = torch.zeros((n_inst, 10), dtype=torch.float32, device="cuda")
    do, dd = api.trace_backward_instances(acc, rays, hits, inst, gt, dV, dS)
    torch.cuda.synchronize()
    return (dV.cpu().numpy().astype(np.float64), dS.cpu().numpy().astype(np.float64),
            do.cpu().numpy().astype(np.float64), dd.cpu().numpy().astype(np.float64))


def _bases(scene):
    return np.concatenate([[0], np.cumsum([m.vertices.shape[0] for m in scene.meshes])])


def test_backward_instances_small_full_check(gpu, orc):
    """8 frames (one mirrored, unnormalised quaternions) of 3 meshes, 8,192
    aimed rays: every pinned hit's ray gradients, and every accumulated vertex
    and frame gradient within the float32 summation bound."""
    torch, api, ctx = gpu
    W = wl.aimed_instances(n_inst=8, n_rays=8192, k=310)
    scene = W.scene
    acc = to_gpu_scene(api, torch, ctx, scene)
    rays, hits, inst = _forward(gpu, acc, W.rays)
    h = hits.cpu().numpy()
    ii = inst.cpu().numpy().view(np.uint32)
    S = orc.OracleScene.from_scene(scene)
    A = orc.accept(S, W.rays)
    check_closest(h, A, inst=ii, label="aimed instances")
    oinst, oprim, _ = orc.closest(S, W.rays)
    prim = h[:, 1].copy().view(np.uint32)
    keep = A.pinned & (oprim != NONE)
    assert (prim[keep] == oprim[keep]).all() and (ii[keep] == oinst[keep]).all()
    assert keep.sum() > 3000
    # float32-representable cotangents: both sides see the same g
    g = wl.rng_for(311).standard_normal((W.rays.shape[0], 3)).astype(np.float32).astype(np.float64)
    g *= keep[:, None]
    base = _bases(scene)
    dV, dS, do, dd = _backward(gpu, acc, rays, hits, inst, g, base[-1], 8)
    # reference: per-ray oracle contributions, their sums and absolute sums
    p_ref = np.where(keep, oprim, NONE).astype(np.uint32)
    rV, rS, ro, rd = orc.adjoint_inst(S, W.rays, oinst, p_ref, g)
    rV = np.concatenate(rV)
    absV = np.zeros_like(rV)
    absS = np.zeros_like(rS)
    cntV = np.zeros(rV.shape[0])
    cntS = np.zeros(8)
    for r in np.flatnonzero(keep):
        v1, s1, _, _ = orc.adjoint_inst(S, W.rays[r:r + 1], oinst[r:r + 1], p_ref[r:r + 1], g[r:r + 1])
        m = int(scene.inst_mesh[oinst[r]])
        tri = scene.meshes[m].indices[oprim[r]].astype(np.int64) + base[m]
        absV[tri] += np.abs(np.concatenate(v1)[tri])
        cntV[tri] += 1
        absS[oinst[r]] += np.abs(s1[oinst[r]])
        cntS[oinst[r]] += 1
    r = np.flatnonzero(keep)
    eo = np.linalg.norm(do[r] - ro[r], axis=1) / np.linalg.norm(ro[r], axis=1)
    ed = np.linalg.norm(dd[r] - rd[r], axis=1) / np.linalg.norm(rd[r], axis=1)
    say("max rel err d_origin", eo.max(), "d_direction", ed.max())
    assert eo.max() <= GRAD_REL and ed.max() <= GRAD_REL
    assert np.abs(do[~keep]).max() == 0 and np.abs(dd[~keep]).max() == 0
    boundV = (cntV[:, None] + 1) * EPS32 * absV + 1e-12
    boundS = (cntS[:, None] + 1) * EPS32 * absS + 1e-12
    say("vertex err / bound", (np.abs(dV - rV) / boundV).max(),
        "frame err / bound", (np.abs(dS - rS) / boundS).max())
    assert (np.abs(dV - rV) <= boundV).all()
    assert (np.abs(dS - rS) <= boundS).all()
    say("frob rel: vertices", np.linalg.norm(dV - rV) / np.linalg.norm(rV),
        "frames", np.linalg.norm(dS - rS) / np.linalg.norm(rS))
    acc.close()


def test_backward_instances_single_rays_vs_finite_differences(gpu, orc):
    """All 25 derivatives of single hits (object vertices, ten frame
    parameters, origin, direction) against FP64 central differences."""
    torch, api, ctx = gpu
    W = wl.aimed_instances(n_inst=8, n_rays=2048, k=312)
    scene = W.scene
    acc = to_gpu_scene(api, torch, ctx, scene)
    rays, hits, inst = _forward(gpu, acc, W.rays)
    S = orc.OracleScene.from_scene(scene)
    A = orc.accept(S, W.rays)
    oinst, oprim, _ = orc.closest(S, W.rays)
    sel = np.flatnonzero(A.pinned & (oprim != NONE))[:40]
    assert sel.size == 40
    g = wl.rng_for(313).standard_normal((W.rays.shape[0], 3)).astype(np.float32).astype(np.float64)
    fd = orc.fd_inst(S, W.rays[sel], oinst[sel], oprim[sel], g[sel], h=1e-6)
    base = _bases(scene)
    for i, r in enumerate(sel):
        dV, dS, do, dd = _backward(gpu, acc, rays[r:r + 1].contiguous(), hits[r:r + 1].contiguous(),
                                   inst[r:r + 1].contiguous(), g[r:r + 1], base[-1], 8)
        m = int(scene.inst_mesh[oinst[r]])
        tri = scene.meshes[m].indices[oprim[r]].astype(np.int64) + base[m]
        got = np.concatenate([dV[tri[0]], dV[tri[1]], dV[tri[2]], dS[oinst[r]], do[0], dd[0]])
        scale = np.abs(fd[i]).max()
        assert np.abs(got - fd[i]).max() <= GRAD_REL * scale, (r, got, fd[i])
    acc.close()


def test_backward_instances_full_size(gpu, orc):
    """1,024 frames, 8,388,608 secondary rays: forward and backward on all
    rays; 256 sampled hits against the oracle's adjoint at the same ids;
    per frame, the translation gradient equals minus the summed origin
    gradients of its rays, and the quaternion gradient is orthogonal to q."""
    torch, api, ctx = gpu
    W = wl.instanced_grids()
    scene = W.scene
    acc = to_gpu_scene(api, torch, ctx, scene)
    rays, hits, inst = _forward(gpu, acc, W.rays)
    h = hits.cpu().numpy()
    ii = inst.cpu().numpy().view(np.uint32)
    prim = h[:, 1].copy().view(np.uint32)
    hit = prim != NONE
    say("hit fraction", hit.mean())
    g = wl.rng_for(314).standard_normal((W.rays.shape[0], 3)).astype(np.float32)
    base = _bases(scene)
    dV, dS, do, dd = _backward(gpu, acc, rays, hits, inst, g, base[-1], 1024)
    cand = np.sort(wl.rng_for(315).choice(W.rays.shape[0], 400, replace=False))
    S = orc.OracleScene.from_scene(scene)
    A = orc.accept(S, W.rays[cand])
    check_closest(h[cand], A, inst=ii[cand], label="instanced sampled")
    # the adjoint is taken at the library's own hit ids (surface-leaving rays
    # are rarely pinned: their origin sits 1e-4 off a triangle)
    idx = cand[hit[cand]][:256]
    assert idx.size >= 200
    _, _, ro, rd = orc.adjoint_inst(S, W.rays[idx], ii[idx], prim[idx], g[idx].astype(np.float64))
    eo = np.linalg.norm(do[idx] - ro, axis=1) / np.linalg.norm(ro, axis=1)
    ed = np.linalg.norm(dd[idx] - rd, axis=1) / np.linalg.norm(rd, axis=1)
    say("sampled max rel err d_origin", eo.max(), "d_direction", ed.max())
    assert eo.max() <= GRAD_REL and ed.max() <= GRAD_REL
    # frame relations on all rays (float64 sums of the float32 ray gradients)
    sum_o = np.zeros((1024, 3))
    abs_o = np.zeros((1024, 3))
    cnt = np.bincount(ii[hit], minlength=1024).astype(np.float64)
    for c in range(3):
        sum_o[:, c] = np.bincount(ii[hit], weights=do[hit, c], minlength=1024)
        abs_o[:, c] = np.bincount(ii[hit], weights=np.abs(do[hit, c]), minlength=1024)
    bound = (cnt[:, None] + 2) * EPS32 * abs_o * 2 + 1e-9
    err = np.abs(dS[:, 7:10] + sum_o)
    say("translation relation err / bound", (err / bound).max())
    assert (err <= bound).all()
    q = scene.inst_srt[:, 3:7].astype(np.float64)
    radial = np.abs((q * dS[:, 3:7]).sum(1)) / np.linalg.norm(q, axis=1)
    assert (radial <= 1e-3 * np.linalg.norm(dS[:, 3:7], axis=1) + 1e-6).all()
    acc.close()


def test_instance_autograd_function(gpu, orc):
    """InstanceRayQueryFn: gradients of a masked loss equal the direct call's."""
    torch, api, ctx = gpu
    W = wl.aimed_instances(n_inst=8, n_rays=4096, k=316)
    scene = W.scene
    Vs = [torch.from_numpy(m.vertices).cuda() for m in scene.meshes]
    Is = [torch.from_numpy(m.indices.view(np.int32)).cuda() for m in scene.meshes]
    acc = api.Accel(ctx, list(zip(Vs, Is)), inst_mesh=scene.inst_mesh, inst_srt=scene.inst_srt)
    V = torch.cat(Vs).requires_grad_(True)
    srt = torch.from_numpy(scene.inst_srt.copy()).requires_grad_(True)
    rays = torch.from_numpy(W.rays).cuda()
    o = rays[:, 0:3].clone().requires_grad_(True)
    d = rays[:, 4:7].clone().requires_grad_(True)
    t, u, v, prim, ins = api.InstanceRayQueryFn.apply(acc, V, srt, o, d, 0.0, float("inf"))
    abc = torch.from_numpy(wl.rng_for(317).standard_normal((4096, 3)).astype(np.float32)).cuda()
    hit = prim >= 0
    assert int(hit.sum()) > 1500
    loss = (abc[hit, 0] * t[hit] + abc[hit, 1] * u[hit] + abc[hit, 2] * v[hit]).sum()
    loss.backward()
    hits, inst = api.trace_closest(acc, rays, want_inst=True)
    g = torch.zeros((4096, 3), dtype=torch.float32, device="cuda")
    g[hit] = abc[hit]
    dV = torch.zeros_like(V)
    dS = torch.zeros((8, 10), dtype=torch.float32, device="cuda")
    do, dd = api.trace_backward_instances(acc, rays, hits, inst, g.contiguous(), dV, dS)
    torch.cuda.synchronize()
    assert srt.grad.device.type == "cpu"
    assert torch.allclose(o.grad, do, rtol=1e-6, atol=1e-6)
    assert torch.allclose(d.grad, dd, rtol=1e-6, atol=1e-6)
    assert torch.allclose(V.grad, dV, rtol=1e-4, atol=1e-5)
    assert torch.allclose(srt.grad, dS.cpu(), rtol=1e-4, atol=1e-4)
    assert (ins[~hit] == -1).all()
    acc.close()


def test_backward_instances_errors(gpu):
    torch, api, ctx = gpu
    from paper_2603_00292_amd import _capi
    import ctypes as C

    W = wl.aimed_instances(n_inst=2, n_rays=16, k=318)
    acc = to_gpu_scene(api, torch, ctx, W.scene)
    rays, hits, inst = _forward(gpu, acc, W.rays)
    g = torch.zeros((16, 3), dtype=torch.float32, device="cuda")
    do = torch.empty((16, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(_capi.RtError) as e:
        _capi.call("rt_trace_backward_instances", acc.handle, C.c_void_p(rays.data_ptr()),
                   C.c_void_p(hits.data_ptr()), None, C.c_void_p(g.data_ptr()), 16, None, None,
                   C.c_void_p(do.data_ptr()), C.c_void_p(do.data_ptr()), None)
    assert e.value.status == _capi.RT_ERROR_INVALID_VALUE
    # n = 0 does nothing; no vertex or frame buffers is allowed
    api.trace_backward_instances(acc, rays[:0], hits[:0], inst[:0], g[:0])
    api.trace_backward_instances(acc, rays, hits, inst, g)
    # ids that are no instance contribute nothing
    bad = torch.full((16,), 7, dtype=torch.int32, device="cuda")
    dS = torch.zeros((2, 10), dtype=torch.float32, device="cuda")
    do2, dd2 = api.trace_backward_instances(acc, rays, hits, bad, torch.ones_like(g), None, dS)
    torch.cuda.synchronize()
    assert float(do2.abs().max()) == 0.0 and float(dS.abs().max()) == 0.0
    acc.close()
    # a single-level accel is refused
    m = W.scene.meshes[0]
    acc1 = api.Accel(ctx, [(torch.from_numpy(m.vertices).cuda(),
                            torch.from_numpy(m.indices.view(np.int32)).cuda())])
    with pytest.raises(_capi.RtError) as e:
        api.trace_backward_instances(acc1, rays, hits, inst, g)
    assert e.value.status == _capi.RT_ERROR_UNSUPPORTED
    acc1.close()


def test_backward_instances_deterministic(gpu):
    """Vertex and frame gradients are summed in a fixed order: repeated
    calls are bit-identical, and a call adds to what the buffers held."""
    torch, api, ctx = gpu
    W = wl.aimed_instances(n_inst=8, n_rays=32768, k=319)
    acc = to_gpu_scene(api, torch, ctx, W.scene)
    rays, hits, inst = _forward(gpu, acc, W.rays)
    g = torch.from_numpy(wl.rng_for(320).standard_normal((W.rays.shape[0], 3)).astype(np.float32)).cuda()
    nv = int(_bases(W.scene)[-1])
    outs = []
    for _ in range(2):
        dV = torch.zeros((nv, 3), dtype=torch.float32, device="cuda")
        dS = torch.zeros((8, 10), dtype=torch.float32, device="cuda")
        do, dd = api.trace_backward_instances(acc, rays, hits, inst, g, dV, dS)
        torch.cuda.synchronize()
        outs.append((dV, dS, do, dd))
    for a, b in zip(outs[0], outs[1]):
        assert torch.equal(a, b)
    dV, dS = outs[0][0].clone(), outs[0][1].clone()
    api.trace_backward_instances(acc, rays, hits, inst, g, dV, dS)
    torch.cuda.synchronize()
    assert torch.allclose(dV, 2 * outs[0][0], rtol=1e-6, atol=1e-7)
    assert torch.allclose(dS, 2 * outs[0][1], rtol=1e-6, atol=1e-7)
    # only frame gradients, only vertex gradients
    dS2 = torch.zeros((8, 10), dtype=torch.float32, device="cuda")
    api.trace_backward_instances(acc, rays, hits, inst, g, None, dS2)
    dV2 = torch.zeros((nv, 3), dtype=torch.float32, device="cuda")
    api.trace_backward_instances(acc, rays, hits, inst, g, dV2, None)
    torch.cuda.synchronize()
    assert torch.equal(dS2, outs[0][1]) and torch.equal(dV2, outs[0][0])
    acc.close()


def test_backward_instances_independent_of_ray_order(gpu):
    """The rays are grouped by triangle range and by instance and each group
    sums exactly: the vertex and frame gradients of a permutation of the
    rays are bit-identical (1,024 frames, 2^20 rays)."""
    torch, api, ctx = gpu
    W = wl.instanced_grids(n_rays=1 << 20, k=321)
    acc = to_gpu_scene(api, torch, ctx, W.scene)
    nv = int(_bases(W.scene)[-1])
    g = wl.rng_for(322).standard_normal((W.rays.shape[0], 3)).astype(np.float32)
    perm = wl.rng_for(323).permutation(W.rays.shape[0])
    res = []
    for order in (np.arange(W.rays.shape[0]), perm):
        rays, hits, inst = _forward(gpu, acc, W.rays[order])
        res.append(_backward(gpu, acc, rays, hits, inst, g[order], nv, 1024))
    (v0, s0, o0, d0), (v1, s1, o1, d1) = res
    assert np.array_equal(v0, v1) and np.array_equal(s0, s1)
    assert np.array_equal(o0[perm], o1) and np.array_equal(d0[perm], d1)
    acc.close()


def test_backward_instances_bucketed_matches_atomic_rows(gpu, monkeypatch):
    """The bucketed sums against the fixed-point atomic rows (the path for
    more instances than LDS counters, forced with RT_BACKWARD_ATOMIC=1 at
    context creation): ray gradients identical; frame and vertex gradients
    equal within two float32 roundings of their values (both are exact sums
    of the same float64 contributions, the vertex route rounds per corner
    to float64 first)."""
    torch, api, ctx = gpu
    W = wl.instanced_grids(n_rays=1 << 20, k=324)
    nv = int(_bases(W.scene)[-1])
    g = wl.rng_for(325).standard_normal((W.rays.shape[0], 3)).astype(np.float32)
    acc = to_gpu_scene(api, torch, ctx, W.scene)
    rays, hits, inst = _forward(gpu, acc, W.rays)
    a = _backward(gpu, acc, rays, hits, inst, g, nv, 1024)
    monkeypatch.setenv("RT_BACKWARD_ATOMIC", "1")
    ctx2 = api.Context(0)
    monkeypatch.delenv("RT_BACKWARD_ATOMIC")
    acc2 = to_gpu_scene(api, torch, ctx2, W.scene)
    b = _backward((torch, api, ctx2), acc2, rays, hits, inst, g, nv, 1024)
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])
    for x, y, name in ((a[0], b[0], "vertices"), (a[1], b[1], "frames")):
        tol = 2 * EPS32 * np.maximum(np.abs(x), np.abs(y)) + 1e-9 * np.abs(x).max()
        say(name, "identical entries", float((x == y).mean()), "max err/tol", float((np.abs(x - y) / tol).max()))
        assert (np.abs(x - y) <= tol).all()
    acc2.close()
    ctx2.close()
    acc.close()


def test_backward_instances_after_refit(gpu):
    """The two-level adjoint reads a copy of every triangle's object-space
    vertices; a refit makes the next call refresh it: gradients after moving
    the vertices equal those of a fresh accel built on them."""
    torch, api, ctx = gpu
    W = wl.aimed_instances(n_inst=8, n_rays=32768, k=326)
    acc = to_gpu_scene(api, torch, ctx, W.scene)
    nv = int(_bases(W.scene)[-1])
    g = wl.rng_for(327).standard_normal((W.rays.shape[0], 3)).astype(np.float32)
    rays, hits, inst = _forward(gpu, acc, W.rays)
    first = _backward(gpu, acc, rays, hits, inst, g, nv, 8)
    V = np.concatenate([m.vertices for m in W.scene.meshes]).copy()
    V[:, 1] += 0.05 * np.sin(3.0 * V[:, 0])
    acc.refit(torch.from_numpy(V).cuda())
    rays, hits, inst = _forward(gpu, acc, W.rays)
    moved = _backward(gpu, acc, rays, hits, inst, g, nv, 8)
    parts = np.split(V, _bases(W.scene)[1:-1])
    scene2 = wl.Scene([wl.Mesh(p.astype(np.float32), m.indices) for p, m in zip(parts, W.scene.meshes)],
                      W.scene.inst_mesh, W.scene.inst_srt)
    acc2 = to_gpu_scene(api, torch, ctx, scene2)
    rays2, hits2, inst2 = _forward(gpu, acc2, W.rays)
    assert torch.equal(hits.view(torch.int32), hits2.view(torch.int32)) and torch.equal(inst, inst2)
    fresh = _backward(gpu, acc2, rays2, hits2, inst2, g, nv, 8)
    for x, y in zip(moved, fresh):
        assert np.array_equal(x, y)
    assert not np.array_equal(moved[0], first[0])
    acc2.close()
    acc.close()


def test_backward_instances_many_instances(gpu):
    """More instances than LDS counters (20,000 > 16,384): the frame sums go
    through the fixed-point atomic rows.  Repeated calls are bit-identical
    and each frame's translation gradient is minus the sum of its rays'
    origin gradients."""
    torch, api, ctx = gpu
    J = 20000
    W = wl.aimed_instances(n_inst=J, n_rays=65536, k=328)
    acc = to_gpu_scene(api, torch, ctx, W.scene)
    rays, hits, inst = _forward(gpu, acc, W.rays)
    nv = int(_bases(W.scene)[-1])
    g = wl.rng_for(329).standard_normal((W.rays.shape[0], 3)).astype(np.float32)
    a = _backward(gpu, acc, rays, hits, inst, g, nv, J)
    b = _backward(gpu, acc, rays, hits, inst, g, nv, J)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    dV, dS, do, dd = a
    ii = inst.cpu().numpy().view(np.uint32)
    hit = hits.cpu().numpy()[:, 1].copy().view(np.uint32) != NONE
    say("hit fraction", hit.mean())
    assert hit.mean() > 0.5
    cnt = np.bincount(ii[hit], minlength=J).astype(np.float64)
    for c in range(3):
        s_o = np.bincount(ii[hit], weights=do[hit, c], minlength=J)
        a_o = np.bincount(ii[hit], weights=np.abs(do[hit, c]), minlength=J)
        bound = (cnt + 2) * EPS32 * a_o * 2 + 1e-9
        assert (np.abs(dS[:, 7 + c] + s_o) <= bound).all()
    acc.close()


def _large_two_level(rng, n_tri, n_rays):
    """Two soups of n_tri triangles each under four frames (scales 0.8-1.2,
    random rotations, translations 1.5 apart), rays from inside the scene."""
    half = 0.025 * np.sqrt(4096.0 / n_tri) * 4
    meshes = [wl.Mesh(*wl.random_triangle_soup(rng, n_tri, half)) for _ in range(2)]
    srt = np.zeros((4, 10), np.float64)
    srt[:, 0:3] = rng.uniform(0.8, 1.2, (4, 3))
    srt[:, 3:7] = wl.uniform_quaternions(rng, 4)
    srt[:, 7:10] = [[0.0, 0.0, 0.0], [1.5, 0.0, 0.0], [0.0, 1.5, 0.0], [1.5, 1.5, 0.0]]
    scene = wl.Scene(meshes, np.array([0, 1, 0, 1], np.uint32), srt.astype(np.float32))
    return scene, wl.box_rays(rng, n_rays, -0.5, 2.5)


def test_backward_instances_128_triangle_buckets(gpu, orc, monkeypatch):
    """More than 2^20 triangles over the meshes of a two-level scene, so the
    rays are grouped in buckets of 128 triangles (64 up to 2^20): every
    pinned hit's ray gradients and the vertex tensor against the oracle, and
    vertex and frame gradients against the fixed-point atomic rows within
    two float32 roundings."""
    torch, api, ctx = gpu
    scene, rays_np = _large_two_level(wl.rng_for(358), 600_000, 65536)
    acc = to_gpu_scene(api, torch, ctx, scene)
    rays, hits, inst = _forward(gpu, acc, rays_np)
    h = hits.cpu().numpy()
    ii = inst.cpu().numpy().view(np.uint32)
    S = orc.OracleScene.from_scene(scene, accel=True)
    A = orc.accept(S, rays_np)
    oinst, oprim, _ = orc.closest(S, rays_np)
    prim = h[:, 1].copy().view(np.uint32)
    keep = A.pinned & (oprim != NONE)
    assert (prim[keep] == oprim[keep]).all() and (ii[keep] == oinst[keep]).all()
    say("pinned hits", int(keep.sum()))
    assert keep.sum() > 10000
    g = wl.rng_for(359).standard_normal((rays_np.shape[0], 3)).astype(np.float32).astype(np.float64)
    g *= keep[:, None]
    nv = int(_bases(scene)[-1])
    dV, dS, do, dd = _backward(gpu, acc, rays, hits, inst, g, nv, 4)
    rV, rS, ro, rd = orc.adjoint_inst(S, rays_np, oinst, np.where(keep, oprim, NONE).astype(np.uint32), g)
    rV = np.concatenate(rV)
    r = np.flatnonzero(keep)
    eo = np.linalg.norm(do[r] - ro[r], axis=1) / np.linalg.norm(ro[r], axis=1)
    ed = np.linalg.norm(dd[r] - rd[r], axis=1) / np.linalg.norm(rd[r], axis=1)
    assert eo.max() <= GRAD_REL and ed.max() <= GRAD_REL
    fv = np.linalg.norm(dV - rV) / np.linalg.norm(rV)
    fs = np.linalg.norm(dS - rS) / np.linalg.norm(rS)
    say("Frobenius rel err: vertices", fv, "frames", fs)
    assert fv <= 1e-5 and fs <= 1e-5
    monkeypatch.setenv("RT_BACKWARD_ATOMIC", "1")
    ctx2 = api.Context(0)
    monkeypatch.delenv("RT_BACKWARD_ATOMIC")
    acc2 = to_gpu_scene(api, torch, ctx2, scene)
    b = _backward((torch, api, ctx2), acc2, rays, hits, inst, g, nv, 4)
    assert np.array_equal(do, b[2]) and np.array_equal(dd, b[3])
    for x, y, name in ((dV, b[0], "vertices"), (dS, b[1], "frames")):
        tol = 2 * EPS32 * np.maximum(np.abs(x), np.abs(y)) + 1e-9 * np.abs(x).max()
        say(name, "vs atomic rows: max err/tol", float((np.abs(x - y) / tol).max()))
        assert (np.abs(x - y) <= tol).all()
    acc2.close()
    ctx2.close()
    acc.close()
