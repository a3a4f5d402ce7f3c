"""GPU parity of two-level (instanced) scenes against the oracle."""
from __future__ import annotations

import numpy as np
import pytest

from helpers import NONE, check_any, check_closest, to_gpu_scene
from paper_2603_00292_amd import workloads as wl

pytestmark = pytest.mark.gpu


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


def trace(gpu, acc, rays):
    torch, api, _ = gpu
    r = torch.from_numpy(np.ascontiguousarray(rays)).cuda()
    hits, inst = api.trace_closest(acc, r, want_inst=True)
    occ = api.trace_any(acc, r)
    torch.cuda.synchronize()
    return hits.cpu().numpy(), inst.cpu().numpy().view(np.uint32), occ.cpu().numpy()


def test_identity_instance_bit_exact(gpu):
    """One identity instance answers exactly like the single-level accel."""
    torch, api, ctx = gpu
    W = wl.random_triangles(n_tri=4096, n_rays=65536, k=400, half=0.05)
    single = to_gpu_scene(api, torch, ctx, W.scene)
    scene2 = wl.Scene(W.scene.meshes, np.zeros(1, np.uint32),
                      np.array([[1, 1, 1, 0, 0, 0, 1, 0, 0, 0]], np.float32))
    two = to_gpu_scene(api, torch, ctx, scene2)
    h1, _, o1 = trace(gpu, single, W.rays)
    h2, i2, o2 = trace(gpu, two, W.rays)
    assert np.array_equal(h1.view(np.uint32), h2.view(np.uint32))
    assert np.array_equal(o1, o2)
    hit = h1[:, 1].copy().view(np.uint32) != NONE
    assert (i2[hit] == 0).all() and (i2[~hit] == NONE).all()
    single.close()
    two.close()


def test_instanced_small_all_rays(gpu, orc):
    """64 instances of the four displaced grids, 8,192 surface rays: every
    ray (instance and triangle ids, t, u, v) against the oracle.  These rays
    start 1e-4 off a surface at world coordinates up to ~40, where the float32
    world-to-object transform carries a comparable rounding, so the ray's own
    source triangle is a legitimate "maybe" for most rays: membership in the
    acceptable set is checked for all, and agreement with the oracle's own
    answer is required on at least 98% of the rays."""
    torch, api, ctx = gpu
    W = wl.instanced_grids(n_inst=64, n_rays=8192, k=401)
    acc = to_gpu_scene(api, torch, ctx, W.scene)
    say(acc.info)
    h, inst, occ = trace(gpu, acc, W.rays)
    S = orc.OracleScene.from_scene(W.scene)
    A = orc.accept(S, W.rays)
    st = check_closest(h, A, inst=inst, label="instanced small")
    check_any(occ, A, label="instanced small any")
    oi, op, _ = orc.closest(S, W.rays)
    prim = h[:, 1].copy().view(np.uint32)
    agree = ((prim == op) & ((inst == oi) | (op == NONE))).mean()
    say(st, "agreement with the oracle's answer", agree)
    assert agree >= 0.98
    acc.close()


def test_instanced_aimed_rays(gpu, orc):
    """64 instances; 16,384 rays from random points of the scene box aimed at
    random instances: every ray against the oracle.  The acceptable sets
    widen instance hits by 16 float32 ulps of |o| + |T| in object units (up
    to ~1e-4 here, on 0.02-wide triangles), so 93.6% of these rays have a
    single acceptable answer (checked bit-exactly); agreement with the
    oracle's own answer is checked on all rays."""
    torch, api, ctx = gpu
    W = wl.instanced_grids(n_inst=64, n_rays=16, k=401)
    rng = wl.rng_for(408)
    n = 16384
    o = rng.uniform(-25, 25, size=(n, 3))
    tgt = W.scene.inst_srt[rng.integers(0, 64, n), 7:10].astype(np.float64) + rng.uniform(-1, 1, (n, 3))
    d = tgt - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays = wl.pack_rays(o, d)
    acc = to_gpu_scene(api, torch, ctx, W.scene)
    h, inst, occ = trace(gpu, acc, rays)
    S = orc.OracleScene.from_scene(W.scene)
    A = orc.accept(S, rays)
    st = check_closest(h, A, inst=inst, label="instanced aimed")
    check_any(occ, A, label="instanced aimed any")
    oi, op, _ = orc.closest(S, rays)
    prim = h[:, 1].copy().view(np.uint32)
    agree = ((prim == op) & ((inst == oi) | (op == NONE))).mean()
    say(st, "agreement with the oracle's answer", agree)
    assert st["hits"] > 2000 and st["pinned_frac"] > 0.93
    assert agree > 0.995
    acc.close()


def test_instanced_full_size_sampled(gpu, orc):
    """1,024 SRT instances (10,240,000 instanced triangles), 8,388,608
    secondary rays on the GPU; 256 sampled rays against the oracle."""
    torch, api, ctx = gpu
    W = wl.instanced_grids()
    acc = to_gpu_scene(api, torch, ctx, W.scene)
    say(acc.info)
    h, inst, occ = trace(gpu, acc, W.rays)
    prim = h[:, 1].copy().view(np.uint32)
    say("hit fraction", (prim != NONE).mean())
    idx = np.sort(wl.rng_for(402).choice(W.rays.shape[0], 256, replace=False))
    S = orc.OracleScene.from_scene(W.scene)
    A = orc.accept(S, W.rays[idx])
    st = check_closest(h[idx], A, inst=inst[idx], label="instanced sampled")
    check_any(occ[idx], A, label="instanced any sampled")
    say(st)
    assert np.array_equal(occ.astype(bool), prim != NONE)
    acc.close()


def test_instance_transform_kinds(gpu, orc):
    """Translation-only, rotation-only, anisotropic scale and a mirror
    (negative scale) instance, all rays against the oracle."""
    torch, api, ctx = gpu
    W = wl.random_triangles(n_tri=2048, n_rays=32768, k=403, half=0.05)
    q = wl.uniform_quaternions(wl.rng_for(404), 1)[0]
    srt = np.array([
        [1, 1, 1, 0, 0, 0, 1, 3.0, -2.0, 0.5],
        [1, 1, 1, q[0], q[1], q[2], q[3], 0, 0, 0],
        [0.5, 2.0, 1.5, 0, 0, 0, 1, -3, 0, 0],
        [-1, 1, 1, 0, 0, 0, 1, 0, 3, 0],
        [1, 1, 1, 0, 0, 0, 2, 0, 0, -3],     # unnormalised quaternion
    ], np.float32)
    scene = wl.Scene(W.scene.meshes, np.zeros(len(srt), np.uint32), srt)
    rng = wl.rng_for(405)
    rays = wl.box_rays(rng, 32768, -4, 4)
    acc = to_gpu_scene(api, torch, ctx, scene)
    h, inst, occ = trace(gpu, acc, rays)
    S = orc.OracleScene.from_scene(scene)
    A = orc.accept(S, rays)
    st = check_closest(h, A, inst=inst, label="transform kinds")
    check_any(occ, A, label="transform kinds any")
    say(st)
    acc.close()


def test_counters_two_level(gpu):
    """The counting variants on a two-level accel (node visits of both
    levels, triangle tests) give the same hits as the plain query, and counts
    that bound the work: at least one node per ray that enters the top level."""
    torch, api, ctx = gpu
    W = wl.instanced_grids(n_inst=64, n_rays=8192, k=402)
    acc = to_gpu_scene(api, torch, ctx, W.scene)
    rays = torch.from_numpy(W.rays).cuda()
    h, _ = api.trace_closest(acc, rays, want_inst=True)
    occ = api.trace_any(acc, rays)
    (nodes, tris, spills), hc = api.trace_counters(acc, rays)
    (nodes_a, tris_a, _), oc = api.trace_counters(acc, rays, any_hit=True)
    torch.cuda.synchronize()
    assert torch.equal(h.view(torch.int32), hc.view(torch.int32))
    assert torch.equal(occ, oc)
    n = rays.shape[0]
    say("two-level counters per ray: closest", nodes / n, tris / n, spills / n, "any", nodes_a / n, tris_a / n)
    assert nodes >= n and tris > 0 and nodes_a <= nodes and tris_a <= tris
    acc.close()


def test_build_argument_errors(gpu):
    torch, api, ctx = gpu
    from paper_2603_00292_amd import _capi

    W = wl.random_triangles(n_tri=64, n_rays=16, k=406, half=0.2)
    m = W.scene.meshes[0]
    V = torch.from_numpy(m.vertices).cuda()
    I = torch.from_numpy(m.indices.view(np.int32)).cuda()
    bad = [
        (np.array([1], np.uint32), np.array([[1, 1, 1, 0, 0, 0, 1, 0, 0, 0]], np.float32), _capi.RT_ERROR_INDEX_OUT_OF_RANGE),
        (np.array([0], np.uint32), np.array([[0, 1, 1, 0, 0, 0, 1, 0, 0, 0]], np.float32), _capi.RT_ERROR_INVALID_VALUE),
        (np.array([0], np.uint32), np.array([[1, 1, 1, 0, 0, 0, 0, 0, 0, 0]], np.float32), _capi.RT_ERROR_INVALID_VALUE),
        (np.array([0], np.uint32), np.array([[1, np.inf, 1, 0, 0, 0, 1, 0, 0, 0]], np.float32), _capi.RT_ERROR_INVALID_VALUE),
    ]
    for im, srt, code in bad:
        with pytest.raises(_capi.RtError) as e:
            api.Accel(ctx, [(V, I)], im, srt)
        assert e.value.status == code
    I2 = I.clone()
    I2[3, 1] = m.vertices.shape[0]
    with pytest.raises(_capi.RtError) as e:
        api.Accel(ctx, [(V, I2)])
    assert e.value.status == _capi.RT_ERROR_INDEX_OUT_OF_RANGE
    for opts in ({"node_width": 3}, {"max_leaf_size": 16}):
        with pytest.raises(_capi.RtError) as e:
            api.Accel(ctx, [(V, I)], **opts)
        assert e.value.status == _capi.RT_ERROR_INVALID_VALUE
