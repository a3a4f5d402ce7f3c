"""GPU parity of the dynamic two-level paths.  rt_update_instances (new
frames; the top-level boxes refit over the kept topology, the meshes' trees
untouched) and rt_refit of a two-level accel (new vertices for every mesh;
their trees and the top level refit) must answer bit for bit like a fresh
build of the changed scene -- closest hits with instance ids, any-hit, masked
queries and the two-level adjoint -- for host and device builds, stay inside
the oracle's acceptable sets, and return to the first answers when the first
frames or vertices are restored."""
from __future__ import annotations

import numpy as np
import pytest

from helpers import check_closest, to_gpu_scene
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


def moved(srt, rng, shift):
    """New frames: translations moved by U[-shift, shift]^3, quaternions
    perturbed (the frame normalises them), scales multiplied by U[0.8, 1.25]."""
    new = srt.astype(np.float64).copy()
    new[:, 7:10] += rng.uniform(-shift, shift, size=(srt.shape[0], 3))
    new[:, 3:7] += rng.normal(0.0, 0.2, size=(srt.shape[0], 4))
    new[:, 0:3] *= rng.uniform(0.8, 1.25, size=(srt.shape[0], 3))
    return new.astype(np.float32)


def answers(torch, api, acc, rays, ray_masks, d_tuv):
    hits, inst = api.trace_closest(acc, rays, want_inst=True)
    occ = api.trace_any(acc, rays)
    hm, im = api.trace_closest_ex(acc, rays, ray_masks=ray_masks, want_inst=True)
    dv = torch.zeros((sum(acc.vertex_counts), 3), dtype=torch.float32, device=rays.device)
    ds = torch.zeros((acc.instance_count, 10), dtype=torch.float32, device=rays.device)
    do, dd = api.trace_backward_instances(acc, rays, hits, inst, d_tuv, dv, ds)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (hits, inst, occ, hm, im, do, dd, dv, ds)]


def same(a, b, label):
    for k, (x, y) in enumerate(zip(a, b)):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32)), f"{label}: output {k} differs"


@pytest.mark.parametrize("device_build", [False, True])
def test_update_matches_fresh_build(gpu, orc, device_build):
    torch, api, ctx = gpu
    W = wl.aimed_instances(n_inst=12, n_rays=8192, k=350)
    rng = wl.rng_for(351)
    rays = torch.from_numpy(W.rays).cuda()
    rmask = torch.from_numpy(rng.integers(0, 4, size=W.rays.shape[0]).astype(np.int32)).cuda()
    imask = rng.integers(1, 4, size=12).astype(np.uint32)
    d_tuv = torch.from_numpy(rng.standard_normal((W.rays.shape[0], 3)).astype(np.float32)).cuda()
    acc = to_gpu_scene(api, torch, ctx, W.scene, device_build=device_build)
    acc.set_instance_masks(imask)
    first = answers(torch, api, acc, rays, rmask, d_tuv)
    sah0 = acc.info["sah_cost"]
    srt1 = moved(W.scene.inst_srt, rng, 1.0)
    acc.update_instances(srt1)
    got = answers(torch, api, acc, rays, rmask, d_tuv)
    scene1 = wl.Scene(W.scene.meshes, W.scene.inst_mesh, srt1)
    fresh = to_gpu_scene(api, torch, ctx, scene1, device_build=device_build)
    fresh.set_instance_masks(imask)
    want = answers(torch, api, fresh, rays, rmask, d_tuv)
    say("device" if device_build else "host", "sah before", sah0, "after update", acc.info["sah_cost"],
        "fresh", fresh.info["sah_cost"])
    fresh.close()
    same(got, want, "update vs fresh build")
    S1 = orc.OracleScene.from_scene(scene1)
    st = check_closest(got[0], orc.accept(S1, W.rays), inst=got[1], label="moved instances")
    say(st)
    assert st["hits"] > 500
    # back to the first frames: the first answers again
    acc.update_instances(W.scene.inst_srt)
    same(answers(torch, api, acc, rays, rmask, d_tuv), first, "restored frames")
    acc.close()


def test_update_errors(gpu):
    torch, api, ctx = gpu
    from paper_2603_00292_amd import _capi
    import ctypes as C

    W = wl.aimed_instances(n_inst=4, n_rays=1024, k=352)
    rays = torch.from_numpy(W.rays).cuda()
    acc = to_gpu_scene(api, torch, ctx, W.scene)
    h0, i0 = api.trace_closest(acc, rays, want_inst=True)
    bad = W.scene.inst_srt.copy()
    bad[2, 1] = 0.0  # zero scale
    with pytest.raises(_capi.RtError) as e:
        acc.update_instances(bad)
    assert e.value.status == _capi.RT_ERROR_INVALID_VALUE
    bad = W.scene.inst_srt.copy()
    bad[1, 8] = np.nan
    with pytest.raises(_capi.RtError) as e:
        acc.update_instances(bad)
    assert e.value.status == _capi.RT_ERROR_INVALID_VALUE
    with pytest.raises(ValueError):
        acc.update_instances(W.scene.inst_srt[:3])
    with pytest.raises(_capi.RtError) as e:
        _capi.call("rt_update_instances", acc.handle, None, None)
    assert e.value.status == _capi.RT_ERROR_INVALID_VALUE
    # nothing changed by the rejected calls
    h1, i1 = api.trace_closest(acc, rays, want_inst=True)
    torch.cuda.synchronize()
    assert torch.equal(h0.view(torch.int32), h1.view(torch.int32)) and torch.equal(i0, i1)
    acc.close()
    m = W.scene.meshes[0]
    single = api.Accel(ctx, [(torch.from_numpy(m.vertices).cuda(), torch.from_numpy(m.indices.view(np.int32)).cuda())])
    srt = np.zeros((1, 10), np.float32)
    with pytest.raises(_capi.RtError) as e:
        _capi.call("rt_update_instances", single.handle, C.c_void_p(srt.ctypes.data), None)
    assert e.value.status == _capi.RT_ERROR_UNSUPPORTED
    single.close()


def test_update_instanced_workload(gpu):
    """The 1,024-instance workload with every instance moved: closest hits
    and instance ids of 2,097,152 of its rays equal a fresh build's."""
    torch, api, ctx = gpu
    W = wl.instanced_grids()
    rays = torch.from_numpy(W.rays[: 1 << 21]).cuda()
    acc = to_gpu_scene(api, torch, ctx, W.scene)
    srt1 = moved(W.scene.inst_srt, wl.rng_for(353), 0.5)
    acc.update_instances(srt1)
    h, i = api.trace_closest(acc, rays, want_inst=True)
    fresh = to_gpu_scene(api, torch, ctx, wl.Scene(W.scene.meshes, W.scene.inst_mesh, srt1))
    hf, if_ = api.trace_closest(fresh, rays, want_inst=True)
    torch.cuda.synchronize()
    hn = h.cpu().numpy()
    say("hit fraction", float((hn[:, 1].view(np.uint32) != 0xFFFFFFFF).mean()), "sah after update",
        acc.info["sah_cost"], "fresh", fresh.info["sah_cost"])
    assert torch.equal(h.view(torch.int32), hf.view(torch.int32)) and torch.equal(i, if_)
    acc.close()
    fresh.close()


@pytest.mark.parametrize("device_build", [False, True])
def test_two_level_refit_matches_fresh_build(gpu, orc, device_build):
    """New vertices for every mesh (heights and a shear changed; mesh 1
    collapsed to a point, so its triangles drop out) through rt_refit."""
    torch, api, ctx = gpu
    W = wl.aimed_instances(n_inst=12, n_rays=8192, k=354)
    rng = wl.rng_for(355)
    rays = torch.from_numpy(W.rays).cuda()
    rmask = torch.from_numpy(rng.integers(0, 4, size=W.rays.shape[0]).astype(np.int32)).cuda()
    imask = rng.integers(1, 4, size=12).astype(np.uint32)
    d_tuv = torch.from_numpy(rng.standard_normal((W.rays.shape[0], 3)).astype(np.float32)).cuda()
    acc = to_gpu_scene(api, torch, ctx, W.scene, device_build=device_build)
    acc.set_instance_masks(imask)
    first = answers(torch, api, acc, rays, rmask, d_tuv)
    new_meshes = []
    for k, m in enumerate(W.scene.meshes):
        v = m.vertices.astype(np.float64).copy()
        if k == 1:
            v[:] = v[0]
        else:
            v[:, 1] += 0.15 * np.sin(3.0 * v[:, 0]) + 0.1 * v[:, 2]
        new_meshes.append(wl.Mesh(v.astype(np.float32), m.indices))
    rows = torch.from_numpy(np.concatenate([m.vertices for m in new_meshes])).cuda()
    acc.refit(rows)
    got = answers(torch, api, acc, rays, rmask, d_tuv)
    scene1 = wl.Scene(new_meshes, W.scene.inst_mesh, W.scene.inst_srt)
    fresh = to_gpu_scene(api, torch, ctx, scene1, device_build=device_build)
    fresh.set_instance_masks(imask)
    want = answers(torch, api, fresh, rays, rmask, d_tuv)
    fresh.close()
    same(got[:5], want[:5], "refit vs fresh build (queries)")
    # the adjoint's vertex rows: mesh 1's triangles are absent in both
    same(got[5:], want[5:], "refit vs fresh build (adjoint)")
    S1 = orc.OracleScene.from_scene(scene1)
    st = check_closest(got[0], orc.accept(S1, W.rays), inst=got[1], label="refit two-level")
    say("device" if device_build else "host", st)
    assert st["hits"] > 500
    assert not np.isin(got[1][got[0][:, 1].view(np.uint32) != 0xFFFFFFFF],
                       np.flatnonzero(W.scene.inst_mesh == 1)).any()
    rows0 = torch.from_numpy(np.concatenate([m.vertices for m in W.scene.meshes])).cuda()
    acc.refit(rows0)
    same(answers(torch, api, acc, rays, rmask, d_tuv), first, "refit back")
    acc.close()
