"""rt_refit: fitting the boxes to moved vertices on the device, keeping the
topology, answers like a fresh build (and like the oracle) on the new
vertices; refitting back reproduces the original answers bit for bit."""
from __future__ import annotations

import numpy as np
import pytest

from helpers import NONE, check_closest
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


def _trace(api, torch, acc, rays):
    h, _ = api.trace_closest(acc, rays)
    torch.cuda.synchronize()
    return h.cpu().numpy()


def test_refit_matches_fresh_build_and_oracle(gpu, orc):
    torch, api, ctx = gpu
    W = wl.displaced_grid(nx=96, nz=48, n_rays=32768, k=700)
    m = W.scene.meshes[0]
    V0 = torch.from_numpy(m.vertices).cuda()
    I = torch.from_numpy(m.indices.view(np.int32)).cuda()
    rays = torch.from_numpy(W.rays).cuda()
    acc = api.Accel(ctx, [(V0, I)])
    h0 = _trace(api, torch, acc, rays)
    # move the vertices: new heights and a lateral shear
    rng = wl.rng_for(701)
    V1n = m.vertices.astype(np.float64).copy()
    V1n[:, 1] += rng.normal(0, 0.08, V1n.shape[0])
    V1n[:, 0] += 0.2 * np.sin(V1n[:, 2] / 7.0)
    V1n = V1n.astype(np.float32)
    V1 = torch.from_numpy(V1n).cuda()
    acc.refit(V1)
    h1 = _trace(api, torch, acc, rays)
    fresh = api.Accel(ctx, [(V1, I)])
    h1f = _trace(api, torch, fresh, rays)
    p1, pf = h1[:, 1].copy().view(np.uint32), h1f[:, 1].copy().view(np.uint32)
    same = p1 == pf
    say("refit vs fresh: same ids", same.mean())
    assert same.mean() > 0.9999
    assert np.array_equal(h1[same].view(np.uint32), h1f[same].view(np.uint32))
    scene1 = wl.Scene([wl.Mesh(V1n, m.indices)])
    S1 = orc.OracleScene.from_scene(scene1)
    check_closest(h1, orc.accept(S1, W.rays), label="refit")
    # refit back: same topology and boxes as the original build
    acc.refit(V0)
    h0b = _trace(api, torch, acc, rays)
    assert np.array_equal(h0.view(np.uint32), h0b.view(np.uint32))
    fresh.close()
    acc.close()


def test_refit_disables_and_restores_degenerate(gpu, orc):
    torch, api, ctx = gpu
    W = wl.random_triangles(n_tri=2048, n_rays=32768, k=702, half=0.05)
    m = W.scene.meshes[0]
    V0 = torch.from_numpy(m.vertices).cuda()
    I = torch.from_numpy(m.indices.view(np.int32)).cuda()
    rays = torch.from_numpy(W.rays).cuda()
    acc = api.Accel(ctx, [(V0, I)])
    h0 = _trace(api, torch, acc, rays)
    p0 = h0[:, 1].copy().view(np.uint32)
    hit_ids, counts = np.unique(p0[p0 != NONE], return_counts=True)
    victim = int(hit_ids[np.argmax(counts)])
    Vd = m.vertices.copy()
    tri = m.indices[victim]
    Vd[tri[1]] = Vd[tri[0]]          # two equal vertices: zero normal (the soup has
                                     # no shared vertices, so no other triangle moves)
    acc.refit(torch.from_numpy(Vd).cuda())
    hd = _trace(api, torch, acc, rays)
    assert not (hd[:, 1].copy().view(np.uint32) == victim).any()
    S = orc.OracleScene([(Vd, m.indices)])
    check_closest(hd, orc.accept(S, W.rays), label="degenerate after refit")
    acc.refit(V0)
    assert np.array_equal(_trace(api, torch, acc, rays).view(np.uint32), h0.view(np.uint32))
    acc.close()


def test_backward_after_refit(gpu):
    torch, api, ctx = gpu
    W = wl.displaced_grid(nx=32, nz=16, n_rays=4096, k=703)
    m = W.scene.meshes[0]
    I = torch.from_numpy(m.indices.view(np.int32)).cuda()
    V0 = torch.from_numpy(m.vertices).cuda()
    V1n = m.vertices.copy()
    V1n[:, 1] += np.float32(0.05)
    V1 = torch.from_numpy(V1n).cuda()
    rays = torch.from_numpy(W.rays).cuda()
    g = torch.from_numpy(W.extra["abc"]).cuda()
    acc = api.Accel(ctx, [(V0, I)])
    acc.refit(V1)
    fresh = api.Accel(ctx, [(V1, I)])
    outs = []
    for a in (acc, fresh):
        h, _ = api.trace_closest(a, rays)
        dV = torch.zeros_like(V1)
        do, dd = api.trace_backward(a, rays, h, g, dV)
        torch.cuda.synchronize()
        outs.append((h.cpu().numpy(), do.cpu().numpy(), dd.cpu().numpy(), dV.cpu().numpy()))
    (h1, o1, d1, v1), (h2, o2, d2, v2) = outs
    assert np.array_equal(h1[:, 1].view(np.uint32), h2[:, 1].view(np.uint32))
    assert np.array_equal(o1, o2) and np.array_equal(d1, d2)
    assert np.allclose(v1, v2, rtol=1e-5, atol=1e-6)
    acc.close()
    fresh.close()


def test_refit_errors(gpu):
    torch, api, ctx = gpu
    from paper_2603_00292_amd import _capi

    W = wl.random_triangles(n_tri=64, n_rays=8, k=704, half=0.2)
    m = W.scene.meshes[0]
    V = torch.from_numpy(m.vertices).cuda()
    I = torch.from_numpy(m.indices.view(np.int32)).cuda()
    acc = api.Accel(ctx, [(V, I)], inst_mesh=np.zeros(1, np.uint32),
                    inst_srt=np.array([[1, 1, 1, 0, 0, 0, 1, 0, 0, 0]], np.float32))
    acc.refit(V)  # a two-level accel takes its meshes' rows one after another
    with pytest.raises(_capi.RtError) as e:
        _capi.call("rt_refit", acc.handle, None, None)
    assert e.value.status == _capi.RT_ERROR_INVALID_VALUE
    with pytest.raises(ValueError):
        acc.refit(torch.cat([V, V]))
    acc.close()
    acc = api.Accel(ctx, [(V, I)])
    with pytest.raises(ValueError):
        acc.refit(V[:-1].contiguous())
    acc.close()
