"""GPU parity of the query variants: all-hit lists (rt_trace_all), ray masks
against instance masks and the self-intersection filter
(rt_trace_closest_ex / rt_trace_any_ex), against the oracle's all-hit
candidates and acceptable sets computed with the same options."""
from __future__ import annotations

import numpy as np
import pytest

from helpers import NONE, check_all, check_any, check_closest, to_gpu_scene
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


def _t(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _all(gpu, acc, rays, cap, **opt):
    torch, api, _ = gpu
    h, i, c = api.trace_all(acc, _t(torch, rays), cap, want_inst=True, **opt)
    torch.cuda.synchronize()
    return h.cpu().numpy(), i.cpu().numpy().view(np.uint32), c.cpu().numpy()


def test_all_hits_stack_closed_form(gpu, orc):
    """Seven triangles in the planes z = 1..7 (shuffled ids), rays up the z
    axis: counts, ids in t order and t = z exactly, u = v = 3/8."""
    torch, api, ctx = gpu
    order = np.random.default_rng(5).permutation(7)
    V, I = [], []
    for slot, z in enumerate(order + 1):
        V += [[-4, -4, z], [4, -4, z], [-4, 4, z]]
        I.append([3 * slot, 3 * slot + 1, 3 * slot + 2])
    scene = wl.Scene([wl.Mesh(np.array(V, np.float32), np.array(I, np.uint32))])
    rays = np.array([[-1, -1, 0, 0, 0, 0, 1, np.inf],
                     [-1, -1, 0, 0, 0, 0, 1, 4.5],
                     [-1, -1, 0, 2, 0, 0, 1, np.inf],
                     [-1, -1, 0, 3, 0, 0, 1, 3.0],
                     [-1, -1, 10, 0, 0, 0, 1, np.inf]], np.float32)
    acc = to_gpu_scene(api, torch, ctx, scene)
    for cap in (8, 3):
        h, ii, c = _all(gpu, acc, rays, cap)
        assert c.tolist() == [7, 4, 6, 1, 0]
        slot_of_z = {int(z): s for s, z in enumerate(order + 1)}
        k = min(7, cap)
        assert h[0, :k, 1].copy().view(np.uint32).tolist() == [slot_of_z[z] for z in range(1, k + 1)]
        assert h[0, :k, 0].tolist() == list(range(1, k + 1))
        assert (h[0, :k, 2:] == 0.375).all() and (ii[0, :k] == 0).all()
        assert (h[4, :, 1].copy().view(np.uint32) == NONE).all() and (ii[4] == NONE).all()
    acc.close()


@pytest.mark.parametrize("width", [4, 2, 8])
def test_all_hits_dense_soup(gpu, orc, width):
    """3,001 random triangles, several layers deep; 20,011 rays (ragged);
    lists of 8 against the oracle's candidates; the first entry equals the
    closest-hit query bit for bit."""
    torch, api, ctx = gpu
    rng = wl.rng_for(220)
    V, I = wl.random_triangle_soup(rng, 3001, 0.08)
    rays = wl.box_rays(rng, 20011, 0.0, 1.0)
    scene = wl.Scene([wl.Mesh(V, I)])
    acc = to_gpu_scene(api, torch, ctx, scene, node_width=width)
    h, ii, c = _all(gpu, acc, rays, 8)
    S = orc.OracleScene.from_scene(scene)
    C = orc.classify_all(S, rays, 64)
    st = check_all(h, ii, c, C, label=f"all W={width}")
    say(st)
    assert st["max_count"] > 8 and (c > 8).sum() > 100
    hc, _ = api.trace_closest(acc, _t(torch, rays))
    hc = hc.cpu().numpy()
    assert np.array_equal(hc.view(np.uint32), h[:, 0].view(np.uint32))
    acc.close()


def test_all_hits_instances(gpu, orc):
    torch, api, ctx = gpu
    W = wl.aimed_instances(n_inst=8, n_rays=8192, k=221)
    acc = to_gpu_scene(api, torch, ctx, W.scene)
    h, ii, c = _all(gpu, acc, W.rays, 4)
    S = orc.OracleScene.from_scene(W.scene)
    C = orc.classify_all(S, W.rays, 64)
    st = check_all(h, ii, c, C, label="all instances")
    say(st)
    assert (c >= 2).sum() > 500
    hc, ic = api.trace_closest(acc, _t(torch, W.rays), want_inst=True)
    hc = hc.cpu().numpy()
    assert np.array_equal(hc.view(np.uint32), h[:, 0].view(np.uint32))
    assert np.array_equal(ic.cpu().numpy().view(np.uint32), ii[:, 0])
    acc.close()


def test_masks_two_level(gpu, orc):
    """Instance j has mask bit (j mod 4); random 4-bit ray masks: closest,
    any and all-hit queries against the oracle with the same masks."""
    torch, api, ctx = gpu
    W = wl.aimed_instances(n_inst=8, n_rays=8192, k=222)
    n = W.rays.shape[0]
    inst_mask = (1 << (np.arange(8) % 4)).astype(np.uint32)
    ray_mask = wl.rng_for(223).integers(0, 16, n).astype(np.uint32)
    acc = to_gpu_scene(api, torch, ctx, W.scene)
    rays = _t(torch, W.rays)
    plain, _ = api.trace_closest(acc, rays)
    # all-ones masks change nothing
    ones, _ = api.trace_closest_ex(acc, rays, ray_masks=_t(torch, np.full(n, 0xFFFFFFFF, np.uint32).view(np.int32)))
    assert torch.equal(plain.view(torch.int32), ones.view(torch.int32))
    acc.set_instance_masks(inst_mask)
    rm = _t(torch, ray_mask.view(np.int32))
    h, ii = api.trace_closest_ex(acc, rays, ray_masks=rm, want_inst=True)
    occ = api.trace_any_ex(acc, rays, ray_masks=rm)
    ha, ia, ca = api.trace_all(acc, rays, 4, ray_masks=rm, want_inst=True)
    torch.cuda.synchronize()
    S = orc.OracleScene.from_scene(W.scene)
    opts = orc.Opts(inst_mask=inst_mask, ray_mask=ray_mask)
    A = orc.accept(S, W.rays, opts=opts)
    st = check_closest(h.cpu().numpy(), A, inst=ii.cpu().numpy().view(np.uint32), label="masked closest")
    check_any(occ.cpu().numpy(), A, label="masked any")
    C = orc.classify_all(S, W.rays, 64, opts=opts)
    check_all(ha.cpu().numpy(), ia.cpu().numpy().view(np.uint32), ca.cpu().numpy(), C, label="masked all")
    say(st)
    assert st["hits"] > 1000
    none = ray_mask == 0
    assert (h.cpu().numpy()[none, 1].view(np.uint32) == NONE).all()
    # restoring all-ones instance masks restores the plain answers
    acc.set_instance_masks(np.full(8, 0xFFFFFFFF, np.uint32))
    again, _ = api.trace_closest_ex(acc, rays, ray_masks=_t(torch, np.full(n, 1, np.int32)))
    assert torch.equal(plain.view(torch.int32), again.view(torch.int32))
    acc.close()


def test_skip_filter_surface_rays(gpu, orc):
    """Secondary rays leaving instanced surfaces skip their source triangle:
    every ray against the oracle with the same filter; the filter turns the
    source triangle from a 'maybe' into no candidate, so most rays are
    pinned (93% of them here, against 6% without it)."""
    torch, api, ctx = gpu
    W = wl.instanced_grids(n_inst=64, n_rays=8192, k=401)
    si, sp = W.extra["src_inst"], W.extra["src_prim"]
    acc = to_gpu_scene(api, torch, ctx, W.scene)
    rays = _t(torch, W.rays)
    ski, skp = _t(torch, si.view(np.int32)), _t(torch, sp.view(np.int32))
    h, ii = api.trace_closest_ex(acc, rays, skip_inst=ski, skip_prim=skp, want_inst=True)
    occ = api.trace_any_ex(acc, rays, skip_inst=ski, skip_prim=skp)
    torch.cuda.synchronize()
    S = orc.OracleScene.from_scene(W.scene)
    opts = orc.Opts(skip_inst=si, skip_prim=sp)
    A = orc.accept(S, W.rays, opts=opts)
    hn, iin = h.cpu().numpy(), ii.cpu().numpy().view(np.uint32)
    st = check_closest(hn, A, inst=iin, label="filtered surface rays")
    check_any(occ.cpu().numpy(), A, label="filtered surface any")
    say(st)
    assert st["pinned_frac"] > 0.9
    src_hit = (hn[:, 1].copy().view(np.uint32) == sp) & (iin == si)
    assert not src_hit.any()
    acc.close()


def test_skip_closest_gives_second_entry(gpu):
    """Skipping each ray's closest hit returns the second entry of its
    all-hit list, bit for bit (single level and two-level)."""
    torch, api, ctx = gpu
    rng = wl.rng_for(224)
    V, I = wl.random_triangle_soup(rng, 3001, 0.08)
    soup = (wl.Scene([wl.Mesh(V, I)]), wl.box_rays(rng, 16384, 0.0, 1.0))
    Wi = wl.aimed_instances(n_inst=8, n_rays=8192, k=225)
    for scene, rays_np in (soup, (Wi.scene, Wi.rays)):
        acc = to_gpu_scene(api, torch, ctx, scene)
        rays = _t(torch, rays_np)
        ha, ia, ca = api.trace_all(acc, rays, 2, want_inst=True)
        first_p = ha[:, 0, 1].contiguous().view(torch.int32)
        first_i = ia[:, 0].contiguous()
        h2, i2 = api.trace_closest_ex(acc, rays, skip_inst=first_i, skip_prim=first_p, want_inst=True)
        torch.cuda.synchronize()
        assert torch.equal(h2.view(torch.int32), ha[:, 1].contiguous().view(torch.int32))
        two = ca >= 2
        assert int(two.sum()) > 1000
        if scene.inst_mesh is not None:
            assert torch.equal(i2[two], ia[two, 1])
        acc.close()


def test_query_errors(gpu):
    torch, api, ctx = gpu
    from paper_2603_00292_amd import _capi

    W = wl.aimed_instances(n_inst=2, n_rays=64, k=226)
    acc = to_gpu_scene(api, torch, ctx, W.scene)
    rays = _t(torch, W.rays)
    for cap in (0, 65):
        with pytest.raises(_capi.RtError) as e:
            api.trace_all(acc, rays, cap)
        assert e.value.status == _capi.RT_ERROR_INVALID_VALUE
    with pytest.raises(_capi.RtError) as e:
        api.trace_closest_ex(acc, rays, skip_prim=torch.zeros(64, dtype=torch.int32, device="cuda"))
    assert e.value.status == _capi.RT_ERROR_INVALID_VALUE
    h, i, c = api.trace_all(acc, rays[:0], 4)
    assert h.shape == (0, 4, 4)
    acc.close()
    m = W.scene.meshes[0]
    single = api.Accel(ctx, [(torch.from_numpy(m.vertices).cuda(),
                              torch.from_numpy(m.indices.view(np.int32)).cuda())])
    with pytest.raises(_capi.RtError) as e:
        single.set_instance_masks(np.zeros(0, np.uint32))
    assert e.value.status in (_capi.RT_ERROR_UNSUPPORTED,)
    zero = torch.zeros(64, dtype=torch.int32, device="cuda")
    h, _ = api.trace_closest_ex(single, rays, ray_masks=zero)
    occ = api.trace_any_ex(single, rays, ray_masks=zero)
    torch.cuda.synchronize()
    assert (h[:, 1].contiguous().view(torch.int32) == -1).all() and int(occ.sum()) == 0
    single.close()
