"""Batched plans: one persistent launch (and its HIP graph) over many meshes
equals separate per-mesh launches bit for bit, and matches the oracle."""
from __future__ import annotations

import numpy as np
import pytest

from helpers import check_chunked, check_closest, to_gpu_scene
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


def _setup(gpu, works):
    torch, api, ctx = gpu
    accs = [to_gpu_scene(api, torch, ctx, w.scene) for w in works]
    rays = [torch.from_numpy(w.rays).cuda() for w in works]
    return accs, rays


def _per_mesh(gpu, accs, rays):
    torch, api, _ = gpu
    out = [api.trace_closest(a, r)[0] for a, r in zip(accs, rays)]
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out]


def _check_equal(batched, per):
    for b, p in zip(batched, per):
        assert np.array_equal(b.view(np.uint32), p.view(np.uint32))


def test_batched_small_uneven(gpu, orc):
    """Twelve meshes (0 to 60k triangles) with uneven ray counts, including
    empty batches: plan launch and graph replays equal per-mesh launches."""
    torch, api, ctx = gpu
    rng = wl.rng_for(500)
    works = []
    for m, (nt, nr) in enumerate([(1000, 1), (60000, 50000), (0, 100), (5000, 0), (2000, 7777),
                                  (30000, 64), (1, 65), (12345, 30000), (800, 1000), (40000, 3),
                                  (7000, 20000), (3, 1)]):
        half = 0.025 * np.sqrt(4096.0 / max(nt, 1))
        V, I = wl.random_triangle_soup(rng, nt, half)
        works.append(wl.Workload(f"b{m}", wl.Scene([wl.Mesh(V, I)]), wl.box_rays(rng, nr, -1, 2)))
    accs, rays = _setup(gpu, works)
    per = _per_mesh(gpu, accs, rays)
    plan = api.BatchPlan(ctx, accs, rays)
    plan.launch()
    torch.cuda.synchronize()
    _check_equal([h.cpu().numpy() for h in plan.hits], per)
    # graph: capture once, replay several times with eager work in between
    s = torch.cuda.Stream()
    g = plan.graph_exec(s)
    for rep in range(3):
        for h in plan.hits:
            h.fill_(-1.0)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            api.graph_launch(g, s)
        s.synchronize()
        _check_equal([h.cpu().numpy() for h in plan.hits], per)
        _ = (rays[1] * 2).sum().item()  # unrelated eager work between replays
    # oracle on a few batches
    for b in (1, 4, 7, 10):
        if works[b].rays.shape[0] == 0:
            continue
        k = min(256, works[b].rays.shape[0])
        S = orc.OracleScene.from_scene(works[b].scene)
        check_closest(per[b][:k], orc.accept(S, works[b].rays[:k]), label=f"batch {b}")
    plan.close()
    for a in accs:
        a.close()


def test_batched_full_size(gpu, orc):
    """256 meshes with log-uniform triangle (1k-500k) and ray (1k-1M) counts,
    all traced in one persistent launch (its HIP graph) and by 256 per-mesh
    launches: every ray compared bit for bit, and every ray of every mesh
    (35,362,456) checked against the oracle's acceptable sets."""
    torch, api, ctx = gpu
    works = wl.batched_meshes()
    say("triangles", sum(w.scene.meshes[0].n_tri for w in works), "rays", sum(w.rays.shape[0] for w in works))
    accs, rays = _setup(gpu, works)
    per = _per_mesh(gpu, accs, rays)
    plan = api.BatchPlan(ctx, accs, rays)
    s = torch.cuda.Stream()
    g = plan.graph_exec(s)
    with torch.cuda.stream(s):
        api.graph_launch(g, s)
    s.synchronize()
    batched = [h.cpu().numpy() for h in plan.hits]
    _check_equal(batched, per)
    plan.close()
    for a in accs:
        a.close()
    del rays, per
    total = pinned = 0
    for b, w in enumerate(works):
        S = orc.OracleScene.from_scene(w.scene, accel=True)
        st = check_chunked(orc, S, w.rays, hits=batched[b], label=f"batch {b}")
        total += st.get("rays", 0)
        pinned += round(st.get("pinned_frac", 0.0) * st.get("rays", 0))
        if b % 32 == 31:
            say(f"oracle checked meshes 0..{b}: {total} rays, pinned {pinned / max(total, 1):.5f}")
    assert total == sum(w.rays.shape[0] for w in works)


def test_batched_two_level(gpu, orc):
    """A plan over five two-level scenes (instanced displaced grids and aimed
    instances of different sizes, one batch without rays): the batched launch
    and its graph replays equal per-accel closest-hit queries bit for bit,
    instance ids included, and a sample matches the oracle."""
    torch, api, ctx = gpu
    from paper_2603_00292_amd import _capi

    works = [wl.instanced_grids(n_inst=64, n_rays=50000, k=510),
             wl.aimed_instances(n_inst=8, n_rays=20000, k=511),
             wl.instanced_grids(n_inst=16, n_rays=0, k=512),
             wl.instanced_grids(n_inst=200, n_rays=120000, k=513),
             wl.aimed_instances(n_inst=30, n_rays=7777, k=514)]
    accs, rays = _setup(gpu, works)
    per = [api.trace_closest(a, r, want_inst=True) for a, r in zip(accs, rays)]
    torch.cuda.synchronize()
    per_h = [h.cpu().numpy() for h, _ in per]
    per_i = [i.cpu().numpy() for _, i in per]
    plan = api.BatchPlan(ctx, accs, rays, want_inst=True)
    plan.launch()
    torch.cuda.synchronize()
    _check_equal([h.cpu().numpy() for h in plan.hits], per_h)
    _check_equal([i.cpu().numpy() for i in plan.inst_ids], per_i)
    s = torch.cuda.Stream()
    g = plan.graph_exec(s)
    for rep in range(3):
        for h in plan.hits:
            h.zero_()
        for i in plan.inst_ids:
            i.fill_(-7)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            api.graph_launch(g, s)
        s.synchronize()
        _check_equal([h.cpu().numpy() for h in plan.hits], per_h)
        _check_equal([i.cpu().numpy() for i in plan.inst_ids], per_i)
    plan.close()
    # without instance ids
    plan2 = api.BatchPlan(ctx, accs, rays)
    plan2.launch()
    torch.cuda.synchronize()
    _check_equal([h.cpu().numpy() for h in plan2.hits], per_h)
    plan2.close()
    rng = wl.rng_for(515)
    for b in (0, 3, 4):
        idx = np.sort(rng.choice(works[b].rays.shape[0], 64, replace=False))
        S = orc.OracleScene.from_scene(works[b].scene)
        check_closest(per_h[b][idx], orc.accept(S, works[b].rays[idx]), inst=per_i[b][idx], label=f"batch {b}")
    # a plan mixing single-level and two-level accels, or asking for
    # instance ids of a single-level accel, is refused
    m = works[0].scene.meshes[0]
    single = api.Accel(ctx, [(torch.from_numpy(m.vertices).cuda(), torch.from_numpy(m.indices.view(np.int32)).cuda())])
    with pytest.raises(_capi.RtError) as e:
        api.BatchPlan(ctx, [accs[0], single], [rays[0], rays[1]])
    assert e.value.status == _capi.RT_ERROR_INVALID_VALUE
    with pytest.raises(_capi.RtError) as e:
        api.BatchPlan(ctx, [single], [rays[1]], want_inst=True)
    assert e.value.status == _capi.RT_ERROR_INVALID_VALUE
    single.close()
    for a in accs:
        a.close()


def _context_with_refill(api, refill):
    import os

    old = os.environ.get("RT_REFILL")
    os.environ["RT_REFILL"] = str(refill)
    try:
        return api.Context(0)
    finally:
        if old is None:
            del os.environ["RT_REFILL"]
        else:
            os.environ["RT_REFILL"] = old


def _soup_works(seed, sizes):
    rng = wl.rng_for(seed)
    works = []
    for m, (nt, nr) in enumerate(sizes):
        half = 0.025 * np.sqrt(4096.0 / max(nt, 1))
        V, I = wl.random_triangle_soup(rng, nt, half)
        works.append(wl.Workload(f"b{m}", wl.Scene([wl.Mesh(V, I)]), wl.box_rays(rng, nr, -1, 2)))
    return works


def test_plan_keeps_its_variant(gpu):
    """A plan launches with the variant its context had at creation: changing
    the context's variant (stack and workgroup) before the launch and before
    a graph capture changes neither the launch nor the answers."""
    torch, api, _ = gpu
    ctx = api.Context(0, stack_entries=16, workgroup=256)
    works = _soup_works(503, [(20000, 30000), (500, 4000), (9000, 12345)])
    accs = [to_gpu_scene(api, torch, ctx, w.scene) for w in works]
    rays = [torch.from_numpy(w.rays).cuda() for w in works]
    per = _per_mesh(gpu, accs, rays)
    plan = api.BatchPlan(ctx, accs, rays)
    ctx.set_variant(8, 64)
    plan.launch()
    torch.cuda.synchronize()
    _check_equal([h.cpu().numpy() for h in plan.hits], per)
    s = torch.cuda.Stream()
    g = plan.graph_exec(s)
    for h in plan.hits:
        h.fill_(-1.0)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        api.graph_launch(g, s)
    s.synchronize()
    _check_equal([h.cpu().numpy() for h in plan.hits], per)
    plan.close()
    for a in accs:
        a.close()
    ctx.close()


def test_batched_overflow_ranges(gpu):
    """A refill threshold of one idle lane (ranges of a few rays per refill)
    changes neither the batched answers nor the per-mesh ones, whose waves
    then overflow their finalize range lists: plan launch and graph replay
    equal per-mesh launches bit for bit."""
    torch, api, _ = gpu
    works = _soup_works(504, [(30000, 400000), (2000, 300000), (0, 1000), (15000, 500000), (7, 3)])
    ctx = _context_with_refill(api, 1)
    accs = [to_gpu_scene(api, torch, ctx, w.scene) for w in works]
    rays = [torch.from_numpy(w.rays).cuda() for w in works]
    per = _per_mesh(gpu, accs, rays)
    plan = api.BatchPlan(ctx, accs, rays)
    plan.launch()
    torch.cuda.synchronize()
    _check_equal([h.cpu().numpy() for h in plan.hits], per)
    s = torch.cuda.Stream()
    g = plan.graph_exec(s)
    for rep in range(2):
        for h in plan.hits:
            h.fill_(-1.0)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            api.graph_launch(g, s)
        s.synchronize()
        _check_equal([h.cpu().numpy() for h in plan.hits], per)
    plan.close()
    for a in accs:
        a.close()
    ctx.close()
