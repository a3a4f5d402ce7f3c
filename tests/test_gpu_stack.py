"""The traversal stack (§7.5: a per-thread stack in shared memory with global
memory as the fallback): rays that push far past the LDS part spill to the
global stack and still return the oracle's answers, bit-identical for every
LDS depth; the deepest fill any ray reaches stays within the builder's bound;
a lane that would exceed its bound is reported on the context's next call."""
from __future__ import annotations

import os

import numpy as np
import pytest

from helpers import NONE, check_chunked, to_gpu_scene
from paper_2603_00292_amd import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def gpu():
    import torch

    from paper_2603_00292_amd import api

    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    torch.cuda.set_device(0)
    ctx = api.Context(0)
    yield torch, api, ctx
    torch.cuda.synchronize()


def layered_scene(layers: int = 65536, seed: int = 700):
    """`layers` large triangles stacked along z (spacing 1e-4, jittered in x
    and y) and rays crossing the whole stack from above and below at up to
    ~15 degrees off the z axis: a ray enters every child box on its way
    down the tree, so its stack fills to about (W - 1) x depth."""
    rng = wl.rng_for(seed)
    z = np.arange(layers) * 1e-4
    c = rng.uniform(-0.2, 0.2, (layers, 2))
    base = 4.0 * np.array([[-1.0, -1.0], [1.5, -0.8], [-0.7, 1.4]])
    V = np.zeros((layers, 3, 3))
    V[:, :, 0:2] = base[None, :, :] + c[:, None, :]
    V[:, :, 2] = z[:, None]
    V = V.reshape(-1, 3).astype(np.float32)
    I = np.arange(3 * layers, dtype=np.uint32).reshape(-1, 3)
    n = 32768
    top = rng.random(n) < 0.5
    o = np.stack([rng.uniform(-0.3, 0.3, n), rng.uniform(-0.3, 0.3, n),
                  np.where(top, z[-1] + 1.0, -1.0)], 1)
    d = np.stack([rng.uniform(-0.25, 0.25, n), rng.uniform(-0.25, 0.25, n), np.where(top, -1.0, 1.0)], 1)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays = wl.pack_rays(o, d)
    # some rays end inside the stack (tmax), some start inside it
    rays[: n // 8, 7] = np.float32(0.5 + z[-1] / 2)
    mid = slice(n // 8, n // 4)
    rays[mid, 2] = np.float32(z[-1] / 3)
    return wl.Scene([wl.Mesh(V, I)]), rays


@pytest.mark.parametrize("width", [4, 8])
def test_forced_spill_matches_oracle(gpu, orc, width):
    torch, api, _ = gpu
    scene, rays = layered_scene()
    r = torch.from_numpy(rays).cuda()
    S = orc.OracleScene.from_scene(scene, accel=True)
    outs = {}
    for s in (8, 16, 32):
        ctx = api.Context(0, stack_entries=s, workgroup=256)
        acc = to_gpu_scene(api, torch, ctx, scene, node_width=width)
        info = acc.info
        h, _ = api.trace_closest(acc, r)
        occ = api.trace_any(acc, r)
        torch.cuda.synchronize()
        outs[s] = (h.cpu().numpy(), occ.cpu().numpy())
        if s == 16:
            (nodes, tris, spills, peak), hc = api.trace_counters(acc, r, peak=True)
            (_, _, spills_a, peak_a), oc = api.trace_counters(acc, r, any_hit=True, peak=True)
            torch.cuda.synchronize()
            say(f"W={width} max_stack {info['max_stack']} depth {info['max_depth']}: spills/ray "
                f"{spills / len(rays):.2f} (any {spills_a / len(rays):.2f}), deepest fill {peak} (any {peak_a})")
            # the rays spill (stack 16 of the counting variant, and so also 8)
            assert info["max_stack"] > 16 and spills > len(rays) and spills_a > 0
            assert 16 < peak <= info["max_stack"] and peak_a <= info["max_stack"]
            assert np.array_equal(hc.cpu().numpy().view(np.uint32), outs[16][0].view(np.uint32))
            assert np.array_equal(oc.cpu().numpy(), outs[16][1])
        acc.close()
        ctx.close()
    for s in (8, 32):
        assert np.array_equal(outs[s][0].view(np.uint32), outs[16][0].view(np.uint32)), s
        assert np.array_equal(outs[s][1], outs[16][1]), s
    # every ray of the spilling launches against the oracle
    h, occ = outs[8]
    st = check_chunked(orc, S, rays, hits=h, occ=occ, label=f"layered W={width}")
    say(st)
    prim = h[:, 1].copy().view(np.uint32)
    assert (prim != NONE).mean() > 0.8


def test_deepest_fill_within_bound(gpu):
    """Headline mesh (all 4,194,304 incoherent rays) and a 1,024-instance
    two-level scene: the deepest stack fill of any ray, closest and any-hit,
    stays within the accel's max_stack."""
    torch, api, ctx = gpu
    for W, kw in ((wl.icosphere_incoherent(), {}), (wl.instanced_grids(n_rays=1 << 20), {}),
                  (wl.random_triangles(), {"node_width": 8})):
        acc = to_gpu_scene(api, torch, ctx, W.scene, **kw)
        r = torch.from_numpy(W.rays).cuda()
        (_, _, sp, peak), _ = api.trace_counters(acc, r, peak=True)
        (_, _, _, peak_a), _ = api.trace_counters(acc, r, any_hit=True, peak=True)
        info = acc.info
        say(W.name, "max_stack", info["max_stack"], "deepest fill", peak, "any", peak_a, "spills", sp)
        assert 0 < peak <= info["max_stack"] and peak_a <= info["max_stack"]
        acc.close()


def test_phase_counters_consistent(gpu):
    """The wave-level loop counts of rt_trace_counters_ex on the headline
    workload and a two-level scene: the first four counters agree with
    rt_trace_counters' (to 0.5%: which rays share a wave, and so when a
    lane's postponed leaves are tested and its cull distance shrinks, depends
    on the order in which waves take rays), a wave iteration serves at most
    64 lanes (node visits <= 64 x node-loop iterations, triangle tests <= 64
    x leaf-loop iterations), refills <= outer passes, and the query's answers
    are those of the plain kernel."""
    torch, api, ctx = gpu
    for W in (wl.icosphere_incoherent(), wl.instanced_grids(n_rays=1 << 20)):
        acc = to_gpu_scene(api, torch, ctx, W.scene)
        r = torch.from_numpy(W.rays).cuda()
        (nodes, tris, sp, peak), h4 = api.trace_counters(acc, r, peak=True)
        c = api.trace_phase_counters(acc, r)
        h, _ = api.trace_closest(acc, r)
        say(W.name, {k: (round(v, 3) if isinstance(v, float) else v) for k, v in c.items()})
        assert abs(c["node_visits"] - nodes) <= 5e-3 * nodes and abs(c["tri_tests"] - tris) <= 5e-3 * tris
        assert 0 < c["deepest"] <= acc.info["max_stack"] and 0 < peak <= acc.info["max_stack"]
        assert 0 < c["node_visits"] <= 64 * c["node_iters"] and 0 < c["tri_tests"] <= 64 * c["leaf_iters"]
        assert 0 < c["refills"] <= c["outer_passes"]
        assert c["refills"] * 64 >= W.rays.shape[0]
        assert torch.equal(h4[:, 1].contiguous().view(torch.int32), h[:, 1].contiguous().view(torch.int32))
        acc.close()


def test_overflow_reported_on_next_call(gpu):
    """A context whose lanes may hold only 20 entries (below the accel's
    bound of 26 and the 22 the deepest ray needs; set from the host, so
    every kernel still finishes normally): the counting traversal drops the
    entries it cannot hold, and the context's next query fails with
    RT_ERROR_STACK_OVERFLOW and clears the flag.  A context without the cap
    never reports it."""
    torch, api, _ = gpu
    from paper_2603_00292_amd import _capi

    scene, rays = layered_scene()
    r = torch.from_numpy(rays).cuda()
    os.environ["RT_STACK_LIMIT"] = "20"
    try:
        ctx = api.Context(0)
    finally:
        del os.environ["RT_STACK_LIMIT"]
    acc = to_gpu_scene(api, torch, ctx, scene)
    assert acc.info["max_stack"] > 20
    (_, _, _, peak), _ = api.trace_counters(acc, r, peak=True)
    torch.cuda.synchronize()
    assert peak == 20
    with pytest.raises(_capi.RtError) as e:
        api.trace_any(acc, r)
    assert e.value.status == _capi.RT_ERROR_STACK_OVERFLOW
    api.trace_any(acc, r)       # flag cleared: the query kernels do not raise it
    api.trace_closest(acc, r)
    torch.cuda.synchronize()
    api.trace_closest(acc, r)
    torch.cuda.synchronize()
    acc.close()
    ctx.close()
    ctx2 = api.Context(0)
    acc2 = to_gpu_scene(api, torch, ctx2, scene)
    for _ in range(2):
        api.trace_counters(acc2, r)
        torch.cuda.synchronize()
        api.trace_closest(acc2, r)
        api.trace_any(acc2, r)
    torch.cuda.synchronize()
    acc2.close()
    ctx2.close()
