"""Out-of-memory paths, driven by the allocation hook of librtq: with
RT_FAULT_ALLOC = k set when a context is created, the k-th device or pinned
allocation after that fails (once).  For every k up to the number of
allocations of a pipeline that exercises every allocating call (context,
host and device builds, closest / any / counting / all-hit queries, the
backward and its first-call lists, a two-level build and backward, a
batched plan), the failing call reports RT_ERROR_OUT_OF_MEMORY, closing what
was created returns the device memory, and a clean run afterwards gives
the same answers as before (the failure left no shared state behind)."""
from __future__ import annotations

import hashlib

import numpy as np
import pytest

from helpers import to_gpu_scene
from paper_2603_00292_amd import workloads as wl

pytestmark = pytest.mark.gpu

SLACK = 4 << 20   # bytes: pool and driver granularity


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def setup():
    import torch

    from paper_2603_00292_amd import _capi as capi
    from paper_2603_00292_amd import api

    torch.cuda.set_device(0)
    W = wl.displaced_grid(nx=256, nz=128, n_rays=65536, k=410)
    A = wl.aimed_instances(n_inst=8, n_rays=4096, k=411)
    data = {
        "V": torch.from_numpy(W.scene.meshes[0].vertices).cuda(),
        "I": torch.from_numpy(W.scene.meshes[0].indices.view(np.int32)).cuda(),
        "rays": torch.from_numpy(W.rays).cuda(),
        "g": torch.from_numpy(W.extra["abc"]).cuda(),
        "scene2": A.scene,
        "rays2": torch.from_numpy(A.rays).cuda(),
        "g2": torch.from_numpy(np.random.default_rng(412).normal(size=(A.rays.shape[0], 3)).astype(np.float32)).cuda(),
    }
    yield torch, api, capi, data
    torch.cuda.synchronize()


def _pipeline(torch, api, data, opened):
    h = hashlib.sha256()

    def put(*ts):
        torch.cuda.synchronize()
        for t in ts:
            h.update(t.cpu().numpy().tobytes())

    ctx = api.Context(0)
    opened.append(ctx)
    acc = api.Accel(ctx, [(data["V"], data["I"])])
    opened.append(acc)
    rays = data["rays"]
    hits, _ = api.trace_closest(acc, rays)
    put(hits)
    put(api.trace_any(acc, rays))
    c = api.trace_counters(acc, rays, peak=True)
    put(hits)
    dV = torch.zeros_like(data["V"])
    do, dd = api.trace_backward(acc, rays, hits, data["g"], dV)
    put(dV, do, dd)
    dacc = api.Accel(ctx, [(data["V"], data["I"])], device_build=True)
    opened.append(dacc)
    dh, _ = api.trace_closest(dacc, rays)
    put(dh)
    ah, _, cnt = api.trace_all(acc, rays[:4096], 4)
    put(ah, cnt)
    two = to_gpu_scene(api, torch, ctx, data["scene2"])
    opened.append(two)
    h2, i2 = api.trace_closest(two, data["rays2"], want_inst=True)
    put(h2, i2)
    nv = sum(m.vertices.shape[0] for m in data["scene2"].meshes)
    dv2 = torch.zeros((nv, 3), dtype=torch.float32, device="cuda")
    ds = torch.zeros((two.instance_count, 10), dtype=torch.float32, device="cuda")
    do2, dd2 = api.trace_backward_instances(two, data["rays2"], h2, i2, data["g2"], dv2, ds)
    put(dv2, ds, do2, dd2)
    plan = api.BatchPlan(ctx, [acc, dacc], [rays[:1000], rays[1000:5000]])
    opened.append(plan)
    plan.launch()
    put(*plan.hits)
    del c
    return h.hexdigest()


def _close(torch, opened):
    for o in reversed(opened):
        o.close()
    opened.clear()
    torch.cuda.synchronize()


def test_every_allocation_failure(setup, monkeypatch):
    torch, api, capi, data = setup
    opened = []
    monkeypatch.delenv("RT_FAULT_ALLOC", raising=False)
    ref = _pipeline(torch, api, data, opened)
    _close(torch, opened)
    free0 = torch.cuda.mem_get_info()[0]
    failed_at = []
    k = 0
    try:
        while True:
            k += 1
            assert k < 400, "the pipeline never completed"
            monkeypatch.setenv("RT_FAULT_ALLOC", str(k))
            done = None
            try:
                done = _pipeline(torch, api, data, opened)
            except capi.RtError as e:
                assert e.status == capi.RT_ERROR_OUT_OF_MEMORY, str(e)
                failed_at.append(str(e).split(":")[0])
            finally:
                _close(torch, opened)
            free = torch.cuda.mem_get_info()[0]
            assert free >= free0 - SLACK, f"k={k}: {(free0 - free) / 2**20:.1f} MiB not returned"
            if done is not None:
                assert done == ref
                break
    finally:
        monkeypatch.delenv("RT_FAULT_ALLOC", raising=False)
        # disarm the hook for whatever runs next in this process
        api.Context(0).close()
    say(f"{len(failed_at)} allocations failed one at a time; calls that reported them:",
        sorted(set(failed_at)))
    assert len(failed_at) == k - 1 and len(failed_at) >= 10
    # the clean run afterwards
    again = _pipeline(torch, api, data, opened)
    _close(torch, opened)
    assert again == ref
