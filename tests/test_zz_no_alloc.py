"""rt_trace_closest_noalloc (scratch in the library's fixed per-GPU array, no
allocation) against rt_trace_closest through the C ABI: bit-identical hits
and instance ids on two calls in a row, the second with a smaller input, and
a clear error for a ray count whose scratch would not fit."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest

from helpers import to_gpu_scene
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
    yield torch, api
    torch.cuda.synchronize()


def _both(gpu, acc, rays, want_inst=False):
    torch, api = gpu
    r = torch.from_numpy(np.ascontiguousarray(rays)).cuda()
    ref, ref_i = api.trace_closest(acc, r, want_inst=want_inst)
    hits = torch.full((r.shape[0], 4), -1.0, dtype=torch.float32, device="cuda")
    inst = torch.full((r.shape[0],), -7, dtype=torch.int32, device="cuda") if want_inst else None
    api.trace_closest_noalloc(acc, r, hits, inst)
    torch.cuda.synchronize()
    assert torch.equal(hits.view(torch.int32), ref.view(torch.int32))
    if want_inst:
        assert torch.equal(inst, ref_i)
    return hits


def test_noalloc_matches_trace_closest(gpu):
    torch, api = gpu
    ctx = api.Context(0)
    # first call: the headline workload (1,310,720 triangles, 4,194,304 rays)
    W = wl.icosphere_incoherent()
    acc = to_gpu_scene(api, torch, ctx, W.scene)
    h = _both(gpu, acc, W.rays)
    say("headline: identical,", int((h[:, 1].view(torch.int32) != -1).sum()), "hits")
    acc.close()
    # second call, smaller: the 4,096-triangle soup, 65,536 rays
    W2 = wl.random_triangles()
    acc2 = to_gpu_scene(api, torch, ctx, W2.scene)
    _both(gpu, acc2, W2.rays)
    _both(gpu, acc2, W2.rays[:1000])
    acc2.close()
    # a two-level accel with instance ids
    W3 = wl.instanced_grids(n_inst=64, n_rays=50000, k=410)
    acc3 = to_gpu_scene(api, torch, ctx, W3.scene)
    _both(gpu, acc3, W3.rays, want_inst=True)
    acc3.close()
    ctx.close()


def test_noalloc_other_variants_and_contexts(gpu):
    """Stack 8 / workgroup 64 (more spilling, a larger grid) and a second
    context on the same device share the one array one call after another."""
    torch, api = gpu
    W = wl.random_triangles(n_tri=20000, n_rays=300000, k=411, half=0.03)
    for s, wg in ((8, 64), (32, 128), (16, 256)):
        ctx = api.Context(0, stack_entries=s, workgroup=wg)
        acc = to_gpu_scene(api, torch, ctx, W.scene)
        _both(gpu, acc, W.rays)
        acc.close()
        ctx.close()


def test_noalloc_rejects_oversized_launch(gpu):
    torch, api = gpu
    from paper_2603_00292_amd import _capi

    ctx = api.Context(0)
    W = wl.random_triangles(n_tri=256, n_rays=64, k=412, half=0.2)
    acc = to_gpu_scene(api, torch, ctx, W.scene)
    r = torch.from_numpy(W.rays).cuda()
    hits = torch.empty((64, 4), dtype=torch.float32, device="cuda")
    # 2^31 - 1 rays need far more range-list scratch than the fixed array
    # holds: refused on the host before anything is enqueued
    st = _capi.load().rt_trace_closest_noalloc(acc.handle, C.c_void_p(r.data_ptr()), 0x7FFFFFFF,
                                                C.c_void_p(hits.data_ptr()), None, None)
    assert st == _capi.RT_ERROR_INVALID_VALUE
    # the entry point still works afterwards
    _both(gpu, acc, W.rays)
    acc.close()
    ctx.close()
