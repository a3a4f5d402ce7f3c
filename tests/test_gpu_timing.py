"""rt_context_set_timing / rt_context_read_timing: HIP events recorded around
the traversal kernel alone.  The answers are unchanged with timing on, the
durations are positive and no longer than the whole call (traversal, finalize
and queue reset), the ring keeps the most recent launches, and a read empties
it."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest

from paper_2603_00292_amd import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def test_timing_ring():
    import torch

    from paper_2603_00292_amd import _capi, api

    torch.cuda.set_device(0)
    ctx = api.Context(0)
    W = wl.random_triangles()
    m = W.scene.meshes[0]
    V = torch.from_numpy(m.vertices).cuda()
    I = torch.from_numpy(m.indices.view(np.int32)).cuda()
    acc = api.Accel(ctx, [(V, I)])
    rays = torch.from_numpy(W.rays).cuda()
    h0, _ = api.trace_closest(acc, rays)
    torch.cuda.synchronize()
    assert ctx.read_timing() == []  # timing off: nothing recorded

    ctx.set_timing(4)
    s = torch.cuda.current_stream()
    whole = []
    for _ in range(6):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        h, _ = api.trace_closest(acc, rays)
        e1.record(s)
        whole.append((e0, e1))
    occ = api.trace_any(acc, rays)
    torch.cuda.synchronize()
    assert torch.equal(h.view(torch.int32), h0.view(torch.int32))
    ms = ctx.read_timing()
    say("traversal ms", ms, "whole calls ms", [a.elapsed_time(b) for a, b in whole[-3:]])
    assert len(ms) == 4  # the ring holds the last four of seven launches
    assert all(t > 0.0 for t in ms)
    # launches 4..6 are closest calls: each traversal lies inside its call
    for t, (a, b) in zip(ms[:3], whole[3:]):
        assert t <= a.elapsed_time(b) + 1e-3
    assert ctx.read_timing() == []  # a read empties the ring
    api.trace_any(acc, rays)
    assert len(ctx.read_timing(capacity=8)) == 1
    occ_ref = api.trace_any(acc, rays)
    torch.cuda.synchronize()
    assert torch.equal(occ, occ_ref)
    ctx.set_timing(0)
    api.trace_closest(acc, rays)
    assert ctx.read_timing() == []
    with pytest.raises(_capi.RtError) as e:
        ctx.set_timing(4097)
    assert e.value.status == _capi.RT_ERROR_INVALID_VALUE
    cnt = C.c_uint32()
    with pytest.raises(_capi.RtError) as e:
        _capi.call("rt_context_read_timing", ctx.handle, None, 4, C.byref(cnt))
    assert e.value.status == _capi.RT_ERROR_INVALID_VALUE
    acc.close()
    ctx.close()
