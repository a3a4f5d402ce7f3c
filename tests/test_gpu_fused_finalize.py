"""The float64 finalize of closest hits on one accel runs inside the traversal
kernel: each wave finalizes the ray ranges it took from the queue, and ranges
beyond its list go to an overflow list finalized by a follow-up kernel.  With
a refill threshold of one idle lane (RT_REFILL=1) a wave takes ranges of a few
rays each, so on the full incoherent workload (about 585 rays per wave) nearly
every wave overflows its 128-entry list; the answers must equal, bit for bit,
those of the default threshold (ranges of 32 or more rays, no overflow), which
the other tests pin to the oracle.  Instance ids of a single-level accel are 0
for hits and invalid for misses on both paths."""
from __future__ import annotations

import os

import numpy as np
import pytest

from paper_2603_00292_amd import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def context_with_refill(api, refill):
    old = os.environ.get("RT_REFILL")
    os.environ["RT_REFILL"] = str(refill)
    try:
        return api.Context(0)
    finally:
        if old is None:
            del os.environ["RT_REFILL"]
        else:
            os.environ["RT_REFILL"] = old


@pytest.mark.parametrize("n_rays", [4194304, 100003])
def test_overflow_ranges_bit_identical(n_rays):
    import torch

    from paper_2603_00292_amd import api

    torch.cuda.set_device(0)
    W = wl.icosphere_incoherent()
    m = W.scene.meshes[0]
    V = torch.from_numpy(m.vertices).cuda()
    I = torch.from_numpy(m.indices.view(np.int32)).cuda()
    rays = torch.from_numpy(np.ascontiguousarray(W.rays[:n_rays])).cuda()
    out = []
    for refill in (32, 1):
        ctx = context_with_refill(api, refill)
        acc = api.Accel(ctx, [(V, I)])
        for _ in range(2):  # the second call reuses the range buffers
            h, inst = api.trace_closest(acc, rays, want_inst=True)
        torch.cuda.synchronize()
        out.append((h.cpu().numpy().view(np.uint32).copy(), inst.cpu().numpy().view(np.uint32).copy()))
        acc.close()
        ctx.close()
    (h32, i32), (h1, i1) = out
    hit = h32[:, 1] != 0xFFFFFFFF
    say(f"rays {n_rays}: hits {int(hit.sum())}")
    assert np.array_equal(h32, h1)
    assert np.array_equal(i32, i1)
    assert np.array_equal(i32[hit], np.zeros(int(hit.sum()), np.uint32))
    assert (i32[~hit] == 0xFFFFFFFF).all()
    # sane values: ids in range, (u, v) inside the triangle up to the
    # rounding of edge hits (the oracle tests bound these to 1e-5)
    prims = h32[hit, 1]
    assert prims.max() < m.n_tri
    u = h32[hit, 2].view(np.float32)
    v = h32[hit, 3].view(np.float32)
    say(f"min u {u.min():.3g}, min v {v.min():.3g}, max u+v {(u + v).max():.8g}")
    assert (u >= -1e-3).all() and (v >= -1e-3).all() and (u + v <= 1 + 1e-3).all()


def test_overflow_ranges_two_level():
    """The same for a two-level accel (float64 instance frames in the
    finalize): 2,097,152 rays of the 1,024-instance workload."""
    import torch

    from helpers import to_gpu_scene
    from paper_2603_00292_amd import api

    torch.cuda.set_device(0)
    W = wl.instanced_grids()
    rays = torch.from_numpy(np.ascontiguousarray(W.rays[: 1 << 21])).cuda()
    out = []
    for refill in (32, 1):
        ctx = context_with_refill(api, refill)
        acc = to_gpu_scene(api, torch, ctx, W.scene)
        for _ in range(2):
            h, inst = api.trace_closest(acc, rays, want_inst=True)
        torch.cuda.synchronize()
        out.append((h.cpu().numpy().view(np.uint32).copy(), inst.cpu().numpy().view(np.uint32).copy()))
        acc.close()
        ctx.close()
    (h32, i32), (h1, i1) = out
    hit = h32[:, 1] != 0xFFFFFFFF
    say(f"two-level: hits {int(hit.sum())} of {h32.shape[0]}")
    assert hit.sum() > 100000
    assert np.array_equal(h32, h1)
    assert np.array_equal(i32, i1)
    assert (i32[hit] < W.scene.inst_mesh.shape[0]).all() and (i32[~hit] == 0xFFFFFFFF).all()
