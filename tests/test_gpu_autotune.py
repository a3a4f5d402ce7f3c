"""The autotuner (rt_autotune): measures every (node width, stack entries,
workgroup) configuration, returns the fastest (keeping the default unless
another is faster by more than 1%), sets the context's variant,
and the tuned configuration answers exactly like the default one."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2603_00292_amd import workloads as wl

pytestmark = pytest.mark.gpu


def test_autotune_picks_fastest_and_keeps_results():
    import torch

    from paper_2603_00292_amd import api, autotune

    torch.cuda.set_device(0)
    W = wl.random_triangles(n_tri=20000, n_rays=65536, k=600, half=0.02)
    m = W.scene.meshes[0]
    V = torch.from_numpy(m.vertices).cuda()
    I = torch.from_numpy(m.indices.view(np.int32)).cuda()
    rays = torch.from_numpy(W.rays).cuda()
    ctx = api.Context(0)
    best, table = autotune.autotune(ctx, V, I, rays[:16384], repeats=3)
    print(best, flush=True)
    assert len(table) == 27
    combos = {(e["node_width"], e["stack_entries"], e["workgroup"]) for e in table}
    assert combos == {(w, s, g) for w in (2, 4, 8) for s in (8, 16, 32) for g in (64, 128, 256)}
    fastest = min(e["ms"] for e in table)
    default = [e for e in table if (e["node_width"], e["stack_entries"], e["workgroup"]) == (4, 16, 256)][0]
    # the default stays unless another configuration is faster by more than 1%
    if default["ms"] <= fastest * 1.01:
        assert best == default
    else:
        assert best["ms"] == fastest
    assert ctx.variant == (best["stack_entries"], best["workgroup"])
    tuned = api.Accel(ctx, [(V, I)], node_width=best["node_width"])
    h1, _ = api.trace_closest(tuned, rays)
    ctx2 = api.Context(0)
    ref = api.Accel(ctx2, [(V, I)])
    h2, _ = api.trace_closest(ref, rays)
    torch.cuda.synchronize()
    a, b = h1.cpu().numpy(), h2.cpu().numpy()
    # ids are identical unless an exact tie sits in different leaves of the two
    # trees; values of equal ids are identical (same float64 finalize)
    pa, pb = a[:, 1].view(np.uint32), b[:, 1].view(np.uint32)
    assert (pa == pb).mean() > 0.9999
    same = pa == pb
    assert np.array_equal(a[same].view(np.uint32), b[same].view(np.uint32))
    tuned.close(); ref.close(); ctx.close(); ctx2.close()
