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
    # the answer is the lexicographic minimum of (float32 t, id) over all hit
    # triangles, with t computed from the same record whatever the tree or
    # variant, and culling is conservative: identical bit for bit
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    tuned.close(); ref.close(); ctx.close(); ctx2.close()


def test_autotune_cache(tmp_path, monkeypatch):
    """choose() measures once per (device, scene class), then serves the
    cached configuration and sets the context's variant from it."""
    import torch

    from paper_2603_00292_amd import api, autotune

    monkeypatch.setenv("RTQ_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    torch.cuda.set_device(0)
    W = wl.random_triangles(n_tri=8000, n_rays=16384, k=601, half=0.02)
    m = W.scene.meshes[0]
    V = torch.from_numpy(m.vertices).cuda()
    I = torch.from_numpy(m.indices.view(np.int32)).cuda()
    rays = torch.from_numpy(W.rays).cuda()
    ctx = api.Context(0)
    best, cached = autotune.choose(ctx, V, I, rays, rays.shape[0], repeats=2)
    assert not cached
    ctx2 = api.Context(0, stack_entries=8, workgroup=64)
    again, cached = autotune.choose(ctx2, V, I, rays, rays.shape[0])
    assert cached and again == best
    assert ctx2.variant == (best["stack_entries"], best["workgroup"])
    ctx.close(); ctx2.close()
