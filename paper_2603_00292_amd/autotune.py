"""Autotuner front end: picks node width, stack entries and workgroup size by
measurement (rt_autotune in librtq) and caches the choice per device and
scene class.

    python -m paper_2603_00292_amd.autotune --workload icosphere_incoherent

The measurement itself (builds at each node width, HIP-event timing of every
variant on a probe batch) runs in the library; this module marshals tensors,
keys the cache and reads/writes it as JSON.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import math
import os

import torch

from . import _capi as capi
from . import api

CACHE = os.path.join(os.path.expanduser("~"), ".cache", "rtq", "autotune.json")


def scene_class(n_triangles: int, n_rays: int) -> str:
    """Cache key part: triangle and ray counts by power-of-four bucket."""
    tb = int(math.log(max(n_triangles, 1), 4))
    rb = int(math.log(max(n_rays, 1), 4))
    return f"tri4^{tb}_ray4^{rb}"


def device_key(device: int) -> str:
    p = torch.cuda.get_device_properties(device)
    arch = getattr(p, "gcnArchName", "unknown").split(":")[0]
    return f"{arch}_cu{p.multi_processor_count}"


def choose(ctx: api.Context, vertices: torch.Tensor, indices: torch.Tensor, probe_rays: torch.Tensor,
           n_rays: int, repeats: int = 3, use_cache: bool = True):
    """The configuration for a mesh of this size traced with n_rays rays on
    this device: the cached choice for (device, scene class) when there is
    one, otherwise rt_autotune on the probe rays, saved to the cache.  Sets
    the context's variant; returns (choice, from_cache)."""
    dev = ctx.device
    cls = scene_class(indices.shape[0], n_rays)
    if use_cache:
        hit = cached_choice(dev, cls)
        if hit is not None:
            ctx.set_variant(hit["stack_entries"], hit["workgroup"])
            return hit, True
    best, _ = autotune(ctx, vertices, indices, probe_rays, repeats)
    if use_cache:
        save_choice(dev, cls, best)
    return best, False


def autotune(ctx: api.Context, vertices: torch.Tensor, indices: torch.Tensor, probe_rays: torch.Tensor,
             repeats: int = 3):
    """Runs rt_autotune; returns (best, table) as dicts.  The context's
    variant is set to the best one; build the accel with best['node_width']."""
    api._require(vertices, "vertices", torch.float32, 3)
    api._require(probe_rays, "probe_rays", torch.float32, 8)
    desc = capi.rt_mesh_desc(vertices.data_ptr(), vertices.shape[0], 12, indices.data_ptr(), indices.shape[0], 12)
    best = capi.rt_tune_entry()
    cap = 64
    table = (capi.rt_tune_entry * cap)()
    n = C.c_uint32(0)
    capi.call("rt_autotune", ctx.handle, C.byref(desc), C.c_void_p(probe_rays.data_ptr()), probe_rays.shape[0],
              int(repeats), C.c_void_p(api._stream()), C.byref(best), table, cap, C.byref(n))
    to = lambda e: {"node_width": e.node_width, "stack_entries": e.stack_entries, "workgroup": e.workgroup,
                    "ms": round(float(e.ms), 5)}
    return to(best), [to(table[i]) for i in range(min(n.value, cap))]


VARIANTS = [(s, wg) for s in (8, 16, 32) for wg in (64, 128, 256)]
DEFAULT_VARIANT = (16, 256)


def tune_variant(ctx: api.Context, make_run, repeats: int = 3, margin: float = 0.01):
    """Picks (stack entries, workgroup) for any query on an existing accel:
    for every variant the context is set to it, ``make_run()`` returns a
    callable that enqueues one query on the current stream (for a batched
    plan: a plan created under that variant, whose launch it returns), which
    is timed with HIP events (median of ``repeats`` after a warm-up).  The
    default variant stays unless another is faster by more than ``margin``.
    Sets the context's variant to the choice; returns (choice, table)."""
    stream = torch.cuda.current_stream()
    table = []
    for s, wg in VARIANTS:
        ctx.set_variant(s, wg)
        run = make_run()
        run()
        torch.cuda.synchronize()
        times = []
        for _ in range(repeats):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            run()
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        table.append({"stack_entries": s, "workgroup": wg, "ms": round(sorted(times)[len(times) // 2], 5)})
    default = next(e for e in table if (e["stack_entries"], e["workgroup"]) == DEFAULT_VARIANT)
    fastest = min(table, key=lambda e: e["ms"])
    best = default if default["ms"] <= fastest["ms"] * (1 + margin) else fastest
    ctx.set_variant(best["stack_entries"], best["workgroup"])
    return best, table


def cache_path() -> str:
    return os.environ.get("RTQ_AUTOTUNE_CACHE", CACHE)


def load_cache() -> dict:
    """The cache's contents; a missing, unreadable or malformed file reads as
    empty (it is a cache: the next save rewrites it)."""
    p = cache_path()
    try:
        with open(p) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return {}
    return c if isinstance(c, dict) and all(isinstance(v, dict) for v in c.values()) else {}


def save_choice(device, cls: str, best: dict) -> None:
    """device: a HIP device id, or a device key string."""
    key = device if isinstance(device, str) else device_key(device)
    c = load_cache()
    c.setdefault(key, {})[cls] = best
    p = cache_path()
    os.makedirs(os.path.dirname(p) or ".", exist_ok=True)
    tmp = p + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1)
    os.replace(tmp, p)


def cached_choice(device, cls: str):
    """The cached configuration of (device, scene class), or None (also for an
    entry that does not name a node width, stack depth and workgroup)."""
    key = device if isinstance(device, str) else device_key(device)
    hit = load_cache().get(key, {}).get(cls)
    if not isinstance(hit, dict):
        return None
    if not all(isinstance(hit.get(k), int) for k in ("node_width", "stack_entries", "workgroup")):
        return None
    return hit


def main():
    import numpy as np

    from . import workloads

    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="icosphere_incoherent",
                    choices=["icosphere_incoherent", "random_triangles", "displaced_grid"])
    ap.add_argument("--probe", type=int, default=262144)
    args = ap.parse_args()
    W = getattr(workloads, args.workload)()
    m = W.scene.meshes[0]
    torch.cuda.set_device(0)
    ctx = api.Context(0)
    V = torch.from_numpy(m.vertices).cuda()
    I = torch.from_numpy(m.indices.view(np.int32)).cuda()
    probe = torch.from_numpy(W.rays[: args.probe]).cuda()
    best, table = autotune(ctx, V, I, probe)
    cls = scene_class(m.n_tri, W.rays.shape[0])
    save_choice(0, cls, best)
    print(json.dumps({"class": cls, "best": best, "table": table}))


if __name__ == "__main__":
    main()
