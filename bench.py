"""Benchmark: incoherent closest-hit ray queries at about a million triangles.

Workload (synthetic, seeded): the noisy icosphere with 1,310,720 triangles
(radius 1 +- 0.02) and 4,194,304 rays with origins uniform in [-1,1]^3 and
directions uniform on the sphere, tmin = 0, tmax = +inf.  A step is one
closest-hit query over all rays (rt_trace_closest: persistent traversal
kernel with the float64 finalize), inputs and outputs resident in HBM.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRI_BYTES = 48
RAY_BYTES = 32
HIT_BYTES = 16
FINALIZE_BYTES = 12 + 36  # indices + vertices of the winning triangle


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target host time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--width", type=int, default=4)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the ray-query path is built and measured on a single "
              "MI355X (rays shard across GPUs with the structure replicated; not measured here).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2603_00292_amd import api, workloads

    torch.cuda.set_device(0)
    t0 = time.time()
    W = workloads.icosphere_incoherent()
    mesh = W.scene.meshes[0]
    n = W.rays.shape[0]
    log(f"workload generated in {time.time() - t0:.1f}s: {mesh.n_tri} triangles, {n} rays")
    ctx = api.Context(0)
    dev = torch.device("cuda:0")
    V = torch.from_numpy(mesh.vertices).to(dev)
    I = torch.from_numpy(mesh.indices.view(np.int32)).to(dev)
    t0 = time.time()
    acc = api.Accel(ctx, [(V, I)], node_width=args.width)
    info = acc.info
    log(f"build {time.time() - t0:.1f}s: {info}")
    rays = torch.from_numpy(W.rays).to(dev)
    hits = torch.empty((n, 4), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()

    # per-ray traversal statistics from the counting variant (same query)
    (nodes, tris, spills), _ = api.trace_counters(acc, rays)
    node_bytes = 32 * info["node_width"]
    hit_rows = None

    def launch():
        from paper_2603_00292_amd import _capi
        import ctypes as C
        _capi.call("rt_trace_closest", acc.handle, C.c_void_p(rays.data_ptr()), n,
                   C.c_void_p(hits.data_ptr()), None, C.c_void_p(int(torch.cuda.current_stream().cuda_stream)))

    for _ in range(args.warmup):
        launch()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    t_begin = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_begin.record(stream)
    for i in range(args.steps):
        starts[i].record(stream)
        launch()
        ends[i].record(stream)
    t_end.record(stream)
    torch.cuda.synchronize()
    total_ms = t_begin.elapsed_time(t_end)
    per = sorted(s.elapsed_time(e) for s, e in zip(starts, ends))
    ms_per_step = total_ms / args.steps
    mean_launch_ms = sum(per) / len(per)
    value = n / (ms_per_step * 1e-3) / 1e6
    h = hits.cpu().numpy()
    hit_rows = int((h[:, 1].copy().view(np.uint32) != 0xFFFFFFFF).sum())
    bytes_per_launch = (n * (RAY_BYTES + HIT_BYTES) + nodes * node_bytes + tris * TRI_BYTES
                        + hit_rows * FINALIZE_BYTES)
    achieved = bytes_per_launch / (mean_launch_ms * 1e-3) / 1e9
    log(f"closest: {ms_per_step:.3f} ms/step, {value:.1f} Mrays/s; nodes/ray {nodes / n:.2f}, "
        f"tris/ray {tris / n:.2f}, spills/ray {spills / n:.3f}, hits {hit_rows}")

    # secondary: any-hit on the same rays
    occ = torch.empty((n,), dtype=torch.uint8, device=dev)

    def launch_any():
        from paper_2603_00292_amd import _capi
        import ctypes as C
        _capi.call("rt_trace_any", acc.handle, C.c_void_p(rays.data_ptr()), n,
                   C.c_void_p(occ.data_ptr()), C.c_void_p(int(torch.cuda.current_stream().cuda_stream)))

    for _ in range(2):
        launch_any()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        launch_any()
    e1.record(stream)
    torch.cuda.synchronize()
    any_mrays = n / (e0.elapsed_time(e1) / args.steps * 1e-3) / 1e6
    log(f"any-hit: {any_mrays:.1f} Mrays/s")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        S = oracle.OracleScene.from_scene(W.scene)
        sample = 16
        t0 = time.time()
        oracle.closest(S, W.rays[:sample])
        dt = time.time() - t0
        m = int(min(n, max(sample, sample * args.cpu_seconds / max(dt, 1e-3))))
        t0 = time.time()
        oracle.closest(S, W.rays[:m])
        dt = time.time() - t0
        cpu = {"value": m / dt / 1e6, "unit": "Mrays/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"first {m} of the {n} rays, brute force over all {mesh.n_tri} triangles "
                         f"(FP64 linear search), {dt:.1f} s"}
        log(f"oracle: {cpu}")

    out = {
        "metric": "Mrays/s closest-hit incoherent @1M tris",
        "value": round(value, 3),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "icosphere_incoherent", "triangles": int(mesh.n_tri), "rays": int(n),
                   "origins": "U[-1,1]^3", "directions": "uniform sphere", "node_width": info["node_width"],
                   "variant": list(ctx.variant), "query": "closest"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_ray": round(bytes_per_launch / n, 1),
                     "nodes_per_ray": round(nodes / n, 3), "tris_per_ray": round(tris / n, 3),
                     "kernel_ms": round(mean_launch_ms, 4)},
        "cpu_baseline": cpu,
        "secondary": {"any_hit_mrays": round(any_mrays, 3),
                      "launch_ms_min": round(per[0], 4), "launch_ms_median": round(per[len(per) // 2], 4)},
    }
    print(json.dumps(out), flush=True)
    acc.close()
    ctx.close()


if __name__ == "__main__":
    main()
