"""Benchmark: incoherent closest-hit ray queries at about a million triangles.

Headline workload (synthetic, seeded): the noisy icosphere with 1,310,720
triangles (radius 1 +- 0.02) and 4,194,304 rays with origins uniform in
[-1,1]^3 and directions uniform on the sphere, tmin = 0, tmax = +inf.  A step
is one closest-hit query over all rays (rt_trace_closest: the persistent
traversal kernel with the float64 finalize); inputs, accel and outputs are
resident in HBM before timing starts.

Secondary figures (same JSON line, "secondary"): any-hit on the same rays,
the adjoint (rt_trace_backward) on the 262,144-triangle displaced grid with
1,048,576 rays, and 256 meshes traced by one batched launch (HIP graph)
versus 256 per-mesh launches.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import ctypes as C
import hashlib
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
FINALIZE_BYTES = 48  # the winning triangle's record, read again by the float64 finalize
BACKWARD_HIT_BYTES = 32 + 16 + 12 + 12 + 36 + 24 + 36  # per hit ray
BACKWARD_MISS_BYTES = 32 + 16 + 12 + 24
# two-level hit ray: the above, its instance id, instance record and float64
# map, the frame read and its ten gradient words written (miss: + instance id)
BACKWARD_INST_HIT_BYTES = BACKWARD_HIT_BYTES + 4 + 8 + 96 + 40 + 40
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "trace_closest_icosphere_incoherent_pmc_traffic.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2603_00292_amd", "csrc", "rt_kernels.hip")
SQ_FILE = os.path.join(ROOT, "profiles", "trace_closest_icosphere_incoherent_sq_counters.txt")
CU_COUNT, CLOCK_HZ = 256, 2.4e9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sha() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(info, variant):
    """HBM-side bytes per launch of the closest-hit kernel from the committed
    rocprofv3 PMC summary (FETCH_SIZE and WRITE_SIZE, calibrated on a copy of
    known size), or None when the kernel source or configuration differs."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    name = "trace_kernel<%d, %d, %d, false, false, 0, false>" % (
        info["node_width"], variant[0], variant[1])
    sha, val = None, None
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if "rt_kernels.hip sha256[:16] =" in line:
                sha = line.split("=")[-1].strip()
            elif name in line:
                val = int(line.split()[-1])
    return val if sha == kernel_sha() else None


def measured_valu(info, variant):
    """Wave-level VALU instructions and active-lane fraction per launch of the
    closest-hit traversal from the committed SQ counter summary, or None when
    the kernel source or configuration differs."""
    if not os.path.exists(SQ_FILE):
        return None
    name = "trace_kernel<%d, %d, %d, false, false, 0, false>" % (
        info["node_width"], variant[0], variant[1])
    sha, kern, ctr = None, None, {}
    with open(SQ_FILE) as f:
        for line in f:
            if "rt_kernels.hip sha256[:16] =" in line:
                sha = line.split("=")[-1].strip()
            elif line.startswith("# kernel:"):
                kern = line
            elif line.startswith("SQ_"):
                k, v = line.split()
                ctr[k] = int(v)
    if sha != kernel_sha() or kern is None or name not in kern:
        return None
    if not all(k in ctr for k in ("SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_THREAD_CYCLES_VALU")):
        return None
    lanes = ctr["SQ_THREAD_CYCLES_VALU"] / (ctr["SQ_ACTIVE_INST_VALU"] * 64.0)
    return ctr["SQ_INSTS_VALU"], lanes


def copy_bandwidth(torch, stream, dev, reps=5):
    """Achievable HBM bandwidth (GB/s, bytes read + written) of a 1 GiB
    device-to-device copy, mean over `reps` copies timed with HIP events."""
    x = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    x.fill_(1.0)
    y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        y.copy_(x)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 2 * x.numel() * 4
    del x, y
    torch.cuda.empty_cache()
    return nbytes / (ms * 1e-3) / 1e9


def timed(fn, steps, stream, torch):
    """Mean and per-launch durations (ms) of fn() with HIP events on `stream`."""
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    tb, te = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    tb.record(stream)
    for i in range(steps):
        starts[i].record(stream)
        fn()
        ends[i].record(stream)
    te.record(stream)
    torch.cuda.synchronize()
    per = sorted(s.elapsed_time(e) for s, e in zip(starts, ends))
    return tb.elapsed_time(te) / steps, per


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target host time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 512 MiB device copy first (for HBM counter calibration)")
    ap.add_argument("--width", type=int, default=4, help="node width when not autotuning")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--probe", type=int, default=0,
                    help="rays the autotuner times (0: all rays of the workload)")
    ap.add_argument("--only", choices=["backward", "batched", "instanced", "camera", "ao", "phases"],
                    help="run one secondary leg alone and print its figures (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the ray-query path is built and measured on a single "
              "MI355X (rays shard across GPUs with the structure replicated; not measured here).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2603_00292_amd import _capi, api, workloads

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    sptr = C.c_void_p(int(stream.cuda_stream))
    if args.only:
        ctx = api.Context(0)
        legs = {"backward": lambda: backward_bench(args, torch, np, api, workloads, ctx, stream),
                "batched": lambda: batched_bench(args, torch, np, api, _capi, workloads, ctx, stream),
                "instanced": lambda: instanced_bench(args, torch, np, api, workloads, ctx, stream),
                "camera": lambda: camera_bench(args, torch, np, api, workloads, ctx, stream),
                "ao": lambda: ao_bench(args, torch, np, api, workloads, ctx, stream),
                "phases": lambda: phases_bench(args, torch, np, api, workloads, ctx, stream)}
        print(json.dumps({"leg": args.only, **legs[args.only]()}), flush=True)
        ctx.close()
        return
    if args.copy_calibration:
        x = torch.empty(128 * 1024 * 1024, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        x.fill_(1.0)
        y.copy_(x)
        torch.cuda.synchronize()
        log("copy calibration: 536870912 bytes read, 536870912 bytes written")
        del x, y

    t0 = time.time()
    W = workloads.icosphere_incoherent()
    mesh = W.scene.meshes[0]
    n = W.rays.shape[0]
    log(f"workload generated in {time.time() - t0:.1f}s: {mesh.n_tri} triangles, {n} rays")
    ctx = api.Context(0)
    V = torch.from_numpy(mesh.vertices).to(dev)
    I = torch.from_numpy(mesh.indices.view(np.int32)).to(dev)
    rays = torch.from_numpy(W.rays).to(dev)
    tuned = None
    cached = False
    width = args.width
    if not args.no_autotune:
        # untimed: pick node width, stack entries and workgroup on a probe of
        # the workload's own rays (rt_autotune)
        from paper_2603_00292_amd import autotune

        t0 = time.time()
        probe = rays if args.probe <= 0 else rays[: args.probe].contiguous()
        tuned, cached = autotune.choose(ctx, V, I, probe, n, repeats=5)
        width = tuned["node_width"]
        log(f"autotune {time.time() - t0:.1f}s ({'cached' if cached else 'measured'}): {tuned}")
    torch.cuda.synchronize()
    t0 = time.time()
    acc = api.Accel(ctx, [(V, I)], node_width=width)
    build_host_s = time.time() - t0
    info = acc.info
    log(f"build {build_host_s:.3f}s: {info}")
    hits = torch.empty((n, 4), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()

    (nodes, tris, spills), _ = api.trace_counters(acc, rays)
    node_bytes = 32 * info["node_width"]

    def launch():
        _capi.call("rt_trace_closest", acc.handle, C.c_void_p(rays.data_ptr()), n,
                   C.c_void_p(hits.data_ptr()), None, sptr)

    for _ in range(args.warmup):
        launch()
    # HIP events around each timed launch's traversal kernel (rt_context_set_timing)
    ctx.set_timing(args.steps)
    ms_per_step, per = timed(launch, args.steps, stream, torch)
    kernel_ms = ctx.read_timing(args.steps)
    ctx.set_timing(0)
    if len(kernel_ms) != args.steps:
        raise RuntimeError(f"timing ring returned {len(kernel_ms)} of {args.steps} launches")
    mean_kernel_ms = sum(kernel_ms) / len(kernel_ms)
    mean_launch_ms = sum(per) / len(per)
    value = n / (ms_per_step * 1e-3) / 1e6
    h = hits.cpu().numpy()
    hit_rows = int((h[:, 1].copy().view(np.uint32) != 0xFFFFFFFF).sum())
    # the traversal kernel's algorithmic bytes: rays in, hits out, node and
    # triangle fetches, and the float64 finalize its waves run at exit (the
    # ray and hit read again, the winner's record, the final hit written)
    # algorithmic bytes of the query as defined for the roofline: the ray in,
    # the hit out, node and triangle fetches; the float64 finalize that the
    # same kernel runs at exit (ray and hit read again, the winner's record,
    # the final hit written) is reported beside it, not counted in `frac`
    finalize_bytes = n * (RAY_BYTES + 2 * HIT_BYTES) + hit_rows * FINALIZE_BYTES
    bytes_per_launch = n * (RAY_BYTES + HIT_BYTES) + nodes * node_bytes + tris * TRI_BYTES
    achieved = bytes_per_launch / (mean_kernel_ms * 1e-3) / 1e9
    achieved_with_finalize = (bytes_per_launch + finalize_bytes) / (mean_kernel_ms * 1e-3) / 1e9
    log(f"closest: {ms_per_step:.3f} ms/step, {value:.1f} Mrays/s; nodes/ray {nodes / n:.2f}, "
        f"tris/ray {tris / n:.2f}, spills/ray {spills / n:.3f}, hits {hit_rows}")

    traffic = measured_traffic(info, ctx.variant)
    valu = measured_valu(info, ctx.variant)
    copy_gbs = copy_bandwidth(torch, stream, dev)
    log(f"traversal kernel {mean_kernel_ms:.4f} ms (events), whole call {mean_launch_ms:.4f} ms; "
        f"1 GiB copy {copy_gbs:.0f} GB/s")

    secondary = {"launch_ms_min": round(per[0], 4), "launch_ms_median": round(per[len(per) // 2], 4),
                 "nodes_per_ray": round(nodes / n, 3), "tris_per_ray": round(tris / n, 3),
                 "spills_per_ray": round(spills / n, 4)}

    # any-hit on the same rays
    occ = torch.empty((n,), dtype=torch.uint8, device=dev)

    def launch_any():
        _capi.call("rt_trace_any", acc.handle, C.c_void_p(rays.data_ptr()), n,
                   C.c_void_p(occ.data_ptr()), sptr)

    launch_any()
    ms_any, _ = timed(launch_any, args.steps, stream, torch)
    (nodes_a, tris_a, _), _ = api.trace_counters(acc, rays, any_hit=True)
    any_bytes = n * (RAY_BYTES + 1) + nodes_a * node_bytes + tris_a * TRI_BYTES
    secondary["any_hit_mrays"] = round(n / (ms_any * 1e-3) / 1e6, 3)
    secondary["any_hit_bytes_per_ray"] = round(any_bytes / n, 1)
    secondary["any_hit_hbm_frac"] = round(any_bytes / (ms_any * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    log(f"any-hit: {secondary['any_hit_mrays']} Mrays/s, {any_bytes / n:.1f} B/ray")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        # the oracle's float64 BVH walk (answers identical to its linear
        # search), on all host cores and on one; the tree build is not timed
        t0 = time.time()
        S = oracle.OracleScene.from_scene(W.scene, accel=True)
        build_s = time.time() - t0
        cores = oracle.num_threads()

        def oracle_rate(threads, budget):
            oracle.set_num_threads(threads)
            m = 4096
            while True:
                t0 = time.time()
                oracle.closest(S, W.rays[:m])
                dt = time.time() - t0
                if dt >= budget / 3 or m >= n:
                    return m, dt
                m = min(n, int(m * max(2.0, budget / max(dt, 1e-3))))

        m_all, dt_all = oracle_rate(cores, args.cpu_seconds)
        m_one, dt_one = oracle_rate(1, args.cpu_seconds / 2)
        oracle.set_num_threads(cores)
        cpu = {"value": m_all / dt_all / 1e6, "unit": "Mrays/s", "cores": cores, "kind": "oracle",
               "sample": f"first {m_all} of the {n} rays, closest hits by the float64 oracle's BVH walk "
                         f"(bit-identical to its linear search over all {mesh.n_tri} triangles), "
                         f"{dt_all:.1f} s; tree build {build_s:.1f} s not timed",
               "one_thread": {"value": m_one / dt_one / 1e6, "unit": "Mrays/s", "cores": 1,
                              "sample": f"first {m_one} rays, {dt_one:.1f} s"}}
        log(f"oracle: {cpu}")
    acc.close()
    del rays, hits, occ

    if not args.no_secondary:
        secondary.update(device_build_bench(args, torch, api, ctx, stream, V, I, W, width, build_host_s))
        secondary.update(camera_bench(args, torch, np, api, workloads, ctx, stream))
        secondary.update(instanced_bench(args, torch, np, api, workloads, ctx, stream))
        secondary.update(backward_bench(args, torch, np, api, workloads, ctx, stream))
        secondary.update(batched_bench(args, torch, np, api, _capi, workloads, ctx, stream))
        secondary.update(ao_bench(args, torch, np, api, workloads, ctx, stream))

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
                   "variant": list(ctx.variant), "autotuned": tuned is not None,
                   "autotune_cached": bool(tuned is not None and cached), "query": "closest",
                   "inputs_sha256": W.checksum()[:16]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "trace_kernel<%d, %d, %d> closest-hit traversal + float64 finalize" % (
                         info["node_width"], ctx.variant[0], ctx.variant[1]),
                     "bytes_per_ray": round(bytes_per_launch / n, 1), "kernel_ms": round(mean_kernel_ms, 4),
                     "call_ms": round(mean_launch_ms, 4),
                     "finalize_bytes_per_ray": round(finalize_bytes / n, 1),
                     "frac_with_finalize": round(achieved_with_finalize / HBM_PEAK_GBS, 4),
                     "traffic_frac": None if traffic is None else round(
                         traffic / (mean_kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "limiter": "VALU issue (see valu): the measured HBM traffic is below the "
                                "algorithmic bytes, most fetches hit the caches",
                     "copy_GBs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4),
                     "valu": None if valu is None else {
                         "bound": "alu", "wave_instructions": valu[0],
                         "issue_ms": round(valu[0] / (CU_COUNT * CLOCK_HZ) * 1e3, 4),
                         "frac": round(valu[0] / (CU_COUNT * CLOCK_HZ) * 1e3 / mean_kernel_ms, 4),
                         "peak": "1 wave instruction per CU per cycle (256 CUs, 2.4 GHz)",
                         "active_lanes": round(valu[1], 4)}},
        "cpu_baseline": cpu,
        "secondary": secondary,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def backward_bench(args, torch, np, api, workloads, ctx, stream):
    """Adjoint throughput on the displaced grid (262,144 triangles, 1,048,576
    rays): forward once, then time rt_trace_backward."""
    W = workloads.displaced_grid()
    m = W.scene.meshes[0]
    dev = torch.device("cuda:0")
    V = torch.from_numpy(m.vertices).to(dev)
    I = torch.from_numpy(m.indices.view(np.int32)).to(dev)
    acc = api.Accel(ctx, [(V, I)])
    rays = torch.from_numpy(W.rays).to(dev)
    hits, _ = api.trace_closest(acc, rays)
    g = torch.from_numpy(W.extra["abc"]).to(dev)
    dV = torch.zeros_like(V)
    do = torch.empty((rays.shape[0], 3), dtype=torch.float32, device=dev)
    dd = torch.empty_like(do)
    from paper_2603_00292_amd import _capi
    sptr = C.c_void_p(int(stream.cuda_stream))
    n = rays.shape[0]

    def bwd():
        _capi.call("rt_trace_backward", acc.handle, C.c_void_p(rays.data_ptr()), C.c_void_p(hits.data_ptr()),
                   C.c_void_p(g.data_ptr()), n, C.c_void_p(dV.data_ptr()), C.c_void_p(do.data_ptr()),
                   C.c_void_p(dd.data_ptr()), sptr)

    def fwd():
        _capi.call("rt_trace_closest", acc.handle, C.c_void_p(rays.data_ptr()), n,
                   C.c_void_p(hits.data_ptr()), None, sptr)

    bwd()
    ms_b, per_b = timed(bwd, args.steps, stream, torch)
    ms_f, _ = timed(fwd, args.steps, stream, torch)
    # the same calls back to back between one pair of events (the per-call
    # events above add their own gaps to a 0.1 ms call)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        bwd()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_bb = e0.elapsed_time(e1) / args.steps
    nh = int((hits[:, 1].contiguous().view(torch.int32) != -1).sum().item())
    alg = nh * BACKWARD_HIT_BYTES + (n - nh) * BACKWARD_MISS_BYTES
    mean_b = sum(per_b) / len(per_b)
    r = {"backward_mrays": round(n / (ms_b * 1e-3) / 1e6, 3),
         "backward_ms_per_call": round(ms_b, 4),
         "backward_ms_back_to_back": round(ms_bb, 4),
         "backward_forward_mrays": round(n / (ms_f * 1e-3) / 1e6, 3),
         "backward_workload": "displaced_grid_512x256 (262144 triangles), 1048576 rays",
         "backward_hbm_frac": round(alg / (mean_b * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
         "backward_hbm_frac_back_to_back": round(alg / (ms_bb * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    log(f"backward: {r}")
    acc.close()
    return r


def ao_bench(args, torch, np, api, workloads, ctx, stream):
    """The ambient-occlusion workload (§4) on the library: 1024 x 1024 camera
    rays over a 131,072-triangle terrain, 16 AO samples per pixel; one step =
    closest hits, AO rays, any-hit queries and the occluded fraction."""
    W = workloads.ao_terrain()
    m = W.scene.meshes[0]
    dev = torch.device("cuda:0")
    V = torch.from_numpy(m.vertices).to(dev)
    I = torch.from_numpy(m.indices.view(np.int32)).to(dev)
    acc = api.Accel(ctx, [(V, I)])
    rays = torch.from_numpy(W.rays).to(dev)
    xi = torch.from_numpy(W.extra["xi"]).to(dev)
    off, rad = W.extra["offset"], W.extra["radius"]

    def step():
        api.ambient_occlusion(acc, rays, xi, off, rad)

    step()
    ms, _ = timed(step, args.steps, stream, torch)
    n_ao = rays.shape[0] * W.extra["samples"]
    r = {"ao_pipeline_ms": round(ms, 4),
         "ao_mrays": round((rays.shape[0] + n_ao) / (ms * 1e-3) / 1e6, 3),
         "ao_workload": f"{W.name}: {m.indices.shape[0]} triangles, {rays.shape[0]} camera rays, "
                        f"{n_ao} AO rays (closest + AO ray generation + any-hit + resolve)"}
    log(f"ao: {r}")
    acc.close()
    return r


def camera_bench(args, torch, np, api, workloads, ctx, stream):
    """The coherent configuration: 2048^2 pinhole primary rays on the same
    icosphere (closest) and as many shadow rays toward a point light
    (any-hit)."""
    W = workloads.icosphere_camera()
    m = W.scene.meshes[0]
    dev = torch.device("cuda:0")
    acc = api.Accel(ctx, [(torch.from_numpy(m.vertices).to(dev), torch.from_numpy(m.indices.view(np.int32)).to(dev))])
    rays = torch.from_numpy(W.rays).to(dev)
    shadow = torch.from_numpy(W.extra["shadow_rays"]).to(dev)
    ms_c, _ = timed(lambda: api.trace_closest(acc, rays), args.steps, stream, torch)
    ms_a, _ = timed(lambda: api.trace_any(acc, shadow), args.steps, stream, torch)
    r = {"camera_closest_mrays": round(rays.shape[0] / (ms_c * 1e-3) / 1e6, 3),
         "shadow_any_mrays": round(shadow.shape[0] / (ms_a * 1e-3) / 1e6, 3),
         "camera_workload": f"{W.name}: {m.indices.shape[0]} triangles, {rays.shape[0]} primary + "
                            f"{shadow.shape[0]} shadow rays"}
    log(f"camera: {r}")
    acc.close()
    return r


def phases_bench(args, torch, np, api, workloads, ctx, stream):
    """Closest-hit queries on five single-level workloads of different
    coherence and depth, each as one untimed and `steps` timed launches of
    the query kernel followed by one launch of its counting variant with the
    wave-level loop counts (rt_trace_counters_ex).  Under `rocprofv3 --pmc SQ_INSTS_VALU`
    the per-dispatch instruction counts of the query launches, fitted against
    these loop counts, split the kernel's instructions by phase."""
    dev = torch.device("cuda:0")
    ao = workloads.ao_terrain()
    sets = [("icosphere_incoherent", workloads.icosphere_incoherent()),
            ("icosphere_camera", workloads.icosphere_camera()),
            ("displaced_grid", workloads.displaced_grid()),
            ("random_triangles_262144", workloads.random_triangles(n_tri=262144, n_rays=1048576, k=7)),
            ("ao_terrain_camera", ao)]
    out = {}
    for name, W in sets:
        m = W.scene.meshes[0]
        acc = api.Accel(ctx, [(torch.from_numpy(m.vertices).to(dev), torch.from_numpy(m.indices.view(np.int32)).to(dev))],
                        node_width=4)
        rays = torch.from_numpy(W.rays).to(dev)
        api.trace_closest(acc, rays)
        ms, _ = timed(lambda: api.trace_closest(acc, rays), args.steps, stream, torch)
        c = api.trace_phase_counters(acc, rays)
        c["query_ms"] = round(ms, 4)
        c["query_launches"] = args.steps
        out[name] = c
        log(f"phases {name}: {c}")
        acc.close()
    return {"phases": out}


def instanced_bench(args, torch, np, api, workloads, ctx, stream):
    """The two-level configuration: 1,024 SRT instances of four 10k-triangle
    grids, 8,388,608 secondary rays (closest, with instance ids)."""
    W = workloads.instanced_grids()
    dev = torch.device("cuda:0")
    meshes = [(torch.from_numpy(m.vertices).to(dev), torch.from_numpy(m.indices.view(np.int32)).to(dev))
              for m in W.scene.meshes]
    acc = api.Accel(ctx, meshes, W.scene.inst_mesh, W.scene.inst_srt)
    rays = torch.from_numpy(W.rays).to(dev)
    ms, _ = timed(lambda: api.trace_closest(acc, rays, want_inst=True), args.steps, stream, torch)
    (nodes, tris, _), _ = api.trace_counters(acc, rays)
    n = rays.shape[0]
    width = acc.info["node_width"]
    # algorithmic bytes per ray: ray, hit and instance id, node visits of both
    # levels, triangle tests, and the finalize's record and float64 map (the
    # instance records read on entry are not counted: a lower bound)
    bpr = 32 + 16 + 4 + nodes / n * 32 * width + tris / n * 48 + 48 + 96
    # the two-level adjoint on the same rays: vertex and frame gradients
    hits, inst = api.trace_closest(acc, rays, want_inst=True)
    g = torch.from_numpy(np.random.default_rng(316).standard_normal((n, 3)).astype(np.float32)).to(dev)
    dV = torch.zeros((sum(m.vertices.shape[0] for m in W.scene.meshes), 3), dtype=torch.float32, device=dev)
    dS = torch.zeros((W.scene.inst_srt.shape[0], 10), dtype=torch.float32, device=dev)
    bwd = lambda: api.trace_backward_instances(acc, rays, hits, inst, g, dV, dS)
    bwd()
    ms_b, _ = timed(bwd, max(3, args.steps // 4), stream, torch)
    nh = int((hits[:, 1].contiguous().view(torch.int32) != -1).sum().item())
    alg_b = nh * BACKWARD_INST_HIT_BYTES + (n - nh) * BACKWARD_MISS_BYTES
    r = {"instanced_closest_mrays": round(n / (ms * 1e-3) / 1e6, 3),
         "instanced_nodes_per_ray": round(nodes / n, 3), "instanced_tris_per_ray": round(tris / n, 3),
         "instanced_bytes_per_ray": round(bpr, 1),
         "instanced_hbm_frac": round(bpr * n / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
         "instanced_backward_mrays": round(n / (ms_b * 1e-3) / 1e6, 3),
         "instanced_backward_ms": round(ms_b, 4),
         "instanced_backward_hbm_frac": round(alg_b / (ms_b * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
         "instanced_workload": f"{W.name}: 1024 instances of 4 x 10000 triangles, {n} rays"}
    log(f"instanced: {r}")
    acc.close()
    return r


def device_build_bench(args, torch, api, ctx, stream, V, I, W, width, build_host_s):
    """Build times of the host SAH build and the device build of the
    headline mesh (not part of the metric) and closest-hit throughput on the
    device-built tree."""
    rays = torch.from_numpy(W.rays).to(V.device)
    api.Accel(ctx, [(V, I)], node_width=width, device_build=True).close()  # warm-up
    torch.cuda.synchronize()
    t0 = time.time()
    acc = api.Accel(ctx, [(V, I)], node_width=width, device_build=True)
    torch.cuda.synchronize()
    build_dev_s = time.time() - t0
    ms, _ = timed(lambda: api.trace_closest(acc, rays), args.steps, stream, torch)
    r = {"build_host_ms": round(build_host_s * 1e3, 2), "build_device_ms": round(build_dev_s * 1e3, 2),
         "device_tree_closest_mrays": round(rays.shape[0] / (ms * 1e-3) / 1e6, 3),
         "device_tree_sah_cost": round(acc.info["sah_cost"], 2)}
    log(f"device build: {r}")
    acc.close()
    return r


def batched_bench(args, torch, np, api, _capi, workloads, ctx, stream):
    """256 meshes (log-uniform 1k-500k triangles, 1k-1M rays each): one
    batched persistent launch replayed from a HIP graph versus 256 per-mesh
    rt_trace_closest launches on one stream."""
    t0 = time.time()
    works = workloads.batched_meshes()
    dev = torch.device("cuda:0")
    accs, rays = [], []
    for w in works:
        m = w.scene.meshes[0]
        accs.append(api.Accel(ctx, [(torch.from_numpy(m.vertices).to(dev),
                                     torch.from_numpy(m.indices.view(np.int32)).to(dev))]))
        rays.append(torch.from_numpy(w.rays).to(dev))
    total = sum(r.shape[0] for r in rays)
    log(f"batched set up in {time.time() - t0:.1f}s: {total} rays, "
        f"{sum(w.scene.meshes[0].n_tri for w in works)} triangles")
    plan = api.BatchPlan(ctx, accs, rays)
    hits = [torch.empty_like(h) for h in plan.hits]
    sptr = C.c_void_p(int(stream.cuda_stream))

    def per_mesh():
        for a, r, h in zip(accs, rays, hits):
            _capi.call("rt_trace_closest", a.handle, C.c_void_p(r.data_ptr()), r.shape[0],
                       C.c_void_p(h.data_ptr()), None, sptr)

    s2 = torch.cuda.Stream()
    g = plan.graph_exec(s2)

    def batched():
        api.graph_launch(g, stream)

    per_mesh()
    batched()
    steps = max(3, args.steps // 4)
    ms_pm, _ = timed(per_mesh, steps, stream, torch)
    ms_b, _ = timed(batched, steps, stream, torch)
    # fixed costs of one rt_trace_closest call: the host time to enqueue it
    # (Python ctypes call included; the first 64 meshes' calls, so the
    # queue never fills) and the device time of a 64-ray launch (fill,
    # persistent traversal and overflow-finalize kernels back to back)
    torch.cuda.synchronize()
    t_host = time.perf_counter()
    for a, r, h in list(zip(accs, rays, hits))[:64]:
        _capi.call("rt_trace_closest", a.handle, C.c_void_p(r.data_ptr()), r.shape[0],
                   C.c_void_p(h.data_ptr()), None, sptr)
    host_us = (time.perf_counter() - t_host) / 64 * 1e6
    torch.cuda.synchronize()
    small, hsmall = rays[0][:64].contiguous(), torch.empty((64, 4), dtype=torch.float32, device=dev)

    def tiny():
        for _ in range(100):
            _capi.call("rt_trace_closest", accs[0].handle, C.c_void_p(small.data_ptr()), 64,
                       C.c_void_p(hsmall.data_ptr()), None, sptr)

    tiny()
    ms_tiny, _ = timed(tiny, 3, stream, torch)
    same = all(torch.equal(a.view(torch.int32), b.view(torch.int32)) for a, b in zip(hits, plan.hits))
    # algorithmic bytes of the whole plan: sum over meshes of rays x (ray +
    # hit + finalize) plus their node and triangle fetches (counting variant)
    alg = 0
    footprint = 0
    for a, r, h in zip(accs, rays, hits):
        (nodes, tris, _), _ = api.trace_counters(a, r)
        n_hit = int((h[:, 1].view(torch.int32) != -1).sum().item())
        nb = 32 * a.info["node_width"]
        alg += r.shape[0] * (RAY_BYTES + HIT_BYTES) + nodes * nb + tris * TRI_BYTES
        alg += r.shape[0] * (RAY_BYTES + 2 * HIT_BYTES) + n_hit * FINALIZE_BYTES
        footprint += a.info["device_bytes"]
    r = {"batched_mrays": round(total / (ms_b * 1e-3) / 1e6, 3),
         "per_mesh_mrays": round(total / (ms_pm * 1e-3) / 1e6, 3),
         "batched_vs_per_mesh": round(ms_pm / ms_b, 3),
         "batched_identical": bool(same),
         "batched_bytes_per_ray": round(alg / total, 1),
         "batched_hbm_frac": round(alg / (ms_b * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
         "batched_accel_bytes": int(footprint),
         "batched_workload": f"256 meshes, {total} rays",
         "per_call_host_us": round(host_us, 2),
         "per_call_64_rays_device_us": round(ms_tiny * 1e3 / 100, 2)}
    log(f"batched: {r}")
    plan.close()
    for a in accs:
        a.close()
    return r


if __name__ == "__main__":
    main()
