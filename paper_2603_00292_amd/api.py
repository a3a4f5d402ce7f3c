"""Torch-facing wrappers over the C ABI (device memory and streams only).

Every query runs in librtq's HIP kernels; these functions only check tensor
shapes/devices, allocate outputs with torch and pass raw pointers and the
current HIP stream.  ``RayQueryFn`` adds the adjoint as a
``torch.autograd.Function``.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _capi as capi


def _stream() -> int:
    return int(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor | None):
    return None if t is None else C.c_void_p(t.data_ptr())


def _require(t: torch.Tensor, name: str, dtype, last: int | None = None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU (got {t.device})")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if last is not None and (t.dim() != 2 or t.shape[1] != last):
        raise ValueError(f"{name} must have shape (n, {last}) (got {tuple(t.shape)})")


class Context:
    """An rt_context on one HIP device (default: torch's current device)."""

    def __init__(self, device: int | None = None, stack_entries: int | None = None,
                 workgroup: int | None = None):
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        h = C.c_void_p()
        capi.call("rt_context_create", self.device, C.byref(h))
        self.handle = h
        if stack_entries is not None or workgroup is not None:
            v = self.variant
            self.set_variant(stack_entries or v[0], workgroup or v[1])

    @property
    def variant(self):
        v = capi.rt_variant()
        capi.call("rt_context_get_variant", self.handle, C.byref(v))
        return int(v.stack_entries), int(v.workgroup)

    def set_variant(self, stack_entries: int, workgroup: int):
        v = capi.rt_variant(int(stack_entries), int(workgroup))
        capi.call("rt_context_set_variant", self.handle, C.byref(v))

    def set_timing(self, slots: int):
        """Record HIP events around the traversal kernel of the next query
        calls, in `slots` pairs used round-robin (0: off)."""
        capi.call("rt_context_set_timing", self.handle, int(slots))

    def read_timing(self, capacity: int = 4096):
        """Traversal-kernel durations (ms) of the launches timed since the
        last read, oldest first."""
        buf = (C.c_float * max(int(capacity), 1))()
        cnt = C.c_uint32()
        capi.call("rt_context_read_timing", self.handle, C.cast(buf, C.c_void_p), int(capacity), C.byref(cnt))
        return [float(buf[i]) for i in range(cnt.value)]

    def close(self):
        if self.handle:
            capi.call("rt_context_destroy", self.handle)
            self.handle = None


class Accel:
    """An acceleration structure built with ``rt_build`` (on the host with
    binned SAH, or on the GPU with ``device_build=True``).

    meshes: list of (vertices (V,3) float32 cuda, indices (N,3) int32/uint32
    cuda).  Single level: one mesh and no instances.  Two-level:
    ``inst_mesh`` (J,) and ``inst_srt`` (J,10) host arrays (numpy or CPU
    tensors) of mesh ids and (sx,sy,sz,qx,qy,qz,qw,tx,ty,tz) frames."""

    def __init__(self, ctx: Context, meshes, inst_mesh=None, inst_srt=None, node_width: int = 0,
                 max_leaf_size: int = 0, device_build: bool = False):
        import numpy as np

        self.ctx = ctx
        self._keep = []
        descs = (capi.rt_mesh_desc * len(meshes))()
        for i, (v, f) in enumerate(meshes):
            _require(v, "vertices", torch.float32, 3)
            if f.dtype not in (torch.int32, torch.uint32):
                raise ValueError("indices must be int32 or uint32")
            if not f.is_contiguous() or f.dim() != 2 or f.shape[1] != 3 or f.device.type != "cuda":
                raise ValueError("indices must be a contiguous (N,3) cuda tensor")
            descs[i] = capi.rt_mesh_desc(v.data_ptr() if v.numel() else None, v.shape[0], 12,
                                         f.data_ptr() if f.numel() else None, f.shape[0], 12)
            self._keep += [v, f]
        self.vertex_count = int(meshes[0][0].shape[0])
        self.vertex_counts = [int(v.shape[0]) for v, _ in meshes]
        n_inst = 0
        im_p = srt_p = None
        if inst_mesh is not None:
            im = np.ascontiguousarray(np.asarray(inst_mesh), dtype=np.uint32).reshape(-1)
            srt = np.ascontiguousarray(np.asarray(inst_srt), dtype=np.float32).reshape(-1, 10)
            if srt.shape[0] != im.shape[0]:
                raise ValueError("inst_mesh and inst_srt lengths differ")
            n_inst = im.shape[0]
            self._im, self._srt = im, srt
            im_p = C.c_void_p(im.ctypes.data)
            srt_p = C.c_void_p(srt.ctypes.data)
        opts = capi.rt_build_options(int(node_width), int(max_leaf_size),
                                     capi.RT_BUILD_DEVICE if device_build else 0)
        h = C.c_void_p()
        capi.call("rt_build", ctx.handle, descs, len(meshes), im_p, srt_p, n_inst, C.byref(opts),
                  C.c_void_p(_stream()), C.byref(h))
        self.handle = h
        self.two_level = n_inst > 0
        self.instance_count = n_inst
        self._keep = []

    @property
    def info(self) -> dict:
        i = capi.rt_accel_info()
        capi.call("rt_accel_get_info", self.handle, C.byref(i))
        return {f: getattr(i, f) for f, _ in capi.rt_accel_info._fields_}

    def refit(self, vertices: torch.Tensor) -> None:
        """Fits the boxes to new vertex positions on the device, keeping the
        tree topology (rt_refit).  Two-level accels take every mesh's vertices
        one after another in build order."""
        _require(vertices, "vertices", torch.float32, 3)
        want = sum(self.vertex_counts) if self.two_level else self.vertex_count
        if vertices.shape[0] != want:
            raise ValueError(f"refit needs {want} vertices, got {vertices.shape[0]}")
        capi.call("rt_refit", self.handle, _ptr(vertices), C.c_void_p(_stream()))

    def update_instances(self, inst_srt) -> None:
        """rt_update_instances: new (J,10) frames (host array) for every
        instance; the top-level boxes are refit, the meshes' trees kept."""
        import numpy as np

        srt = np.ascontiguousarray(np.asarray(inst_srt), dtype=np.float32)
        if srt.shape != (self.instance_count, 10):
            raise ValueError(f"need ({self.instance_count}, 10) frames, got {srt.shape}")
        capi.call("rt_update_instances", self.handle, C.c_void_p(srt.ctypes.data), C.c_void_p(_stream()))

    def set_instance_masks(self, masks) -> None:
        """Visibility masks of the instances (host array, one uint32 each),
        ANDed with the ray masks of the _ex and all-hit queries."""
        import numpy as np

        m = np.ascontiguousarray(np.asarray(masks), dtype=np.uint32).reshape(-1)
        if m.shape[0] != self.instance_count:
            raise ValueError(f"need {self.instance_count} masks, got {m.shape[0]}")
        capi.call("rt_accel_set_instance_masks", self.handle, C.c_void_p(m.ctypes.data),
                  C.c_void_p(_stream()))

    def close(self):
        if self.handle:
            capi.call("rt_accel_destroy", self.handle)
            self.handle = None


def trace_closest(accel: Accel, rays: torch.Tensor, want_inst: bool = False):
    """Closest hits of rays (n,8) float32: returns (hits (n,4) float32 with
    columns t, prim_id bits, u, v; inst_ids (n,) int32 or None)."""
    _require(rays, "rays", torch.float32, 8)
    n = rays.shape[0]
    hits = torch.empty((n, 4), dtype=torch.float32, device=rays.device)
    inst = torch.empty((n,), dtype=torch.int32, device=rays.device) if want_inst else None
    capi.call("rt_trace_closest", accel.handle, _ptr(rays), n, _ptr(hits), _ptr(inst),
              C.c_void_p(_stream()))
    return hits, inst


def trace_closest_noalloc(accel: Accel, rays: torch.Tensor, hits: torch.Tensor,
                          inst: torch.Tensor | None = None) -> None:
    """rt_trace_closest_noalloc into caller-provided outputs (hits (n,4)
    float32, inst (n,) int32 or None): the library allocates nothing."""
    _require(rays, "rays", torch.float32, 8)
    n = rays.shape[0]
    _require(hits, "hits", torch.float32, 4)
    if hits.shape[0] != n or (inst is not None and (inst.shape != (n,) or inst.dtype != torch.int32
                                                     or not inst.is_contiguous())):
        raise ValueError("hits must be (n,4) float32 and inst (n,) int32, contiguous")
    capi.call("rt_trace_closest_noalloc", accel.handle, _ptr(rays), n, _ptr(hits), _ptr(inst),
              C.c_void_p(_stream()))


def _u32_vec(t, n, name):
    if t is None:
        return None
    if t.dtype not in (torch.int32, torch.uint32) or not t.is_contiguous() or t.device.type != "cuda" \
            or t.shape != (n,):
        raise ValueError(f"{name} must be a contiguous ({n},) int32 cuda tensor")
    return t


def _options(n, ray_masks, skip_inst, skip_prim):
    """rt_query_options for per-ray tensors (kept alive by the caller)."""
    if ray_masks is None and skip_inst is None and skip_prim is None:
        return None
    o = capi.rt_query_options()
    for f, t in (("ray_masks", ray_masks), ("skip_inst", skip_inst), ("skip_prim", skip_prim)):
        t = _u32_vec(t, n, f)
        setattr(o, f, t.data_ptr() if t is not None and t.numel() else None)
    return o


def trace_closest_ex(accel: Accel, rays: torch.Tensor, ray_masks=None, skip_inst=None,
                     skip_prim=None, want_inst: bool = False):
    """rt_trace_closest_ex: closest hits under ray masks and the per-ray
    skipped triangle; returns (hits (n,4), inst_ids (n,) or None)."""
    _require(rays, "rays", torch.float32, 8)
    n = rays.shape[0]
    opts = _options(n, ray_masks, skip_inst, skip_prim)
    hits = torch.empty((n, 4), dtype=torch.float32, device=rays.device)
    inst = torch.empty((n,), dtype=torch.int32, device=rays.device) if want_inst else None
    capi.call("rt_trace_closest_ex", accel.handle, _ptr(rays), n, C.byref(opts) if opts else None,
              _ptr(hits), _ptr(inst), C.c_void_p(_stream()))
    return hits, inst


def trace_any_ex(accel: Accel, rays: torch.Tensor, ray_masks=None, skip_inst=None, skip_prim=None):
    _require(rays, "rays", torch.float32, 8)
    n = rays.shape[0]
    opts = _options(n, ray_masks, skip_inst, skip_prim)
    occ = torch.empty((n,), dtype=torch.uint8, device=rays.device)
    capi.call("rt_trace_any_ex", accel.handle, _ptr(rays), n, C.byref(opts) if opts else None,
              _ptr(occ), C.c_void_p(_stream()))
    return occ


def trace_all(accel: Accel, rays: torch.Tensor, capacity: int, ray_masks=None, skip_inst=None,
              skip_prim=None, want_inst: bool = False):
    """rt_trace_all: per ray, the number of hits and the `capacity` nearest
    sorted by (t, instance, prim).  Returns (hits (n, capacity, 4),
    inst_ids (n, capacity) or None, counts (n,) int32)."""
    _require(rays, "rays", torch.float32, 8)
    n = rays.shape[0]
    opts = _options(n, ray_masks, skip_inst, skip_prim)
    hits = torch.empty((n, capacity, 4), dtype=torch.float32, device=rays.device)
    inst = torch.empty((n, capacity), dtype=torch.int32, device=rays.device) if want_inst else None
    counts = torch.empty((n,), dtype=torch.int32, device=rays.device)
    capi.call("rt_trace_all", accel.handle, _ptr(rays), n, C.byref(opts) if opts else None,
              int(capacity), _ptr(hits), _ptr(inst), _ptr(counts), C.c_void_p(_stream()))
    return hits, inst, counts


def ao_rays(accel: Accel, rays: torch.Tensor, hits: torch.Tensor, xi: torch.Tensor, offset: float,
            radius: float, inst_ids: torch.Tensor | None = None) -> torch.Tensor:
    """rt_ao_rays (rt_ao_rays_instances with the hits' inst_ids on a
    two-level accel): (n * samples, 8) ambient-occlusion rays from closest
    hits; xi (n, samples, 2) float32 uniforms on the device."""
    _require(rays, "rays", torch.float32, 8)
    _require(hits, "hits", torch.float32, 4)
    n = rays.shape[0]
    if inst_ids is not None and (inst_ids.dtype not in (torch.int32, torch.uint32) or not inst_ids.is_contiguous()
                                 or inst_ids.shape != (n,) or inst_ids.device.type != "cuda"):
        raise ValueError("inst_ids must be a contiguous (n,) int32 cuda tensor")
    if xi.dtype != torch.float32 or not xi.is_contiguous() or xi.dim() != 3 or xi.shape[0] != n \
            or xi.shape[2] != 2 or xi.device.type != "cuda":
        raise ValueError("xi must be a contiguous (n, samples, 2) float32 cuda tensor")
    samples = xi.shape[1]
    out = torch.empty((n * samples, 8), dtype=torch.float32, device=rays.device)
    if inst_ids is None:
        capi.call("rt_ao_rays", accel.handle, _ptr(rays), _ptr(hits), n, samples, _ptr(xi), float(offset),
                  float(radius), _ptr(out), C.c_void_p(_stream()))
    else:
        capi.call("rt_ao_rays_instances", accel.handle, _ptr(rays), _ptr(hits), _ptr(inst_ids), n, samples,
                  _ptr(xi), float(offset), float(radius), _ptr(out), C.c_void_p(_stream()))
    return out


def ao_resolve(occluded: torch.Tensor, samples: int) -> torch.Tensor:
    """rt_ao_resolve: per-ray occluded fraction of `samples` occlusion bytes."""
    if occluded.dtype != torch.uint8 or not occluded.is_contiguous() or occluded.device.type != "cuda":
        raise ValueError("occluded must be a contiguous uint8 cuda tensor")
    n = occluded.numel() // samples
    ao = torch.empty((n,), dtype=torch.float32, device=occluded.device)
    capi.call("rt_ao_resolve", _ptr(occluded), n, int(samples), _ptr(ao), C.c_void_p(_stream()))
    return ao


def ambient_occlusion(accel: Accel, rays: torch.Tensor, xi: torch.Tensor, offset: float,
                      radius: float):
    """The ambient-occlusion workload of §4 on the library: closest hits of
    the primary rays, AO rays from them, any-hit queries, occluded fraction.
    Returns (ao (n,), hits (n,4), ao_rays (n*samples, 8), occluded)."""
    two = bool(getattr(accel, "two_level", False))
    hits, inst = trace_closest(accel, rays, want_inst=two)
    ar = ao_rays(accel, rays, hits, xi, offset, radius, inst_ids=inst)
    occ = trace_any(accel, ar)
    return ao_resolve(occ, xi.shape[1]), hits, ar, occ


def hit_fields(hits: torch.Tensor):
    """(t, prim_id (int64, -1 for a miss), u, v) views of a hit tensor."""
    t = hits[:, 0]
    prim = hits[:, 1].contiguous().view(torch.int32).to(torch.int64)
    return t, prim, hits[:, 2], hits[:, 3]


def trace_any(accel: Accel, rays: torch.Tensor) -> torch.Tensor:
    _require(rays, "rays", torch.float32, 8)
    n = rays.shape[0]
    occ = torch.empty((n,), dtype=torch.uint8, device=rays.device)
    capi.call("rt_trace_any", accel.handle, _ptr(rays), n, _ptr(occ), C.c_void_p(_stream()))
    return occ


def trace_counters(accel: Accel, rays: torch.Tensor, any_hit: bool = False, peak: bool = False):
    """Runs the counting variant; returns (node visits, triangle tests,
    spilled stack entries) summed over the rays (with peak=True also the
    deepest stack fill of any ray), and the query's output."""
    _require(rays, "rays", torch.float32, 8)
    n = rays.shape[0]
    cnt = torch.zeros((4,), dtype=torch.int64, device=rays.device)
    hits = occ = None
    if any_hit:
        occ = torch.empty((n,), dtype=torch.uint8, device=rays.device)
    else:
        hits = torch.empty((n, 4), dtype=torch.float32, device=rays.device)
    capi.call("rt_trace_counters", accel.handle, _ptr(rays), n, int(any_hit), _ptr(hits), _ptr(occ),
              _ptr(cnt), C.c_void_p(_stream()))
    c = cnt.cpu().tolist()
    if peak:
        return (c[0], c[1], c[2], c[3]), (occ if any_hit else hits)
    return (c[0], c[1], c[2]), (occ if any_hit else hits)


def trace_phase_counters(accel: Accel, rays: torch.Tensor, any_hit: bool = False) -> dict:
    """rt_trace_counters_ex with 8 counters: the lane-level work (node
    visits, triangle tests) and the wave-level loop counts of the counting
    kernel (outer passes, refills, node-loop and leaf-loop iterations), with
    the lane occupancy of the node and leaf phases."""
    _require(rays, "rays", torch.float32, 8)
    n = rays.shape[0]
    cnt = torch.zeros((8,), dtype=torch.int64, device=rays.device)
    hits = occ = None
    if any_hit:
        occ = torch.empty((n,), dtype=torch.uint8, device=rays.device)
    else:
        hits = torch.empty((n, 4), dtype=torch.float32, device=rays.device)
    capi.call("rt_trace_counters_ex", accel.handle, _ptr(rays), n, int(any_hit), _ptr(hits), _ptr(occ),
              _ptr(cnt), 8, C.c_void_p(_stream()))
    c = cnt.cpu().tolist()
    return {"rays": n, "node_visits": c[0], "tri_tests": c[1], "spills": c[2], "deepest": c[3],
            "outer_passes": c[4], "refills": c[5], "node_iters": c[6], "leaf_iters": c[7],
            "node_lane_occupancy": c[0] / max(64 * c[6], 1), "leaf_lane_occupancy": c[1] / max(64 * c[7], 1)}


def trace_backward(accel: Accel, rays: torch.Tensor, hits: torch.Tensor, d_tuv: torch.Tensor,
                   d_vertices: torch.Tensor):
    """Adjoint at fixed triangles; d_vertices is accumulated in place.
    Returns (d_origins (n,3), d_directions (n,3))."""
    _require(rays, "rays", torch.float32, 8)
    _require(hits, "hits", torch.float32, 4)
    _require(d_tuv, "d_tuv", torch.float32, 3)
    _require(d_vertices, "d_vertices", torch.float32, 3)
    n = rays.shape[0]
    do = torch.empty((n, 3), dtype=torch.float32, device=rays.device)
    dd = torch.empty((n, 3), dtype=torch.float32, device=rays.device)
    capi.call("rt_trace_backward", accel.handle, _ptr(rays), _ptr(hits), _ptr(d_tuv), n,
              _ptr(d_vertices), _ptr(do), _ptr(dd), C.c_void_p(_stream()))
    return do, dd


def trace_backward_instances(accel: Accel, rays: torch.Tensor, hits: torch.Tensor,
                             inst_ids: torch.Tensor, d_tuv: torch.Tensor,
                             d_vertices: torch.Tensor | None = None,
                             d_srt: torch.Tensor | None = None):
    """Two-level adjoint (rt_trace_backward_instances).  d_vertices
    (sum of vertex counts, 3) holds the meshes' object-space vertex gradients
    one after another in build order; d_srt (instances, 10) the frame
    gradients; both accumulated in place when given.  Returns (d_origins,
    d_directions), each (n,3)."""
    _require(rays, "rays", torch.float32, 8)
    _require(hits, "hits", torch.float32, 4)
    _require(d_tuv, "d_tuv", torch.float32, 3)
    if inst_ids.dtype not in (torch.int32, torch.uint32) or not inst_ids.is_contiguous() \
            or inst_ids.device.type != "cuda" or inst_ids.shape != (rays.shape[0],):
        raise ValueError("inst_ids must be a contiguous (n,) int32 cuda tensor")
    if d_vertices is not None:
        _require(d_vertices, "d_vertices", torch.float32, 3)
        if d_vertices.shape[0] != sum(accel.vertex_counts):
            raise ValueError(f"d_vertices needs {sum(accel.vertex_counts)} rows")
    if d_srt is not None:
        _require(d_srt, "d_srt", torch.float32, 10)
        if d_srt.shape[0] != accel.instance_count:
            raise ValueError(f"d_srt needs {accel.instance_count} rows")
    n = rays.shape[0]
    do = torch.empty((n, 3), dtype=torch.float32, device=rays.device)
    dd = torch.empty((n, 3), dtype=torch.float32, device=rays.device)
    capi.call("rt_trace_backward_instances", accel.handle, _ptr(rays), _ptr(hits), _ptr(inst_ids),
              _ptr(d_tuv), n, _ptr(d_vertices), _ptr(d_srt), _ptr(do), _ptr(dd),
              C.c_void_p(_stream()))
    return do, dd


class RayQueryFn(torch.autograd.Function):
    """Differentiable closest hit.

    forward(accel, vertices, origins, directions, tmin, tmax) ->
    (t, u, v, prim_id).  ``vertices`` must be the (V,3) tensor the accel was
    built from; gradients flow to vertices, origins and directions through
    the hand-written adjoint kernel (rt_trace_backward)."""

    @staticmethod
    def forward(ctx, accel, vertices, origins, directions, tmin, tmax):
        n = origins.shape[0]
        rays = torch.empty((n, 8), dtype=torch.float32, device=origins.device)
        rays[:, 0:3] = origins
        rays[:, 3] = tmin
        rays[:, 4:7] = directions
        rays[:, 7] = tmax
        hits, _ = trace_closest(accel, rays)
        t, prim, u, v = hit_fields(hits)
        ctx.accel = accel
        ctx.save_for_backward(rays, hits)
        ctx.vshape = vertices.shape
        ctx.mark_non_differentiable(prim)
        return t.clone(), u.clone(), v.clone(), prim

    @staticmethod
    def backward(ctx, gt, gu, gv, gprim):
        rays, hits = ctx.saved_tensors
        n = rays.shape[0]
        z = torch.zeros(n, dtype=torch.float32, device=rays.device)
        d_tuv = torch.stack([gt if gt is not None else z, gu if gu is not None else z,
                             gv if gv is not None else z], 1).contiguous().float()
        dV = torch.zeros(ctx.vshape, dtype=torch.float32, device=rays.device)
        do, dd = trace_backward(ctx.accel, rays, hits, d_tuv, dV)
        return None, dV, do, dd, None, None


class InstanceRayQueryFn(torch.autograd.Function):
    """Differentiable closest hit on a two-level accel.

    forward(accel, vertices, srt, origins, directions, tmin, tmax) ->
    (t, u, v, prim_id, inst_id).  ``vertices`` (sum of vertex counts, 3) are
    the meshes' vertices the accel was built from, one mesh after another in
    build order, and ``srt`` (instances, 10) its frames; gradients flow to
    them and to the rays through rt_trace_backward_instances."""

    @staticmethod
    def forward(ctx, accel, vertices, srt, origins, directions, tmin, tmax):
        n = origins.shape[0]
        rays = torch.empty((n, 8), dtype=torch.float32, device=origins.device)
        rays[:, 0:3] = origins
        rays[:, 3] = tmin
        rays[:, 4:7] = directions
        rays[:, 7] = tmax
        hits, inst = trace_closest(accel, rays, want_inst=True)
        t, prim, u, v = hit_fields(hits)
        ctx.accel = accel
        ctx.save_for_backward(rays, hits, inst)
        ctx.vshape = vertices.shape
        ctx.srt_device = srt.device
        inst64 = inst.to(torch.int64)
        inst64[prim < 0] = -1
        ctx.mark_non_differentiable(prim, inst64)
        return t.clone(), u.clone(), v.clone(), prim, inst64

    @staticmethod
    def backward(ctx, gt, gu, gv, gprim, ginst):
        rays, hits, inst = ctx.saved_tensors
        n = rays.shape[0]
        z = torch.zeros(n, dtype=torch.float32, device=rays.device)
        d_tuv = torch.stack([gt if gt is not None else z, gu if gu is not None else z,
                             gv if gv is not None else z], 1).contiguous().float()
        dV = torch.zeros(ctx.vshape, dtype=torch.float32, device=rays.device)
        dS = torch.zeros((ctx.accel.instance_count, 10), dtype=torch.float32, device=rays.device)
        do, dd = trace_backward_instances(ctx.accel, rays, hits, inst, d_tuv, dV, dS)
        return None, dV, dS.to(ctx.srt_device), do, dd, None, None


class BatchPlan:
    """Closest-hit queries of many (accel, rays) pairs in one persistent
    launch; ``graph()`` captures it into a HIP graph for replay."""

    def __init__(self, ctx: Context, accels, rays_list, hits_list=None, want_inst: bool = False):
        """accels all single-level or all two-level; with want_inst (two-level
        plans) ``self.inst_ids`` receives each batch's instance ids."""
        n = len(accels)
        if hits_list is None:
            hits_list = [torch.empty((r.shape[0], 4), dtype=torch.float32, device=r.device)
                         for r in rays_list]
        for r, h in zip(rays_list, hits_list):
            _require(r, "rays", torch.float32, 8)
            _require(h, "hits", torch.float32, 4)
        self.hits = hits_list
        self._rays = rays_list
        self.inst_ids = ([torch.empty((r.shape[0],), dtype=torch.int32, device=r.device) for r in rays_list]
                         if want_inst else None)
        A = (C.c_void_p * n)(*[a.handle.value for a in accels])
        R = (C.c_void_p * n)(*[r.data_ptr() if r.numel() else None for r in rays_list])
        H = (C.c_void_p * n)(*[h.data_ptr() if h.numel() else None for h in hits_list])
        cnt = (C.c_uint32 * n)(*[r.shape[0] for r in rays_list])
        h = C.c_void_p()
        if want_inst:
            I = (C.c_void_p * n)(*[t.data_ptr() if t.numel() else None for t in self.inst_ids])
            capi.call("rt_batch_plan_create_instances", ctx.handle, A, R, H, I, cnt, n, C.byref(h))
        else:
            capi.call("rt_batch_plan_create", ctx.handle, A, R, H, cnt, n, C.byref(h))
        self.handle = h
        self._graph = None

    def launch(self):
        capi.call("rt_batch_plan_launch", self.handle, C.c_void_p(_stream()))

    def graph_exec(self, stream: torch.cuda.Stream) -> int:
        g = C.c_void_p()
        capi.call("rt_batch_plan_graph", self.handle, C.c_void_p(int(stream.cuda_stream)), C.byref(g))
        return int(g.value)

    def close(self):
        if self.handle:
            capi.call("rt_batch_plan_destroy", self.handle)
            self.handle = None


_hip = None


def graph_launch(graph_exec: int, stream: torch.cuda.Stream | None = None) -> None:
    """Replays a graph returned by ``BatchPlan.graph_exec`` (hipGraphLaunch)."""
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipGraphLaunch.argtypes = [C.c_void_p, C.c_void_p]
        _hip.hipGraphLaunch.restype = C.c_int
    s = stream if stream is not None else torch.cuda.current_stream()
    rc = _hip.hipGraphLaunch(C.c_void_p(graph_exec), C.c_void_p(int(s.cuda_stream)))
    if rc != 0:
        raise RuntimeError(f"hipGraphLaunch failed with HIP error {rc}")
