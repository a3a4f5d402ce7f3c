"""FP64 CPU oracle for the ray-query path (TEST INFRASTRUCTURE ONLY).

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The product library never
loads it: it is the independent reference the HIP path is checked against.

The arithmetic lives in ``rt_oracle.c`` (plain C, double precision, OpenMP
over rays); this module compiles it with gcc and marshals numpy arrays.

Every query is defined by the linear search over all triangles (the
paper's §3.3 search for the closest hit) with the plane-then-edge test of
§3.1; a scene built with ``accel=True`` carries an FP64 BVH whose walk only
skips pairs that cannot matter, so it returns the same answers bit for bit
(§6.2: the hierarchy accelerates the search).  See
the header of ``rt_oracle.c`` for the readings taken where the paper is
silent.  ``accept`` implements the FP32 tolerance model (acceptable sets),
``adjoint`` the implicit-function adjoint of (t,u,v) and ``fd`` central finite
differences of the plane formula.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rt_oracle.c")
_HDR = os.path.join(_HERE, "rt_oracle.h")
_OUT_DIR = os.path.join(_HERE, "_build")
LIB_PATH = os.path.join(_OUT_DIR, "librt_oracle.so")

NONE = 0xFFFFFFFF
DELTA = 2.0 ** -20  # relative input slack of the acceptable-set model (16 float32 unit roundoffs)

_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    os.makedirs(_OUT_DIR, exist_ok=True)
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
               "-ffp-contract=off", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            build(force=False)
        lib = C.CDLL(LIB_PATH)
        P = C.c_void_p
        i64 = C.c_int64
        for name, args in {
            "orc_closest": [P, P, i64, P, P, P],
            "orc_any": [P, P, i64, P],
            "orc_closest_ex": [P, P, i64, P, P, P, P],
            "orc_any_ex": [P, P, i64, P, P],
            "orc_all": [P, P, i64, P, C.c_int32, P, P, P, P],
            "orc_accept_ex": [P, P, i64, P, C.c_double, C.c_int32, P, P, P, P, P, P, P],
            "orc_classify_all": [P, P, i64, P, C.c_double, C.c_int32, P, P, P, P, P, P, P, P, P],
            "orc_accept": [P, P, i64, C.c_double, C.c_int32, P, P, P, P, P, P, P],
            "orc_adjoint": [P, P, P, i64, P, P, P, P],
            "orc_fd": [P, P, P, i64, P, C.c_double, P],
            "orc_fixed_tuv": [P, P, P, i64, P],
            "orc_adjoint_inst": [P, P, P, P, i64, P, P, P, P, P],
            "orc_fd_inst": [P, P, P, P, i64, P, C.c_double, P],
            "orc_ao_rays": [P, P, P, P, i64, C.c_int32, P, C.c_double, C.c_double, P],
            "orc_ao_rays_inst": [P, P, P, P, P, i64, C.c_int32, P, C.c_double, C.c_double, P],
        }.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = C.c_int
        lib.orc_num_threads.restype = C.c_int
        lib.orc_set_num_threads.argtypes = [C.c_int]
        lib.orc_bvh_create.argtypes = [C.c_void_p, C.POINTER(C.c_void_p)]
        lib.orc_bvh_create.restype = C.c_int
        lib.orc_bvh_destroy.argtypes = [C.c_void_p]
        lib.orc_bvh_destroy.restype = None
        lib.orc_bvh_stats.argtypes = [C.c_void_p, C.c_void_p]
        lib.orc_bvh_stats.restype = C.c_int
        lib.orc_bvh_check.argtypes = [C.c_void_p, C.c_void_p, i64, C.c_int, C.c_double, C.c_void_p]
        lib.orc_bvh_check.restype = C.c_int
        _lib = lib
        return lib


class _Scene(C.Structure):
    _fields_ = [
        ("n_mesh", C.c_int32),
        ("vertices", C.c_void_p),
        ("n_vertices", C.c_void_p),
        ("indices", C.c_void_p),
        ("n_triangles", C.c_void_p),
        ("n_inst", C.c_int64),
        ("inst_mesh", C.c_void_p),
        ("inst_srt", C.c_void_p),
        ("bvh", C.c_void_p),
    ]


class OracleScene:
    """Holds contiguous float32/uint32 copies of a scene and its C descriptor.

    ``meshes``: list of (vertices (V,3) float32, indices (N,3) uint32).
    ``inst_mesh``/``inst_srt``: optional instance arrays (see workloads).
    ``accel``: also build the FP64 BVH (``orc_bvh_create``); every query then
    walks it instead of scanning every triangle, with identical answers."""

    def __init__(self, meshes, inst_mesh=None, inst_srt=None, accel: bool = False):
        self._bvh = None
        self._v = [np.ascontiguousarray(v, dtype=np.float32).reshape(-1, 3) for v, _ in meshes]
        self._i = [np.ascontiguousarray(i, dtype=np.uint32).reshape(-1, 3) for _, i in meshes]
        n = len(meshes)
        self._vp = (C.c_void_p * n)(*[a.ctypes.data if a.size else None for a in self._v])
        self._ip = (C.c_void_p * n)(*[a.ctypes.data if a.size else None for a in self._i])
        self._nv = np.array([a.shape[0] for a in self._v], dtype=np.int64)
        self._nt = np.array([a.shape[0] for a in self._i], dtype=np.int64)
        if inst_mesh is not None:
            self._im = np.ascontiguousarray(inst_mesh, dtype=np.uint32).reshape(-1)
            self._is = np.ascontiguousarray(inst_srt, dtype=np.float32).reshape(-1, 10)
            ninst = self._im.shape[0]
        else:
            self._im = self._is = None
            ninst = 0
        self.n_inst = ninst
        self.desc = _Scene(
            n, C.cast(self._vp, C.c_void_p), self._nv.ctypes.data, C.cast(self._ip, C.c_void_p),
            self._nt.ctypes.data, ninst,
            self._im.ctypes.data if ninst else None, self._is.ctypes.data if ninst else None, None)
        if accel:
            lib = _load()
            h = C.c_void_p()
            if lib.orc_bvh_create(self.ptr, C.byref(h)) != 0:
                raise ValueError("oracle: BVH build failed (invalid scene or out of memory)")
            self._bvh = h
            self._lib = lib
            self.desc.bvh = h.value

    @classmethod
    def from_scene(cls, scene, accel: bool = False):
        return cls([(m.vertices, m.indices) for m in scene.meshes], scene.inst_mesh, scene.inst_srt,
                   accel=accel)

    @property
    def accel(self) -> bool:
        return self._bvh is not None

    def bvh_stats(self) -> dict:
        """Tree nodes, triangles without a finite box, deepest leaf, instance-tree nodes."""
        if self._bvh is None:
            return {}
        out = np.zeros(4, np.int64)
        self._lib.orc_bvh_stats(self._bvh, out.ctypes.data)
        return {"nodes": int(out[0]), "loose": int(out[1]), "depth": int(out[2]),
                "top_nodes": int(out[3])}

    def linear(self) -> "OracleScene":
        """The same scene without the BVH (the plain linear search)."""
        meshes = list(zip(self._v, self._i))
        return OracleScene(meshes, self._im, self._is, accel=False)

    def __del__(self):
        if getattr(self, "_bvh", None) is not None:
            self.desc.bvh = None
            self._lib.orc_bvh_destroy(self._bvh)
            self._bvh = None

    @property
    def ptr(self):
        return C.addressof(self.desc)


def _rays(rays):
    r = np.ascontiguousarray(rays, dtype=np.float32).reshape(-1, 8)
    return r, r.shape[0]


def _p(a):
    return a.ctypes.data if a is not None and a.size else None


def _check(rc, name):
    if rc != 0:
        raise ValueError(f"oracle {name}: invalid arguments")


class _OptsC(C.Structure):
    _fields_ = [("inst_mask", C.c_void_p), ("ray_mask", C.c_void_p), ("skip_inst", C.c_void_p),
                ("skip_prim", C.c_void_p)]


class Opts:
    """Query options: instance masks (n_inst,), ray masks (n,) and the
    per-ray skipped triangle (skip_inst, skip_prim) (n,) each; any may be
    None.  See ``orc_opts`` in ``rt_oracle.h`` for the semantics."""

    def __init__(self, inst_mask=None, ray_mask=None, skip_inst=None, skip_prim=None):
        def u32(a):
            return None if a is None else np.ascontiguousarray(a, dtype=np.uint32).reshape(-1)
        self._a = [u32(inst_mask), u32(ray_mask), u32(skip_inst), u32(skip_prim)]
        self.desc = _OptsC(*[a.ctypes.data if a is not None and a.size else None for a in self._a])

    @property
    def ptr(self):
        return C.addressof(self.desc)

    def check(self, n):
        for a in self._a[1:]:
            if a is not None and a.shape[0] != n:
                raise ValueError("per-ray option arrays need one entry per ray")


def _optp(opts, n):
    if opts is None:
        return None
    opts.check(n)
    return opts.ptr


def closest(scene: OracleScene, rays, opts: Opts | None = None):
    """Returns (inst (n,) uint32, prim (n,) uint32, tuv (n,3) float64)."""
    lib = _load()
    r, n = _rays(rays)
    inst = np.empty(n, np.uint32)
    prim = np.empty(n, np.uint32)
    tuv = np.empty((n, 3), np.float64)
    if opts is None:
        _check(lib.orc_closest(scene.ptr, _p(r), n, _p(inst), _p(prim), _p(tuv)), "closest")
    else:
        _check(lib.orc_closest_ex(scene.ptr, _p(r), n, _optp(opts, n), _p(inst), _p(prim), _p(tuv)),
               "closest_ex")
    return inst, prim, tuv


def any_hit(scene: OracleScene, rays, opts: Opts | None = None):
    lib = _load()
    r, n = _rays(rays)
    occ = np.empty(n, np.uint8)
    if opts is None:
        _check(lib.orc_any(scene.ptr, _p(r), n, _p(occ)), "any")
    else:
        _check(lib.orc_any_ex(scene.ptr, _p(r), n, _optp(opts, n), _p(occ)), "any_ex")
    return occ


def all_hits(scene: OracleScene, rays, K: int, opts: Opts | None = None):
    """All hits sorted by (t, inst, prim): (count (n,) int64, inst (n,K),
    prim (n,K) uint32, tuv (n,K,3) float64), the first K stored."""
    lib = _load()
    r, n = _rays(rays)
    count = np.empty(n, np.int64)
    inst = np.empty((n, K), np.uint32)
    prim = np.empty((n, K), np.uint32)
    tuv = np.empty((n, K, 3), np.float64)
    _check(lib.orc_all(scene.ptr, _p(r), n, _optp(opts, n), int(K), _p(count), _p(inst), _p(prim),
                       _p(tuv)), "all")
    return count, inst, prim, tuv


class Candidates:
    """Every sure-or-maybe pair per ray for all-hit queries, sorted by
    (t, inst, prim), with the range [lo, hi] of its float32 t."""

    def __init__(self, count, n_sure, inst, prim, tuv, scale, lo, hi, sure, K):
        self.count, self.n_sure, self.inst, self.prim = count, n_sure, inst, prim
        self.tuv, self.scale, self.lo, self.hi, self.sure, self.K = tuv, scale, lo, hi, sure, K


def classify_all(scene: OracleScene, rays, K: int, opts: Opts | None = None,
                 delta: float = DELTA) -> Candidates:
    lib = _load()
    r, n = _rays(rays)
    count = np.empty(n, np.int32)
    n_sure = np.empty(n, np.int32)
    ai = np.empty((n, K), np.uint32)
    ap = np.empty((n, K), np.uint32)
    at = np.empty((n, K, 3), np.float64)
    asc = np.empty((n, K), np.float64)
    lo = np.empty((n, K), np.float64)
    hi = np.empty((n, K), np.float64)
    su = np.empty((n, K), np.uint8)
    _check(lib.orc_classify_all(scene.ptr, _p(r), n, _optp(opts, n), float(delta), int(K), _p(count),
                                _p(n_sure), _p(ai), _p(ap), _p(at), _p(asc), _p(lo), _p(hi), _p(su)),
           "classify_all")
    return Candidates(count, n_sure, ai, ap, at, asc, lo, hi, su.astype(bool), K)


class Accept:
    """Acceptable sets per ray (see ``rt_oracle.c``)."""

    def __init__(self, miss_ok, count, inst, prim, tuv, scale, any_class, K):
        self.miss_ok, self.count, self.inst, self.prim = miss_ok, count, inst, prim
        self.tuv, self.scale, self.any_class, self.K = tuv, scale, any_class, K

    @property
    def pinned(self):
        return (self.count + self.miss_ok.astype(np.int32)) == 1

    def subset(self, rows) -> "Accept":
        """The acceptable sets of the rays ``rows`` only."""
        return Accept(self.miss_ok[rows], self.count[rows], self.inst[rows], self.prim[rows],
                      self.tuv[rows], self.scale[rows], self.any_class[rows], self.K)

    @property
    def overflow(self):
        return self.count > self.K


def accept(scene: OracleScene, rays, delta: float = DELTA, K: int = 8,
           opts: Opts | None = None) -> Accept:
    lib = _load()
    r, n = _rays(rays)
    miss_ok = np.empty(n, np.uint8)
    count = np.empty(n, np.int32)
    ai = np.empty((n, K), np.uint32)
    ap = np.empty((n, K), np.uint32)
    at = np.empty((n, K, 3), np.float64)
    asc = np.empty((n, K), np.float64)
    ac = np.empty(n, np.uint8)
    if opts is None:
        _check(lib.orc_accept(scene.ptr, _p(r), n, float(delta), int(K), _p(miss_ok), _p(count),
                              _p(ai), _p(ap), _p(at), _p(asc), _p(ac)), "accept")
    else:
        _check(lib.orc_accept_ex(scene.ptr, _p(r), n, _optp(opts, n), float(delta), int(K),
                                 _p(miss_ok), _p(count), _p(ai), _p(ap), _p(at), _p(asc), _p(ac)),
               "accept_ex")
    return Accept(miss_ok.astype(bool), count, ai, ap, at, asc, ac, K)


def adjoint(scene: OracleScene, rays, prim, g):
    """Returns (d_vertices (V,3), d_orig (n,3), d_dir (n,3)) in float64."""
    lib = _load()
    r, n = _rays(rays)
    prim = np.ascontiguousarray(prim, dtype=np.uint32).reshape(-1)
    g = np.ascontiguousarray(g, dtype=np.float64).reshape(-1, 3)
    nv = int(scene._nv[0])
    dV = np.zeros((nv, 3), np.float64)
    do = np.empty((n, 3), np.float64)
    dd = np.empty((n, 3), np.float64)
    _check(lib.orc_adjoint(scene.ptr, _p(r), _p(prim), n, _p(g), _p(dV), _p(do), _p(dd)), "adjoint")
    return dV, do, dd


def fd(scene: OracleScene, rays, prim, g, h: float = 1e-6):
    """Central differences: (n,15) = d/d(v0,v1,v2,o,d) of g.(t,u,v)."""
    lib = _load()
    r, n = _rays(rays)
    prim = np.ascontiguousarray(prim, dtype=np.uint32).reshape(-1)
    g = np.ascontiguousarray(g, dtype=np.float64).reshape(-1, 3)
    out = np.empty((n, 15), np.float64)
    _check(lib.orc_fd(scene.ptr, _p(r), _p(prim), n, _p(g), float(h), _p(out)), "fd")
    return out


def fixed_tuv(scene: OracleScene, rays, prim):
    lib = _load()
    r, n = _rays(rays)
    prim = np.ascontiguousarray(prim, dtype=np.uint32).reshape(-1)
    tuv = np.empty((n, 3), np.float64)
    _check(lib.orc_fixed_tuv(scene.ptr, _p(r), _p(prim), n, _p(tuv)), "fixed_tuv")
    return tuv


def adjoint_inst(scene: OracleScene, rays, inst, prim, g):
    """Two-level adjoint.  Returns (list of d_vertices (V_m,3) per mesh,
    d_srt (n_inst,10), d_orig (n,3), d_dir (n,3)), all float64."""
    lib = _load()
    r, n = _rays(rays)
    inst = np.ascontiguousarray(inst, dtype=np.uint32).reshape(-1)
    prim = np.ascontiguousarray(prim, dtype=np.uint32).reshape(-1)
    g = np.ascontiguousarray(g, dtype=np.float64).reshape(-1, 3)
    dV = [np.zeros((int(nv), 3), np.float64) for nv in scene._nv]
    ptrs = (C.c_void_p * len(dV))(*[a.ctypes.data if a.size else None for a in dV])
    dS = np.zeros((scene.n_inst, 10), np.float64)
    do = np.empty((n, 3), np.float64)
    dd = np.empty((n, 3), np.float64)
    _check(lib.orc_adjoint_inst(scene.ptr, _p(r), _p(inst), _p(prim), n, _p(g),
                                C.cast(ptrs, C.c_void_p), _p(dS), _p(do), _p(dd)), "adjoint_inst")
    return dV, dS, do, dd


def fd_inst(scene: OracleScene, rays, inst, prim, g, h: float = 1e-6):
    """Central differences: (n,25) = d/d(v0,v1,v2, sx,sy,sz,qx,qy,qz,qw,tx,ty,tz, o,d)."""
    lib = _load()
    r, n = _rays(rays)
    inst = np.ascontiguousarray(inst, dtype=np.uint32).reshape(-1)
    prim = np.ascontiguousarray(prim, dtype=np.uint32).reshape(-1)
    g = np.ascontiguousarray(g, dtype=np.float64).reshape(-1, 3)
    out = np.empty((n, 25), np.float64)
    _check(lib.orc_fd_inst(scene.ptr, _p(r), _p(inst), _p(prim), n, _p(g), float(h), _p(out)),
           "fd_inst")
    return out


def ao_rays(scene: OracleScene, rays, prim, tuv, xi, offset: float, radius: float, inst=None):
    """Ambient-occlusion rays (§4): (n*N, 8) float32 for the primary rays'
    closest hits (prim, tuv; and inst, their instances, in a two-level scene)
    and uniforms xi (n, N, 2)."""
    lib = _load()
    r, n = _rays(rays)
    prim = np.ascontiguousarray(prim, dtype=np.uint32).reshape(-1)
    tuv = np.ascontiguousarray(tuv, dtype=np.float64).reshape(-1, 3)
    xi = np.ascontiguousarray(xi, dtype=np.float32)
    N = xi.shape[1]
    assert xi.shape == (n, N, 2)
    out = np.empty((n * N, 8), np.float32)
    if inst is None:
        _check(lib.orc_ao_rays(scene.ptr, _p(r), _p(prim), _p(tuv), n, int(N), _p(xi), float(offset),
                               float(radius), _p(out)), "ao_rays")
    else:
        inst = np.ascontiguousarray(inst, dtype=np.uint32).reshape(-1)
        _check(lib.orc_ao_rays_inst(scene.ptr, _p(r), _p(inst), _p(prim), _p(tuv), n, int(N), _p(xi),
                                    float(offset), float(radius), _p(out)), "ao_rays_inst")
    return out


def bvh_check(scene: OracleScene, rays, candidates: bool, delta: float = DELTA):
    """The BVH's culling invariant on every wanted pair of the linear search
    (see ``orc_bvh_check``): returns (pairs checked, violations)."""
    if not scene.accel:
        raise ValueError("bvh_check needs a scene built with accel=True")
    lib = _load()
    r, n = _rays(rays)
    out = np.zeros(2, np.int64)
    _check(lib.orc_bvh_check(scene.ptr, _p(r), n, int(bool(candidates)), float(delta), _p(out)),
           "bvh_check")
    return int(out[0]), int(out[1])


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    _load().orc_set_num_threads(int(n))
