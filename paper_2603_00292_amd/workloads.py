"""Seeded synthetic inputs for the ray-query workloads.

This module only *draws* scenes and rays. It contains none of the query
arithmetic (no ray/box or ray/triangle test, no traversal, no gradient), so
both the HIP path and the FP64 CPU oracle can consume its arrays without
sharing any of the method's code.

Conventions shared by every generator
-------------------------------------
* Random stream ``k`` is ``numpy.random.default_rng([260300292, k])``.
* Values are drawn in float64 and rounded once to float32; the float32 arrays
  are the inputs for both sides.
* Vertices: ``(V, 3) float32``.  Indices: ``(N, 3) uint32``.
* Rays: ``(n, 8) float32`` rows ``(ox, oy, oz, tmin, dx, dy, dz, tmax)``,
  the 32-byte ray record of the library (origin, min length, direction, max
  length; the ray is R(t) = o + t d of the paper's ray equation in §3.1, with
  t measured in units of the given d).
* Instances: ``inst_mesh (J,) uint32`` and ``inst_srt (J, 10) float32`` rows
  ``(sx, sy, sz, qx, qy, qz, qw, tx, ty, tz)`` meaning
  world = T + R(q/|q|) (S * x)  (scale, then rotate, then translate; the
  scale-rotation-translation frame of §7.3).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 260300292


def rng_for(k: int) -> np.random.Generator:
    return np.random.default_rng([SEED_BASE, k])


# ----------------------------------------------------------------------------
# small helpers (sampling only)
# ----------------------------------------------------------------------------

def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def pack_rays(origins, directions, tmin=0.0, tmax=np.inf) -> np.ndarray:
    """Pack float64 origins/directions (n,3) and scalar-or-(n,) tmin/tmax."""
    o = np.asarray(origins, dtype=np.float64)
    d = np.asarray(directions, dtype=np.float64)
    n = o.shape[0]
    r = np.empty((n, 8), dtype=np.float64)
    r[:, 0:3] = o
    r[:, 3] = np.broadcast_to(np.asarray(tmin, dtype=np.float64), (n,))
    r[:, 4:7] = d
    r[:, 7] = np.broadcast_to(np.asarray(tmax, dtype=np.float64), (n,))
    return _f32(r)


def uniform_sphere_dirs(rng: np.random.Generator, n: int) -> np.ndarray:
    """Directions uniform on the unit sphere (normalised Gaussian triples)."""
    g = rng.standard_normal((n, 3))
    nrm = np.linalg.norm(g, axis=1, keepdims=True)
    nrm[nrm == 0.0] = 1.0
    return g / nrm


def random_triangle_soup(rng: np.random.Generator, n_tri: int, half: float = 0.025):
    """Triangles with centres uniform in [0,1]^3 and each vertex offset
    uniformly by +-half per axis. Unshared vertices: indices (3i, 3i+1, 3i+2)."""
    c = rng.random((n_tri, 3))
    off = rng.uniform(-half, half, size=(n_tri, 3, 3))
    v = (c[:, None, :] + off).reshape(-1, 3)
    idx = np.arange(3 * n_tri, dtype=np.uint32).reshape(n_tri, 3)
    return _f32(v), np.ascontiguousarray(idx)


def box_rays(rng: np.random.Generator, n: int, lo: float, hi: float, tmin=0.0, tmax=np.inf):
    """Origins uniform in [lo,hi]^3, directions uniform on the sphere."""
    o = rng.uniform(lo, hi, size=(n, 3))
    d = uniform_sphere_dirs(rng, n)
    return pack_rays(o, d, tmin, tmax)


# ----------------------------------------------------------------------------
# icosphere
# ----------------------------------------------------------------------------

def icosphere(levels: int):
    """Unit icosphere: icosahedron (12 vertices (0,+-1,+-phi) and cyclic
    permutations, 20 faces counter-clockwise seen from outside), subdivided
    ``levels`` times with shared edge midpoints projected to the sphere.
    Children of face f are 4f..4f+3: corner0, corner1, corner2, centre.
    Returns float64 vertices (10*4^L+2, 3) and uint32 faces (20*4^L, 3)."""
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([
        [-1, phi, 0], [1, phi, 0], [-1, -phi, 0], [1, -phi, 0],
        [0, -1, phi], [0, 1, phi], [0, -1, -phi], [0, 1, -phi],
        [phi, 0, -1], [phi, 0, 1], [-phi, 0, -1], [-phi, 0, 1],
    ], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int64)
    for _ in range(levels):
        a, b, c = f[:, 0], f[:, 1], f[:, 2]
        e = np.stack([np.stack([a, b], 1), np.stack([b, c], 1), np.stack([c, a], 1)], 1)  # (F,3,2)
        e_sorted = np.sort(e, axis=2).reshape(-1, 2)
        key = e_sorted[:, 0] * (len(v) + 1) + e_sorted[:, 1]
        uniq, inv = np.unique(key, return_inverse=True)
        ea = uniq // (len(v) + 1)
        eb = uniq % (len(v) + 1)
        mid = v[ea] + v[eb]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        base = len(v)
        v = np.concatenate([v, mid], 0)
        m = (inv.reshape(-1, 3) + base)
        ab, bc, ca = m[:, 0], m[:, 1], m[:, 2]
        f = np.stack([
            np.stack([a, ab, ca], 1),
            np.stack([ab, b, bc], 1),
            np.stack([ca, bc, c], 1),
            np.stack([ab, bc, ca], 1),
        ], 1).reshape(-1, 3)
    return v, f.astype(np.uint32)


def noisy_icosphere(rng: np.random.Generator, levels: int = 8, noise: float = 0.02):
    v, f = icosphere(levels)
    r = 1.0 + rng.uniform(-noise, noise, size=(len(v), 1))
    return _f32(v * r), np.ascontiguousarray(f)


# ----------------------------------------------------------------------------
# displaced grids
# ----------------------------------------------------------------------------

def grid_mesh(nx: int, nz: int, x0: float, x1: float, z0: float, z1: float, heights: np.ndarray):
    """(nx+1)*(nz+1) vertices on a regular x/z grid with the given heights;
    quad (i,j) splits into (a,b,c) and (a,c,d) with a=(i,j), b=(i+1,j),
    c=(i+1,j+1), d=(i,j+1)."""
    xs = np.linspace(x0, x1, nx + 1)
    zs = np.linspace(z0, z1, nz + 1)
    X, Z = np.meshgrid(xs, zs, indexing="xy")  # (nz+1, nx+1)
    H = np.asarray(heights, dtype=np.float64).reshape(nz + 1, nx + 1)
    v = np.stack([X, H, Z], -1).reshape(-1, 3)
    j, i = np.meshgrid(np.arange(nz), np.arange(nx), indexing="ij")
    a = j * (nx + 1) + i
    b = a + 1
    c = a + (nx + 1) + 1
    d = a + (nx + 1)
    t0 = np.stack([a, b, c], -1).reshape(-1, 3)
    t1 = np.stack([a, c, d], -1).reshape(-1, 3)
    f = np.stack([t0, t1], 1).reshape(-1, 3)
    return _f32(v), np.ascontiguousarray(f.astype(np.uint32))


# ----------------------------------------------------------------------------
# rotations (Shoemake's uniform random quaternion)
# ----------------------------------------------------------------------------

def uniform_quaternions(rng: np.random.Generator, n: int) -> np.ndarray:
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a = np.sqrt(1.0 - u1)
    b = np.sqrt(u1)
    qx = a * np.sin(2 * np.pi * u2)
    qy = a * np.cos(2 * np.pi * u2)
    qz = b * np.sin(2 * np.pi * u3)
    qw = b * np.cos(2 * np.pi * u3)
    return np.stack([qx, qy, qz, qw], 1)


def quat_matrix(q: np.ndarray) -> np.ndarray:
    """Rotation matrices (n,3,3) of quaternions (n,4) = (x,y,z,w), normalised."""
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    x, y, z, w = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - z * w)
    R[..., 0, 2] = 2 * (x * z + y * w)
    R[..., 1, 0] = 2 * (x * y + z * w)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - x * w)
    R[..., 2, 0] = 2 * (x * z - y * w)
    R[..., 2, 1] = 2 * (y * z + x * w)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


# ----------------------------------------------------------------------------
# workload containers
# ----------------------------------------------------------------------------

@dataclass
class Mesh:
    vertices: np.ndarray  # (V,3) float32
    indices: np.ndarray   # (N,3) uint32

    @property
    def n_tri(self) -> int:
        return int(self.indices.shape[0])


@dataclass
class Scene:
    meshes: list                      # list[Mesh]
    inst_mesh: np.ndarray | None = None  # (J,) uint32
    inst_srt: np.ndarray | None = None   # (J,10) float32

    @property
    def instanced(self) -> bool:
        return self.inst_mesh is not None


@dataclass
class Workload:
    name: str
    scene: Scene
    rays: np.ndarray                       # (n,8) float32
    extra: dict = field(default_factory=dict)

    def checksum(self) -> str:
        """SHA-256 (hex) of every input array in a fixed order: each mesh's
        vertices and indices, the instance arrays, the rays, then the array
        entries of `extra` by key.  Each array contributes its dtype, shape
        and bytes, so the value pins the generator's output exactly."""
        import hashlib

        h = hashlib.sha256()

        def add(tag, a):
            a = np.ascontiguousarray(a)
            h.update(f"{tag}:{a.dtype.str}:{a.shape};".encode())
            h.update(a.tobytes())

        for i, m in enumerate(self.scene.meshes):
            add(f"v{i}", m.vertices)
            add(f"i{i}", m.indices)
        if self.scene.inst_mesh is not None:
            add("inst_mesh", self.scene.inst_mesh)
            add("inst_srt", self.scene.inst_srt)
        add("rays", self.rays)
        for k in sorted(self.extra):
            if isinstance(self.extra[k], np.ndarray):
                add(f"extra:{k}", self.extra[k])
        return h.hexdigest()


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------

def random_triangles(n_tri: int = 4096, n_rays: int = 65536, k: int = 0, half: float = 0.025) -> Workload:
    """Random-triangle soup in the unit cube with uniform-sphere rays whose
    origins are uniform in [-1,2]^3; tmin = 0, tmax = +inf."""
    rng = rng_for(k)
    v, f = random_triangle_soup(rng, n_tri, half)
    rays = box_rays(rng, n_rays, -1.0, 2.0)
    return Workload(f"random_triangles_{n_tri}", Scene([Mesh(v, f)]), rays)


def icosphere_incoherent(n_rays: int = 4194304, levels: int = 8, k: int = 5) -> Workload:
    """Incoherent closest-hit at about a million triangles: the noisy
    icosphere (levels=8: 1,310,720 triangles, radius 1 +- 0.02) with origins
    uniform in [-1,1]^3 and directions uniform on the sphere."""
    rng = rng_for(k)
    v, f = noisy_icosphere(rng, levels, 0.02)
    rays = box_rays(rng, n_rays, -1.0, 1.0)
    return Workload(f"icosphere{levels}_incoherent", Scene([Mesh(v, f)]), rays)


def pinhole_rays(origin, right, up, width: int, height: int, jitter=None):
    """Primary rays of the pinhole camera of §3.2: forward = normalize(up x right),
    film at distance 1 spanned by +-right and +-up, u = xi/W, v = yi/H,
    ray index xi + W*yi.  ``jitter`` (optional (H*W,2) array in [0,1)) is added
    to (xi, yi) before normalising."""
    origin = np.asarray(origin, dtype=np.float64)
    right = np.asarray(right, dtype=np.float64)
    up = np.asarray(up, dtype=np.float64)
    fwd = np.cross(up, right)
    fwd /= np.linalg.norm(fwd)
    yi, xi = np.meshgrid(np.arange(height), np.arange(width), indexing="ij")
    xi = xi.reshape(-1).astype(np.float64)
    yi = yi.reshape(-1).astype(np.float64)
    if jitter is not None:
        xi = xi + jitter[:, 0]
        yi = yi + jitter[:, 1]
    u = (xi / width)[:, None]
    v = (yi / height)[:, None]
    to = origin + fwd + ((1 - u) * (-right) + u * right) + ((1 - v) * up + v * (-up))
    d = to - origin
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.broadcast_to(origin, d.shape)
    return o, d


def icosphere_camera(width: int = 2048, height: int = 2048, levels: int = 8, k: int = 1) -> Workload:
    """Coherent primary rays from a pinhole camera at (0,0,3), 40 degree FOV,
    onto the noisy icosphere; plus the same number of shadow rays toward a
    point light at (2,2,2) (``extra['shadow_rays']``).

    Shadow-ray origins: the primary ray's entry point on the analytic sphere of
    radius 1.0201 (just outside the largest vertex radius 1.02, so the origin
    is never inside the mesh); primary rays that miss that sphere start at
    o + 3d. Direction = normalised vector to the light, tmin = 0,
    tmax = distance to the light."""
    rng = rng_for(k)
    v, f = noisy_icosphere(rng, levels, 0.02)
    th = math.tan(math.radians(20.0))
    o, d = pinhole_rays((0.0, 0.0, 3.0), (th, 0.0, 0.0), (0.0, th, 0.0), width, height)
    prim = pack_rays(o, d)
    # analytic sphere entry (scene set-up, not the triangle query)
    R = 1.0201
    b = np.einsum("ij,ij->i", o, d)
    c = np.einsum("ij,ij->i", o, o) - R * R
    disc = b * b - c
    hit = disc >= 0
    ts = np.where(hit, -b - np.sqrt(np.maximum(disc, 0.0)), 3.0)
    os_ = o + ts[:, None] * d
    light = np.array([2.0, 2.0, 2.0])
    ld = light - os_
    dist = np.linalg.norm(ld, axis=1)
    sd = ld / dist[:, None]
    shadow = pack_rays(os_, sd, 0.0, dist)
    return Workload(f"icosphere{levels}_camera", Scene([Mesh(v, f)]), prim, {"shadow_rays": shadow})


def instanced_grids(n_inst: int = 1024, n_rays: int = 8388608, k: int = 2) -> Workload:
    """Two-level scene: four 100x50-quad displaced grids (10,000 triangles
    each, heights N(0, sigma_b), sigma_b in {0.01,0.02,0.05,0.1}) instanced
    ``n_inst`` times with scale U[0.5,2]^3, uniform rotation and translation
    U[-20,20]^3 (instance m uses mesh m mod 4).

    Rays: secondary rays leaving the surface. Each ray picks a uniformly random
    instance, triangle and barycentric point, offsets it 1e-4 along the world
    geometric normal turned toward the camera position (0,0,70), and takes a
    cosine-weighted direction about that normal (hemisphere sampling of §4.1
    with the tangent frame of §4.2)."""
    rng = rng_for(k)
    meshes = []
    for s in (0.01, 0.02, 0.05, 0.1):
        h = rng.normal(0.0, s, size=(51 * 101,))
        mv, mf = grid_mesh(100, 50, -1.0, 1.0, -0.5, 0.5, h)
        meshes.append(Mesh(mv, mf))
    inst_mesh = (np.arange(n_inst) % 4).astype(np.uint32)
    S = rng.uniform(0.5, 2.0, size=(n_inst, 3))
    q = uniform_quaternions(rng, n_inst)
    T = rng.uniform(-20.0, 20.0, size=(n_inst, 3))
    srt = _f32(np.concatenate([S, q, T], 1))
    # secondary-ray origins on surfaces (FP64 from the float32 instance data)
    S64 = srt[:, 0:3].astype(np.float64)
    R64 = quat_matrix(srt[:, 3:7].astype(np.float64))
    T64 = srt[:, 7:10].astype(np.float64)
    inst = rng.integers(0, n_inst, size=n_rays)
    tri = rng.integers(0, 10000, size=n_rays)
    r1 = rng.random(n_rays)
    r2 = rng.random(n_rays)
    su = np.sqrt(r1)
    b1 = su * (1 - r2)
    b2 = su * r2
    b0 = 1 - b1 - b2
    o = np.empty((n_rays, 3))
    nrm = np.empty((n_rays, 3))
    t0 = np.empty((n_rays, 3))
    for m in range(4):
        sel = np.nonzero(inst_mesh[inst] == m)[0]
        mv = meshes[m].vertices.astype(np.float64)
        mf = meshes[m].indices.astype(np.int64)[tri[sel]]
        ii = inst[sel]

        def to_world(x):
            return np.einsum("nij,nj->ni", R64[ii], S64[ii] * x) + T64[ii]

        w0, w1, w2 = to_world(mv[mf[:, 0]]), to_world(mv[mf[:, 1]]), to_world(mv[mf[:, 2]])
        o[sel] = b0[sel, None] * w0 + b1[sel, None] * w1 + b2[sel, None] * w2
        nn = np.cross(w1 - w0, w2 - w0)
        nn /= np.linalg.norm(nn, axis=1, keepdims=True)
        t0[sel] = (w1 - w0) / np.linalg.norm(w1 - w0, axis=1, keepdims=True)
        nrm[sel] = nn
    cam = np.array([0.0, 0.0, 70.0])
    flip = np.einsum("ij,ij->i", nrm, cam - o) < 0
    nrm[flip] *= -1
    t1 = np.cross(nrm, t0)
    xi0, xi1 = rng.random(n_rays), rng.random(n_rays)
    ph = 2 * np.pi * xi0
    r = np.sqrt(xi1)
    lx, lz = np.cos(ph) * r, np.sin(ph) * r
    ly = np.sqrt(np.maximum(1 - r * r, 0.0))
    d = t0 * lx[:, None] + t1 * lz[:, None] + nrm * ly[:, None]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = o + 1e-4 * nrm
    rays = pack_rays(o, d)
    extra = {"src_inst": inst.astype(np.uint32), "src_prim": tri.astype(np.uint32)}
    return Workload("instanced_grids", Scene(meshes, inst_mesh, srt), rays, extra)


def aimed_instances(n_inst: int = 8, n_rays: int = 4096, k: int = 130) -> Workload:
    """Small two-level scene for gradient checks: three 12x8-quad displaced
    grids (heights N(0, sigma), sigma in {0.02, 0.05, 0.1}) instanced
    ``n_inst`` times (instance m uses mesh m mod 3) with scale U[0.5,2]^3
    (instance 1 mirrored in z), uniform rotations given as quaternions of
    norm U[0.6,1.8] (the frame normalises them) and translation U[-6,6]^3.
    Rays start uniformly in [-9,9]^3 and aim at uniformly chosen points of
    uniformly chosen instances."""
    rng = rng_for(k)
    meshes = []
    for s in (0.02, 0.05, 0.1):
        mv, mf = grid_mesh(12, 8, -1.0, 1.0, -0.5, 0.5, rng.normal(0, s, 13 * 9))
        meshes.append(Mesh(mv, mf))
    inst_mesh = (np.arange(n_inst) % 3).astype(np.uint32)
    S = rng.uniform(0.5, 2.0, (n_inst, 3))
    if n_inst > 1:
        S[1, 2] *= -1.0
    q = uniform_quaternions(rng, n_inst) * rng.uniform(0.6, 1.8, (n_inst, 1))
    T = rng.uniform(-6, 6, (n_inst, 3))
    srt = _f32(np.concatenate([S, q, T], 1))
    R = quat_matrix(srt[:, 3:7].astype(np.float64))
    j = rng.integers(0, n_inst, n_rays)
    p_obj = np.stack([rng.uniform(-0.9, 0.9, n_rays), np.zeros(n_rays),
                      rng.uniform(-0.4, 0.4, n_rays)], 1)
    tgt = np.einsum("nij,nj->ni", R[j], srt[j, 0:3].astype(np.float64) * p_obj) + srt[j, 7:10]
    o = rng.uniform(-9, 9, (n_rays, 3))
    d = tgt - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return Workload("aimed_instances", Scene(meshes, inst_mesh, srt), pack_rays(o, d))


def ao_terrain(width: int = 1024, height: int = 1024, samples: int = 16, k: int = 6,
               nq: int = 256) -> Workload:
    """Ambient-occlusion workload (§4): a terrain of nq x nq quads over
    [0,16]^2 with heights a sum of six random plane waves (amplitudes
    U[0.2,0.6], wave numbers U[1,4], random directions and phases), seen by
    a width x height pinhole camera (§3.2) at (8, 6, -2) looking at (8, 0, 9)
    with a 60-degree vertical field of view.  ``extra``: ``xi``
    (width*height, samples, 2) float32 uniforms of the cosine-weighted
    sampling, ``samples``, ``radius`` = 1 (the AO ray length of §4.2) and
    ``offset`` = 1e-4 (the self-intersection offset of §4.2)."""
    rng = rng_for(k)
    xs = np.linspace(0.0, 16.0, nq + 1)
    X, Z = np.meshgrid(xs, xs, indexing="xy")
    H = np.zeros_like(X)
    for _ in range(6):
        a = rng.uniform(0.2, 0.6)
        f = rng.uniform(1.0, 4.0)
        th = rng.uniform(0.0, 2 * np.pi)
        ph = rng.uniform(0.0, 2 * np.pi)
        H += a * np.sin(f * (X * np.cos(th) + Z * np.sin(th)) + ph)
    v, f = grid_mesh(nq, nq, 0.0, 16.0, 0.0, 16.0, H.reshape(-1))
    origin = np.array([8.0, 6.0, -2.0])
    fwd = np.array([8.0, 0.0, 9.0]) - origin
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.array([0.0, 1.0, 0.0]))
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    half = math.tan(math.radians(30.0))
    right = right * half * (width / height)
    up = up * half
    o, d = pinhole_rays(origin, right, up, width, height)
    rays = pack_rays(o, d)
    xi = _f32(rng.random((width * height, samples, 2)))
    extra = {"xi": xi, "samples": samples, "radius": 1.0, "offset": 1e-4}
    return Workload(f"ao_terrain_{width}x{height}x{samples}", Scene([Mesh(v, f)]), rays, extra)


def batched_meshes(n_mesh: int = 256, tri_range=(1e3, 5e5), ray_range=(1e3, 1e6), k: int = 3):
    """Independent meshes with log-uniform triangle counts and log-uniform ray
    counts. Mesh m: the random-triangle recipe with offset half-width
    0.025*sqrt(4096/N_m); rays: origins uniform in [-1,2]^3, uniform-sphere
    directions. Returns a list of Workloads."""
    rng = rng_for(k)
    nt = np.rint(np.exp(rng.uniform(math.log(tri_range[0]), math.log(tri_range[1]), n_mesh))).astype(np.int64)
    nr = np.rint(np.exp(rng.uniform(math.log(ray_range[0]), math.log(ray_range[1]), n_mesh))).astype(np.int64)
    out = []
    for m in range(n_mesh):
        half = 0.025 * math.sqrt(4096.0 / nt[m])
        v, f = random_triangle_soup(rng, int(nt[m]), half)
        rays = box_rays(rng, int(nr[m]), -1.0, 2.0)
        out.append(Workload(f"batch_{m}", Scene([Mesh(v, f)]), rays))
    return out


def displaced_grid(nx: int = 512, nz: int = 256, n_rays: int = 1048576, k: int = 4) -> Workload:
    """Differentiable workload: nx*nz unit quads over x in [0,nx], z in [0,nz]
    with heights N(0,0.05); rays start on the bounding box's top face and point
    down within 30 degrees of -y. ``extra['abc']`` holds per-ray weights
    (a,b,c) ~ N(0,1) of L = sum(a t + b u + c v)."""
    rng = rng_for(k)
    h = rng.normal(0.0, 0.05, size=((nx + 1) * (nz + 1),))
    v, f = grid_mesh(nx, nz, 0.0, float(nx), 0.0, float(nz), h)
    ymax = float(v[:, 1].max())
    ox = rng.uniform(0.0, nx, n_rays)
    oz = rng.uniform(0.0, nz, n_rays)
    o = np.stack([ox, np.full(n_rays, ymax), oz], 1)
    ct = rng.uniform(math.cos(math.radians(30.0)), 1.0, n_rays)
    ph = rng.uniform(0.0, 2 * np.pi, n_rays)
    st = np.sqrt(np.maximum(1 - ct * ct, 0.0))
    d = np.stack([st * np.cos(ph), -ct, st * np.sin(ph)], 1)
    rays = pack_rays(o, d)
    abc = _f32(rng.standard_normal((n_rays, 3)))
    return Workload(f"displaced_grid_{nx}x{nz}", Scene([Mesh(v, f)]), rays, {"abc": abc})
