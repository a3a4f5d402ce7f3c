"""Shared checks for the GPU parity tests (compare HIP results with the oracle)."""
from __future__ import annotations

import numpy as np

NONE = 0xFFFFFFFF
T_REL = 1e-5     # |t_gpu - t_k| <= T_REL |t_k| + T_ABS * s
T_ABS = 1e-7
UV_ABS = 1e-5    # barycentrics: 1e-5 of their [0,1] range


def to_gpu_scene(api, torch, ctx, scene, **build):
    dev = torch.device("cuda", torch.cuda.current_device())
    meshes = [(torch.from_numpy(m.vertices).to(dev), torch.from_numpy(m.indices.view(np.int32)).to(dev))
              for m in scene.meshes]
    return api.Accel(ctx, meshes, scene.inst_mesh, scene.inst_srt, **build)


def check_closest(hits: np.ndarray, A, inst: np.ndarray | None = None, label: str = ""):
    """hits (n,4) float32 from the GPU; A = oracle.accept(...) on the same rays.
    Asserts membership in the acceptable set for every ray, and the value
    tolerances for the returned triangle.  Returns a stats dict."""
    n = hits.shape[0]
    prim = hits[:, 1].copy().view(np.uint32)
    hit = prim != NONE
    K = A.K
    cnt = np.minimum(A.count, K)
    match = (A.prim == prim[:, None]) & (np.arange(K)[None, :] < cnt[:, None])
    if inst is not None:
        match &= (A.inst == inst.astype(np.uint32)[:, None])
    in_set = np.where(hit, match.any(1), A.miss_ok)
    unverifiable = hit & ~in_set & A.overflow
    bad = ~in_set & ~unverifiable
    if bad.any():
        i = np.flatnonzero(bad)[:5]
        raise AssertionError(
            f"{label}: {int(bad.sum())} of {n} rays outside the acceptable set; first rays {i.tolist()} "
            f"gpu prim {prim[i].tolist()} accept {[A.prim[j, :cnt[j]].tolist() for j in i]} "
            f"miss_ok {A.miss_ok[i].tolist()}")
    assert unverifiable.sum() == 0, f"{label}: {int(unverifiable.sum())} rays overflow the acceptable list"
    # misses report t = +inf, u = v = 0
    miss = ~hit
    assert np.isinf(hits[miss, 0]).all() and (hits[miss, 0] > 0).all(), f"{label}: miss t != +inf"
    assert (hits[miss, 2] == 0).all() and (hits[miss, 3] == 0).all(), f"{label}: miss u,v != 0"
    # values of the returned triangle
    rows = np.flatnonzero(hit)
    j = match[rows].argmax(1)
    ref = A.tuv[rows, j]
    s = A.scale[rows, j]
    finite = np.isfinite(ref).all(1)
    g = hits[rows][:, [0, 2, 3]].astype(np.float64)
    dt = np.abs(g[:, 0] - ref[:, 0])
    du = np.abs(g[:, 1] - ref[:, 1])
    dv = np.abs(g[:, 2] - ref[:, 2])
    tol_t = T_REL * np.abs(ref[:, 0]) + T_ABS * s
    badv = finite & ((dt > tol_t) | (du > UV_ABS) | (dv > UV_ABS))
    if badv.any():
        k = np.flatnonzero(badv)[:5]
        raise AssertionError(f"{label}: {int(badv.sum())} hits outside the value tolerance; "
                             f"gpu {g[k].tolist()} oracle {ref[k].tolist()}")
    pinned = A.pinned
    return {
        "rays": n,
        "hits": int(hit.sum()),
        "pinned_frac": float(pinned.mean()),
        "max_dt_rel": float((dt[finite] / np.maximum(np.abs(ref[finite, 0]), 1e-30)).max()) if finite.any() else 0.0,
        "max_duv": float(max(du[finite].max(), dv[finite].max())) if finite.any() else 0.0,
    }


def check_any(occ: np.ndarray, A, label: str = ""):
    must = A.any_class == 1
    mustnot = A.any_class == 0
    bad = (must & (occ == 0)) | (mustnot & (occ != 0))
    if bad.any():
        i = np.flatnonzero(bad)[:5]
        raise AssertionError(f"{label}: {int(bad.sum())} any-hit answers outside the acceptable set "
                             f"(rays {i.tolist()}, class {A.any_class[i].tolist()}, gpu {occ[i].tolist()})")
    assert set(np.unique(occ).tolist()) <= {0, 1}
    return {"rays": len(occ), "occluded": int(occ.sum()), "decided": float((A.any_class != 2).mean())}
