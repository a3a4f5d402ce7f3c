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


def check_all(hits: np.ndarray, inst: np.ndarray | None, counts: np.ndarray, C, label: str = ""):
    """All-hit lists from the GPU: hits (n,cap,4), inst (n,cap) or None,
    counts (n,); C = oracle.classify_all(...) with K at least every ray's
    candidate count.  Per ray: every listed pair is a candidate, with t, u, v
    within the value tolerance and no repeats; n_sure <= count <= candidates;
    the list holds every sure candidate (when count <= cap), or every sure
    candidate that must precede its last entry (when it is full); entries are
    ordered up to the candidates' t ranges; entries past the list are misses.
    Returns a stats dict."""
    n, cap = hits.shape[0], hits.shape[1]
    assert (C.count <= C.K).all(), f"{label}: oracle candidate lists overflow K={C.K}"
    prim = hits[:, :, 1].copy().view(np.uint32)
    ins = np.zeros_like(prim) if inst is None else inst.astype(np.uint32)
    counts = counts.astype(np.int64)
    assert ((C.n_sure <= counts) & (counts <= C.count)).all(), (
        f"{label}: counts outside [sure, candidates] for rays "
        f"{np.flatnonzero((C.n_sure > counts) | (counts > C.count))[:5].tolist()}")
    exact = 0
    for r in range(n):
        m = int(min(counts[r], cap))
        assert (prim[r, m:] == NONE).all() and np.isinf(hits[r, m:, 0]).all(), f"{label}: ray {r} tail"
        idx = {}
        for i in range(int(C.count[r])):
            idx[(int(C.inst[r, i]), int(C.prim[r, i]))] = i
        pos = []
        for k in range(m):
            key = (int(ins[r, k]), int(prim[r, k]))
            assert key in idx, f"{label}: ray {r} entry {k} {key} is no candidate {sorted(idx)}"
            pos.append(idx[key])
        assert len(set(pos)) == m, f"{label}: ray {r} repeats a pair"
        for k, i in enumerate(pos):
            ref = C.tuv[r, i]
            if np.isfinite(ref).all():
                g = hits[r, k, [0, 2, 3]].astype(np.float64)
                assert abs(g[0] - ref[0]) <= T_REL * abs(ref[0]) + T_ABS * C.scale[r, i], (label, r, k)
                assert abs(g[1] - ref[1]) <= UV_ABS and abs(g[2] - ref[2]) <= UV_ABS, (label, r, k)
        for a, b in zip(pos, pos[1:]):
            assert C.lo[r, a] <= C.hi[r, b], f"{label}: ray {r} out of order"
        listed = set(pos)
        sure = [i for i in range(int(C.count[r])) if C.sure[r, i]]
        if counts[r] <= cap:
            missing = [i for i in sure if i not in listed]
        else:
            last_lo = C.lo[r, pos[-1]]
            missing = [i for i in sure if i not in listed and C.hi[r, i] < last_lo]
        assert not missing, f"{label}: ray {r} lacks sure hits {missing}"
        exact += int(C.n_sure[r] == C.count[r])
    return {"rays": n, "hits": int(counts.sum()), "max_count": int(counts.max()) if n else 0,
            "all_sure_frac": exact / max(n, 1)}



def _sub_opts(orc, opts, idx):
    """Query options restricted to the rays idx (instance masks kept)."""
    if opts is None:
        return None
    a = opts._a
    pick = lambda x: None if x is None else x[idx]
    return orc.Opts(a[0], pick(a[1]), pick(a[2]), pick(a[3]))


def check_chunked(orc, S, rays, hits=None, inst=None, occ=None, opts=None, chunk: int = 1 << 20,
                  K: int = 8, label: str = ""):
    """check_closest (hits, inst) and/or check_any (occ) on every ray, in
    chunks of `chunk` rays; rays whose acceptable set does not fit K entries
    are classified again with a K that holds it, so no ray is left
    unverifiable.  ``opts``: oracle query options of all rays.  Returns the
    summed statistics."""
    n = rays.shape[0]
    tally = Tally()
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        idx_all = np.arange(lo, hi)
        A = orc.accept(S, rays[lo:hi], K=K, opts=_sub_opts(orc, opts, idx_all))
        ovf = np.flatnonzero(A.overflow)
        ok = np.flatnonzero(~A.overflow)
        parts = [(ok, A.subset(ok) if len(ovf) else A)]
        if len(ovf):
            k2 = int(A.count[ovf].max())
            B = orc.accept(S, rays[lo + ovf], K=k2, opts=_sub_opts(orc, opts, lo + ovf))
            assert not B.overflow.any()
            parts.append((ovf, B))
        for rows, AA in parts:
            if len(rows) == 0:
                continue
            if hits is not None:
                tally.closest(check_closest(hits[lo + rows], AA, None if inst is None else inst[lo + rows],
                                            label=f"{label} [{lo},{hi})"))
            if occ is not None:
                tally.any(check_any(occ[lo + rows], AA, label=f"{label} any [{lo},{hi})"))
    return tally.summary()


class Tally:
    """Sums of the per-chunk statistics of check_closest / check_any."""

    def __init__(self):
        self.rays = self.hits = self.pinned = self.occluded = self.decided = self.any_rays = 0
        self.max_dt_rel = self.max_duv = 0.0

    def closest(self, st):
        self.rays += st["rays"]
        self.hits += st["hits"]
        self.pinned += round(st["pinned_frac"] * st["rays"])
        self.max_dt_rel = max(self.max_dt_rel, st["max_dt_rel"])
        self.max_duv = max(self.max_duv, st["max_duv"])

    def any(self, st):
        self.any_rays += st["rays"]
        self.occluded += st["occluded"]
        self.decided += round(st["decided"] * st["rays"])

    def summary(self):
        out = {}
        if self.rays:
            out.update(rays=self.rays, hits=self.hits, pinned_frac=self.pinned / self.rays,
                       max_dt_rel=self.max_dt_rel, max_duv=self.max_duv)
        if self.any_rays:
            out.update(any_rays=self.any_rays, occluded=self.occluded,
                       any_decided_frac=self.decided / self.any_rays)
        return out
