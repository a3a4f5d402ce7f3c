"""The chunked parity check itself (CPU): the oracle's own answers, written in
the GPU's output layout, pass it on every ray, including rays whose
acceptable set overflows the first classification; planted mistakes fail it."""
from __future__ import annotations

import numpy as np
import pytest

from helpers import NONE, check_chunked
from paper_2603_00292_amd import workloads as wl


def _as_gpu(prim, tuv):
    """Oracle closest answers in the (t, prim bits, u, v) float32 layout."""
    n = prim.shape[0]
    h = np.zeros((n, 4), np.float32)
    hit = prim != NONE
    h[:, 0] = np.where(hit, tuv[:, 0], np.inf)
    h[:, 1] = prim.view(np.float32)
    h[:, 2] = np.where(hit, tuv[:, 1], 0.0)
    h[:, 3] = np.where(hit, tuv[:, 2], 0.0)
    return h


@pytest.fixture(scope="module")
def dense(orc):
    # a dense soup with exact duplicates (ties) so that some rays have large
    # acceptable sets
    rng = wl.rng_for(900)
    V, I = wl.random_triangle_soup(rng, 1500, 0.1)
    I = np.concatenate([I, I[:300], I[:300]])
    scene = wl.Scene([wl.Mesh(V, I)])
    rays = wl.box_rays(rng, 5000, 0.0, 1.0)
    S = orc.OracleScene.from_scene(scene, accel=True)
    _, prim, tuv = orc.closest(S, rays)
    occ = orc.any_hit(S, rays)
    return S, rays, prim, tuv, occ


def test_oracle_answers_pass_every_chunk(orc, dense):
    S, rays, prim, tuv, occ = dense
    A = orc.accept(S, rays, K=2)
    assert A.overflow.sum() > 20          # the re-classification path runs
    st = check_chunked(orc, S, rays, hits=_as_gpu(prim, tuv), occ=occ, chunk=1234, K=2, label="oracle")
    assert st["rays"] == rays.shape[0] and st["any_rays"] == rays.shape[0]
    assert st["max_duv"] < 1e-6


def test_planted_mistakes_fail(orc, dense):
    S, rays, prim, tuv, occ = dense
    A = orc.accept(S, rays, K=2)
    pinned_hit = np.flatnonzero(A.pinned & (prim != NONE))
    r = int(pinned_hit[0])
    bad = prim.copy()
    bad[r] = (int(prim[r]) + 1) % 2100          # another triangle
    with pytest.raises(AssertionError):
        check_chunked(orc, S, rays, hits=_as_gpu(bad, tuv), chunk=1000, K=2)
    bad = prim.copy()
    bad[r] = NONE                               # a miss where a hit is sure
    with pytest.raises(AssertionError):
        check_chunked(orc, S, rays, hits=_as_gpu(bad, tuv), chunk=1000, K=2)
    t2 = tuv.copy()
    t2[r, 1] += 3e-5                            # u off by more than 1e-5
    with pytest.raises(AssertionError):
        check_chunked(orc, S, rays, hits=_as_gpu(prim, t2), chunk=1000, K=2)
    o2 = occ.copy()
    o2[np.flatnonzero(A.any_class == 1)[0]] = 0  # unoccluded where a hit is sure
    with pytest.raises(AssertionError):
        check_chunked(orc, S, rays, occ=o2, chunk=1000, K=2)
    # an overflowing ray answered by a member beyond the first K entries passes
    ov = np.flatnonzero(A.overflow & ~A.miss_ok)
    B = orc.accept(S, rays[ov], K=64)
    alt = prim.copy()
    t3 = tuv.copy()
    for j, rr in enumerate(ov[:10]):
        alt[rr] = B.prim[j, B.count[j] - 1]
        t3[rr] = B.tuv[j, B.count[j] - 1]
    check_chunked(orc, S, rays, hits=_as_gpu(alt, t3), chunk=1000, K=2)
