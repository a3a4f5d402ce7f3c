"""The seeded workload generators still produce exactly the inputs every
figure and parity case was measured on: SHA-256 of each workload's arrays
against tests/golden/workload_checksums.json (written by the script beside
it).  A deliberate generator change rewrites that file in the same commit."""
from __future__ import annotations

import importlib.util
import json
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")


def _maker():
    spec = importlib.util.spec_from_file_location("make_workload_checksums",
                                                  os.path.join(GOLDEN, "make_workload_checksums.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.fixture(scope="module")
def stored():
    with open(os.path.join(GOLDEN, "workload_checksums.json")) as f:
        return json.load(f)


MAKER = _maker()


@pytest.mark.parametrize("name", sorted(MAKER.CASES))
def test_workload_checksum(name, stored):
    assert MAKER.CASES[name]().checksum() == stored[name], f"{name}: generator output changed"


def test_batched_checksum(stored):
    assert MAKER.batched_checksum() == stored["batched_meshes_256"]


def test_checksum_sees_every_array():
    from paper_2603_00292_amd import workloads as wl

    W = wl.random_triangles(n_tri=16, n_rays=8, k=0)
    base = W.checksum()
    W.rays[3, 5] = 0.5
    assert W.checksum() != base
    W = wl.random_triangles(n_tri=16, n_rays=8, k=0)
    W.scene.meshes[0].indices[0, 0] ^= 1
    assert W.checksum() != base
