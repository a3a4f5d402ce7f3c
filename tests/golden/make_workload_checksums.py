"""Writes workload_checksums.json: the SHA-256 of the inputs of each
benchmark and parity workload as the seeded generators produce them.  The
test that reads it guards against an unnoticed change of a generator (which
would change every figure measured on it).  Run:

    python tests/golden/make_workload_checksums.py
"""
from __future__ import annotations

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_2603_00292_amd import workloads as wl  # noqa: E402

# name -> generator call; the large ones are the benchmark configurations
CASES = {
    "random_triangles_4096": lambda: wl.random_triangles(),
    "icosphere8_incoherent": lambda: wl.icosphere_incoherent(),
    "icosphere8_camera": lambda: wl.icosphere_camera(),
    "instanced_grids": lambda: wl.instanced_grids(),
    "displaced_grid_512x256": lambda: wl.displaced_grid(),
    "ao_terrain_1024x1024x16": lambda: wl.ao_terrain(),
    "aimed_instances_8": lambda: wl.aimed_instances(),
}


def batched_checksum() -> str:
    import hashlib

    h = hashlib.sha256()
    for w in wl.batched_meshes():
        h.update(w.checksum().encode())
    return h.hexdigest()


def main():
    out = {name: make().checksum() for name, make in CASES.items()}
    out["batched_meshes_256"] = batched_checksum()
    path = os.path.join(HERE, "workload_checksums.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
