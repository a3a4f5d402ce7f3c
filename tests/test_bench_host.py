"""Host logic of bench.py, without a GPU: the one-GPU refusal, and the
committed rocprofv3 summaries read back only for the kernel source and the
variant they were taken on, with their scaled byte counts consistent with the
raw counters and the calibration they state."""
import os
import re
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")
INFO = {"node_width": 4}
VARIANT = (16, 256)
HEADLINE_RAYS = 4194304


def recorded_sha(path):
    with open(path) as f:
        for line in f:
            if "rt_kernels.hip sha256[:16] =" in line:
                return line.split("=")[-1].strip()
    raise AssertionError(f"{path} records no kernel source hash")


def test_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line for a configuration that was not measured


def test_traffic_only_for_recorded_source_and_variant(monkeypatch):
    sha = recorded_sha(bench.TRAFFIC_FILE)
    monkeypatch.setattr(bench, "kernel_sha", lambda: sha)
    v = bench.measured_traffic(INFO, VARIANT)
    assert isinstance(v, int)
    # L2-to-fabric bytes of one headline launch: below the ~3.1 KB per ray the
    # traversal requests, above the rays and hits it must read and write
    assert (32 + 16) * HEADLINE_RAYS < v < 3200 * HEADLINE_RAYS
    assert bench.measured_traffic(INFO, (32, 256)) is None
    assert bench.measured_traffic(INFO, (16, 128)) is None
    assert bench.measured_traffic({"node_width": 8}, VARIANT) is None
    monkeypatch.setattr(bench, "kernel_sha", lambda: "0" * 16)
    assert bench.measured_traffic(INFO, VARIANT) is None


def test_valu_only_for_recorded_source_and_variant(monkeypatch):
    sha = recorded_sha(bench.SQ_FILE)
    monkeypatch.setattr(bench, "kernel_sha", lambda: sha)
    insts, lanes = bench.measured_valu(INFO, VARIANT)
    assert insts > HEADLINE_RAYS / 64  # at least one wave instruction per wave of rays
    assert 1.0 / 64 <= lanes <= 1.0
    assert bench.measured_valu(INFO, (32, 256)) is None
    assert bench.measured_valu({"node_width": 2}, VARIANT) is None
    monkeypatch.setattr(bench, "kernel_sha", lambda: "f" * 16)
    assert bench.measured_valu(INFO, VARIANT) is None


def test_traffic_summaries_scale_their_counters():
    """Every PMC traffic summary's scaled_bytes column is FETCH_SIZE and
    WRITE_SIZE (KiB) times the calibration factors the file states."""
    files = [f for f in sorted(os.listdir(PROFILES)) if f.endswith("_pmc_traffic.txt")]
    assert files
    for name in files:
        text = open(os.path.join(PROFILES, name)).read()
        m = re.search(r"fetch scale ([0-9.]+); WRITE_SIZE read [0-9.]+ KiB -> write scale ([0-9.]+)", text)
        assert m, name
        fs, ws = float(m.group(1)), float(m.group(2))
        rows = 0
        for line in text.splitlines():
            parts = line.split()
            if line.startswith("#") or len(parts) < 5 or not parts[-1].isdigit():
                continue
            fetch, write, scaled = float(parts[-3]), float(parts[-2]), int(parts[-1])
            want = 1024.0 * (fetch * fs + write * ws)
            # the factors are printed to four decimals
            assert abs(scaled - want) <= 1e-4 * want + 2048, (name, line)
            rows += 1
        assert rows, name


@pytest.mark.parametrize("name", sorted(f for f in os.listdir(PROFILES) if f.endswith(".txt")))
def test_profile_names_its_command_and_source(name):
    """A summary gives the command that made it (committed files only) and
    the hash of the kernel source it was taken on."""
    text = open(os.path.join(PROFILES, name)).read()
    cmds = [l for l in text.splitlines() if "rocprofv3 " in l and " -- " in l]
    assert cmds, name
    for c in cmds:
        assert "_work" not in c, (name, c)
        prog = c.split(" -- ", 1)[1].split()
        assert prog[0] == "python3" and os.path.exists(os.path.join(ROOT, prog[1])), (name, c)
    assert re.fullmatch(r"[0-9a-f]{16}", recorded_sha(os.path.join(PROFILES, name)))
