"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU): the
BVH builder (csrc/bvh_build.cpp) and the oracle (oracle/rt_oracle.c) are
compiled with gcc/g++ and the sanitizers into small drivers
(tests/sanitize/) that run them on seeded scenes with degenerate,
non-finite and empty input and check their results (tree structure; BVH
queries equal to the linear search).  Any sanitizer report aborts the
driver."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _build_and_run(tmp_path, compiler, sources, includes, std, libs):
    if shutil.which(compiler) is None:
        pytest.skip(f"{compiler} not found")
    exe = str(tmp_path / "driver")
    cmd = [compiler, std, *SAN, *[f"-I{i}" for i in includes], *sources, "-o", exe, *libs]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-6000:]
    assert "0 failures" in r.stdout
    return out


def test_builder_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_2603_00292_amd", "csrc")
    _build_and_run(tmp_path, "g++", [os.path.join(HERE, "sanitize", "builder_driver.cpp"),
                                     os.path.join(csrc, "bvh_build.cpp")],
                   [csrc], "-std=c++17", ["-lpthread"])


def test_oracle_under_sanitizers(tmp_path):
    odir = os.path.join(ROOT, "oracle")
    _build_and_run(tmp_path, "gcc", [os.path.join(HERE, "sanitize", "oracle_driver.c"),
                                     os.path.join(odir, "rt_oracle.c")],
                   [odir], "-std=c11", ["-lm"])
