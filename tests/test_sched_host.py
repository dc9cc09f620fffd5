"""The serving scheduler's host logic (csrc/serve_sched.h) under a fake executor (no GPU).

tests/host/sched_check.cpp is compiled with the system C++ compiler against
the library's own scheduling header and run: random streams of requests are
admitted by slot and workspace, stepped stage by stage and retired or
cancelled, and every step checks queue order, arena accounting (no overlap,
coalescing), slot use, one stage per request per step, section-ordered step
layout and that each request ends after exactly its stage count.
"""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# host-only build with the system compiler (no device code): plain, and with
# AddressSanitizer + UndefinedBehaviorSanitizer
BUILDS = {"plain": [], "sanitized": ["-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]}


@pytest.mark.parametrize("build", sorted(BUILDS))
def test_scheduler_invariants_under_fake_executor(tmp_path, build):
    exe = tmp_path / "sched_check"
    src = os.path.join(ROOT, "tests", "host", "sched_check.cpp")
    inc = os.path.join(ROOT, "paper_2501_00675_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", *BUILDS[build], f"-I{inc}", src, "-o", str(exe)],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "scheduler checks passed" in r.stdout
