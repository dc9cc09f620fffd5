"""The C program in paper_2501_00675_amd/examples, which uses the library through its C ABI alone (no
Python): built by the package build step against include/cos.h and the in-tree library, and run on the GPU,
where it checks cos_evaluate at FP64 and FP32-rescaled against the closed form of a complete layered graph
with level-constant factors, a served request against cos_evaluate's bits, and a refused call's status."""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2501_00675_amd")
EXE = os.path.join(PKG, "examples", "evaluate_layered")


def test_c_program_is_built_against_the_in_tree_library():
    assert os.path.exists(EXE), "built by paper_2501_00675_amd/_build.py"
    r = subprocess.run(["ldd", EXE], capture_output=True, text=True, check=True)
    line = next(l for l in r.stdout.splitlines() if "libcosdag.so" in l)
    assert os.path.realpath(line.split("=>")[1].split()[0]) == os.path.realpath(os.path.join(PKG, "libcosdag.so"))


@pytest.mark.gpu
def test_c_program_runs_on_the_gpu():
    print(f"running {EXE}", flush=True)
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout
