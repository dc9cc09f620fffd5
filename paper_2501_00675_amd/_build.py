"""Build libcosdag.so (host runtime + HIP kernels for gfx950) in-tree with hipcc.

    python paper_2501_00675_amd/_build.py

(run as a script: importing the package loads the library it builds)
"""

from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libcosdag.so")
OBJDIR = os.path.join(ROOT, "_build", "cosdag")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", f"-I{INCLUDE}", f"-I{CSRC}",
    # no packed FP32 math (v_pk_*_f32) anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def sources() -> list[str]:
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp", ".h")))


def source_hash() -> str:
    h = hashlib.sha256()
    for p in sources() + [os.path.join(INCLUDE, "cos.h")]:
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _compile(src: str, defines: list[str]) -> str:
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC, *COMMON, *defines, "-c", *lang, src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    bid = source_hash()
    defines = [f'-DCOS_BUILD_ID="{bid}"']
    srcs = [s for s in sources() if not s.endswith(".h")]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, defines), srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    example = build_example()
    if verbose:
        print(f"built {LIB} (build id {bid}) and {example}")
    return LIB


EXAMPLE_SRC = os.path.join(PKG, "examples", "evaluate_layered.c")
EXAMPLE = os.path.join(PKG, "examples", "evaluate_layered")


def build_example() -> str:
    """The C program that uses the library without Python (plain C, the system compiler)."""
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__", f"-I{INCLUDE}",
           f"-I{rocm}/include", EXAMPLE_SRC, f"-L{PKG}", "-lcosdag", f"-L{rocm}/lib", "-lamdhip64", "-lm",
           "-Wl,-rpath,$ORIGIN/..", f"-Wl,-rpath,{rocm}/lib", "-o", EXAMPLE]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"example build failed:\n{r.stderr}")
    return EXAMPLE


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
