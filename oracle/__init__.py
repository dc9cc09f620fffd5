"""CPU oracle for leveled-DAG diagram summation -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library and the library
never calls it.

  level_sweep.c  plain FP64 level-by-level evaluator (C, OpenMP over samples);
                 built a second time with long double arithmetic as a self-check
  path_sum.py    the definition itself: exact rational sum over all paths
  mc.py          the Metropolis chain over sample configurations, with its
                 counter-based generator (Philox4x64-10), step by step

Functions here only marshal numpy arrays into the C evaluator.
"""

from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "level_sweep.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_LD = os.path.join(_HERE, "liboracle_ld.so")
_lib = None
_lib_ld = None

MODES = {"value": 0, "abs": 1, "square": 2}


def _src_hash(src_path: str = _SRC) -> str:
    with open(src_path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def build(out: str = _LIB, src: str = _SRC, defines: tuple = ()) -> str:
    """Compile level_sweep.c with gcc (FP64, no contraction, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", f'-DORACLE_SRC_HASH="{_src_hash(src)}"', *defines,
           "-o", out, src, "-lm"]
    subprocess.run(cmd, check=True)
    with open(out + ".srchash", "w") as f:
        f.write(_src_hash(src))
    return out


def build_long_double(out: str = _LIB_LD) -> str:
    """The self-check build of level_sweep.c: the same sweep carried in long double (x87 80-bit)."""
    return build(out, defines=("-DORACLE_LONG_DOUBLE",))


def _bind(lib):
    i32, i64, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.oracle_src_hash.restype = ctypes.c_char_p
    lib.oracle_check.restype = ctypes.c_int
    lib.oracle_check.argtypes = [i32, p, p, p, p, p, p, p]
    lib.oracle_sweep.restype = ctypes.c_int
    lib.oracle_sweep.argtypes = [i32, p, p, p, p, p, p, p, p, i64, i32, i32, p, p]
    lib.oracle_check_lookup.restype = ctypes.c_int
    lib.oracle_check_lookup.argtypes = [i32, p, p, p, p, p, p, i32]
    lib.oracle_sweep_lookup.restype = ctypes.c_int
    lib.oracle_sweep_lookup.argtypes = [i32, p, p, p, p, p, p, i32, p, i64, i32, i32, p, p]
    lib.oracle_sweep_nodes.restype = ctypes.c_int
    lib.oracle_sweep_nodes.argtypes = [i32, p, p, p, p, p, p, p, p, i64, i32, i32, p, p]
    lib.oracle_sweep_lookup_nodes.restype = ctypes.c_int
    lib.oracle_sweep_lookup_nodes.argtypes = [i32, p, p, p, p, p, p, i32, p, i64, i32, i32, p, p]
    return lib


def load(path: str = _LIB, rebuild_if_stale: bool = True):
    """Load the compiled oracle (building it when missing or out of date)."""
    global _lib
    if path == _LIB and _lib is not None:
        return _lib
    if not os.path.exists(path):
        if not rebuild_if_stale:
            raise FileNotFoundError(path)
        build(path)
    if path == _LIB and rebuild_if_stale:
        # decided from the hash file written beside the library, before any dlopen
        # (a library once loaded stays mapped under its path for the process)
        try:
            with open(path + ".srchash") as f:
                stale = f.read().strip() != _src_hash()
        except OSError:
            stale = True
        if stale:
            build(path)
    lib = _bind(ctypes.CDLL(path))
    if path == _LIB:
        if lib.oracle_src_hash().decode() != _src_hash():
            raise ImportError(f"{path} was built from other sources; rebuild with oracle.build()")
        _lib = lib
    return lib


def load_long_double():
    """The self-check build (every factor, product and sum in long double), built when missing or
    out of date.  Same entry points as load(); results are rounded to binary64 on output."""
    global _lib_ld
    if _lib_ld is not None:
        return _lib_ld
    try:
        with open(_LIB_LD + ".srchash") as f:
            stale = f.read().strip() != _src_hash()
    except OSError:
        stale = True
    if stale or not os.path.exists(_LIB_LD):
        build_long_double()
    lib = _bind(ctypes.CDLL(_LIB_LD))
    if lib.oracle_src_hash().decode() != _src_hash():
        raise ImportError(f"{_LIB_LD} was built from other sources; rebuild with oracle.build_long_double()")
    _lib_ld = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _is_lookup(g) -> bool:
    return getattr(g, "slot", None) is not None


def _arrays(g):
    A = dict(
        widths=np.ascontiguousarray(g.widths, dtype=np.int64),
        epl=np.ascontiguousarray(g.epl, dtype=np.int64),
        src=np.ascontiguousarray(g.src, dtype=np.int32),
        dst=np.ascontiguousarray(g.dst, dtype=np.int32),
    )
    if _is_lookup(g):
        A.update(slot=np.ascontiguousarray(g.slot, dtype=np.int32),
                 coef=np.ascontiguousarray(g.coef, dtype=np.float64))
    else:
        A.update(a=np.ascontiguousarray(g.a, dtype=np.float64),
                 b=np.ascontiguousarray(g.b, dtype=np.float64),
                 k=np.ascontiguousarray(g.k, dtype=np.float64).reshape(-1))
    return A


def check(g, lib=None) -> bool:
    lib = lib or load()
    A = _arrays(g)
    if _is_lookup(g):
        return lib.oracle_check_lookup(g.L, *[_ptr(A[n]) for n in ("widths", "epl", "src", "dst", "slot", "coef")],
                                       int(g.n_slots)) == 0
    return lib.oracle_check(g.L, *[_ptr(A[n]) for n in ("widths", "epl", "src", "dst", "a", "b", "k")]) == 0


def sweep(g, x, mode: str = "value", threads: int = 0, lib=None, return_threads: bool = False):
    """Evaluate the final-node value (or its |w| / w^2 norm sweeps).

    x: float64[3, S] sample coordinates for a graph with rational factors, or
    float64[n_slots, S] per-sample tables for a graph with lookup factors.
    """
    lib = lib or load()
    A = _arrays(g)
    x = np.ascontiguousarray(x, dtype=np.float64)
    rows = int(g.n_slots) if _is_lookup(g) else 3
    if x.ndim != 2 or x.shape[0] != rows:
        raise ValueError(f"x must be float64[{rows}, S]")
    S = x.shape[1]
    out = np.empty(S, dtype=np.float64)
    used = ctypes.c_int32(0)
    if _is_lookup(g):
        rc = lib.oracle_sweep_lookup(g.L, *[_ptr(A[n]) for n in ("widths", "epl", "src", "dst", "slot", "coef")],
                                     int(g.n_slots), _ptr(x), S, MODES[mode], int(threads), _ptr(out),
                                     ctypes.byref(used))
    else:
        rc = lib.oracle_sweep(g.L, *[_ptr(A[n]) for n in ("widths", "epl", "src", "dst", "a", "b", "k")],
                              _ptr(x), S, MODES[mode], int(threads), _ptr(out), ctypes.byref(used))
    if rc != 0:
        raise ValueError(f"oracle sweep failed with code {rc}")
    return (out, used.value) if return_threads else out


def node_values(g, x, mode: str = "value", threads: int = 0, lib=None):
    """Every node's value after the sweep: float64[n_nodes, S] (node n holds the
    sum over root-to-n paths of the product of the factors, or of their |w| or
    w^2 in the norm modes).  Row n_nodes - 1 is what sweep() returns."""
    lib = lib or load()
    A = _arrays(g)
    x = np.ascontiguousarray(x, dtype=np.float64)
    rows = int(g.n_slots) if _is_lookup(g) else 3
    if x.ndim != 2 or x.shape[0] != rows:
        raise ValueError(f"x must be float64[{rows}, S]")
    S = x.shape[1]
    out = np.empty(S, dtype=np.float64)
    nodes = np.empty((int(np.sum(g.widths)), S), dtype=np.float64)
    if _is_lookup(g):
        rc = lib.oracle_sweep_lookup_nodes(g.L, *[_ptr(A[n]) for n in ("widths", "epl", "src", "dst", "slot", "coef")],
                                           int(g.n_slots), _ptr(x), S, MODES[mode], int(threads), _ptr(out),
                                           _ptr(nodes))
    else:
        rc = lib.oracle_sweep_nodes(g.L, *[_ptr(A[n]) for n in ("widths", "epl", "src", "dst", "a", "b", "k")],
                                    _ptr(x), S, MODES[mode], int(threads), _ptr(out), _ptr(nodes))
    if rc != 0:
        raise ValueError(f"oracle sweep failed with code {rc}")
    return nodes


def evaluate(g, x, threads: int = 0, lib=None):
    """(V, A, Q): value, 1-norm and squared 2-norm of the path terms per sample."""
    return (sweep(g, x, "value", threads, lib), sweep(g, x, "abs", threads, lib),
            sweep(g, x, "square", threads, lib))


def scaled_error(y, r, Q):
    """Per-sample error |y - r| / max(|r|, sqrt(Q)).

    Plain relative error is unbounded near the sign changes of V(x) for any
    evaluator; sqrt(Q) (the 2-norm of the individual path terms) is the natural
    scale of the sum there.
    """
    y = np.asarray(y, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    den = np.maximum(np.abs(r), np.sqrt(np.asarray(Q, dtype=np.float64)))
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.abs(y - r) / den
    e[(den == 0) & (y == r)] = 0.0
    return e
