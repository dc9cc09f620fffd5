"""ctypes loader for libcosdag.so (argument marshalling only).

torch is imported first on purpose: torch ships its own HIP runtime with the
same SONAME as the system one, and loading it first makes this library bind to
that same runtime, so torch streams and device pointers are valid here.  The
loader fails loudly when the library is missing, stale, or when two HIP
runtimes ended up in the process.
"""

from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (see module docstring)

from . import _build

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcosdag.so")

COS_OK, COS_EINVAL, COS_ENOMEM, COS_EDEVICE, COS_EAGAIN, COS_ECANCELED = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "COS_OK", -1: "COS_EINVAL", -2: "COS_ENOMEM", -3: "COS_EDEVICE", -4: "COS_EAGAIN",
                -5: "COS_ECANCELED"}
PRECISIONS = {"fp64": 0, "fp32r": 1, "fp32": 2, "fp16r": 3, "bf16r": 4}
KINDS = {"level": 0, "fused": 1, "final_partial": 2, "final_combine": 3, "fill": 4, "serve": 5, "hub": 6}

# every symbol include/cos.h declares (checked by the tests)
EXPORTS = [
    "cos_last_error", "cos_build_id", "cos_abi_version", "cos_create_graph", "cos_graph_get_info",
    "cos_graph_export", "cos_evaluate_workspace_size", "cos_evaluate", "cos_destroy_graph",
    "cos_timing_enable", "cos_timing_read", "cos_graph_set_path", "cos_create_graph_lookup",
    "cos_graph_export_lookup", "cos_evaluate_no_alloc",
    "cos_server_create", "cos_server_add_graph", "cos_server_submit", "cos_server_poll", "cos_server_wait",
    "cos_server_cancel", "cos_server_get_stats", "cos_server_destroy",
    "cos_mc_workspace_size", "cos_mc_run", "cos_server_fail_admission", "cos_server_read_steps",
]
PATHS = {"auto": 0, "streamed": 1, "fused": 2, "panel": 3}
FACTOR_KINDS = {0: "rational", 1: "lookup"}


class CosError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class GraphInfo(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("fused_mask", ctypes.c_int32), ("n_nodes", ctypes.c_int64),
                ("n_edges", ctypes.c_int64), ("max_width", ctypes.c_int64), ("max_in_degree", ctypes.c_int64),
                ("final_in_degree", ctypes.c_int64), ("device_bytes", ctypes.c_uint64),
                ("factor_kind", ctypes.c_int32), ("n_inputs", ctypes.c_int32), ("panel_mask", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class ReqStats(ctypes.Structure):
    _fields_ = [("t_submit_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64),
                ("status", ctypes.c_int32), ("steps", ctypes.c_int32), ("first_step", ctypes.c_int64),
                ("footprint", ctypes.c_int64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("cancelled", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("steps", ctypes.c_int64), ("items", ctypes.c_int64),
                ("max_active", ctypes.c_int64), ("max_step_requests", ctypes.c_int64),
                ("budget_bytes", ctypes.c_uint64), ("peak_bytes", ctypes.c_uint64)]


class StepRecord(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("t_launch_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64),
                ("n_fused", ctypes.c_int32), ("n_streamed", ctypes.c_int32), ("items", ctypes.c_int64)]


def _hip_runtimes_mapped() -> set:
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    paths.add(os.path.realpath(line.split()[-1]))
    except OSError:
        pass
    return paths


def _bind(lib):
    i32, i64, u64, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
    lib.cos_last_error.restype = ctypes.c_char_p
    lib.cos_build_id.restype = ctypes.c_char_p
    lib.cos_abi_version.restype = i32
    lib.cos_create_graph.restype = i32
    lib.cos_create_graph.argtypes = [i32, p, p, p, p, p, p, p, ctypes.POINTER(p)]
    lib.cos_graph_get_info.restype = i32
    lib.cos_graph_get_info.argtypes = [p, ctypes.POINTER(GraphInfo)]
    lib.cos_graph_export.restype = i32
    lib.cos_graph_export.argtypes = [p, p, p, p, p, p]
    lib.cos_create_graph_lookup.restype = i32
    lib.cos_create_graph_lookup.argtypes = [i32, p, p, p, p, p, p, i32, ctypes.POINTER(p)]
    lib.cos_graph_export_lookup.restype = i32
    lib.cos_graph_export_lookup.argtypes = [p, p, p, p, p]
    lib.cos_graph_set_path.restype = i32
    lib.cos_graph_set_path.argtypes = [p, i32]
    lib.cos_evaluate_workspace_size.restype = i32
    lib.cos_evaluate_workspace_size.argtypes = [p, i64, i32, ctypes.POINTER(u64)]
    lib.cos_evaluate.restype = i32
    lib.cos_evaluate.argtypes = [p, p, i64, i32, p, p, p, u64, p]
    lib.cos_evaluate_no_alloc.restype = i32
    lib.cos_evaluate_no_alloc.argtypes = [p, p, i64, i32, p, p, p]
    lib.cos_destroy_graph.restype = i32
    lib.cos_destroy_graph.argtypes = [p]
    lib.cos_timing_enable.restype = i32
    lib.cos_timing_enable.argtypes = [i32]
    lib.cos_timing_read.restype = i32
    lib.cos_timing_read.argtypes = [i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    lib.cos_server_create.restype = i32
    lib.cos_server_create.argtypes = [u64, i32, ctypes.POINTER(p)]
    lib.cos_server_add_graph.restype = i32
    lib.cos_server_add_graph.argtypes = [p, p, ctypes.POINTER(i32)]
    lib.cos_server_submit.restype = i32
    lib.cos_server_submit.argtypes = [p, i32, p, i64, i32, p, p, ctypes.POINTER(u64)]
    for name in ("cos_server_poll", "cos_server_wait"):
        getattr(lib, name).restype = i32
        getattr(lib, name).argtypes = [p, u64, ctypes.POINTER(ReqStats)]
    lib.cos_server_cancel.restype = i32
    lib.cos_server_cancel.argtypes = [p, u64]
    lib.cos_server_get_stats.restype = i32
    lib.cos_server_get_stats.argtypes = [p, ctypes.POINTER(ServerStats)]
    lib.cos_server_destroy.restype = i32
    lib.cos_server_destroy.argtypes = [p]
    lib.cos_server_read_steps.restype = i32
    lib.cos_server_read_steps.argtypes = [p, ctypes.POINTER(StepRecord), i64, ctypes.POINTER(i64)]
    lib.cos_server_fail_admission.restype = i32
    lib.cos_server_fail_admission.argtypes = [p, i64]
    lib.cos_mc_workspace_size.restype = i32
    lib.cos_mc_workspace_size.argtypes = [p, i64, i32, ctypes.POINTER(u64)]
    lib.cos_mc_run.restype = i32
    lib.cos_mc_run.argtypes = [p, i32, i64, p, p, i64, i64, u64, ctypes.c_double, p, p, p, u64, p]
    return lib


def load(path: str = LIB_PATH, check_stale: bool = True):
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run `python paper_2501_00675_amd/_build.py` "
                          "(there is no CPU fallback)")
    lib = _bind(ctypes.CDLL(path, mode=ctypes.RTLD_GLOBAL))
    if check_stale and os.path.isdir(_build.CSRC):
        built, current = lib.cos_build_id().decode(), _build.source_hash()
        if built != current:
            raise ImportError(f"{path} was built from other sources (build id {built}, sources {current}); "
                              "rebuild with `python paper_2501_00675_amd/_build.py`")
    rts = _hip_runtimes_mapped()
    if len(rts) > 1:
        raise ImportError(f"two HIP runtimes are loaded ({sorted(rts)}); import torch before this package")
    return lib


LIB = load()


def check(status: int, what: str = ""):
    if status != COS_OK:
        msg = LIB.cos_last_error().decode(errors="replace")
        raise CosError(status, f"{what}: {msg}" if what else msg)
