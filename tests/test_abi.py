"""The C-ABI library loads, exports what include/cos.h declares, and validates input (no GPU)."""

import ctypes
import os
import re

import numpy as np
import pytest

from workloads import make_config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "cos.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cos_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = header_functions()
    for n in ["cos_create_graph", "cos_evaluate", "cos_destroy_graph", "cos_graph_export", "cos_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2501_00675_amd._lib as L

    lib = ctypes.CDLL(L.LIB_PATH)
    for n in header_functions():
        assert hasattr(lib, n), f"{n} declared in cos.h but not exported"
    assert sorted(L.EXPORTS) == header_functions()


def test_build_id_matches_sources_and_abi_version():
    import paper_2501_00675_amd as P
    from paper_2501_00675_amd import _build

    assert P.LIB.cos_build_id().decode() == _build.source_hash()
    assert P.LIB.cos_abi_version() == 4


def _create(g, **over):
    import paper_2501_00675_amd._lib as L

    arrs = dict(widths=np.asarray(g.widths, np.int64), epl=np.asarray(g.epl, np.int64),
                src=np.asarray(g.src, np.int32), dst=np.asarray(g.dst, np.int32), a=np.asarray(g.a, np.float64),
                b=np.asarray(g.b, np.float64), k=np.asarray(g.k, np.float64).reshape(-1))
    arrs.update(over)
    h = ctypes.c_void_p()
    p = {n: (v.ctypes.data_as(ctypes.c_void_p) if v is not None else None) for n, v in arrs.items()}
    st = L.LIB.cos_create_graph(g.L, p["widths"], p["epl"], p["src"], p["dst"], p["a"], p["b"], p["k"],
                                ctypes.byref(h))
    return st, L.LIB.cos_last_error().decode(), h


@pytest.mark.parametrize("case", ["root_width", "final_width", "zero_width", "src_level", "dst_level",
                                  "nan_a", "neg_b", "inf_k", "neg_epl", "null_src", "c0_overflow",
                                  "g_overflow"])
def test_create_rejects_invalid_input(case):
    g, _ = make_config("tiny", S=1)
    g = g.copy()
    over = {}
    if case == "root_width":
        g.widths[0] = 2
    elif case == "final_width":
        g.widths[-1] = 3
    elif case == "zero_width":
        g.widths[2] = 0
    elif case == "src_level":
        g.src[5] = 0
    elif case == "dst_level":
        g.dst[0] = 11
    elif case == "nan_a":
        g.a[3] = np.nan
    elif case == "neg_b":
        g.b[3] = -0.5
    elif case == "inf_k":
        g.k[2, 1] = np.inf
    elif case == "neg_epl":
        g.epl[1] = -1
    elif case == "null_src":
        over["src"] = None
    elif case == "c0_overflow":  # finite b and k, but 1 + b|k|^2 is not finite in binary64
        g.b[4], g.k[4] = 1e300, (1e10, 0.0, 0.0)
    elif case == "g_overflow":  # 1 + b |k|^2 stays finite, 2 b k overflows
        g.b[4], g.k[4] = 1e308, (1.0, 0.0, 0.0)
    st, msg, h = _create(g, **over)
    assert st == -1, (st, msg)
    assert msg and not h.value


@pytest.mark.parametrize("case", ["slot_high", "slot_negative", "nan_coef", "no_slots", "null_slot"])
def test_create_lookup_rejects_invalid_input(case):
    import paper_2501_00675_amd._lib as L

    g, _ = make_config("tiny", S=1, factor="lookup")
    slot, coef, n_slots = g.slot.copy(), g.coef.copy(), g.n_slots
    if case == "slot_high":
        slot[4] = n_slots
    elif case == "slot_negative":
        slot[0] = -1
    elif case == "nan_coef":
        coef[2] = np.nan
    elif case == "no_slots":
        n_slots = 0
    arrs = [np.asarray(g.widths, np.int64), np.asarray(g.epl, np.int64), np.asarray(g.src, np.int32),
            np.asarray(g.dst, np.int32), slot, coef]
    ptrs = [a.ctypes.data_as(ctypes.c_void_p) for a in arrs]
    if case == "null_slot":
        ptrs[4] = None
    h = ctypes.c_void_p()
    st = L.LIB.cos_create_graph_lookup(g.L, *ptrs, n_slots, ctypes.byref(h))
    assert st == -1 and L.LIB.cos_last_error().decode() and not h.value


def test_evaluate_rejects_null_and_bad_args():
    import paper_2501_00675_amd._lib as L

    assert L.LIB.cos_evaluate(None, None, 4, 0, None, None, None, 0, None) == -1
    assert "NULL" in L.LIB.cos_last_error().decode()
    assert L.LIB.cos_evaluate_no_alloc(None, None, 4, 0, None, None, None) == -1
    assert "cos_evaluate_no_alloc" in L.LIB.cos_last_error().decode()
    v = ctypes.c_uint64()
    assert L.LIB.cos_evaluate_workspace_size(None, 4, 0, ctypes.byref(v)) == -1
    assert L.LIB.cos_graph_get_info(None, None) == -1
    assert L.LIB.cos_destroy_graph(None) == 0
    ms, n = ctypes.c_double(), ctypes.c_int64()
    assert L.LIB.cos_timing_read(99, ctypes.byref(ms), ctypes.byref(n)) == -1


def test_server_rejects_null_and_bad_args():
    # argument checks that come before any device call
    import paper_2501_00675_amd._lib as L

    h = ctypes.c_void_p()
    for slots in (0, -1, 513):
        assert L.LIB.cos_server_create(1 << 20, slots, ctypes.byref(h)) == -1
        assert "max_slots" in L.LIB.cos_last_error().decode() and not h.value
    assert L.LIB.cos_server_create(1 << 20, 4, None) == -1
    gid, t = ctypes.c_int32(), ctypes.c_uint64()
    assert L.LIB.cos_server_add_graph(None, None, ctypes.byref(gid)) == -1
    assert L.LIB.cos_server_submit(None, 0, None, 4, 0, None, None, ctypes.byref(t)) == -1
    assert L.LIB.cos_server_poll(None, 1, None) == -1
    assert L.LIB.cos_server_wait(None, 1, None) == -1
    assert L.LIB.cos_server_cancel(None, 1) == -1
    assert L.LIB.cos_server_get_stats(None, None) == -1
    assert L.LIB.cos_server_fail_admission(None, 0) == -1
    assert L.LIB.cos_server_read_steps(None, None, 0, None) == -1
    assert L.LIB.cos_server_destroy(None) == 0


def test_mc_rejects_null_and_bad_args():
    # argument checks that come before any device call
    import paper_2501_00675_amd._lib as L

    v = ctypes.c_uint64()
    assert L.LIB.cos_mc_workspace_size(None, 16, 0, ctypes.byref(v)) == -1
    assert L.LIB.cos_mc_run(None, 0, 16, None, None, 0, 1, 0, 1.0, None, None, None, 0, None) == -1
    assert "NULL" in L.LIB.cos_last_error().decode()


def test_no_cpu_fallback_in_product_path():
    # the package never imports the oracle and has no torch compute on the path
    pkg = os.path.join(ROOT, "paper_2501_00675_amd")
    for f in os.listdir(pkg):
        if f.endswith(".py"):
            src = open(os.path.join(pkg, f)).read()
            assert "import oracle" not in src and "from oracle" not in src, f
