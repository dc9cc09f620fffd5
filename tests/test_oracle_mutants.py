"""Plant plausible mistakes in the oracle (on the CPU) and check the pins catch each.

Every mutant is a copy of oracle/level_sweep.c with one textual change, built
into a temporary directory.  A mutant that passes every pin would mean the pins
cannot tell that mistake from the correct oracle.
"""

import os

import pytest

import oracle
import pins

MUTANTS = {
    "dropped_last_edge": ("e < edge_first[l]; ++e", "e < edge_first[l] - 1; ++e"),
    "factor_sign": ("return a / ((real)1.0 + b * r2);", "return -a / ((real)1.0 + b * r2);"),
    "offset_sign": ("real d1 = x1 - (real)k[1];", "real d1 = x1 + (real)k[1];"),
    "sample_index": ("x[S + s]", "x[s]"),
    "k_component": ("real d2 = x2 - (real)k[2];", "real d2 = x2 - (real)k[1];"),
    "swapped_a_b": ("return a / ((real)1.0 + b * r2);", "return b / ((real)1.0 + a * r2);"),
    "reads_dst_value": ("+= w * value[(int64_t)src[e]", "+= w * value[(int64_t)dst[e]"),
    "missing_square_norm": ("w = w * w;", "w = REAL_ABS(w);"),
    "r_not_squared": ("return a / ((real)1.0 + b * r2);", "return a / ((real)1.0 + b * sqrt(r2));"),
    "root_not_one": ("value[0 * SAMPLE_BLOCK + j] = 1.0;", "value[0 * SAMPLE_BLOCK + j] = 2.0;"),
    "level_not_cleared": ("value[n * SAMPLE_BLOCK + j] = 0.0;", "value[n * SAMPLE_BLOCK + j] = 1.0;"),
    # lookup factors
    "lookup_constant_dropped": ("w = (real)coef[e] * (real)x[(int64_t)slot[e] * S + s];",
                                "w = (real)x[(int64_t)slot[e] * S + s];"),
    "lookup_wrong_slot": ("w = (real)coef[e] * (real)x[(int64_t)slot[e] * S + s];",
                          "w = (real)coef[e] * (real)x[(int64_t)(slot[e] > 0 ? slot[e] - 1 : 0) * S + s];"),
    "lookup_wrong_sample": ("w = (real)coef[e] * (real)x[(int64_t)slot[e] * S + s];",
                            "w = (real)coef[e] * (real)x[(int64_t)slot[e] * S + s0];"),
    "lookup_constant_squared": ("w = (real)coef[e] * (real)x[(int64_t)slot[e] * S + s];",
                                "w = (real)coef[e] * (real)coef[e] * (real)x[(int64_t)slot[e] * S + s];"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(os.path.join(os.path.dirname(oracle.__file__), "level_sweep.c")).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(old, new, 1))
    lib = oracle.load(oracle.build(str(tmp_path / "libmutant.so"), str(mpath)), rebuild_if_stale=False)
    caught = []
    for pin in pins.ALL_PINS:
        try:
            pin(lib)
        except (AssertionError, ValueError):
            caught.append(pin.__name__)
    assert caught, f"mutant {name} passes every pin"
