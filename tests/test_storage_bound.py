"""The 16-bit storage error bound against a binary64 emulation of the scheme (no GPU)."""

import numpy as np
import pytest

from storage_bound import emulate_storage, headroom16, storage_bound
from workloads import make_config
from workloads.graphs import level_offsets


@pytest.mark.parametrize("precision", ["fp16r", "bf16r"])
@pytest.mark.parametrize("name,factor,S", [("tiny", "rational", 256), ("mid", "rational", 64),
                                           ("precision", "rational", 16), ("mid", "lookup", 64)])
def test_bound_covers_emulated_storage(name, factor, S, precision):
    if precision == "fp16r" and factor == "lookup":
        pytest.skip("binary16 storage takes rational factors only")
    g, x = make_config(name, S=S, factor=factor)
    B, B1, V = storage_bound(g, x, precision)
    err = np.abs(emulate_storage(g, x, precision) - V)
    assert np.all(err <= B)
    # the bound is not vacuous: storage rounding alone uses a visible part of it
    assert np.median(err / B) > 1e-3
    assert np.all(B <= B1 * 8.0 + 1e-300)


def test_bound_is_zero_where_storage_is_exact():
    # all factors 1: integer node values below 2^11 are exact in binary16
    g, x = make_config("tiny", S=8)
    g = g.with_params(a=1.0, b=0.0)
    B, _, V = storage_bound(g, x, "fp16r")
    assert np.all(emulate_storage(g, x, "fp16r") == V)
    assert np.all(B >= 0)


def test_headroom_exponents():
    g, _ = make_config("tiny", S=1)
    assert np.all(headroom16(g) == 0)  # |a| <= 1, in-degree 2
    big = g.with_params(a=g.a * 2.0 ** 20)
    h = headroom16(big)
    off = level_offsets(g.widths)
    for l, sl in enumerate(g.level_slices()[:-1], start=1):
        R = np.zeros(int(g.widths[l]))
        np.add.at(R, g.dst[sl] - off[l], np.abs(big.a[sl]))
        # the smallest h with R * 2^-h <= 2^14
        assert R.max() * 2.0 ** -h[l] <= 2.0 ** 14 < R.max() * 2.0 ** -(h[l] - 1)


def test_emulated_headroom_keeps_values_in_range():
    g, x = make_config("tiny", S=64)
    big = g.with_params(a=g.a * 2.0 ** 20)
    y = emulate_storage(big, x, "fp16r")
    B, _, V = storage_bound(big, x, "fp16r")
    assert np.all(np.isfinite(y)) and np.all(np.abs(y - V) <= B)
