"""The oracle's long-double self-check build (-DORACLE_LONG_DOUBLE).

The same level sweep carried in x87 long double (64-bit significand) bounds
the binary64 oracle's own rounding error (Sec. III, numerical stability).  It
is pinned like the binary64 build, and more tightly against the exact path
sums, and then used to show on the mid and precision workloads what the error
metric of the parity tests rests on: the binary64 oracle itself fails a plain
per-sample relative bar of 1e-12 at samples near a zero of V(x), while its
error scaled by max(|V|, sqrt(Q)) stays below 1e-14.
"""

from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest

import oracle
import pins
from oracle.path_sum import path_sum
from workloads import make_config

U_LD = 2.0 ** -64  # unit roundoff of the x87 extended format


@pytest.fixture(scope="module")
def ld_lib():
    return oracle.load_long_double()


def gamma_ld(K: int) -> float:
    return K * U_LD / (1 - K * U_LD)


def test_long_double_build_passes_the_pins(ld_lib):
    pins.pin_paper_figure(ld_lib)
    pins.pin_exact_path_sum(ld_lib)
    pins.pin_level_constant_closed_form(ld_lib)
    pins.pin_all_ones_counts(ld_lib)
    pins.pin_transpose(ld_lib)
    pins.pin_pow2_scaling(ld_lib)


def test_long_double_build_is_within_its_own_bound(ld_lib, oracle_lib):
    """Exact rational path sums (dyadic inputs): the long-double result, rounded once to binary64, is within
    gamma_K(2^-64) * A + 2^-53 |V|.  The binary64 build misses this tighter bound on some of the same cases,
    so the self-check is more precise than what it checks."""
    rng = np.random.default_rng(91)
    graphs = [pins.random_small_graph(rng) for _ in range(10)]
    tiny, _ = make_config("tiny", S=4)
    graphs.append(pins.dyadic_params(tiny, rng))
    misses64 = 0
    for g in graphs:
        x = pins.dyadic(rng, (3, 4), -1, 1)
        Vld = oracle.sweep(g, x, "value", lib=ld_lib)
        V64 = oracle.sweep(g, x, "value", lib=oracle_lib)
        K = pins.error_K(g)
        for j in range(x.shape[1]):
            ex = path_sum(g, x[:, j])
            A = path_sum(g, x[:, j], weight=abs)
            bound = Fraction(gamma_ld(K)) * A + Fraction(2.0 ** -53) * abs(ex)
            assert abs(Fraction(float(Vld[j])) - ex) <= bound, (g.widths, j)
            misses64 += abs(Fraction(float(V64[j])) - ex) > bound
    assert misses64 > 0


@pytest.mark.parametrize("name,S", [("mid", 16384), ("precision", 1024)])
def test_binary64_oracle_against_long_double(ld_lib, oracle_lib, name, S):
    g, x = make_config(name)
    x = np.ascontiguousarray(x[:, :S])
    V64 = oracle.sweep(g, x, "value", lib=oracle_lib)
    Vld = oracle.sweep(g, x, "value", lib=ld_lib)
    Q = oracle.sweep(g, x, "square", lib=oracle_lib)
    with np.errstate(divide="ignore", invalid="ignore"):
        plain = np.abs(V64 - Vld) / np.abs(Vld)
    scaled = oracle.scaled_error(V64, Vld, Q)
    # a plain per-sample bar of 1e-12 fails for the binary64 oracle itself ...
    assert plain.max() > 1e-12, plain.max()
    # ... at samples where |V| is far below the scale of its path terms
    bad = plain > 1e-12
    assert np.all(np.abs(Vld[bad]) < 1e-2 * np.sqrt(Q[bad]))
    # while the scaled error stays two orders of magnitude below the FP64 bar
    assert scaled.max() <= 1e-14, scaled.max()
