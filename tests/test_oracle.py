"""The CPU oracle against its pins (no GPU)."""

import numpy as np
import pytest

import oracle
import pins
from workloads import make_config


def test_paper_figure_path_count(oracle_lib):
    pins.pin_paper_figure(oracle_lib)


def test_exact_path_sum(oracle_lib):
    pins.pin_exact_path_sum(oracle_lib)


def test_level_constant_closed_form(oracle_lib):
    pins.pin_level_constant_closed_form(oracle_lib)


def test_all_ones_path_counts(oracle_lib):
    pins.pin_all_ones_counts(oracle_lib)


@pytest.mark.slow
def test_all_ones_path_count_large(oracle_lib):
    # 3^30 * 2^46 paths on the 12M-edge graph, exact in binary64 (3^30 < 2^53)
    pins.pin_all_ones_counts(oracle_lib, include_large=True)


def test_transpose_invariance(oracle_lib):
    pins.pin_transpose(oracle_lib)


def test_pow2_scaling_exact(oracle_lib):
    pins.pin_pow2_scaling(oracle_lib)


def test_lookup_exact_path_sum(oracle_lib):
    pins.pin_lookup_exact_path_sum(oracle_lib)


def test_lookup_level_constant_closed_form(oracle_lib):
    pins.pin_lookup_level_constant(oracle_lib)


def test_lookup_all_ones_path_counts(oracle_lib):
    pins.pin_lookup_all_ones(oracle_lib)


def test_lookup_sign_scale_and_relabel_exact(oracle_lib):
    pins.pin_lookup_sign_and_scale(oracle_lib)


def test_lookup_transpose_invariance(oracle_lib):
    pins.pin_lookup_transpose(oracle_lib)


def test_lookup_rejects_bad_slots(oracle_lib):
    g, T = make_config("tiny", S=4, factor="lookup")
    bad = g.with_lookup(g.slot, g.coef, g.n_slots)
    bad.slot[3] = g.n_slots  # outside the table
    with pytest.raises(ValueError):
        oracle.sweep(bad, T, lib=oracle_lib)
    with pytest.raises(ValueError):  # the table must have n_slots rows
        oracle.sweep(g, T[:-1], lib=oracle_lib)


def test_thread_count_does_not_change_bits(oracle_lib):
    g, x = make_config("mid", S=100)
    v1 = oracle.sweep(g, x, threads=1, lib=oracle_lib)
    v4 = oracle.sweep(g, x, threads=4, lib=oracle_lib)
    assert np.array_equal(v1, v4)


def test_norm_sweeps_bound_value(oracle_lib):
    g, x = make_config("tiny", S=256)
    V, A, Q = oracle.evaluate(g, x, lib=oracle_lib)
    assert np.all(A >= np.abs(V) * (1 - 1e-15))
    assert np.all(Q >= 0)
    # all factors positive: value and 1-norm coincide
    gp = g.with_params(a=np.abs(g.a))
    Vp, Ap, _ = oracle.evaluate(gp, x, lib=oracle_lib)
    assert np.array_equal(Vp, Ap)


def test_chain_is_product_of_factors(oracle_lib):
    # all widths 1: a single path, V = prod_l w_l(x)
    from workloads import layered_graph

    rng = np.random.default_rng(5)
    g = layered_graph([1] * 8, 1, rng)
    g = g.with_params(a=rng.uniform(-1, 1, 7), b=rng.uniform(0, 2, 7), k=rng.uniform(-1, 1, (7, 3)))
    x = rng.normal(size=(3, 50))
    w = g.a[:, None] / (1 + g.b[:, None] * ((x[None, :, :] - g.k[:, :, None]) ** 2).sum(1))
    v = oracle.sweep(g, x, lib=oracle_lib)
    np.testing.assert_allclose(v, w.prod(0), rtol=100 * 2.0 ** -53)


@pytest.mark.parametrize("case", ["root_width", "final_width", "src_level", "dst_level", "nan_a",
                                  "neg_b", "inf_k"])
def test_oracle_rejects_invalid(oracle_lib, case):
    g, _ = make_config("tiny", S=1)
    g = g.copy()
    if case == "root_width":
        g.widths[0] = 2
    elif case == "final_width":
        g.widths[-1] = 2
    elif case == "src_level":
        g.src[5] = 0  # edge of level 2 with its source in level 0
    elif case == "dst_level":
        g.dst[0] = 11
    elif case == "nan_a":
        g.a[3] = np.nan
    elif case == "neg_b":
        g.b[3] = -0.5
    elif case == "inf_k":
        g.k[2, 1] = np.inf
    assert not oracle.check(g, lib=oracle_lib)
    with pytest.raises(ValueError):
        oracle.sweep(g, np.zeros((3, 1)), lib=oracle_lib)


def test_zero_in_degree_and_empty_level(oracle_lib):
    # a node without in-edges holds 0; a level with no edges zeroes the result
    from workloads import LeveledGraph

    g = LeveledGraph(np.array([1, 2, 1]), np.array([1, 2]), np.array([0, 1, 2], np.int32),
                     np.array([1, 3, 3], np.int32), np.array([0.5, 1.0, 7.0]), np.zeros(3), np.zeros((3, 3)))
    assert oracle.sweep(g, np.zeros((3, 2)), lib=oracle_lib).tolist() == [0.5, 0.5]
    g2 = LeveledGraph(np.array([1, 2, 1]), np.array([2, 0]), np.array([0, 0], np.int32),
                      np.array([1, 2], np.int32), np.ones(2), np.zeros(2), np.zeros((2, 3)))
    assert oracle.sweep(g2, np.zeros((3, 3)), lib=oracle_lib).tolist() == [0.0] * 3


@pytest.mark.parametrize("factor", ["rational", "lookup"])
@pytest.mark.parametrize("name", ["tiny", "mid"])
def test_node_values_level_identity(oracle_lib, name, factor):
    # forward node values v_n (root -> n) and backward ones G_n (n -> final,
    # the forward values of the transposed graph): every level l cuts each
    # path exactly once, so sum_{n in l} v_n G_n = V for every l
    from workloads import transpose
    from workloads.graphs import level_offsets

    g, x = make_config(name, S=16, factor=factor)
    v = oracle.node_values(g, x)
    t = oracle.node_values(transpose(g), x)
    V = oracle.sweep(g, x)
    assert np.array_equal(v[-1], V) and np.all(v[0] == 1.0)
    off, off_t = level_offsets(g.widths), level_offsets(g.widths[::-1])
    for l in range(g.L + 1):
        fw = v[off[l]:off[l + 1]]
        bw = t[off_t[g.L - l]:off_t[g.L - l + 1]]  # (level l, i) <-> transposed (level L-l, i)
        s = np.sum(fw * bw, axis=0)
        assert np.all(np.abs(s - V) <= 1e-12 * np.sum(np.abs(fw * bw), axis=0)), l


def test_node_values_count_paths(oracle_lib):
    g, x = make_config("mid", S=2)
    g = g.with_params(a=1.0, b=0.0)
    count = np.zeros(g.n_nodes)
    count[0] = 1.0
    for s, d in zip(g.src.tolist(), g.dst.tolist()):  # level-major order
        count[d] += count[s]
    v = oracle.node_values(g, x)
    assert np.all(v == count[:, None])
