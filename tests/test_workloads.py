"""Structure of the seeded synthetic graphs (no GPU)."""

import numpy as np
import pytest

from workloads import level_offsets, make_config, serving_mix, transpose

EXPECT = {  # edges per level and total, from the in-degree readings
    "tiny": ([3, 8, 6, 3], 20, 12),
    "mid": ([256] + [1024] * 10 + [256], 10752, 2818),
    "precision": ([4096] + [32768] * 22 + [4096], 729088, 94210),
}


@pytest.mark.parametrize("name", sorted(EXPECT))
def test_config_shapes(name):
    g, x = make_config(name, S=8)
    epl, E, N = EXPECT[name]
    assert g.epl.tolist() == epl and g.n_edges == E and g.n_nodes == N
    assert x.shape == (3, 8)


@pytest.mark.parametrize("name", ["tiny", "mid", "precision"])
def test_structure_invariants(name):
    g, _ = make_config(name, S=1)
    off = level_offsets(g.widths)
    for l, sl in enumerate(g.level_slices(), start=1):
        s, d = g.src[sl], g.dst[sl]
        assert s.min() >= off[l - 1] and s.max() < off[l]
        assert d.min() >= off[l] and d.max() < off[l + 1]
        # no parallel edges (sources drawn without replacement)
        pairs = s.astype(np.int64) * (1 << 32) + d
        assert len(np.unique(pairs)) == len(pairs)
        # every previous-level node has an out-edge, every node an in-edge
        assert len(np.unique(s)) == g.widths[l - 1]
        assert len(np.unique(d)) == g.widths[l]
        # edges are in (src, dst) order within the level
        assert np.all(np.diff(pairs) > 0)


def test_seed_determinism():
    g1, x1 = make_config("mid", S=16)
    g2, x2 = make_config("mid", S=16)
    assert np.array_equal(g1.src, g2.src) and np.array_equal(g1.a, g2.a) and np.array_equal(x1, x2)
    g3, _ = make_config("mid", S=16, seed=99)
    assert not np.array_equal(g1.src, g3.src)


def test_transpose_is_involution():
    g, _ = make_config("tiny", S=1)
    gtt = transpose(transpose(g))
    order = np.lexsort((gtt.dst, gtt.src))
    order0 = np.lexsort((g.dst, g.src))
    assert np.array_equal(gtt.src[order], g.src[order0]) and np.array_equal(gtt.a[order], g.a[order0])


def test_serving_mix_shapes():
    graphs, reqs = serving_mix(n_graphs=16, n_requests=32, max_width=64)
    assert len(graphs) == 16 and len(reqs) == 32
    for g in graphs:
        assert 4 <= g.L <= 20 and g.widths[0] == 1 and g.widths[-1] == 1
    for r in reqs:
        assert 256 <= r["S"] <= 8192 and r["x"].shape == (3, r["S"])
