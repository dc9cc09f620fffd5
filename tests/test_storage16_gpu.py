"""16-bit level storage (fp16r, bf16r) through the C ABI, against the FP64 oracle.

The bar is the per-sample bound |y - V| <= B(x) derived in storage_bound.py
(binary16 or bfloat16 rounding of every stored level value, binary32
arithmetic, the subnormal floor; probabilistic model with lambda = 8), from
the oracle's node values of the graph and of its transpose.  The ratios to
the bound and the scaled errors are printed for the record.
"""

import numpy as np
import pytest
import torch

import oracle
from gpu_util import gpu_eval, sample_subset, say, to_dev
from storage_bound import headroom16, storage_bound
from workloads import make_config

pytestmark = pytest.mark.gpu

P16 = ("fp16r", "bf16r")


@pytest.fixture(scope="module")
def P():
    import paper_2501_00675_amd as P

    assert torch.cuda.is_available()
    return P


def check_bound(g, x, y, precision, label, idx=None):
    xs = x if idx is None else np.ascontiguousarray(x[:, idx])
    B, B1, V = storage_bound(g, xs, precision)
    Q = oracle.sweep(g, xs, "square")
    err = np.abs(y - V)
    ratio = err / np.where(B > 0, B, 1.0)
    scaled = oracle.scaled_error(y, V, Q)
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.median(err / np.abs(V))
    say(f"{label} {precision}: |y-V|/B max {ratio.max():.3f} p50 {np.median(ratio):.3f}, "
        f"|y-V|/B_first max {np.max(err / np.where(B1 > 0, B1, 1.0)):.3f}, scaled error max {scaled.max():.2e} "
        f"p50 {np.median(scaled):.2e}, |y-V|/|V| p50 {rel:.2e}")
    bad = np.flatnonzero(~(err <= B))
    assert bad.size == 0, f"{label} {precision}: {bad.size} samples above the bound, first {bad[0]}"
    return scaled


@pytest.mark.parametrize("precision", P16)
def test_tiny_within_bound(P, precision):
    g, x = make_config("tiny")
    G = P.Graph.from_leveled(g)
    check_bound(g, x, gpu_eval(G, x, precision), precision, "tiny")


@pytest.mark.parametrize("precision", P16)
@pytest.mark.parametrize("S", [1, 63, 257, 1000])
def test_ragged_sample_counts(P, precision, S):
    g, x = make_config("tiny", S=S, seed=11)
    G = P.Graph.from_leveled(g)
    check_bound(g, x, gpu_eval(G, x, precision), precision, f"tiny S={S}")


@pytest.mark.parametrize("precision", P16)
@pytest.mark.parametrize("name,n", [("mid", 256), ("precision", 64)])
def test_full_size_sampled(P, precision, name, n):
    g, x = make_config(name)
    G = P.Graph.from_leveled(g)
    y = gpu_eval(G, x, precision)
    idx = sample_subset(x.shape[1], n)
    check_bound(g, x, y[idx], precision, name, idx)
    assert np.all(np.isfinite(y))


@pytest.mark.parametrize("precision", P16)
def test_large_full_size_sampled(P, precision):
    g, x = make_config("large")
    G = P.Graph.from_leveled(g)
    y = gpu_eval(G, x, precision)
    idx = sample_subset(x.shape[1], 8)
    check_bound(g, x, y[idx], precision, "large", idx)


def test_bf16r_lookup_within_bound(P):
    g, x = make_config("mid", S=2048, factor="lookup")
    G = P.Graph.from_leveled(g)
    y = gpu_eval(G, x, "bf16r")
    idx = sample_subset(x.shape[1], 128)
    check_bound(g, x, y[idx], "bf16r", "mid lookup", idx)


def test_fp16r_is_more_accurate_than_bf16r(P):
    g, x = make_config("precision", S=1024)
    G = P.Graph.from_leveled(g)
    idx = sample_subset(x.shape[1], 64)
    V = oracle.sweep(g, np.ascontiguousarray(x[:, idx]))
    e16 = np.abs(gpu_eval(G, x, "fp16r")[idx] - V)
    eb16 = np.abs(gpu_eval(G, x, "bf16r")[idx] - V)
    # 3 more significand bits: about 8x smaller errors
    assert np.median(e16) * 2 < np.median(eb16)


@pytest.mark.parametrize("precision", P16)
def test_bit_reproducible_and_chunked(P, precision):
    g, x = make_config("mid", S=3000)
    G = P.Graph.from_leveled(g)
    y1 = gpu_eval(G, x, precision)
    y2 = gpu_eval(G, x, precision)
    assert np.array_equal(y1, y2)
    # a workspace for 256 samples: the library sweeps in chunks, bit-identically
    ws = torch.empty(G.workspace_bytes(256, precision), dtype=torch.uint8, device="cuda:0")
    y3 = gpu_eval(G, x, precision, workspace=ws)
    assert np.array_equal(y1, y3)


def test_fp16r_headroom_keeps_large_factors_finite_and_scale_exact(P):
    # a_e scaled by 2^20: level values up to ~2^22 times the previous level's
    # largest, beyond binary16's 65504 without the headroom shift
    g, x = make_config("tiny", S=512)
    big = g.with_params(a=g.a * 2.0 ** 20)
    bigger = g.with_params(a=g.a * 2.0 ** 21)
    assert np.all(headroom16(big)[1:] > 0)
    Gb, Gbb = P.Graph.from_leveled(big), P.Graph.from_leveled(bigger)
    xd = to_dev(x)
    e1 = torch.empty(x.shape[1], dtype=torch.int32, device="cuda:0")
    e2 = torch.empty_like(e1)
    m1 = Gb.evaluate(xd, "fp16r", out_exp=e1).cpu().numpy()
    m2 = Gbb.evaluate(xd, "fp16r", out_exp=e2).cpu().numpy()
    torch.cuda.synchronize()
    assert np.all(np.isfinite(m1))
    check_bound(big, x, np.ldexp(m1, e1.cpu().numpy()), "fp16r", "tiny a*2^20")
    # every level has headroom here, so doubling every factor shifts each
    # interior level's exponent by one and leaves the stored values
    # bit-identical; the binary64 final sum doubles exactly
    assert np.array_equal(m2, 2.0 * m1)
    assert np.all(e2.cpu().numpy() - e1.cpu().numpy() == g.L - 1)


def test_fp16r_refuses_unbounded_factors(P):
    g, x = make_config("tiny", S=8)
    a = g.a.copy()
    a[5] = 1e35  # a level row sum above 2^110 (still finite in binary32)
    G = P.Graph.from_leveled(g.with_params(a=a))
    with pytest.raises(P.CosError, match="binary16"):
        G.evaluate(to_dev(x), "fp16r")
    y = gpu_eval(G, x, "bf16r")  # bfloat16 has binary32's range
    assert y.shape == (8,)


def test_fp16r_refuses_lookup_factors(P):
    g, x = make_config("tiny", S=8, factor="lookup")
    G = P.Graph.from_leveled(g)
    with pytest.raises(P.CosError, match="binary16"):
        G.evaluate(to_dev(x), "fp16r")


@pytest.mark.parametrize("precision", P16)
def test_16bit_is_streamed_only(P, precision):
    g, x = make_config("tiny", S=8)
    G = P.Graph.from_leveled(g)
    assert not (G.info()["fused_mask"] >> P.PRECISIONS[precision]) & 1
    G.set_path("fused")
    with pytest.raises(P.CosError, match="streamed"):
        G.evaluate(to_dev(x), precision)


@pytest.mark.parametrize("precision", P16)
@pytest.mark.parametrize("S", [8, 300])
def test_server_serves_16bit_on_the_streamed_plan(P, precision, S):
    # the tiny graph takes the whole-graph plan at 32 and 64 bits; 16-bit requests run streamed
    # (one step per level, then the final node's two) with cos_evaluate's bits
    g, x = make_config("tiny", S=S)
    G = P.Graph.from_leveled(g)
    ref = gpu_eval(G, x, precision)
    srv = P.Server(hbm_budget=1 << 24, max_slots=4)
    try:
        gid = srv.add_graph(G)
        t = srv.submit(gid, to_dev(x), precision)
        st = srv.wait(t)
        assert st["status"] == 0 and st["steps"] == g.L + 1
        assert np.array_equal(t.out.cpu().numpy().view(np.uint64), ref.view(np.uint64))
    finally:
        srv.close()


@pytest.mark.parametrize("precision", P16)
def test_short_graphs_and_empty_rows(P, precision):
    from workloads import LeveledGraph, layered_graph

    rng = np.random.default_rng(4)
    x = rng.uniform(-1, 1, (3, 100))
    # L = 1: root joined to the final node by three parallel edges (no stored level)
    g1 = LeveledGraph(np.array([1, 1]), np.array([3]), np.zeros(3, np.int32), np.ones(3, np.int32),
                      np.array([0.5, -0.25, 2.0]), np.array([0.0, 1.0, 0.5]), np.zeros((3, 3)))
    check_bound(g1, x, gpu_eval(P.Graph.from_leveled(g1), x, precision), precision, "L=1")
    # L = 2: one stored level
    g2 = layered_graph([1, 7, 1], [1, 7], rng)
    g2 = g2.with_params(a=rng.uniform(-1, 1, g2.n_edges), b=rng.uniform(0, 2, g2.n_edges),
                        k=rng.uniform(-1, 1, (g2.n_edges, 3)))
    check_bound(g2, x, gpu_eval(P.Graph.from_leveled(g2), x, precision), precision, "L=2")
    # rows without in-edges and a level whose nodes all lose their in-edges
    g = layered_graph([1, 5, 6, 4, 1], [1, 2, 2, 4], rng, cover=False)
    g = g.with_params(a=rng.uniform(-1, 1, g.n_edges), b=rng.uniform(0, 2, g.n_edges),
                      k=rng.uniform(-1, 1, (g.n_edges, 3)))
    keep = np.ones(g.n_edges, bool)
    sl = g.level_slices()[2]
    keep[sl.start:sl.start + 3] = False
    g3 = LeveledGraph(g.widths, np.array([int(keep[s].sum()) for s in g.level_slices()]), g.src[keep],
                      g.dst[keep], g.a[keep], g.b[keep], g.k[keep])
    check_bound(g3, x, gpu_eval(P.Graph.from_leveled(g3), x, precision), precision, "zero-in-degree")
    g4 = LeveledGraph(np.array([1, 2, 1]), np.array([2, 0]), np.zeros(2, np.int32), np.array([1, 2], np.int32),
                      np.ones(2), np.zeros(2), np.zeros((2, 3)))
    assert np.all(gpu_eval(P.Graph.from_leveled(g4), x, precision) == 0.0)
