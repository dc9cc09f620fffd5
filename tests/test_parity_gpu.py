"""GPU path (through the C ABI) against the CPU oracle, element by element.

Tolerances: per-sample |y - r| / max(|r|, sqrt(Q)) <= 1e-12 for FP64 and
<= 1e-5 for the FP32 paths, where r is the oracle's FP64 value and Q the
squared 2-norm of the path terms; integer-valued results (path counts) must be
bit-exact.
"""

import numpy as np
import pytest
import torch

import oracle
import pins
from gpu_util import PRECISIONS, assert_parity, gpu_eval, oracle_ref, sample_subset, say, to_dev
from workloads import LeveledGraph, layered_graph, make_config, transpose

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2501_00675_amd as P

    assert torch.cuda.is_available()
    return P


def graph(P, g):
    return P.Graph.from_leveled(g)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_paper_figure_all_ones(P, precision):
    g, expect = pins.load_figure_graph()
    x = np.random.default_rng(1).uniform(-1, 1, (3, 300))
    y = gpu_eval(graph(P, g), x, precision)
    assert np.all(y == expect)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_tiny_parity(P, precision):
    g, x = make_config("tiny")
    say(f"tiny {precision} S={x.shape[1]}")
    y = gpu_eval(graph(P, g), x, precision)
    V, Q = oracle_ref(g, x)
    assert_parity(y, V, Q, precision, "tiny")


@pytest.mark.parametrize("S", [1, 2, 63, 64, 65, 127, 255, 257, 1000])
@pytest.mark.parametrize("precision", ["fp64", "fp32r"])
@pytest.mark.parametrize("path", ["fused", "streamed"])
def test_ragged_sample_counts(P, S, precision, path):
    g, x = make_config("mid", S=S, width=40, L=6)
    say(f"ragged {precision} {path} S={S}")
    y = gpu_eval(graph(P, g).set_path(path), x, precision)
    V, Q = oracle_ref(g, x)
    assert_parity(y, V, Q, precision, f"ragged S={S}")


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("name,S,over", [("tiny", 1024, {}), ("mid", 1000, {}), ("mid", 4096, {}),
                                         ("mid", 777, dict(width=300, L=5, degree=7))])
def test_fused_and_streamed_bit_identical(P, precision, name, S, over):
    g, x = make_config(name, S=S, **over)
    G = graph(P, g)
    code = {"fp64": 0, "fp32r": 1, "fp32": 2}[precision]
    if not (G.info()["fused_mask"] >> code) & 1:
        pytest.skip("graph does not fit the fused plan at this precision")
    say(f"fused vs streamed {name} {precision} S={S} {over}")
    yf = gpu_eval(G.set_path("fused"), x, precision)
    ys = gpu_eval(G.set_path("streamed"), x, precision)
    assert np.array_equal(yf.view(np.uint64), ys.view(np.uint64))
    V, Q = oracle_ref(g, x)
    assert_parity(yf, V, Q, precision, f"{name} fused")


def test_fused_plan_rejected_when_too_wide(P):
    g, x = make_config("precision", S=64)
    G = graph(P, g)
    assert G.info()["fused_mask"] == 0
    G.set_path("fused")
    with pytest.raises(P.CosError) as ei:
        gpu_eval(G, x, "fp64")
    assert ei.value.status == -1


@pytest.mark.parametrize("precision", PRECISIONS)
def test_mid_full_size_sampled(P, precision):
    g, x = make_config("mid")
    say(f"mid full {precision}")
    y = gpu_eval(graph(P, g), x, precision)
    idx = sample_subset(x.shape[1], 512)
    V, Q = oracle_ref(g, x, idx)
    assert np.all(np.isfinite(y))
    assert_parity(y[idx], V, Q, precision, "mid")


@pytest.mark.parametrize("precision", PRECISIONS)
def test_precision_full_size_sampled(P, precision):
    g, x = make_config("precision")
    say(f"precision full {precision}")
    y = gpu_eval(graph(P, g), x, precision)
    idx = sample_subset(x.shape[1], 192)
    V, Q = oracle_ref(g, x, idx)
    assert_parity(y[idx], V, Q, precision, "precision")


@pytest.mark.slow
def test_large_full_size_sampled(P):
    g, x = make_config("large")
    G = graph(P, g)
    idx = sample_subset(x.shape[1], 24)
    V, Q = oracle_ref(g, x, idx)
    for precision in ("fp64", "fp32r"):
        say(f"large full {precision}")
        y = gpu_eval(G, x, precision)
        assert_parity(y[idx], V, Q, precision, "large")


@pytest.mark.slow
def test_large_graph_beyond_one_sweep_is_chunked(P):
    # the large graph's level buffer for 4500 samples (65536 rows x 4608 x 8 B) exceeds the 2 GiB a sweep
    # addresses with 32-bit offsets: the library sweeps 3840 samples, then the remaining 660
    g, x = make_config("large", S=4500, seed=17)
    G = graph(P, g)
    assert G.workspace_bytes(4500, "fp64") < 2 * 65536 * 4608 * 8  # the plan is a chunk, not the whole S
    idx = np.unique(np.concatenate([sample_subset(4500, 14, seed=3), [3839, 3840, 4499]]))
    V, Q = oracle_ref(g, x, idx)
    for precision in ("fp64", "fp32r"):
        say(f"large S=4500 {precision}")
        y = gpu_eval(G, x, precision)
        assert_parity(y[idx], V, Q, precision, "large chunked")


@pytest.mark.parametrize("name,expect", [("tiny", 12), ("mid", 2 ** 28), ("precision", 2 ** 78)])
@pytest.mark.parametrize("precision", PRECISIONS)
def test_all_ones_path_counts_exact(P, name, expect, precision):
    g, x = make_config(name, S=300)
    g1 = g.with_params(a=1.0, b=0.0, k=0.0)
    y = gpu_eval(graph(P, g1), x, precision)
    assert np.all(y == float(expect)), (y[:4], expect)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_level_constant_closed_form(P, precision):
    rng = np.random.default_rng(7)
    g, x = make_config("mid", S=512)
    gc, (al, bl, kl) = pins.level_constant_graph(g, rng)
    d = pins.in_degrees(g)
    cf = np.ones(x.shape[1])
    for l in range(g.L):
        cf = cf * (d[l] * al[l] / (1.0 + bl[l] * ((x - kl[l][:, None]) ** 2).sum(0)))
    y = gpu_eval(graph(P, gc), x, precision)
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert np.max(np.abs(y - cf) / np.abs(cf)) <= tol


@pytest.mark.parametrize("precision", PRECISIONS)
def test_bit_reproducible(P, precision):
    g, x = make_config("precision", S=1000)
    G = graph(P, g)
    y1 = gpu_eval(G, x, precision)
    y2 = gpu_eval(G, x, precision)
    assert np.array_equal(y1.view(np.uint64), y2.view(np.uint64))


def test_input_permutation_gives_identical_graph_and_bits(P):
    g, x = make_config("mid", S=700)
    rng = np.random.default_rng(3)
    gp = g.copy()
    for sl in g.level_slices():
        perm = rng.permutation(sl.stop - sl.start) + sl.start
        gp.src[sl], gp.dst[sl], gp.a[sl], gp.b[sl], gp.k[sl] = (g.src[perm], g.dst[perm], g.a[perm], g.b[perm],
                                                                 g.k[perm])
    G1, G2 = graph(P, g), graph(P, gp)
    e1, e2 = G1.export(), G2.export()
    for n in e1:
        assert np.array_equal(e1[n], e2[n])
    for precision in ("fp64", "fp32r"):
        assert np.array_equal(gpu_eval(G1, x, precision), gpu_eval(G2, x, precision))


def test_export_is_canonical_sort_of_input(P):
    g, _ = make_config("tiny", S=1, order="shuffle")
    e = graph(P, g).export()
    for sl in g.level_slices():
        bits = [np.asarray(v).view(np.uint64) for v in (g.k[sl, 2], g.k[sl, 1], g.k[sl, 0], g.b[sl], g.a[sl])]
        order = np.lexsort((*bits, g.src[sl], g.dst[sl])) + sl.start
        assert np.array_equal(e["dst"][sl], g.dst[order]) and np.array_equal(e["src"][sl], g.src[order])
        assert np.array_equal(e["a"][sl], g.a[order]) and np.array_equal(e["k"][sl], g.k[order])


def test_fp32_rescaled_equals_unscaled_on_benign_graph(P):
    # power-of-two scaling is exact: with no under/overflow the two FP32 paths agree bit for bit
    g, x = make_config("mid", S=1024)
    G = graph(P, g)
    assert np.array_equal(gpu_eval(G, x, "fp32r"), gpu_eval(G, x, "fp32"))


def test_out_exp_form(P):
    g, x = make_config("precision", S=300)
    G = graph(P, g)
    xd = to_dev(x)
    e = torch.empty(x.shape[1], dtype=torch.int32, device=xd.device)
    m = G.evaluate(xd, "fp32r", out_exp=e)
    y = G.evaluate(xd, "fp32r")
    torch.cuda.synchronize()
    assert np.array_equal(np.ldexp(m.cpu().numpy(), e.cpu().numpy()), y.cpu().numpy())
    e64 = torch.full((x.shape[1],), 7, dtype=torch.int32, device=xd.device)
    G.evaluate(xd, "fp64", out_exp=e64)
    torch.cuda.synchronize()
    assert int(e64.abs().max()) == 0


def test_rescale_prevents_fp32_underflow(P):
    # 40 levels of factors ~2^-6: the value ~2^-240 underflows binary32 but not binary64
    rng = np.random.default_rng(11)
    g = layered_graph([1] + [8] * 39 + [1], 2, rng)
    E = g.n_edges
    g = g.with_params(a=rng.uniform(0.5, 1.0, E) * 2.0 ** -7, b=rng.uniform(0.5, 2, E), k=rng.uniform(-1, 1, (E, 3)))
    x = rng.uniform(-1, 1, (3, 256))
    V, Q = oracle_ref(g, x)
    assert np.all(np.abs(V) < 2.0 ** -200)
    G = graph(P, g)
    assert_parity(gpu_eval(G, x, "fp32r"), V, Q, "fp32r", "underflow")
    assert np.all(gpu_eval(G, x, "fp32") == 0.0)
    assert_parity(gpu_eval(G, x, "fp64"), V, Q, "fp64", "underflow")


@pytest.mark.parametrize("precision", PRECISIONS)
def test_single_edge_level_and_parallel_edges(P, precision):
    # L = 1: root joined to the final node by three parallel edges
    g = LeveledGraph(np.array([1, 1]), np.array([3]), np.zeros(3, np.int32), np.ones(3, np.int32),
                     np.array([0.5, -0.25, 2.0]), np.array([0.0, 1.0, 0.5]), np.zeros((3, 3)))
    x = np.random.default_rng(2).uniform(-1, 1, (3, 70))
    V, Q = oracle_ref(g, x)
    assert_parity(gpu_eval(graph(P, g), x, precision), V, Q, precision, "L=1")


@pytest.mark.parametrize("precision", PRECISIONS)
def test_zero_in_degree_nodes_and_empty_level(P, precision):
    rng = np.random.default_rng(4)
    g = layered_graph([1, 5, 6, 4, 1], [1, 2, 2, 4], rng, cover=False)
    g = g.with_params(a=rng.uniform(-1, 1, g.n_edges), b=rng.uniform(0, 2, g.n_edges),
                      k=rng.uniform(-1, 1, (g.n_edges, 3)))
    keep = np.ones(g.n_edges, bool)
    sl = g.level_slices()[2]
    keep[sl.start:sl.start + 3] = False  # some level-3 nodes lose in-edges
    g2 = LeveledGraph(g.widths, np.array([int(keep[s].sum()) for s in g.level_slices()]), g.src[keep], g.dst[keep],
                      g.a[keep], g.b[keep], g.k[keep])
    x = rng.uniform(-1, 1, (3, 100))
    V, Q = oracle_ref(g2, x)
    assert_parity(gpu_eval(graph(P, g2), x, precision), V, Q, precision, "zero-in-degree")
    g3 = LeveledGraph(np.array([1, 2, 1]), np.array([2, 0]), np.zeros(2, np.int32), np.array([1, 2], np.int32),
                      np.ones(2), np.zeros(2), np.zeros((2, 3)))
    assert np.all(gpu_eval(graph(P, g3), x, precision) == 0.0)


def _hub_graph(W, fan, rng):
    # level 2 is a single node fed by all W nodes of level 1 (an interior in-degree of W), which
    # then fans out to `fan` nodes; factors drawn as for the synthetic workloads
    ar = np.arange(W)
    widths = np.array([1, W, 1, fan, 1])
    first = np.concatenate([[0], np.cumsum(widths)])
    src = np.concatenate([np.zeros(W, int), first[1] + ar, np.full(fan, first[2]), first[3] + np.arange(fan)])
    dst = np.concatenate([first[1] + ar, np.full(W, first[2]), first[3] + np.arange(fan), np.full(fan, first[4])])
    E = len(src)
    return LeveledGraph(widths, np.array([W, W, fan, fan]), src.astype(np.int32), dst.astype(np.int32),
                        rng.uniform(-1, 1, E), rng.uniform(0.5, 2, E), rng.uniform(-1, 1, (E, 3)))


def _parallel_hub_graph(W, mult, fan, rng):
    # as _hub_graph, but the hub takes `mult` parallel edges from each of the W nodes of level 1, so a
    # narrow graph (one that fits the whole-graph plan) holds a node of W * mult in-edges
    widths = np.array([1, W, 1, fan, 1])
    first = np.concatenate([[0], np.cumsum(widths)])
    n = W * mult
    src = np.concatenate([np.zeros(W, int), first[1] + np.tile(np.arange(W), mult), np.full(fan, first[2]),
                          first[3] + np.arange(fan)])
    dst = np.concatenate([first[1] + np.arange(W), np.full(n, first[2]), first[3] + np.arange(fan),
                          np.full(fan, first[4])])
    E = len(src)
    return LeveledGraph(widths, np.array([W, n, fan, fan]), src.astype(np.int32), dst.astype(np.int32),
                        rng.uniform(-1, 1, E), rng.uniform(0.5, 2, E), rng.uniform(-1, 1, (E, 3)))


def _serve_one(P, G, x, precision):
    srv = P.Server(1 << 30, 4)
    gid = srv.add_graph(G)
    xd = to_dev(x)
    out = torch.empty(x.shape[1], dtype=torch.float64, device=xd.device)
    srv.wait(srv.submit(gid, xd, precision, out=out))
    torch.cuda.synchronize()
    y = out.cpu().numpy()
    srv.close()
    return y


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("W", [200, 4096, 32768])
def test_interior_node_of_high_in_degree(P, precision, W):
    # a hub of W in-edges: up to kHubEdges (1024) summed edge after edge by one wave, above it in chunks
    # of 256 (chunk sums computed by a launch of their own on the streamed plan, by the wave itself in
    # the serving runtime); the result must meet the bar, and every plan must give the same bits
    rng = np.random.default_rng(W)
    g = _hub_graph(W, 64, rng)
    x = rng.uniform(-1, 1, (3, 300))
    V, Q = oracle_ref(g, x)
    G = graph(P, g)
    say(f"hub in-degree {W} {precision}")
    ys = gpu_eval(G.set_path("streamed"), x, precision)
    assert_parity(ys, V, Q, precision, f"hub W={W}")
    code = {"fp64": 0, "fp32r": 1, "fp32": 2}[precision]
    if (G.info()["fused_mask"] >> code) & 1:
        yf = gpu_eval(G.set_path("fused"), x, precision)
        assert np.array_equal(yf.view(np.uint64), ys.view(np.uint64))
    else:
        assert W > 1000
    if precision != "fp32":  # the serving runtime takes FP64 and FP32-rescaled requests
        yv = _serve_one(P, G.set_path("auto"), x, precision)
        assert np.array_equal(yv.view(np.uint64), ys.view(np.uint64))


@pytest.mark.parametrize("precision", PRECISIONS)
def test_hub_of_parallel_edges_same_bits_on_every_plan(P, precision):
    # a hub of 256 * 8 = 2048 in-edges (parallel edges) in a graph narrow enough for the whole-graph
    # plan: chunked sums on the streamed plan (separate launch), the fused plan and the serving runtime
    # (each wave by itself) give identical bits, within the bar of the oracle
    rng = np.random.default_rng(11)
    g = _parallel_hub_graph(256, 8, 48, rng)
    x = rng.uniform(-1, 1, (3, 700))
    V, Q = oracle_ref(g, x)
    G = graph(P, g)
    say(f"parallel-edge hub {precision}")
    ys = gpu_eval(G.set_path("streamed"), x, precision)
    assert_parity(ys, V, Q, precision, "parallel hub")
    yf = gpu_eval(G.set_path("fused"), x, precision)
    assert np.array_equal(yf.view(np.uint64), ys.view(np.uint64))
    if precision != "fp32":
        for path in ("fused", "streamed"):
            yv = _serve_one(P, G.set_path(path), x, precision)
            assert np.array_equal(yv.view(np.uint64), ys.view(np.uint64)), path


def _level_ms(P, G, xd, precision, reps=5):
    ws = torch.empty(G.workspace_bytes(xd.shape[1], precision), dtype=torch.uint8, device=xd.device)
    for _ in range(2):
        G.evaluate(xd, precision, workspace=ws)
    torch.cuda.synchronize()
    for k in ("level", "hub"):
        P.timing_read(k)
    P.timing_enable(True)
    for _ in range(reps):
        G.evaluate(xd, precision, workspace=ws)
    torch.cuda.synchronize()
    P.timing_enable(False)
    return sum(P.timing_read(k)[0] for k in ("level", "hub")) / reps


@pytest.mark.parametrize("precision", ["fp64", "fp32r"])
def test_hub_of_32768_in_edges_runs_near_the_spread_graph(P, precision):
    # the same 32768 in-edges into one node, or spread over 4096 nodes of in-degree 8: the interior
    # launches of the hub graph (chunk sums + levels) must take at most 1.5x those of the spread graph
    rng = np.random.default_rng(5)
    W = 32768
    hub = _hub_graph(W, W, rng)
    first = np.concatenate([[0], np.cumsum([1, W, 4096, W, 1])])
    src = np.concatenate([np.zeros(W, int), first[1] + np.arange(W), first[2] + np.arange(W) % 4096,
                          first[3] + np.arange(W)])
    dst = np.concatenate([first[1] + np.arange(W), first[2] + np.arange(W) // 8, first[3] + np.arange(W),
                          np.full(W, first[4])])
    E = len(src)
    spread = LeveledGraph(np.array([1, W, 4096, W, 1]), np.array([W, W, W, W]), src.astype(np.int32),
                          dst.astype(np.int32), rng.uniform(-1, 1, E), rng.uniform(0.5, 2, E),
                          rng.uniform(-1, 1, (E, 3)))
    x = rng.uniform(-1, 1, (3, 4096))
    xd = to_dev(x)
    t_hub = _level_ms(P, graph(P, hub).set_path("streamed"), xd, precision)
    t_spread = _level_ms(P, graph(P, spread).set_path("streamed"), xd, precision)
    say(f"hub 32768 {precision}: {t_hub:.3f} ms vs spread {t_spread:.3f} ms (ratio {t_hub / t_spread:.2f})")
    assert t_hub <= 1.5 * t_spread


def test_transpose_agrees(P):
    g, x = make_config("mid", S=256, seed=9)
    y = gpu_eval(graph(P, g), x, "fp64")
    yt = gpu_eval(graph(P, transpose(g)), x, "fp64")
    V, Q = oracle_ref(g, x)
    assert_parity(y, V, Q, "fp64", "G")
    assert_parity(yt, V, Q, "fp64", "G^T")


def test_zero_samples_queue_nothing(P):
    g, _ = make_config("tiny", S=1)
    G = graph(P, g)
    xd = torch.empty((3, 0), dtype=torch.float64, device="cuda:0")
    out = G.evaluate(xd, "fp64")
    assert out.numel() == 0


def test_workspace_checks(P):
    g, x = make_config("tiny", S=100)
    G = graph(P, g)
    xd = to_dev(x)
    G.set_path("streamed")
    need = G.workspace_bytes(100, "fp64")
    ws = torch.empty(need + 512, dtype=torch.uint8, device=xd.device)
    with pytest.raises(P.CosError):
        G.evaluate(xd, "fp64", workspace=ws[: need - 8])  # not even one 256-sample sweep fits
    with pytest.raises(P.CosError):
        G.evaluate(xd, "fp64", workspace=ws[8:])  # misaligned
    y = G.evaluate(xd, "fp64", workspace=ws)
    torch.cuda.synchronize()
    V, Q = oracle_ref(g, x)
    assert_parity(y.cpu().numpy(), V, Q, "fp64", "workspace")


@pytest.mark.parametrize("precision", PRECISIONS)
def test_small_workspace_sweeps_in_chunks_bit_identical(P, precision):
    # a workspace sized for 1000 samples evaluates 4100 samples in 5 sweeps (ragged last one)
    g, x = make_config("mid", S=4100, width=96, L=7)
    G = graph(P, g).set_path("streamed")
    xd = to_dev(x)
    full = G.evaluate(xd, precision)
    small = torch.empty(G.workspace_bytes(1000, precision), dtype=torch.uint8, device=xd.device)
    assert small.numel() < G.workspace_bytes(4100, precision)
    chunked = G.evaluate(xd, precision, workspace=small)
    torch.cuda.synchronize()
    assert np.array_equal(full.cpu().numpy(), chunked.cpu().numpy())
    V, Q = oracle_ref(g, x)
    assert_parity(chunked.cpu().numpy(), V, Q, precision, "chunked")


def test_side_stream(P):
    g, x = make_config("mid", S=2048, width=64)
    G = graph(P, g)
    xd = to_dev(x)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        y = G.evaluate(xd, "fp64", stream=s)
    s.synchronize()
    V, Q = oracle_ref(g, x)
    assert_parity(y.cpu().numpy(), V, Q, "fp64", "side stream")


def test_side_stream_outside_its_context(P):
    """evaluate(stream=s) while the current stream is another one: s waits for the samples written on the
    current stream, and the temporary workspace and output stay reserved until s has finished (memory
    allocated and overwritten on the current stream right after the call must not land in them)."""
    g, x = make_config("precision", S=2048)
    G = graph(P, g)
    V, Q = oracle_ref(g, x)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    say("side stream outside its context: precision fp32r S=2048")
    for precision in ("fp64", "fp32r"):
        xd = torch.zeros((3, x.shape[1]), dtype=torch.float64, device="cuda:0")
        xd.copy_(torch.from_numpy(x).to("cuda:0"))  # written on the current stream
        y = G.evaluate(xd, precision, stream=s)
        del xd
        scribble = [torch.full((G.workspace_bytes(x.shape[1], precision) // 8 + 1,), float("nan"),
                               dtype=torch.float64, device="cuda:0") for _ in range(2)]
        s.synchronize()
        torch.cuda.synchronize()
        assert_parity(y.cpu().numpy(), V, Q, precision, "side stream, outside its context")
        del scribble


def test_walkers_on_side_stream(P):
    """Walkers created on the current stream and run on another: the side stream waits for the state the
    constructor wrote, and the same chain results as on the current stream (bit for bit)."""
    g, x = make_config("tiny", S=512)
    G = graph(P, g)
    ref = P.Walkers(G, to_dev(x), "fp64", seed=3, sigma=0.7).run(20)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    W = P.Walkers(G, to_dev(x), "fp64", seed=3, sigma=0.7, stream=s).run(20)
    s.synchronize()
    for a, b in ((W.x, ref.x), (W.v, ref.v), (W.accepted, ref.accepted), (W.acc, ref.acc)):
        assert torch.equal(a, b)


def test_binary32_range_guard(P):
    """A parameter that is finite in binary64 but rounds to infinity in binary32: FP64 evaluates it (parity
    with the oracle); every binary32 precision is refused with a message, by cos_evaluate, by the server
    and by the Monte Carlo walkers."""
    g, x = make_config("tiny")
    g = g.copy()
    g.a[3] = 1e39
    G = graph(P, g)
    V, Q = oracle_ref(g, x)
    assert_parity(gpu_eval(G, x, "fp64"), V, Q, "fp64", "a beyond binary32")
    xd = to_dev(x)
    for p in ("fp32r", "fp32", "fp16r", "bf16r"):
        with pytest.raises(P.CosError, match="binary32 range"):
            G.evaluate(xd, p)
    srv = P.Server(1 << 26, 4)
    try:
        gid = srv.add_graph(G)
        with pytest.raises(P.CosError, match="binary32 range"):
            srv.submit(gid, xd, "fp32r")
    finally:
        srv.close()
    with pytest.raises(P.CosError, match="binary32 range"):
        P.Walkers(G, xd, "fp32r")


def test_timing_probe_counts_launches(P):
    g, x = make_config("mid", S=1024)
    G = graph(P, g)
    xd = to_dev(x)
    for kind in ("level", "final_partial", "final_combine", "fill", "fused"):
        P.timing_read(kind)
    P.timing_enable(True)
    try:
        G.set_path("streamed").evaluate(xd, "fp64")
        torch.cuda.synchronize()
        ms_l, n_l = P.timing_read("level")
        ms_p, n_p = P.timing_read("final_partial")
        G.set_path("fused").evaluate(xd, "fp64")
        torch.cuda.synchronize()
        ms_f, n_f = P.timing_read("fused")
    finally:
        P.timing_enable(False)
    assert n_l == g.L - 1 and ms_l > 0
    assert n_p == 1 and ms_p > 0
    assert n_f == 1 and ms_f > 0


@pytest.mark.parametrize("name,precision,factor", [("mid", "fp64", "rational"), ("mid", "fp32r", "rational"),
                                                   ("precision", "fp16r", "rational"),
                                                   ("precision", "fp32r", "rational"),
                                                   ("mid", "fp32r", "lookup"), ("precision", "bf16r", "lookup")])
def test_evaluate_captured_in_a_graph_replays_bit_identical(P, name, precision, factor):
    # cos_evaluate with a caller workspace issues kernels only (no allocation, no memset), so it
    # can be captured in a HIP graph; every replay, with new samples written in between, must
    # give the eager result's bits (the lookup cases include the binary32 table copy, on the
    # fused and on the streamed plan)
    g, x = make_config(name, S=2048, factor=factor)
    G = graph(P, g)
    rng = np.random.default_rng(5)
    xs = [x] + [x + rng.normal(0, 0.05, x.shape) for _ in range(3)]
    eager = [gpu_eval(G, xi, precision) for xi in xs]
    xd = to_dev(xs[0])
    out = torch.empty(x.shape[1], dtype=torch.float64, device="cuda:0")
    ws = torch.empty(G.workspace_bytes(x.shape[1], precision), dtype=torch.uint8, device="cuda:0")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        G.evaluate(xd, precision, out=out, workspace=ws, stream=s)  # warm-up outside the capture
    s.synchronize()
    graph_ = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph_, stream=s):
        G.evaluate(xd, precision, out=out, workspace=ws, stream=s)
    for i in (1, 2, 0, 3):
        xd.copy_(to_dev(xs[i]))
        torch.cuda.synchronize()
        graph_.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager[i]), f"replay with samples {i}"
        gpu_eval(G, xs[(i + 1) % 4], precision)  # eager work between replays


@pytest.mark.parametrize("precision", ["fp32r", "fp32"])
@pytest.mark.parametrize("S", [300, 1000])
def test_panel_plan_bit_identical_to_streamed(P, precision, S):
    # wide levels (8192 nodes): row panels with their records in LDS over 32-sample tiles, level values
    # tile-major; the same arithmetic and order as the row-streamed kernel, so the same bits
    g, x = make_config("precision", S=S, width=8192, L=5, degree=6, seed=21)
    G = graph(P, g)
    say(f"panel vs streamed {precision} S={S}")
    yp = gpu_eval(G.set_path("panel"), x, precision)
    ys = gpu_eval(G.set_path("streamed"), x, precision)
    assert np.array_equal(yp.view(np.uint64), ys.view(np.uint64))
    idx = sample_subset(S, 96, seed=2)
    V, Q = oracle_ref(g, x, idx)
    assert_parity(yp[idx], V, Q, precision, "panel")


@pytest.mark.parametrize("precision", ["fp16r", "bf16r"])
@pytest.mark.parametrize("S", [1, 300, 1000])
def test_panel_plan_16bit_bit_identical_to_streamed(P, precision, S):
    # 16-bit storage: 64-sample tiles (one 128-byte line per node), 16 lanes per row and 8-byte gathers;
    # the graph with a scaled by 2^16 makes binary16 shift every level after the first by its headroom
    # (h_next > 0 in the maxima the kernel folds)
    g, x = make_config("precision", S=S, width=8192, L=5, degree=6, seed=22)
    for gg in (g, g.with_params(a=g.a * 2.0 ** 16)):
        G = graph(P, gg)
        assert (G.info()["panel_mask"] >> P.PRECISIONS[precision]) & 1
        say(f"panel vs streamed {precision} S={S}")
        yp = gpu_eval(G.set_path("panel"), x, precision)
        ys = gpu_eval(G.set_path("streamed"), x, precision)
        assert np.all(np.isfinite(yp))
        assert np.array_equal(yp.view(np.uint64), ys.view(np.uint64))


@pytest.mark.parametrize("precision", ["fp32r", "fp32"])
@pytest.mark.parametrize("S", [70, 1000])
def test_panel_plan_lookup_factors_bit_identical_to_streamed(P, precision, S):
    # lookup factors (w = coef32 * T_s[slot] from the binary32 tables, tile-major on the panel plan): the
    # streamed plan's bits; binary32 storage only (16-bit storage of lookup graphs stays streamed)
    g, T = make_config("precision", S=S, width=8192, L=5, degree=6, seed=23, factor="lookup")
    G = graph(P, g)
    mask = G.info()["panel_mask"]
    assert (mask >> P.PRECISIONS[precision]) & 1 and not (mask >> P.PRECISIONS["bf16r"]) & 1
    say(f"lookup panel vs streamed {precision} S={S}")
    yp = gpu_eval(G.set_path("panel"), T, precision)
    ys = gpu_eval(G.set_path("streamed"), T, precision)
    assert np.array_equal(yp.view(np.uint64), ys.view(np.uint64))
    small = torch.empty(G.workspace_bytes(256, precision), dtype=torch.uint8, device="cuda:0")
    yc = gpu_eval(G.set_path("panel"), T, precision, workspace=small)  # sweeps of 256 samples
    assert np.array_equal(yc.view(np.uint64), ys.view(np.uint64))
    idx = sample_subset(S, 48, seed=3)
    V, Q = oracle_ref(g, T, idx)
    assert_parity(yp[idx], V, Q, precision, "lookup panel")


def test_panel_plan_uneven_rows_and_chunked_sweeps(P):
    # irregular in-degrees (1..13), rows without in-edges, a ragged sample count and a workspace that
    # forces sweeps of 512 samples: the panel plan keeps the streamed plan's bits
    rng = np.random.default_rng(8)
    W, L = 5000, 4
    g = layered_graph([1] + [W] * (L - 1) + [1], rng.integers(1, 14, L), rng)
    from workloads import draw_params
    draw_params(g, rng)
    keep = np.ones(g.n_edges, bool)
    l2, l3 = g.level_slices()[1], g.level_slices()[2]
    keep[l2.start:l2.stop] = rng.random(l2.stop - l2.start) > 0.3  # uneven in-degrees in level 2
    keep[l3.start:l3.stop] = g.dst[l3] % 97 != 5  # some rows of level 3 lose every in-edge
    g2 = LeveledGraph(g.widths, np.array([int(keep[s].sum()) for s in g.level_slices()]), g.src[keep],
                      g.dst[keep], g.a[keep], g.b[keep], g.k[keep])
    x = rng.uniform(-1, 1, (3, 1500))
    G = graph(P, g2)
    for precision in ("fp32r", "fp16r", "bf16r"):
        ys = gpu_eval(G.set_path("streamed"), x, precision)
        yp = gpu_eval(G.set_path("panel"), x, precision)
        assert np.array_equal(yp.view(np.uint64), ys.view(np.uint64)), precision
        small = torch.empty(G.workspace_bytes(512, precision), dtype=torch.uint8, device="cuda:0")
        yc = gpu_eval(G, x, precision, workspace=small)
        assert np.array_equal(yc.view(np.uint64), ys.view(np.uint64)), precision
        if precision == "fp32r":
            V, Q = oracle_ref(g2, x, sample_subset(1500, 64))
            assert_parity(yp[sample_subset(1500, 64)], V, Q, "fp32r", "panel uneven")


def test_panel_plan_refused_where_it_does_not_apply(P):
    g, x = make_config("precision", S=64, width=8192, L=4, seed=3)
    G = graph(P, g).set_path("panel")
    with pytest.raises(P.CosError) as ei:
        gpu_eval(G, x, "fp64")  # binary64 keeps the row-streamed kernel
    assert ei.value.status == -1 and "panel" in str(ei.value)
    gn, xn = make_config("mid", S=64)
    Gn = graph(P, gn).set_path("panel")
    with pytest.raises(P.CosError):
        gpu_eval(Gn, xn, "fp32r")  # narrow graph: no panel plan


@pytest.mark.slow
def test_large_panel_plan_bit_identical_to_streamed(P):
    g, x = make_config("large")
    G = graph(P, g)
    for precision in ("fp32r", "fp16r", "bf16r"):
        say(f"large panel vs streamed {precision}")
        yp = gpu_eval(G.set_path("panel"), x, precision)
        ys = gpu_eval(G.set_path("streamed"), x, precision)
        assert np.array_equal(yp.view(np.uint64), ys.view(np.uint64)), precision


@pytest.mark.parametrize("precision", ["fp32r", "fp32", "fp16r", "bf16r"])
@pytest.mark.parametrize("S", [1, 70, 257])
def test_panel_plan_mixed_widths_and_small_S(P, precision, S):
    # a wide graph whose other levels are narrow (100 and 3 nodes) and sample counts below one tile
    # quarter: every level runs on the panel plan, with the streamed plan's bits
    rng = np.random.default_rng(S)
    from workloads import draw_params
    g = layered_graph([1, 5000, 100, 7000, 3, 1], [1, 5, 4, 9, 3], rng, cover=False)
    draw_params(g, rng)
    x = rng.uniform(-1, 1, (3, S))
    G = graph(P, g)
    assert (G.info()["panel_mask"] >> P.PRECISIONS[precision]) & 1
    yp = gpu_eval(G.set_path("panel"), x, precision)
    ys = gpu_eval(G.set_path("streamed"), x, precision)
    assert np.array_equal(yp.view(np.uint64), ys.view(np.uint64))
    if precision in ("fp32r", "fp32"):  # 16-bit storage: its per-sample bound is checked on the streamed plan
        V, Q = oracle_ref(g, x)
        assert_parity(yp, V, Q, precision, f"panel mixed S={S}")


def test_panel_plan_captured_in_a_graph_replays_bit_identical(P):
    # the panel plan queues kernel launches only (and fill kernels), so it can be captured and replayed
    g, x = make_config("precision", S=2048, width=8192, L=5, degree=6, seed=4)
    G = graph(P, g).set_path("panel")
    rng = np.random.default_rng(6)
    xs = [x] + [x + rng.normal(0, 0.05, x.shape) for _ in range(2)]
    eager = [gpu_eval(G, xi, "fp32r") for xi in xs]
    xd = to_dev(xs[0])
    out = torch.empty(x.shape[1], dtype=torch.float64, device="cuda:0")
    ws = torch.empty(G.workspace_bytes(x.shape[1], "fp32r"), dtype=torch.uint8, device="cuda:0")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        G.evaluate(xd, "fp32r", out=out, workspace=ws, stream=s)
    s.synchronize()
    graph_ = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph_, stream=s):
        G.evaluate(xd, "fp32r", out=out, workspace=ws, stream=s)
    for i in (1, 2, 0):
        xd.copy_(to_dev(xs[i]))
        torch.cuda.synchronize()
        graph_.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager[i]), f"replay with samples {i}"
        gpu_eval(G, xs[(i + 1) % 3], "fp32r")
