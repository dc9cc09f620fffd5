"""Lookup edge factors on the GPU (w_e = c_e * T_s[slot_e]) against the oracle.

Same bars as the rational factors: per-sample |y - r| / max(|r|, sqrt(Q)) <= 1e-12
(FP64) and <= 1e-5 (binary32 paths) against the FP64 oracle; exact results where
the inputs make them exact (path counts, sign flips); both plans bit-identical.
"""

import numpy as np
import pytest
import torch

import oracle
import pins
from gpu_util import PRECISIONS, assert_parity, gpu_eval, oracle_ref, sample_subset, say, to_dev
from workloads import LeveledGraph, make_config, transpose

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2501_00675_amd as P

    assert torch.cuda.is_available()
    return P


def graph(P, g):
    return P.Graph.from_leveled(g)


def bits(y):
    return np.asarray(y, np.float64).view(np.uint64)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_tiny_parity(P, precision):
    g, T = make_config("tiny", factor="lookup")
    say(f"lookup tiny {precision}")
    G = graph(P, g)
    assert G.info()["kind"] == "lookup" and G.n_inputs == g.n_slots
    y = gpu_eval(G, T, precision)
    V, Q = oracle_ref(g, T)
    assert_parity(y, V, Q, precision, "lookup tiny")


@pytest.mark.parametrize("S", [1, 63, 65, 257, 1000])
@pytest.mark.parametrize("precision", ["fp64", "fp32r"])
@pytest.mark.parametrize("path", ["fused", "streamed"])
def test_ragged_sample_counts(P, S, precision, path):
    g, T = make_config("mid", S=S, width=40, L=6, factor="lookup")
    say(f"lookup ragged {precision} {path} S={S}")
    y = gpu_eval(graph(P, g).set_path(path), T, precision)
    V, Q = oracle_ref(g, T)
    assert_parity(y, V, Q, precision, f"lookup ragged S={S}")


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("name,S,over", [("tiny", 1024, {}), ("mid", 2000, {}),
                                         ("mid", 777, dict(width=300, L=5, degree=7))])
def test_fused_and_streamed_bit_identical(P, precision, name, S, over):
    g, T = make_config(name, S=S, factor="lookup", **over)
    G = graph(P, g)
    code = {"fp64": 0, "fp32r": 1, "fp32": 2}[precision]
    if not (G.info()["fused_mask"] >> code) & 1:
        pytest.skip("graph does not fit the fused plan at this precision")
    say(f"lookup fused vs streamed {name} {precision} S={S} {over}")
    yf = gpu_eval(G.set_path("fused"), T, precision)
    ys = gpu_eval(G.set_path("streamed"), T, precision)
    assert np.array_equal(bits(yf), bits(ys))
    V, Q = oracle_ref(g, T)
    assert_parity(yf, V, Q, precision, f"lookup {name}")


@pytest.mark.parametrize("precision", PRECISIONS)
def test_mid_full_size_sampled(P, precision):
    g, T = make_config("mid", factor="lookup")
    say(f"lookup mid full size {precision}")
    y = gpu_eval(graph(P, g), T, precision)
    idx = sample_subset(T.shape[1], 512, seed=3)
    V, Q = oracle_ref(g, T, idx)
    assert_parity(y[idx], V, Q, precision, "lookup mid")


@pytest.mark.parametrize("precision", PRECISIONS)
def test_precision_full_size_sampled(P, precision):
    g, T = make_config("precision", factor="lookup")
    say(f"lookup precision full size {precision}")
    y = gpu_eval(graph(P, g), T, precision)
    idx = sample_subset(T.shape[1], 128, seed=4)
    V, Q = oracle_ref(g, T, idx)
    assert_parity(y[idx], V, Q, precision, "lookup precision")


@pytest.mark.slow
@pytest.mark.parametrize("precision", ["fp64", "fp32r"])
def test_large_full_size_sampled(P, precision):
    g, T = make_config("large", factor="lookup")
    say(f"lookup large full size {precision}")
    y = gpu_eval(graph(P, g), T, precision)
    idx = sample_subset(T.shape[1], 16, seed=5)
    V, Q = oracle_ref(g, T, idx)
    assert_parity(y[idx], V, Q, precision, "lookup large")


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("name,count", [("tiny", 12), ("mid", 4 ** 10 * 256), ("precision", 8 ** 22 * 4096)])
def test_all_ones_path_counts_exact(P, name, count, precision):
    g, _ = make_config(name, S=300)
    g1 = g.with_lookup(1, 1.0, 2)
    T = np.stack([np.full(300, 7.0), np.ones(300)])  # only entry 1 is read
    y = gpu_eval(graph(P, g1), T, precision)
    assert np.all(y == float(count)), (name, precision, y[:4])


@pytest.mark.parametrize("precision", PRECISIONS)
def test_level_constant_closed_form(P, precision):
    rng = np.random.default_rng(61)
    g, _ = make_config("mid", S=512)
    d = pins.in_degrees(g)
    sl = rng.integers(0, 5, g.L)
    cl = rng.uniform(-2, 2, g.L)
    lev = np.repeat(np.arange(g.L), g.epl)
    gl = g.with_lookup(sl[lev], cl[lev], 5)
    T = rng.uniform(-1, 1, (5, 512))
    y = gpu_eval(graph(P, gl), T, precision)
    cf = np.ones(512)
    for l in range(g.L):
        cf = cf * (d[l] * cl[l] * T[sl[l]])
    V, Q = oracle_ref(gl, T)
    assert_parity(y, V, Q, precision, "lookup level-constant")
    tol = {"fp64": 1e-12, "fp32r": 1e-5, "fp32": 1e-5}[precision]
    assert np.max(np.abs(y - cf) / np.abs(cf)) <= tol


@pytest.mark.parametrize("precision", ["fp64", "fp32r"])
def test_level_sign_flip_is_exact(P, precision):
    g, T = make_config("mid", S=700, width=64, L=8, factor="lookup")
    G = graph(P, g)
    y = gpu_eval(G, T, precision)
    lev = np.repeat(np.arange(g.L), g.epl)
    c = g.coef.copy()
    c[lev == 3] *= -1.0
    yf = gpu_eval(graph(P, g.with_lookup(g.slot, c, g.n_slots)), T, precision)
    assert np.array_equal(yf, -y)


def test_export_is_canonical_and_permutation_invariant(P):
    g, T = make_config("mid", S=300, width=48, L=6, factor="lookup")
    rng = np.random.default_rng(9)
    perm = np.concatenate([s.start + rng.permutation(s.stop - s.start) for s in g.level_slices()])
    gp = LeveledGraph(g.widths, g.epl, g.src[perm], g.dst[perm], g.a[perm], g.b[perm], g.k[perm],
                      slot=g.slot[perm], coef=g.coef[perm], n_slots=g.n_slots)
    G, Gp = graph(P, g), graph(P, gp)
    ex, exp_ = G.export(), Gp.export()
    for key in ("src", "dst", "slot", "coef"):
        assert np.array_equal(ex[key], exp_[key]), key
    order = np.lexsort((g.coef.view(np.uint64), g.slot, g.src, g.dst))
    assert np.array_equal(ex["dst"], g.dst[order]) and np.array_equal(ex["slot"], g.slot[order])
    for precision in ("fp64", "fp32r"):
        assert np.array_equal(bits(gpu_eval(G, T, precision)), bits(gpu_eval(Gp, T, precision)))


@pytest.mark.parametrize("precision", PRECISIONS)
def test_single_level_parallel_edges(P, precision):
    g = LeveledGraph(np.array([1, 1]), np.array([3]), np.zeros(3, np.int32), np.ones(3, np.int32),
                     np.zeros(3), np.zeros(3), np.zeros((3, 3)), slot=np.array([0, 2, 0], np.int32),
                     coef=np.array([1.0, -1.0, 0.5]), n_slots=3)
    T = np.random.default_rng(2).uniform(-1, 1, (3, 70))
    V, Q = oracle_ref(g, T)
    assert_parity(gpu_eval(graph(P, g), T, precision), V, Q, precision, "lookup L=1")


def test_transpose_agrees(P):
    g, T = make_config("mid", S=256, width=64, L=7, factor="lookup")
    y = gpu_eval(graph(P, g), T, "fp64")
    yt = gpu_eval(graph(P, transpose(g)), T, "fp64")
    V, Q = oracle_ref(g, T)
    assert oracle.scaled_error(yt, y, Q).max() <= 1e-12


def test_wrong_input_rows_rejected(P):
    g, T = make_config("tiny", S=64, factor="lookup")
    G = graph(P, g)
    with pytest.raises(ValueError):
        G.evaluate(to_dev(np.zeros((3, 64))), "fp64")
    with P.Server(1 << 20, 2) as srv:
        gid = srv.add_graph(G)  # served since lookup graphs take the lookup sections of a step
        with pytest.raises(ValueError):
            srv.submit(gid, to_dev(np.zeros((3, 64))), "fp64")


def test_lookup_graph_file_round_trip_bit_identical(P, tmp_path):
    g, T = make_config("mid", S=512, factor="lookup")
    G = P.Graph.from_leveled(g)
    G.save(tmp_path / "g.npz")
    G2 = P.Graph.load(tmp_path / "g.npz")
    assert G2.info()["kind"] == "lookup" and G2.n_inputs == g.n_slots
    for precision in ("fp64", "fp32r"):
        assert np.array_equal(gpu_eval(G, T, precision), gpu_eval(G2, T, precision))


@pytest.mark.parametrize("path", ["fused", "streamed"])
def test_binary32_table_copy_workspace(P, path):
    # the binary32 paths of a lookup graph copy the tables into the workspace: its size covers
    # them on both plans, a fused-plan workspace without room for them is refused, and a small
    # streamed workspace sweeps in chunks with the same bits
    g, T = make_config("mid", S=3000, factor="lookup")
    G = graph(P, g).set_path(path)
    S, n = T.shape[1], T.shape[0]
    need32, need64 = G.workspace_bytes(S, "fp32r"), G.workspace_bytes(S, "fp64")
    assert need32 >= n * S * 4
    say(f"lookup table copy workspace {path}: {need32} bytes (FP64 {need64})")
    xd = to_dev(T)
    ref = gpu_eval(G, T, "fp32r")
    if path == "fused":
        small = torch.empty(256, dtype=torch.uint8, device="cuda:0")
        with pytest.raises(P.CosError):
            G.evaluate(xd, "fp32r", workspace=small)
    else:
        small = torch.empty(G.workspace_bytes(700, "fp32r"), dtype=torch.uint8, device="cuda:0")
        y = G.evaluate(xd, "fp32r", workspace=small)
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy().view(np.uint64), ref.view(np.uint64))
