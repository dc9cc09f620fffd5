"""cos_evaluate_no_alloc (the fixed-workspace entry point for callers that cannot allocate) against
cos_evaluate on the same inputs: results must be bit-identical, on two calls in a row, the second with
fewer samples; a graph whose plan does not fit the fixed workspace is refused with a message."""

import ctypes

import numpy as np
import pytest
import torch

from gpu_util import assert_parity, oracle_ref, say, to_dev
from workloads import draw_params, draw_samples, layered_graph, make_config

pytestmark = pytest.mark.gpu

SCRATCH = 64 << 20


@pytest.fixture(scope="module")
def P():
    import paper_2501_00675_amd as P

    assert torch.cuda.is_available()
    return P


def _bits(t):
    return t.cpu().numpy().view(np.int64)


def _both(P, G, x, precision):
    """(no-alloc result, allocating cos_evaluate result) on the same samples, each through the C ABI."""
    xd = to_dev(x)
    y0 = G.evaluate_no_alloc(xd, precision)
    y1 = G.evaluate(xd, precision)
    torch.cuda.synchronize()
    return y0, y1


@pytest.mark.parametrize("cfg,precision,S1,S2", [("tiny", "fp64", 1024, 300), ("mid", "fp64", 4096, 1000),
                                                  ("mid", "fp32r", 4096, 1000),
                                                  ("precision", "fp64", 4096, 700),
                                                  ("precision", "fp32r", 4096, 700)])
def test_no_alloc_matches_cos_evaluate_twice(P, cfg, precision, S1, S2):
    g, x = make_config(cfg, S=S1)
    G = P.Graph.from_leveled(g)
    ws = G.workspace_bytes(S1, precision)
    say(f"no_alloc {cfg} {precision} S={S1} then {S2} (workspace {ws} bytes, scratch {SCRATCH})")
    for S in (S1, S2):  # the second call: fewer samples, the scratch holds the first call's contents
        xs = np.ascontiguousarray(x[:, :S])
        y0, y1 = _both(P, G, xs, precision)
        assert np.array_equal(_bits(y0), _bits(y1)), f"{cfg} {precision} S={S}: bits differ"
        idx = np.unique(np.linspace(0, S - 1, 64).astype(int))
        V, Q = oracle_ref(g, xs, idx)
        assert_parity(y0.cpu().numpy()[idx], V, Q, precision, f"no_alloc {cfg}")
    G.close()


def test_no_alloc_sweeps_in_chunks_when_the_level_exceeds_the_scratch(P):
    # precision-shaped levels at S = 4096 in FP64: two level buffers of 128 MiB, so the fixed
    # workspace holds only a chunk of the samples per sweep
    g, x = make_config("precision", S=4096)
    G = P.Graph.from_leveled(g)
    assert G.workspace_bytes(4096, "fp64") > SCRATCH
    y0, y1 = _both(P, G, x, "fp64")
    assert np.array_equal(_bits(y0), _bits(y1))
    G.close()


def test_no_alloc_refuses_a_graph_too_wide_for_the_scratch(P):
    rng = np.random.default_rng(7)
    g = layered_graph([1, 40000, 1], 1, rng)
    draw_params(g, rng)
    G = P.Graph.from_leveled(g).set_path("streamed")
    x = draw_samples(300, "uniform", rng)
    with pytest.raises(P.CosError) as e:
        G.evaluate_no_alloc(to_dev(x), "fp64")
    assert e.value.status == -1 and "too small" in str(e.value) and "cos_evaluate_no_alloc" in str(e.value)
    # the allocating entry point evaluates the same graph
    y = G.evaluate(to_dev(x), "fp64")
    torch.cuda.synchronize()
    V, Q = oracle_ref(g, x)
    assert_parity(y.cpu().numpy(), V, Q, "fp64", "wide")
    G.close()
