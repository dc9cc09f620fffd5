"""Shared helpers of the GPU tests: run the library, run the oracle, compare."""

from __future__ import annotations

import sys

import numpy as np
import torch

import oracle

# per-sample tolerance on |y - r| / max(|r|, sqrt(Q)) against the FP64 oracle
TOL = {"fp64": 1e-12, "fp32r": 1e-5, "fp32": 1e-5}
PRECISIONS = ("fp64", "fp32r", "fp32")


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def dev():
    return torch.device("cuda:0")


def to_dev(x: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(dev())


def gpu_eval(G, x: np.ndarray, precision: str, **kw) -> np.ndarray:
    xd = to_dev(x)
    out = G.evaluate(xd, precision, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def oracle_ref(g, x: np.ndarray, idx=None):
    """(V, Q) from the oracle, optionally on a subset of samples (samples are independent)."""
    xs = x if idx is None else np.ascontiguousarray(x[:, idx])
    return oracle.sweep(g, xs, "value"), oracle.sweep(g, xs, "square")


def assert_parity(y, V, Q, precision: str, label: str = ""):
    err = oracle.scaled_error(y, V, Q)
    tol = TOL[precision]
    bad = np.flatnonzero(~(err <= tol))
    assert bad.size == 0, (f"{label} {precision}: {bad.size} samples above {tol}; worst {err.max():.3e} at "
                           f"{int(np.argmax(err))} (y={y[bad[0]]!r}, ref={V[bad[0]]!r})")
    return float(err.max())


def sample_subset(S: int, n: int, seed: int = 0) -> np.ndarray:
    """Seeded subset of n sample indices, always including the first and last (ragged tail)."""
    if n >= S:
        return np.arange(S)
    rng = np.random.default_rng(seed)
    idx = rng.choice(S, n - 2, replace=False)
    return np.unique(np.concatenate([[0, S - 1], idx]))
