"""Python face of the Monte Carlo walkers (cos_mc_run in include/cos.h).

Argument marshalling only: proposals, the level sweep of the proposals and the
Metropolis decisions run in the library's kernels.  The walkers' state and
sums live in device tensors owned by this object.
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import LIB, PRECISIONS, check
from .graph import Graph


class Walkers:
    """C Metropolis walkers for the density |V(x)| on a graph with rational factors.

    x0: float64[3, C] starting points on the device.  Their values V(x0) are
    computed at construction (cos_evaluate).  run(n) advances every walker n
    steps; the per-walker sums (sign V, |x|^2, accepted proposals) accumulate
    until reset_sums().
    """

    def __init__(self, graph: Graph, x0: torch.Tensor, precision: str = "fp64", seed: int = 0, sigma: float = 1.0,
                 stream: torch.cuda.Stream | None = None):
        if not (isinstance(x0, torch.Tensor) and x0.is_cuda and x0.dtype == torch.float64 and x0.dim() == 2
                and x0.shape[0] == 3 and x0.shape[1] >= 1):
            raise ValueError("x0 must be a float64 CUDA tensor of shape [3, C]")
        self.graph, self.precision, self.seed, self.sigma = graph, precision, int(seed), float(sigma)
        self.C = int(x0.shape[1])
        self.stream = stream if stream is not None else torch.cuda.current_stream(x0.device)
        dev = x0.device
        self.x = x0.contiguous().clone()
        self.v = torch.empty(self.C, dtype=torch.float64, device=dev)
        self.accepted = torch.zeros(self.C, dtype=torch.int64, device=dev)
        self.acc = torch.zeros(2, self.C, dtype=torch.float64, device=dev)
        nb = ctypes.c_uint64()
        check(LIB.cos_mc_workspace_size(graph.handle, self.C, PRECISIONS[precision], ctypes.byref(nb)),
              "cos_mc_workspace_size")
        self.workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=dev)
        self._adopt(torch.cuda.current_stream(dev))
        with torch.cuda.stream(self.stream):
            graph.evaluate(self.x, precision, out=self.v, stream=self.stream)
        self.step = 0          # global step index of the next step
        self.steps_summed = 0  # steps in the current sums

    def _adopt(self, made_on: torch.cuda.Stream) -> None:
        """The state tensors were allocated and written on `made_on`; when the walkers run on another
        stream, that stream waits for those writes and the tensors are marked as in use on it (the
        caching allocator then keeps their memory until the walkers' own work is done)."""
        if self.stream.cuda_stream != made_on.cuda_stream:
            self.stream.wait_stream(made_on)
            for t in (self.x, self.v, self.accepted, self.acc, self.workspace):
                t.record_stream(self.stream)

    def save(self, path) -> None:
        """Checkpoint the walkers (positions, values, sums, step index, seed, sigma) to a .npz file.
        Random numbers depend on (seed, walker, step) only, so Walkers.load(...).run(n) continues
        with exactly the bits an uninterrupted run would produce."""
        self.stream.synchronize()
        np.savez(path, x=self.x.cpu().numpy(), v=self.v.cpu().numpy(), accepted=self.accepted.cpu().numpy(),
                 acc=self.acc.cpu().numpy(), step=np.int64(self.step), steps_summed=np.int64(self.steps_summed),
                 seed=np.uint64(self.seed), sigma=np.float64(self.sigma), precision=np.str_(self.precision))

    @classmethod
    def load(cls, graph: Graph, path, stream: torch.cuda.Stream | None = None) -> "Walkers":
        """Walkers restored from save() on the same graph (plain arrays only: nothing in the file is executed)."""
        with np.load(path, allow_pickle=False) as z:
            st = {k: z[k] for k in z.files}
        dev = torch.device("cuda", torch.cuda.current_device())
        w = cls.__new__(cls)
        w.graph, w.precision, w.seed, w.sigma = graph, str(st["precision"]), int(st["seed"]), float(st["sigma"])
        w.x = torch.from_numpy(np.ascontiguousarray(st["x"])).to(dev)
        w.C = int(w.x.shape[1])
        w.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        w.v = torch.from_numpy(np.ascontiguousarray(st["v"])).to(dev)
        w.accepted = torch.from_numpy(np.ascontiguousarray(st["accepted"])).to(dev)
        w.acc = torch.from_numpy(np.ascontiguousarray(st["acc"])).to(dev)
        nb = ctypes.c_uint64()
        check(LIB.cos_mc_workspace_size(graph.handle, w.C, PRECISIONS[w.precision], ctypes.byref(nb)),
              "cos_mc_workspace_size")
        w.workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=dev)
        w.step, w.steps_summed = int(st["step"]), int(st["steps_summed"])
        w._adopt(torch.cuda.current_stream(dev))
        return w

    def run(self, n_steps: int) -> "Walkers":
        check(LIB.cos_mc_run(self.graph.handle, PRECISIONS[self.precision], self.C, self.x.data_ptr(),
                             self.v.data_ptr(), self.step, int(n_steps), self.seed, self.sigma,
                             self.accepted.data_ptr(), self.acc.data_ptr(), self.workspace.data_ptr(),
                             self.workspace.numel(), self.stream.cuda_stream), "cos_mc_run")
        self.step += int(n_steps)
        self.steps_summed += int(n_steps)
        return self

    def reset_sums(self) -> "Walkers":
        with torch.cuda.stream(self.stream):
            self.accepted.zero_()
            self.acc.zero_()
        self.steps_summed = 0
        return self

    def estimates(self) -> dict:
        """<sign V> and <|x|^2> over walkers and summed steps, with standard errors
        from the spread of the (independent) walkers' own averages."""
        self.stream.synchronize()
        n = max(self.steps_summed, 1)
        per = self.acc.cpu().numpy() / n
        se = per.std(axis=1) / np.sqrt(self.C) if self.C > 1 else np.full(2, np.nan)
        return {"sign": float(per[0].mean()), "sign_se": float(se[0]), "x2": float(per[1].mean()),
                "x2_se": float(se[1]), "acceptance": float(self.accepted.cpu().numpy().mean() / n),
                "steps": self.steps_summed, "walkers": self.C}
