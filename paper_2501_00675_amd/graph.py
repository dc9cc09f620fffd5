"""Python face of the C ABI: device-resident graphs and their evaluation.

Only argument marshalling happens here; every step of the evaluation runs in
the library's HIP kernels.  torch provides device memory and the stream.
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import FACTOR_KINDS, KINDS, LIB, PATHS, PRECISIONS, GraphInfo, check


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


class Graph:
    """A leveled DAG held on the current HIP device.

    Rational factors (cos_create_graph): pass a, b, k.  Lookup factors
    (cos_create_graph_lookup): pass slot, coef and n_slots instead.
    """

    def __init__(self, L, widths, edges_per_level, src, dst, a=None, b=None, k=None, *, slot=None, coef=None,
                 n_slots=None):
        keep = []

        def ptr(v, dt):
            arr, p = _c(v, dt)
            keep.append(arr)
            return p

        h = ctypes.c_void_p()
        if slot is not None:
            st = LIB.cos_create_graph_lookup(int(L), ptr(widths, np.int64), ptr(edges_per_level, np.int64),
                                             ptr(src, np.int32), ptr(dst, np.int32), ptr(slot, np.int32),
                                             ptr(coef, np.float64), int(n_slots), ctypes.byref(h))
            check(st, "cos_create_graph_lookup")
        else:
            st = LIB.cos_create_graph(int(L), ptr(widths, np.int64), ptr(edges_per_level, np.int64),
                                      ptr(src, np.int32), ptr(dst, np.int32), ptr(a, np.float64),
                                      ptr(b, np.float64), ptr(np.reshape(k, -1), np.float64), ctypes.byref(h))
            check(st, "cos_create_graph")
        self._h = h
        # host copy of the level sizes (for save)
        self._L = int(L)
        self._widths = np.array(widths, dtype=np.int64)
        self._epl = np.array(edges_per_level, dtype=np.int64)

    @classmethod
    def from_leveled(cls, g) -> "Graph":
        """From any object with L, widths, epl, src, dst and either a, b, k or slot, coef, n_slots
        (e.g. workloads.LeveledGraph)."""
        if getattr(g, "slot", None) is not None:
            return cls(g.L, g.widths, g.epl, g.src, g.dst, slot=g.slot, coef=g.coef, n_slots=g.n_slots)
        return cls(g.L, g.widths, g.epl, g.src, g.dst, g.a, g.b, g.k)

    @property
    def handle(self) -> int:
        if self._h is None:
            raise ValueError("graph was destroyed")
        return self._h.value

    def info(self) -> dict:
        gi = GraphInfo()
        check(LIB.cos_graph_get_info(self.handle, ctypes.byref(gi)), "cos_graph_get_info")
        d = {f: getattr(gi, f) for f, _ in GraphInfo._fields_}
        d["kind"] = FACTOR_KINDS[d["factor_kind"]]
        return d

    @property
    def n_inputs(self) -> int:
        """Rows of the per-sample input: 3 coordinates, or the table entries of a lookup graph."""
        if getattr(self, "_n_inputs", None) is None:
            self._n_inputs = self.info()["n_inputs"]
        return self._n_inputs

    def set_path(self, path: str = "auto") -> "Graph":
        """Kernel plan for later evaluations: 'auto', 'streamed', 'fused' or 'panel' (cos_graph_set_path)."""
        check(LIB.cos_graph_set_path(self.handle, PATHS[path]), "cos_graph_set_path")
        return self

    def export(self) -> dict:
        info = self.info()
        E = info["n_edges"]
        if info["kind"] == "lookup":
            out = dict(src=np.empty(E, np.int32), dst=np.empty(E, np.int32), slot=np.empty(E, np.int32),
                       coef=np.empty(E))
            check(LIB.cos_graph_export_lookup(self.handle, *[out[n].ctypes.data_as(ctypes.c_void_p)
                                                             for n in ("src", "dst", "slot", "coef")]),
                  "cos_graph_export_lookup")
            return out
        out = dict(src=np.empty(E, np.int32), dst=np.empty(E, np.int32), a=np.empty(E), b=np.empty(E),
                   k=np.empty((E, 3)))
        check(LIB.cos_graph_export(self.handle, *[out[n].ctypes.data_as(ctypes.c_void_p)
                                                  for n in ("src", "dst", "a", "b", "k")]), "cos_graph_export")
        return out

    def save(self, path) -> None:
        """Write the graph to a .npz file: level sizes and the canonical edge lists (export()).
        Graph.load re-creates it; the canonical order makes the re-created graph, and every
        result on it, bit-identical."""
        info = self.info()
        np.savez(path, L=np.int64(self._L), widths=self._widths, epl=self._epl, kind=np.str_(info["kind"]),
                 n_slots=np.int64(info["n_inputs"]), **self.export())

    @classmethod
    def load(cls, path) -> "Graph":
        """Re-create a graph written by save() (plain arrays only: nothing in the file is executed)."""
        with np.load(path, allow_pickle=False) as z:
            if str(z["kind"]) == "lookup":
                return cls(int(z["L"]), z["widths"], z["epl"], z["src"], z["dst"], slot=z["slot"], coef=z["coef"],
                           n_slots=int(z["n_slots"]))
            return cls(int(z["L"]), z["widths"], z["epl"], z["src"], z["dst"], z["a"], z["b"], z["k"])

    def workspace_bytes(self, S: int, precision: str = "fp64") -> int:
        v = ctypes.c_uint64()
        check(LIB.cos_evaluate_workspace_size(self.handle, int(S), PRECISIONS[precision], ctypes.byref(v)),
              "cos_evaluate_workspace_size")
        return int(v.value)

    def evaluate(self, x: torch.Tensor, precision: str = "fp64", out: torch.Tensor | None = None,
                 out_exp: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
                 stream: torch.cuda.Stream | None = None) -> torch.Tensor:
        """Final-node value per sample, queued on `stream`.

        x: float64[R, S] on the device, R = 3 (coordinates) for rational factors or
        n_slots (each sample's table) for lookup factors.

        Stream order: tensors are allocated (and x, out, workspace are usually
        written) on the current stream.  When `stream` is another stream it first
        waits for the current one, and every tensor the call uses is marked as in
        use on `stream`, so the caching allocator cannot hand its memory out again
        before the evaluation has finished there.
        """
        rows = self.n_inputs
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float64 and x.dim() == 2
                and x.shape[0] == rows and x.is_contiguous()):
            raise ValueError(f"x must be a contiguous float64 CUDA tensor of shape [{rows}, S]")
        S = x.shape[1]
        if out is None:
            out = torch.empty(S, dtype=torch.float64, device=x.device)
        if not (out.is_cuda and out.dtype == torch.float64 and out.numel() >= S and out.is_contiguous()):
            raise ValueError("out must be a contiguous float64 CUDA tensor with >= S elements")
        if out_exp is not None and not (out_exp.is_cuda and out_exp.dtype == torch.int32
                                        and out_exp.numel() >= S and out_exp.is_contiguous()):
            raise ValueError("out_exp must be a contiguous int32 CUDA tensor with >= S elements")
        if workspace is None:
            workspace = torch.empty(self.workspace_bytes(S, precision), dtype=torch.uint8, device=x.device)
        # a workspace smaller than workspace_bytes(S) makes the library sweep in sample chunks
        cur = torch.cuda.current_stream(x.device)
        st = stream if stream is not None else cur
        side = st.cuda_stream != cur.cuda_stream
        if side:
            st.wait_stream(cur)
        check(LIB.cos_evaluate(self.handle, x.data_ptr(), S, PRECISIONS[precision], out.data_ptr(),
                               out_exp.data_ptr() if out_exp is not None else None, workspace.data_ptr(),
                               workspace.numel() * workspace.element_size(), st.cuda_stream), "cos_evaluate")
        if side:
            for t in (x, out, out_exp, workspace):
                if t is not None:
                    t.record_stream(st)
        return out

    def evaluate_no_alloc(self, x: torch.Tensor, precision: str = "fp64", out: torch.Tensor | None = None,
                          out_exp: torch.Tensor | None = None) -> torch.Tensor:
        """cos_evaluate_no_alloc on the current stream: the library's fixed device workspace instead of an
        allocated one (the same results as evaluate).  Calls that overlap on one device race on that
        workspace.  Allocates `out` here only when it is not given."""
        rows = self.n_inputs
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float64 and x.dim() == 2
                and x.shape[0] == rows and x.is_contiguous()):
            raise ValueError(f"x must be a contiguous float64 CUDA tensor of shape [{rows}, S]")
        S = x.shape[1]
        if out is None:
            out = torch.empty(S, dtype=torch.float64, device=x.device)
        if not (out.is_cuda and out.dtype == torch.float64 and out.numel() >= S and out.is_contiguous()):
            raise ValueError("out must be a contiguous float64 CUDA tensor with >= S elements")
        if out_exp is not None and not (out_exp.is_cuda and out_exp.dtype == torch.int32
                                        and out_exp.numel() >= S and out_exp.is_contiguous()):
            raise ValueError("out_exp must be a contiguous int32 CUDA tensor with >= S elements")
        st = torch.cuda.current_stream(x.device)
        check(LIB.cos_evaluate_no_alloc(self.handle, x.data_ptr(), S, PRECISIONS[precision], out.data_ptr(),
                                        out_exp.data_ptr() if out_exp is not None else None, st.cuda_stream),
              "cos_evaluate_no_alloc")
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            check(LIB.cos_destroy_graph(self._h.value), "cos_destroy_graph")
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def timing_enable(on: bool = True):
    check(LIB.cos_timing_enable(1 if on else 0), "cos_timing_enable")


def timing_read(kind: str) -> tuple[float, int]:
    """(total device ms, launches) recorded for a kernel class since the last read."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    check(LIB.cos_timing_read(KINDS[kind], ctypes.byref(ms), ctypes.byref(n)), "cos_timing_read")
    return ms.value, n.value
