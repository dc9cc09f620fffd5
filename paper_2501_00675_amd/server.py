"""Python face of the serving API (cos_server_* in include/cos.h).

Argument marshalling only: admission, batching and every evaluation step run
in the library (scheduling thread in C++, step kernels in HIP).  The server
keeps a reference to each request's tensors until the request has ended.
"""

from __future__ import annotations

import ctypes

import torch

from ._lib import (COS_EAGAIN, COS_ECANCELED, COS_EINVAL, COS_OK, LIB, PRECISIONS, CosError, ReqStats, ServerStats,
                   StepRecord, check)
from .graph import Graph


def _stats_dict(st: ReqStats) -> dict:
    return {f: getattr(st, f) for f, _ in ReqStats._fields_}


class Ticket(int):
    """A request's ticket number, carrying its output tensors (out, out_exp)."""

    def __new__(cls, value: int, out: torch.Tensor, out_exp: torch.Tensor | None):
        t = super().__new__(cls, value)
        t.out, t.out_exp = out, out_exp
        return t


class Server:
    """Continuous-batching evaluator over resident graphs on the current device.

    hbm_budget: device bytes for the workspaces of admitted requests (graphs
    whose widest level fits in LDS need none); max_slots: requests admitted at
    once (1..512).
    """

    def __init__(self, hbm_budget: int, max_slots: int = 64):
        h = ctypes.c_void_p()
        check(LIB.cos_server_create(int(hbm_budget), int(max_slots), ctypes.byref(h)), "cos_server_create")
        self._h = h
        self._graphs: list[Graph] = []
        self._live: dict[int, tuple] = {}

    @property
    def handle(self) -> int:
        if self._h is None:
            raise ValueError("server was destroyed")
        return self._h.value

    def add_graph(self, graph: Graph) -> int:
        gid = ctypes.c_int32()
        check(LIB.cos_server_add_graph(self.handle, graph.handle, ctypes.byref(gid)), "cos_server_add_graph")
        self._graphs.append(graph)
        return gid.value

    def submit(self, gid: int, x: torch.Tensor, precision: str = "fp64", out: torch.Tensor | None = None,
               out_exp: torch.Tensor | None = None, sync_inputs: bool = True) -> Ticket:
        """Queue a request; returns its ticket (with .out and .out_exp).

        x: float64[R, S] on the device, R = 3 (coordinates) for rational factors
        or n_slots (each sample's table) for lookup factors.  The server reads
        x on its own stream, so x must be complete when the request is
        admitted: with sync_inputs the current torch stream is synchronised
        first.
        """
        # the row count of the graph's input (an unknown id is left for the library to refuse)
        rows = self._graphs[int(gid)].n_inputs if 0 <= int(gid) < len(self._graphs) else x.shape[0]
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
        if sync_inputs:
            torch.cuda.current_stream(x.device).synchronize()
        t = ctypes.c_uint64()
        check(LIB.cos_server_submit(self.handle, int(gid), x.data_ptr(), S, PRECISIONS[precision], out.data_ptr(),
                                    out_exp.data_ptr() if out_exp is not None else None, ctypes.byref(t)),
              "cos_server_submit")
        self._live[t.value] = (x, out, out_exp)
        return Ticket(t.value, out, out_exp)

    def _finish(self, ticket: int, st: int, stats: ReqStats) -> dict:
        d = _stats_dict(stats)
        d["status"] = st
        self._live.pop(int(ticket), None)
        if st not in (COS_OK, COS_ECANCELED):
            raise CosError(st, f"request {ticket} failed")
        return d

    def poll(self, ticket: int) -> dict | None:
        """None while queued or running; the request's stats once it has ended (forgets the ticket)."""
        stats = ReqStats()
        st = LIB.cos_server_poll(self.handle, int(ticket), ctypes.byref(stats))
        if st == COS_EAGAIN:
            return None
        if st == COS_EINVAL:  # unknown ticket
            check(st, "cos_server_poll")
        return self._finish(ticket, st, stats)

    def wait(self, ticket: int) -> dict:
        """Block until the request has ended; its stats (status COS_OK or COS_ECANCELED)."""
        stats = ReqStats()
        st = LIB.cos_server_wait(self.handle, int(ticket), ctypes.byref(stats))
        if st == COS_EINVAL:  # unknown ticket
            check(st, "cos_server_wait")
        return self._finish(ticket, st, stats)

    def cancel(self, ticket: int) -> bool:
        """Cancel a request not yet admitted: True if cancelled, False if it is already running."""
        st = LIB.cos_server_cancel(self.handle, int(ticket))
        if st == COS_EAGAIN:
            return False
        check(st, "cos_server_cancel")
        return True

    def read_steps(self, cap: int = 65536) -> list:
        """Trace records of the steps completed since the last read (cos_server_read_steps), oldest first."""
        buf = (StepRecord * max(int(cap), 1))()
        n = ctypes.c_int64()
        check(LIB.cos_server_read_steps(self.handle, buf, int(cap), ctypes.byref(n)), "cos_server_read_steps")
        return [{f: getattr(buf[i], f) for f, _ in StepRecord._fields_} for i in range(n.value)]

    def fail_admission(self, admission_index: int) -> "Server":
        """Test hook (cos_server_fail_admission): the admission with this index fails its set-up."""
        check(LIB.cos_server_fail_admission(self.handle, int(admission_index)), "cos_server_fail_admission")
        return self

    def stats(self) -> dict:
        s = ServerStats()
        check(LIB.cos_server_get_stats(self.handle, ctypes.byref(s)), "cos_server_get_stats")
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            check(LIB.cos_server_destroy(self._h.value), "cos_server_destroy")
        self._h = None
        self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
