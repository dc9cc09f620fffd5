"""Leveled-DAG diagram summation on AMD Instinct MI355X (gfx950).

Evaluates the combinatorial-summation graph of Sturt & Kozik (arXiv
2501.00675, Sec. II): the root holds 1, each edge multiplies its source value
by an edge factor and adds it into its destination, and the final node holds
the sum over all root-to-final paths of the products of their factors -- for
many sample points at once.  The work runs in hand-written HIP kernels behind
the C ABI of include/cos.h (libcosdag.so); this package only marshals
arguments.  There is no CPU fallback: importing fails if the library is not
built.
"""

from ._lib import LIB, PRECISIONS, CosError  # noqa: F401
from .graph import Graph, timing_enable, timing_read  # noqa: F401
from .mc import Walkers  # noqa: F401
from .server import Server, Ticket  # noqa: F401

__all__ = ["Graph", "Server", "Ticket", "Walkers", "CosError", "PRECISIONS", "timing_enable", "timing_read", "LIB"]
