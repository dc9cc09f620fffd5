"""Seeded synthetic inputs for leveled-DAG evaluation.

This package only *draws* inputs: graph structure (per-level edge lists), edge
parameters and per-sample inputs (coordinates, or tables for lookup factors).  It holds none of the evaluation arithmetic, so
that the CPU oracle and the GPU library can both consume it without sharing any
code that computes a result.

The graphs stand in for the combinatorial-summation (CoS) graphs of the paper
(Sec. II.B, Fig. ``combinedgraphflat``), which are not reproducible from the
paper alone: a single root at level 0, a single final node at level L, edges
only between consecutive levels, nodes numbered contiguously level by level.
"""

from .graphs import (  # noqa: F401
    LeveledGraph,
    layered_graph,
    draw_lookup,
    draw_params,
    draw_samples,
    draw_table,
    level_offsets,
    transpose,
)
from .configs import (  # noqa: F401
    CONFIGS,
    lookup_slots,
    make_config,
    serving_mix,
)
