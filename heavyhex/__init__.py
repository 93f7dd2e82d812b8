"""Workload inputs shared by the oracle, the tests and the bench.

This package holds only input generation: the qubit graphs of the paper's
lattices (heavy-hexagon patches, a 12-site ring, small trees), a deterministic
proper edge colouring that fixes the order in which the two-qubit gates of one
Trotter layer are applied, and the seeded parameter recipes of the benchmark
workloads.  It contains none of the simple-update arithmetic, so both the
oracle and the GPU path can consume it without sharing code with each other.
"""

from .graphs import (
    Graph,
    heavy_hex,
    eagle127,
    heavy_hex_cell10,
    ring,
    path,
    tree_from_edges,
    kempe_edge_colouring,
    check_proper_colouring,
    bfs_ball,
)
from .workloads import WORKLOADS, Workload, Instance, make_workload

__all__ = [
    "Graph",
    "heavy_hex",
    "eagle127",
    "heavy_hex_cell10",
    "ring",
    "path",
    "tree_from_edges",
    "kempe_edge_colouring",
    "check_proper_colouring",
    "bfs_ball",
    "WORKLOADS",
    "Workload",
    "Instance",
    "make_workload",
]
