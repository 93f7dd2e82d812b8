"""Seeded workload recipes: graphs, angles, bond dimension, steps, precision.

Every workload is the kicked-Ising Trotter circuit of Eq. 2-3 of the paper
(RX(theta_h) on every qubit, then RZZ(theta_J) on every edge, repeated n times
from |0...0>) on one or more qubit graphs.  theta_J = -pi/2 reproduces the
exp(+i pi/4 Z Z) gate of Eq. 2 under RZZ(theta) = exp(-i theta Z Z / 2).

The recipes mirror the paper's workloads at the sizes a single GPU runs:
  ring12_d4_c128     12-qubit ring (one heavy-hex face), D=4, complex128, 5 steps
  eagle127_d16       127-qubit heavy-hex, theta_h=0.7, D=16, 20 steps (Fig. 3b-like)
  eagle127_sweep_d32 32 theta_h instances on [0, pi/2], D=32, 20 steps (Fig. 3b sweep)
  mixed_d32          435 + 1123 + 8 x 127 qubit graphs, cap D=32, 40 steps (Fig. 4 sizes)
  eagle127_sweep_d16 the 127-qubit graph, 256 instances theta_h=linspace(0, pi/2, 256), D=16, 20 steps
  eagle127_grad_d16  127-qubit heavy-hex, theta_h=0.6, D=16, 20 steps (adjoint workload)
  eagle127_grad_d32  the same at D=32
  eagle127_weight_d32 the 32 theta_h instances of the sweep, D=32, 5 steps then 5 inverse steps
                     U(pi/2)^dagger (Appendix B weight-10 / weight-17 observables, Fig. 3)
  heavyhex_inf_d32   infinite heavy-hex lattice (10-qubit periodic unit cell), 256 theta_h
                     instances on [0, pi/2], D=32, 20 steps (Fig. 4 infinite-size curve)
  heavyhex_inf_weight_d32 the same cell, 32 theta_h instances, 5 steps then 5 inverse steps
                     (Table I: Q = 2 on the infinite lattice)
  long_theta1_d{8,16,32} long-time evolution (Figs. 5-6): the 127-, 435- and 1123-qubit graphs,
                     theta_h = 1.0, 39 steps, one workload per bond dimension of the ladder
  eagle127_d64       127-qubit heavy-hex, theta_h = 0.7 and 1.0, D=64, 8 steps (bond dimension beyond
                     32, Fig. 3(b)'s chi = 64)
  eagle127_d64_t20   127-qubit heavy-hex, theta_h = 0.7, D=64, 20 steps
  long_theta1_d64_127 the D = 64 rung of the long-time ladder on the 127-qubit graph, 39 steps
The only random draw is the per-graph theta_h of mixed_d32:
numpy.random.default_rng(0).uniform(0.1, 1.0, 10), in graph order.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Callable, Dict, List

import numpy as np

from .graphs import Graph, eagle127, heavy_hex, heavy_hex_cell10, ring

C64 = "c64"    # site tensors complex64, QR / SVD / lambda in float64
C128 = "c128"  # everything complex128 / float64


@dataclasses.dataclass
class Instance:
    graph: int       # index into Workload.graphs
    theta_h: float
    theta_j: float


@dataclasses.dataclass
class Workload:
    name: str
    graphs: List[Graph]
    instances: List[Instance]
    d_max: int
    steps: int
    precision: str
    trunc_rel: float
    description: str
    inverse_steps: int = 0              # applications of U(theta_h_inverse)^dagger after the steps
    theta_h_inverse: float = math.pi / 2

    @property
    def rows(self) -> int:
        """History rows of the whole evolution: forward steps, then inverse steps."""
        return self.steps + self.inverse_steps

    @property
    def edge_updates(self) -> int:
        """Two-qubit gate applications of the whole evolution."""
        return sum(self.graphs[i.graph].n_edges for i in self.instances) * self.rows

    def scaled(self, steps: int | None = None, instances: List[int] | None = None) -> "Workload":
        """A copy with fewer steps and/or a subset of instances (parity-test sizes)."""
        ins = self.instances if instances is None else [self.instances[k] for k in instances]
        return dataclasses.replace(self, steps=self.steps if steps is None else steps, instances=list(ins))


THETA_J = -math.pi / 2


def _ring12() -> Workload:
    return Workload("ring12_d4_c128", [ring(12)], [Instance(0, 0.5, THETA_J)], 4, 5, C128, 1e-12,
                    "12-qubit ring, theta_h=0.5, D=4, complex128, 5 steps")


def _eagle_d16() -> Workload:
    return Workload("eagle127_d16", [eagle127()], [Instance(0, 0.7, THETA_J)], 16, 20, C64, 1e-6,
                    "127-qubit heavy-hex, theta_h=0.7, D=16, complex64 + float64 QR/SVD, 20 steps")


def _eagle_sweep_d32() -> Workload:
    ths = np.linspace(0.0, math.pi / 2, 32)
    return Workload("eagle127_sweep_d32", [eagle127()], [Instance(0, float(t), THETA_J) for t in ths],
                    32, 20, C64, 1e-6,
                    "127-qubit heavy-hex, 32 instances theta_h=linspace(0, pi/2, 32), D=32, 20 steps")


def _eagle_sweep_d16() -> Workload:
    ths = np.linspace(0.0, math.pi / 2, 256)
    return Workload("eagle127_sweep_d16", [eagle127()], [Instance(0, float(t), THETA_J) for t in ths],
                    16, 20, C64, 1e-6,
                    "127-qubit heavy-hex, 256 instances theta_h=linspace(0, pi/2, 256), D=16, 20 steps")


def _mixed_d32() -> Workload:
    g = [heavy_hex(13, 27, False), heavy_hex(21, 43, False)] + [eagle127()]
    graph_of = [0, 1] + [2] * 8
    ths = np.random.default_rng(0).uniform(0.1, 1.0, 10)
    ins = [Instance(gi, float(t), THETA_J) for gi, t in zip(graph_of, ths)]
    return Workload("mixed_d32", g, ins, 32, 40, C64, 1e-8,
                    "435 + 1123 + 8 x 127 qubit heavy-hex graphs, cap D=32, cutoff 1e-8, 40 steps")


def _eagle_grad_d16() -> Workload:
    return Workload("eagle127_grad_d16", [eagle127()], [Instance(0, 0.6, THETA_J)], 16, 20, C64, 1e-6,
                    "127-qubit heavy-hex, theta_h=0.6, D=16, 20 steps, gradient of mean <Z>")


def _eagle_grad_d32() -> Workload:
    return Workload("eagle127_grad_d32", [eagle127()], [Instance(0, 0.6, THETA_J)], 32, 20, C64, 1e-6,
                    "127-qubit heavy-hex, theta_h=0.6, D=32, 20 steps, gradient of mean <Z>")


def _eagle_weight_d32() -> Workload:
    ths = np.linspace(0.0, math.pi / 2, 32)
    return Workload("eagle127_weight_d32", [eagle127()], [Instance(0, float(t), THETA_J) for t in ths],
                    32, 5, C64, 1e-6,
                    "127-qubit heavy-hex, 32 instances theta_h=linspace(0, pi/2, 32), D=32, 5 steps then "
                    "5 steps of U(pi/2)^dagger; <Z_13>, <Z_58> give the weight-10 / weight-17 observables",
                    inverse_steps=5)


def _inf_d32() -> Workload:
    ths = np.linspace(0.0, math.pi / 2, 256)
    return Workload("heavyhex_inf_d32", [heavy_hex_cell10()], [Instance(0, float(t), THETA_J) for t in ths],
                    32, 20, C64, 1e-6,
                    "infinite heavy-hex lattice (10-qubit periodic unit cell), 256 instances "
                    "theta_h=linspace(0, pi/2, 256), D=32, 20 steps")


def _inf_weight_d32() -> Workload:
    ths = np.linspace(0.0, math.pi / 2, 32)
    return Workload("heavyhex_inf_weight_d32", [heavy_hex_cell10()], [Instance(0, float(t), THETA_J) for t in ths],
                    32, 5, C64, 1e-6,
                    "infinite heavy-hex lattice (10-qubit cell), 32 instances theta_h=linspace(0, pi/2, 32), "
                    "D=32, 5 steps then 5 steps of U(pi/2)^dagger; <Z_2> of the last row",
                    inverse_steps=5)


def _eagle_d64() -> Workload:
    return Workload("eagle127_d64", [eagle127()], [Instance(0, 0.7, THETA_J), Instance(0, 1.0, THETA_J)],
                    64, 8, C64, 1e-6,
                    "127-qubit heavy-hex, theta_h = 0.7 and 1.0, D=64, 8 steps (bonds saturate at t = 6, "
                    "truncation from t = 7)")


def _eagle_d64_t20() -> Workload:
    return Workload("eagle127_d64_t20", [eagle127()], [Instance(0, 0.7, THETA_J)], 64, 20, C64, 1e-6,
                    "127-qubit heavy-hex, theta_h=0.7, D=64, complex64 + float64 QR/SVD, 20 steps")


def _long_d64_127() -> Workload:
    return Workload("long_theta1_d64_127", [eagle127()], [Instance(0, 1.0, THETA_J)], 64, 39, C64, 1e-8,
                    "127-qubit heavy-hex, theta_h=1.0, D=64, cutoff 1e-8, 39 steps (the D = 64 rung of the "
                    "long-time ladder on the 127-qubit lattice)")


def _long(d: int) -> Callable[[], Workload]:
    def make() -> Workload:
        g = [eagle127(), heavy_hex(13, 27, False), heavy_hex(21, 43, False)]
        return Workload(f"long_theta1_d{d}", g, [Instance(k, 1.0, THETA_J) for k in range(3)], d, 39, C64, 1e-8,
                        f"127 + 435 + 1123 qubit heavy-hex graphs, theta_h=1.0, D={d}, cutoff 1e-8, 39 steps "
                        "(long-time evolution, one rung of the bond-dimension ladder)")
    return make


WORKLOADS: Dict[str, Callable[[], Workload]] = {
    "ring12_d4_c128": _ring12,
    "eagle127_d16": _eagle_d16,
    "eagle127_sweep_d32": _eagle_sweep_d32,
    "eagle127_sweep_d16": _eagle_sweep_d16,
    "mixed_d32": _mixed_d32,
    "eagle127_grad_d16": _eagle_grad_d16,
    "eagle127_grad_d32": _eagle_grad_d32,
    "eagle127_weight_d32": _eagle_weight_d32,
    "heavyhex_inf_d32": _inf_d32,
    "heavyhex_inf_weight_d32": _inf_weight_d32,
    "long_theta1_d8": _long(8),
    "long_theta1_d16": _long(16),
    "long_theta1_d32": _long(32),
    "eagle127_d64": _eagle_d64,
    "eagle127_d64_t20": _eagle_d64_t20,
    "long_theta1_d64_127": _long_d64_127,
}


def make_workload(name: str) -> Workload:
    return WORKLOADS[name]()
