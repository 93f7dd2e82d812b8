"""Exact references that pin the oracle: state vectors, light cones, Pauli propagation.

These share nothing with the oracle's simple update: they evolve the full
wavefunction (or a Clifford Pauli string) under the circuit of Eq. 2-3 of the
paper directly.

* statevector_z: brute-force evolution of U(theta_h)^t |0...0> on <= ~20 qubits.
  The RZZ layer is diagonal, so it is one phase vector exp(-i theta_J/2 sum_<ij> z_i z_j).
* lightcone_z: <Z_i> after t steps depends only on the gates inside the ball of
  radius t-1 around i (U^dag Z_i U keeps support {i}; each further step adds one
  hop), so the state vector of that ball's induced subgraph gives the exact
  value on a large graph.
* propagate_pauli: conjugation O -> U O U^dag of a Pauli string at the Clifford
  point theta_h = pi/2, theta_J = -pi/2 (Appendix B of the paper uses
  W = U^n Z_q U^{dag n}).
"""

from __future__ import annotations

import math
from typing import Dict, List, Sequence, Tuple

import numpy as np


def _apply_rx_all(psi: np.ndarray, n: int, theta_h: float) -> np.ndarray:
    c, s = math.cos(theta_h / 2), math.sin(theta_h / 2)
    m = np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)
    t = psi.reshape((2,) * n)
    for q in range(n):
        t = np.moveaxis(np.tensordot(m, t, axes=([1], [q])), 0, q)
    return t.reshape(-1)


def _zz_phase(n: int, edges: Sequence[Tuple[int, int]], theta_j: float) -> np.ndarray:
    idx = np.arange(2 ** n, dtype=np.int64)
    # qubit q is bit (n-1-q) of the basis index (qubit 0 most significant)
    z = 1 - 2 * ((idx[:, None] >> (n - 1 - np.arange(n)[None, :])) & 1)
    acc = np.zeros(2 ** n, dtype=np.float64)
    for u, v in edges:
        acc += z[:, u] * z[:, v]
    return np.exp(-0.5j * theta_j * acc)


def _z_expect(psi: np.ndarray, n: int) -> np.ndarray:
    p = (np.abs(psi) ** 2).reshape((2,) * n)
    out = np.empty(n)
    for q in range(n):
        m = np.moveaxis(p, q, 0).reshape(2, -1).sum(axis=1)
        out[q] = m[0] - m[1]
    return out / p.sum()


def statevector_z(n: int, edges: Sequence[Tuple[int, int]], theta_h: float, theta_j: float,
                  steps: int) -> np.ndarray:
    """<Z_q> for every qubit after every step: array [steps, n]."""
    psi = np.zeros(2 ** n, dtype=np.complex128)
    psi[0] = 1.0
    phase = _zz_phase(n, edges, theta_j)
    out = np.empty((steps, n))
    for t in range(steps):
        psi = _apply_rx_all(psi, n, theta_h)
        psi = psi * phase
        out[t] = _z_expect(psi, n)
    return out


def statevector(n: int, edges: Sequence[Tuple[int, int]], theta_h: float, theta_j: float,
                steps: int) -> np.ndarray:
    """U(theta_h)^steps |0...0> as a vector of 2^n amplitudes (qubit 0 most significant)."""
    psi = np.zeros(2 ** n, dtype=np.complex128)
    psi[0] = 1.0
    phase = _zz_phase(n, edges, theta_j)
    for _ in range(steps):
        psi = _apply_rx_all(psi, n, theta_h) * phase
    return psi


def pauli_expect(psi: np.ndarray, n: int, phase: complex, ops: Dict[int, str]) -> complex:
    """<psi| phase * P |psi> for the Pauli string P (dict qubit -> letter), applied factor by factor."""
    mats = {"X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
            "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
            "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128)}
    t = psi.reshape((2,) * n)
    for q, p in ops.items():
        t = np.moveaxis(np.tensordot(mats[p], t, axes=([1], [q])), 0, q)
    return complex(phase * np.vdot(psi, t.reshape(-1)))


def ball(adj: List[List[int]], centre: int, radius: int) -> List[int]:
    dist = {centre: 0}
    frontier = [centre]
    for r in range(radius):
        nxt = []
        for x in frontier:
            for y in adj[x]:
                if y not in dist:
                    dist[y] = r + 1
                    nxt.append(y)
        frontier = nxt
    return sorted(dist)


def lightcone_z(n_nodes: int, edges: np.ndarray, site: int, theta_h: float, theta_j: float,
                steps: int) -> float:
    """Exact <Z_site> after ``steps`` Trotter steps on a large graph via its light cone."""
    adj: List[List[int]] = [[] for _ in range(n_nodes)]
    for u, v in edges:
        adj[int(u)].append(int(v))
        adj[int(v)].append(int(u))
    sub = ball(adj, site, max(steps - 1, 0))
    pos = {q: k for k, q in enumerate(sub)}
    sub_edges = [(pos[int(u)], pos[int(v)]) for u, v in edges if int(u) in pos and int(v) in pos]
    z = statevector_z(len(sub), sub_edges, theta_h, theta_j, steps)
    return float(z[-1, pos[site]])


# ----- Clifford Pauli propagation ------------------------------------------------------------

# single-qubit Pauli products: (a, b) -> (phase, c) with a.b = phase * c
_MUL: Dict[Tuple[str, str], Tuple[complex, str]] = {}
for _p in "IXYZ":
    _MUL[("I", _p)] = (1, _p)
    _MUL[(_p, "I")] = (1, _p)
for _a, _b, _c in [("X", "Y", "Z"), ("Y", "Z", "X"), ("Z", "X", "Y")]:
    _MUL[(_a, _b)] = (1j, _c)
    _MUL[(_b, _a)] = (-1j, _c)
for _p in "XYZ":
    _MUL[(_p, _p)] = (1, "I")


def _mul(phase: complex, ops: Dict[int, str], other: Dict[int, str]) -> Tuple[complex, Dict[int, str]]:
    """(phase * ops) . other, both Pauli strings (dict qubit -> letter)."""
    out = dict(ops)
    for q, b in other.items():
        a = out.get(q, "I")
        ph, c = _MUL[(a, b)]
        phase *= ph
        if c == "I":
            out.pop(q, None)
        else:
            out[q] = c
    return phase, out


def propagate_pauli(edges: np.ndarray, ops: Dict[int, str], steps: int) -> Tuple[complex, Dict[int, str]]:
    """U^steps O U^{dag steps} at theta_h = pi/2, theta_J = -pi/2, U = ZZ-layer . RX-layer.

    O -> U O U^dag = ZZ (RX O RX^dag) ZZ^dag.  With RX = exp(-i pi/4 X):
    X -> X, Y -> Z, Z -> -Y.  With G = exp(+i pi/4 Z_a Z_b): a string that
    anticommutes with Z_a Z_b maps to O . (-i Z_a Z_b); one that commutes is unchanged.
    """
    phase: complex = 1
    cur = dict(ops)
    for _ in range(steps):
        nxt: Dict[int, str] = {}
        for q, p in cur.items():
            if p == "Y":
                nxt[q] = "Z"
            elif p == "Z":
                nxt[q] = "Y"
                phase *= -1
            else:
                nxt[q] = p
        cur = nxt
        for u, v in edges:
            u, v = int(u), int(v)
            anti = sum(1 for q in (u, v) if cur.get(q, "I") in ("X", "Y")) % 2
            if anti:
                phase, cur = _mul(phase * (-1j), cur, {u: "Z", v: "Z"})
    return phase, cur
