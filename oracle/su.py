"""Plain FP64 CPU oracle of the gPEPS simple update for the kicked-Ising circuit.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module; the GPU library never
calls it and shares no code with it.

What is computed (paper: Model section, Eq. 1-3; Method section):
  * the state |psi(theta_h, n)> = U(theta_h)^n |0...0> with
    U = prod_<ij> exp(+i pi/4 Z_i Z_j) * prod_i exp(-i theta_h X_i / 2)  (Eq. 2-3);
    the ZZ angle is generalised to RZZ(theta_J) = exp(-i theta_J Z Z / 2), so
    theta_J = -pi/2 is Eq. 2 exactly;
  * as a graph PEPS (gPEPS): one tensor Gamma_v per qubit with a physical leg
    of dimension 2 and one virtual leg per incident edge, and one positive
    weight vector lambda_e per edge (Method section, "gPEPS");
  * evolved with the simple update: each two-qubit gate is applied locally,
    using the lambda vectors of the neighbouring edges as the environment, and
    the bond is truncated back to at most chi = D singular values (Method
    section, "simple update", "bond dimension chi");
  * read out in the mean-field (lambda) environment: the one-site density
    matrix of v is Gamma_v contracted with its conjugate over every virtual
    leg weighted by lambda^2 (Method section and Appendix B, "mean-field
    approximation of the environment").

The paper cites the simple update without writing it out; the steps below are
the standard one, in this order, for edge e = (i, j):
  1. absorb lambda_e' into Gamma_i on every other leg e' != e, and arrange it
     as a matrix A_i whose rows run over the other legs and whose columns run
     over (physical s, leg e); same for j;
  2. when A has more rows than columns, QR-reduce it: A = Q R; else R = A;
  3. Theta = R_i . diag(lambda_e) . R_j^T over the shared bond, times the
     diagonal gate g(s, t) = exp(-i theta_J z_s z_t / 2), z_0 = +1, z_1 = -1;
  4. SVD Theta = U S V^H, singular values descending;
  5. keep chi = max(1, min(D, #{S_k > eps * S_0})) values;
     lambda_e <- S[:chi] / ||S[:chi]||_2;
  6. Gamma_i <- Q_i U[:, :chi] with lambda_e'^{-1} on every other leg; Gamma_j
     likewise from the rows of V^H.
Weight-N observables (Appendix B): at the Clifford point theta_h = pi/2 the
expectation of W = U(pi/2)^n Z_q U(pi/2)^{dagger n} in |psi(theta_h, n)> equals
<Z_q> in |omega> = U(pi/2)^{dagger n} |psi(theta_h, n)>; evolve(inverse_steps=n)
continues the simple update with n applications of U(pi/2)^dagger.

Readings where the paper is silent (gate order inside a layer = ascending
colour classes, then ascending edge id; relative cutoff eps; lambda
normalisation; RX layer first) are listed with the workload definitions.

Tensor layout (oracle only): Gamma_v has shape (2, d_{e_1}, ..., d_{e_k}) with
the virtual legs in ascending incident-edge id; bond dimensions are variable
(start at 1, grow up to D); lambda_e holds only strictly positive entries.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

Z_SIGN = np.array([1.0, -1.0])


def rx_matrix(theta_h: float) -> np.ndarray:
    """exp(-i theta_h X / 2) (Eq. 2, field layer)."""
    c, s = math.cos(theta_h / 2.0), math.sin(theta_h / 2.0)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


def rzz_diagonal(theta_j: float) -> np.ndarray:
    """Diagonal of exp(-i theta_J Z Z / 2) as a 2x2 array g[s, t] (Eq. 2, coupling layer)."""
    zz = np.outer(Z_SIGN, Z_SIGN)
    return np.exp(-0.5j * theta_j * zz)


@dataclasses.dataclass
class PEPS:
    """gPEPS state: site tensors, bond weights and the graph they live on."""

    n_nodes: int
    edges: np.ndarray          # [E, 2]
    incident: List[List[int]]  # ascending incident edge ids per vertex
    gammas: List[np.ndarray]   # Gamma_v, shape (2, d_e1, ..., d_ek)
    lambdas: List[np.ndarray]  # lambda_e, float64, strictly positive

    def bond_dims(self) -> np.ndarray:
        return np.array([lam.shape[0] for lam in self.lambdas], dtype=np.int64)


def product_state(n_nodes: int, edges: np.ndarray) -> PEPS:
    """|0...0> as a gPEPS: all bonds of dimension 1, lambda = [1] (Eq. 3 initial state)."""
    incident: List[List[int]] = [[] for _ in range(n_nodes)]
    for e, (u, v) in enumerate(edges):
        incident[int(u)].append(e)
        incident[int(v)].append(e)
    gammas = []
    for v in range(n_nodes):
        g = np.zeros((2,) + (1,) * len(incident[v]), dtype=np.complex128)
        g[(0,) + (0,) * len(incident[v])] = 1.0
        gammas.append(g)
    lambdas = [np.ones(1, dtype=np.float64) for _ in range(len(edges))]
    return PEPS(n_nodes, np.asarray(edges), incident, gammas, lambdas)


def apply_rx_layer(peps: PEPS, theta_h: float) -> None:
    """Gamma_v[s, ...] <- sum_s' RX[s, s'] Gamma_v[s', ...] on every site."""
    m = rx_matrix(theta_h)
    for v in range(peps.n_nodes):
        peps.gammas[v] = np.tensordot(m, peps.gammas[v], axes=([1], [0]))


def _side_matrix(peps: PEPS, v: int, e: int):
    """Step 1 for one end of edge e: absorb the other legs' lambdas, reshape.

    Returns (A, other_edges, other_dims, pos) where A is [M, 2 * d_e] with rows
    over the other legs (in ascending edge id) and columns over (s, leg e).
    """
    legs = peps.incident[v]
    pos = legs.index(e)
    g = peps.gammas[v].copy()
    others = [f for f in legs if f != e]
    for f in others:
        ax = 1 + legs.index(f)
        shape = [1] * g.ndim
        shape[ax] = peps.lambdas[f].shape[0]
        g = g * peps.lambdas[f].reshape(shape)
    # axes order: other legs..., physical, leg e
    order = [1 + legs.index(f) for f in others] + [0, 1 + pos]
    a = np.transpose(g, order)
    other_dims = [peps.lambdas[f].shape[0] for f in others]
    m = int(np.prod(other_dims)) if other_dims else 1
    a = a.reshape(m, 2 * peps.lambdas[e].shape[0])
    return a, others, other_dims, pos


def _restore_site(peps: PEPS, v: int, e: int, x: np.ndarray, others, other_dims, pos: int) -> None:
    """Step 6 for one end: x is [M, 2, chi]; divide other legs by lambda, restore leg order."""
    chi = x.shape[2]
    t = x.reshape(tuple(other_dims) + (2, chi))
    for k, f in enumerate(others):
        shape = [1] * t.ndim
        shape[k] = other_dims[k]
        t = t / peps.lambdas[f].reshape(shape)
    legs = peps.incident[v]
    # current axes: others..., s, e ; target: s, legs in ascending order
    cur = others + ["s", e]
    target = ["s"] + legs
    perm = [cur.index(lbl) for lbl in target]
    peps.gammas[v] = np.transpose(t, perm).copy()


@dataclasses.dataclass
class EdgeRecord:
    """Diagnostics of one simple-update step on one edge."""

    edge: int
    chi: int
    discarded_weight: float  # sum of discarded S_k^2 / sum of all S_k^2
    cut_gap: float           # (S_{chi-1} - S_chi) / S_0, inf when nothing was cut


def kept_rank(s: np.ndarray, d_max: int, eps: float) -> int:
    """Step 5: chi = max(1, min(D, #{S_k > eps * S_0})) for descending singular values S."""
    return max(1, min(d_max, int(np.count_nonzero(s > eps * s[0]))))


def simple_update_edge(peps: PEPS, e: int, theta_j: float, d_max: int, eps: float) -> EdgeRecord:
    """One RZZ(theta_J) gate on edge e by the simple update (steps 1-6 above)."""
    i, j = int(peps.edges[e, 0]), int(peps.edges[e, 1])
    de = peps.lambdas[e].shape[0]

    # steps 1-2: environment absorption and QR reduction of both ends
    a_i, oth_i, dims_i, pos_i = _side_matrix(peps, i, e)
    a_j, oth_j, dims_j, pos_j = _side_matrix(peps, j, e)
    q_i = q_j = None
    if a_i.shape[0] > a_i.shape[1]:
        q_i, r_i = np.linalg.qr(a_i, mode="reduced")
    else:
        r_i = a_i
    if a_j.shape[0] > a_j.shape[1]:
        q_j, r_j = np.linalg.qr(a_j, mode="reduced")
    else:
        r_j = a_j
    ri, rj = r_i.shape[0], r_j.shape[0]
    r_i3 = r_i.reshape(ri, 2, de)
    r_j3 = r_j.reshape(rj, 2, de)

    # step 3: two-site matrix with the bond weight and the diagonal gate
    theta = np.einsum("ask,k,btk->astb", r_i3, peps.lambdas[e], r_j3)
    theta = theta * rzz_diagonal(theta_j)[None, :, :, None]
    theta = theta.reshape(ri * 2, 2 * rj)

    # step 4: SVD
    u, s, vh = np.linalg.svd(theta, full_matrices=False)

    # step 5: truncation and renormalisation
    if s[0] <= 0.0:
        raise FloatingPointError("simple update produced a zero two-site tensor")
    chi = kept_rank(s, d_max, eps)
    total = float(np.sum(s * s))
    disc = float(np.sum(s[chi:] ** 2)) / total if total > 0 else 0.0
    gap = float((s[chi - 1] - s[chi]) / s[0]) if chi < s.shape[0] else math.inf
    lam = s[:chi] / np.linalg.norm(s[:chi])

    # step 6: new site tensors with the environment removed again
    x_i = u[:, :chi].reshape(ri, 2, chi)
    if q_i is not None:
        x_i = np.tensordot(q_i, x_i, axes=([1], [0]))
    x_j = vh[:chi, :].reshape(chi, 2, rj).transpose(2, 1, 0)
    if q_j is not None:
        x_j = np.tensordot(q_j, x_j, axes=([1], [0]))
    peps.lambdas[e] = lam
    _restore_site(peps, i, e, x_i, oth_i, dims_i, pos_i)
    _restore_site(peps, j, e, x_j, oth_j, dims_j, pos_j)
    return EdgeRecord(edge=e, chi=chi, discarded_weight=disc, cut_gap=gap)


def site_z(peps: PEPS) -> np.ndarray:
    """Mean-field <Z_v> for every site: (rho_00 - rho_11) / (rho_00 + rho_11).

    rho_v[s, s'] = sum over virtual indices of Gamma_v[s, ...] conj(Gamma_v[s', ...])
    times the product of lambda_e^2 over every leg of v (Method section; Appendix B).
    """
    out = np.empty(peps.n_nodes, dtype=np.float64)
    for v in range(peps.n_nodes):
        g = peps.gammas[v]
        w = np.ones(g.shape[1:], dtype=np.float64)
        for k, f in enumerate(peps.incident[v]):
            shape = [1] * (g.ndim - 1)
            shape[k] = peps.lambdas[f].shape[0]
            w = w * (peps.lambdas[f] ** 2).reshape(shape)
        p = np.abs(g) ** 2
        rho00 = float(np.sum(p[0] * w))
        rho11 = float(np.sum(p[1] * w))
        out[v] = (rho00 - rho11) / (rho00 + rho11)
    return out


@dataclasses.dataclass
class Trajectory:
    """Per-step results of one evolution."""

    z: np.ndarray                 # [steps, n_nodes], <Z_v> after each full Trotter step
    bond_dims: np.ndarray         # [steps, n_edges]
    min_cut_gap: np.ndarray       # [steps], smallest relative cut gap among truncated bonds
    discarded: np.ndarray         # [steps], largest discarded weight of any bond update
    peps: Optional[PEPS] = None   # final state

    @property
    def magnetisation(self) -> np.ndarray:
        return self.z.mean(axis=1)


def trotter_step(peps: PEPS, classes: Sequence[Sequence[int]], theta_h: float, theta_j: float,
                 d_max: int, eps: float) -> List[EdgeRecord]:
    """One application of U(theta_h): RX on every qubit, then the RZZ gates class by class."""
    apply_rx_layer(peps, theta_h)
    recs = []
    for cls in classes:
        for e in cls:
            recs.append(simple_update_edge(peps, e, theta_j, d_max, eps))
    return recs


def regauge_sweep(peps: PEPS, classes: Sequence[Sequence[int]], d_max: int, eps: float) -> List[EdgeRecord]:
    """One sweep of the simple update with the identity gate over every edge, class by class.

    The state is unchanged (up to singular values under the cutoff), only its gauge moves; the
    fixed point of these sweeps is the fixed point of belief propagation on the norm network
    (Results: the simple update and BP share their fixed point), so repeated sweeps are BP
    gauging, and at convergence the mean-field readout equals the BP readout.
    """
    return [simple_update_edge(peps, e, 0.0, d_max, eps) for cls in classes for e in cls]


def inverse_trotter_step(peps: PEPS, classes: Sequence[Sequence[int]], theta_h: float, theta_j: float,
                         d_max: int, eps: float) -> List[EdgeRecord]:
    """One application of U(theta_h)^dagger (Appendix B): RZZ(-theta_J) gates, then RX(-theta_h).

    U is the RZZ layer after the RX layer, so its inverse undoes the RZZ layer first.  The RZZ
    gates commute with one another; they run in the same class order as in trotter_step (the
    order matters only through truncation).
    """
    recs = []
    for cls in classes:
        for e in cls:
            recs.append(simple_update_edge(peps, e, -theta_j, d_max, eps))
    apply_rx_layer(peps, -theta_h)
    return recs


def evolve(n_nodes: int, edges: np.ndarray, colour: np.ndarray, theta_h: float, theta_j: float,
           d_max: int, steps: int, eps: float = 1e-12, keep_state: bool = False,
           inverse_steps: int = 0, theta_h_inverse: float = math.pi / 2, regauge: int = 0) -> Trajectory:
    """Simple-update evolution of |0...0> under U(theta_h)^steps, <Z_v> after every step.

    With inverse_steps = m > 0 the evolution continues with m applications of
    U(theta_h_inverse)^dagger at the same theta_J, giving the state
    |omega(theta_h, n)> = U(pi/2)^{dagger m} |psi(theta_h, n)> of Appendix B (weight-N
    observables at the Clifford point); their rows follow the forward rows.
    With regauge = k > 0, k identity-gate sweeps (BP gauging, regauge_sweep) follow the gates
    of every step, before its readout.
    """
    edges = np.asarray(edges)
    colour = np.asarray(colour)
    n_col = int(colour.max()) + 1 if len(colour) else 0
    classes = [[int(e) for e in np.nonzero(colour == c)[0]] for c in range(n_col)]
    peps = product_state(n_nodes, edges)
    zs, dims, gaps, disc = [], [], [], []
    for t in range(steps + inverse_steps):
        if t < steps:
            recs = trotter_step(peps, classes, theta_h, theta_j, d_max, eps)
        else:
            recs = inverse_trotter_step(peps, classes, theta_h_inverse, theta_j, d_max, eps)
        for _ in range(regauge):
            regauge_sweep(peps, classes, d_max, eps)
        zs.append(site_z(peps))
        dims.append(peps.bond_dims())
        g = [r.cut_gap for r in recs if math.isfinite(r.cut_gap)]
        gaps.append(min(g) if g else math.inf)
        disc.append(max((r.discarded_weight for r in recs), default=0.0))
    rows = steps + inverse_steps
    return Trajectory(z=np.array(zs).reshape(rows, n_nodes), bond_dims=np.array(dims).reshape(rows, -1),
                      min_cut_gap=np.array(gaps), discarded=np.array(disc),
                      peps=peps if keep_state else None)


def evolve_graph(graph, theta_h: float, theta_j: float, d_max: int, steps: int, eps: float = 1e-12,
                 keep_state: bool = False, inverse_steps: int = 0,
                 theta_h_inverse: float = math.pi / 2, regauge: int = 0) -> Trajectory:
    """evolve() on a graph object exposing n_nodes, edges and colour."""
    return evolve(graph.n_nodes, graph.edges, graph.colour, theta_h, theta_j, d_max, steps, eps, keep_state,
                  inverse_steps, theta_h_inverse, regauge)
