"""Plain FP64 CPU oracle: belief propagation (BP) on the norm network of a gPEPS.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module; the GPU library never
calls it and shares no code with it.

The paper also runs BP gauging after each Trotter step and finds that it does not
improve on the simple update, whose lambda environment is BP's fixed point
(Results, discussion of Fig. 3(a)).  This module runs BP on a given state and
reads <Z> out of its messages, which measures how far the simple-update gauge
is from that fixed point:
  * site tensors in the symmetric gauge: A_v = Gamma_v times sqrt(lambda_e) on
    every leg e, so that contracting the A's over every bond gives |psi>;
  * one message m_{u->v} per directed edge e = (u, v): a d_e x d_e matrix over
    the ket and bra copies of the bond index, starting at identity / d_e;
  * parallel (Jacobi) update of every message from the previous ones:
        m_{v->w}[a, a'] = sum over s and every other leg f of v of
            A_v[s, .., a, ..] conj(A_v[s, .., a', ..]) prod_f m_{u_f->v}[b_f, b'_f],
    then divided by its trace;
  * BP readout: rho_v[s, s'] = the same sum with s, s' open and every leg of v
    closed by its incoming message; <Z_v> = (rho_00 - rho_11) / (rho_00 + rho_11).
On a tree BP is exact after as many iterations as the tree's diameter.  For a
state in the Vidal gauge (a tree evolved by the untruncated simple update) the
fixed point is m = diag(lambda_e) / sum(lambda_e), and the BP readout equals the
mean-field one.
"""

from __future__ import annotations

import dataclasses
from typing import Dict, List, Tuple

import numpy as np

from .su import PEPS


def symmetric_tensors(peps: PEPS) -> List[np.ndarray]:
    """A_v = Gamma_v with sqrt(lambda_e) on every leg (legs in ascending incident edge id)."""
    out = []
    for v in range(peps.n_nodes):
        a = peps.gammas[v].copy()
        for k, e in enumerate(peps.incident[v]):
            shape = [1] * a.ndim
            shape[1 + k] = peps.lambdas[e].shape[0]
            a = a * np.sqrt(peps.lambdas[e]).reshape(shape)
        out.append(a)
    return out


def _close_legs(a: np.ndarray, msgs: List[np.ndarray], open_leg: int) -> np.ndarray:
    """sum A[s, ..] conj(A[s', ..]) prod_k msgs[k][b_k, b'_k] over every leg except `open_leg`.

    With open_leg = -1 every leg is closed and the result is rho[s, s'];
    otherwise s is summed too and the result is indexed [a, a'] on the open leg.
    """
    k_legs = a.ndim - 1
    ket = [0] + list(range(1, k_legs + 1))           # s, legs
    bra = [10] + list(range(11, 11 + k_legs))        # s', legs'
    if open_leg >= 0:
        bra[0] = 0  # the physical index is summed: ket and bra share it
    ops = [a, ket, np.conj(a), bra]
    for k in range(k_legs):
        if k == open_leg:
            continue
        ops += [msgs[k], [1 + k, 11 + k]]
    out = [0, 10] if open_leg < 0 else [1 + open_leg, 11 + open_leg]
    return np.einsum(*ops, out, optimize=True)


@dataclasses.dataclass
class BPResult:
    z: np.ndarray                                # [n_nodes] BP <Z_v>
    residual: float                              # largest Frobenius change of a message, last iteration
    messages: Dict[Tuple[int, int], np.ndarray]  # (edge, to_vertex) -> m_{other -> to_vertex}


def run(peps: PEPS, iters: int) -> BPResult:
    """`iters` parallel BP iterations from identity messages, then the BP readout."""
    a = symmetric_tensors(peps)
    msgs: Dict[Tuple[int, int], np.ndarray] = {}
    for e, (u, v) in enumerate(peps.edges):
        d = peps.lambdas[e].shape[0]
        for w in (int(u), int(v)):
            msgs[(e, w)] = np.eye(d, dtype=np.complex128) / d
    residual = 0.0
    for _ in range(iters):
        new = {}
        residual = 0.0
        for e, (u, v) in enumerate(peps.edges):
            for src, dst in ((int(u), int(v)), (int(v), int(u))):
                legs = peps.incident[src]
                into = [msgs[(f, src)] for f in legs]
                m = _close_legs(a[src], into, legs.index(e))
                m = m / np.trace(m).real
                residual = max(residual, float(np.linalg.norm(m - msgs[(e, dst)])))
                new[(e, dst)] = m
        msgs = new
    z = np.empty(peps.n_nodes)
    for v in range(peps.n_nodes):
        rho = _close_legs(a[v], [msgs[(f, v)] for f in peps.incident[v]], -1)
        z[v] = float((rho[0, 0].real - rho[1, 1].real) / (rho[0, 0].real + rho[1, 1].real))
    return BPResult(z=z, residual=residual, messages=msgs)
