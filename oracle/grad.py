"""FP64 CPU oracle of the gradient d<M>/d(theta_h, theta_J) of the simple-update evolution.

TEST INFRASTRUCTURE ONLY (imported by tests and the benchmark's CPU-baseline leg).

Loss: L = (1/m) sum_v <Z_v> after the last Trotter step, the average magnetisation of
Fig. 2a, with the state evolved by the simple update of oracle.su (Eq. 2-3; Method
section).  The gradient is a hand-written reverse sweep with per-step checkpoints:
the forward pass stores the state at the start of every step; the backward pass
restores each step's checkpoint, re-runs that step while recording every gate's
inputs, and walks the gates back in reverse colour-class order, then the RX layer.

Per gate the reverse sweep differentiates the two-site formulation that the QR
reduction of oracle.su only makes cheaper: Phi[(a,s),(t,b)] = g(s,t) sum_k
A_i[a,(s,k)] lambda_k A_j[b,(t,k)] with A = Gamma times the other legs' lambdas,
Phi = U S V^H, lambda_e' = S[:chi]/||S[:chi]||, Gamma_i' = U[:, :chi] / w_i,
Gamma_j' = V^H[:chi] / w_j.  (The QR step changes neither the singular values nor
the new tensors, so this is the same function of the inputs.)  The complex SVD
adjoint, with J = U^H dU-bar, K = V^H dV-bar over all r = min(m, n) singular triplets:

  A-bar = U [ (F o (J - J^H)) S + S (F o (K - K^H)) + diag(S-bar)
              + i diag(Im J_kk - Im K_kk) / (2 s_k) ] V^H
          + (I - U U^H) U-bar S^-1 V^H + U S^-1 V-bar^H (I - V V^H)

with F_kl = 1/(s_l^2 - s_k^2) = 1/((s_l - s_k)(s_l + s_k)) broadened on the difference of
singular values: F_kl = d/(d^2 + eps_F) / (s_l + s_k), d = s_l - s_k, both in units of s_0
(the Lorentzian of Liao et al., PRX 9, 031041, 2019), eps_F = 1e-12, and F_kl = 0 when both
values are zero.  Broadening the difference of squares instead biased dL/dtheta by ~1e-4
relative at D = 16, 20 steps.  U-bar and V-bar vanish on the
discarded triplets, so 1/s only meets kept values s_k > eps * s_0 and is used exactly.
The truncation rank chi is held fixed (the loss is piecewise smooth in the angles).
Complex adjoints follow x-bar = dL/dRe x + i dL/dIm x.
"""

from __future__ import annotations

import copy
import dataclasses
import math
from typing import List

import numpy as np

from . import su


def _gate_and_derivative(theta_j: float):
    zz = np.outer(su.Z_SIGN, su.Z_SIGN)
    g = np.exp(-0.5j * theta_j * zz)
    return g, -0.5j * zz * g


def _rx_and_derivative(theta_h: float):
    m = su.rx_matrix(theta_h)
    x = np.array([[0.0, 1.0], [1.0, 0.0]], dtype=np.complex128)
    return m, -0.5j * x @ m


@dataclasses.dataclass
class _GateRecord:
    e: int
    i: int
    j: int
    gam_i: np.ndarray
    gam_j: np.ndarray
    lam_e: np.ndarray
    oth_i: list
    oth_j: list
    dims_i: list
    dims_j: list
    w_i: np.ndarray   # [M_i] product of the other legs' lambdas
    w_j: np.ndarray
    a_i: np.ndarray   # [M_i, 2, de] raw Gamma_i rows (without w)
    a_j: np.ndarray   # [M_j, 2, de]
    u: np.ndarray     # [2 M_i, r]
    s: np.ndarray     # [r]
    vh: np.ndarray    # [r, 2 M_j]
    chi: int
    new_i: np.ndarray  # [M_i, 2, chi]  Gamma_i' rows
    new_j: np.ndarray  # [M_j, 2, chi]


def _rows(peps: su.PEPS, v: int, e: int, gam: np.ndarray):
    """Gamma_v as [M, 2, d_e] with rows over the other legs (ascending id) and w over rows."""
    legs = peps.incident[v]
    others = [f for f in legs if f != e]
    order = [1 + legs.index(f) for f in others] + [0, 1 + legs.index(e)]
    t = np.transpose(gam, order)
    dims = [peps.lambdas[f].shape[0] for f in others]
    m = int(np.prod(dims)) if dims else 1
    w = np.ones(m)
    if others:
        w = peps.lambdas[others[0]].copy()
        for f in others[1:]:
            w = np.outer(w, peps.lambdas[f]).reshape(-1)
    return t.reshape(m, 2, gam.shape[1 + legs.index(e)]), others, dims, w


def _unrows(peps: su.PEPS, v: int, e: int, x: np.ndarray, others, dims) -> np.ndarray:
    """Inverse of _rows for an array [M, 2, d] -> tensor with legs in ascending order."""
    legs = peps.incident[v]
    t = x.reshape(tuple(dims) + (2, x.shape[2]))
    cur = others + ["s", e]
    target = ["s"] + legs
    return np.transpose(t, [cur.index(lbl) for lbl in target]).copy()


def _gate_forward(peps: su.PEPS, e: int, theta_j: float, d_max: int, eps: float) -> _GateRecord:
    """One simple-update gate in the two-site formulation, recording what the adjoint needs."""
    i, j = int(peps.edges[e, 0]), int(peps.edges[e, 1])
    g, _ = _gate_and_derivative(theta_j)
    lam = peps.lambdas[e].copy()
    a_i, oth_i, dims_i, w_i = _rows(peps, i, e, peps.gammas[i])
    a_j, oth_j, dims_j, w_j = _rows(peps, j, e, peps.gammas[j])
    mi, mj = a_i.shape[0], a_j.shape[0]
    ai = a_i * w_i[:, None, None]
    aj = a_j * w_j[:, None, None]
    phi = np.einsum("ask,k,btk,st->astb", ai, lam, aj, g).reshape(2 * mi, 2 * mj)
    u, s, vh = np.linalg.svd(phi, full_matrices=False)
    keep = int(np.count_nonzero(s > eps * s[0]))
    chi = max(1, min(d_max, keep))
    new_i = u[:, :chi].reshape(mi, 2, chi) / w_i[:, None, None]
    new_j = vh[:chi, :].reshape(chi, 2, mj).transpose(2, 1, 0) / w_j[:, None, None]
    rec = _GateRecord(e, i, j, peps.gammas[i], peps.gammas[j], lam, oth_i, oth_j, dims_i, dims_j,
                      w_i, w_j, a_i, a_j, u, s, vh, chi, new_i, new_j)
    peps.lambdas[e] = s[:chi] / np.linalg.norm(s[:chi])
    peps.gammas[i] = _unrows(peps, i, e, new_i, oth_i, dims_i)
    peps.gammas[j] = _unrows(peps, j, e, new_j, oth_j, dims_j)
    return rec


def _svd_backward(u, s, vh, ubar, vbar, sbar, eps_f, broaden="difference"):
    """Reverse of the thin complex SVD A = U diag(s) V^H (all r triplets); returns A-bar.

    broaden = "difference": F_kl = d/(d^2 + eps_f)/(s_l + s_k), d = s_l - s_k (the reading used);
    broaden = "squares": F_kl = q/(q^2 + eps_f), q = s_l^2 - s_k^2 (the Lorentzian written on the
    squared differences), both with s in units of s_0.
    """
    v = vh.conj().T
    r = s.shape[0]
    s0 = s[0]
    sn = s / s0
    ds = sn[None, :] - sn[:, None]             # ds[k, l] = (s_l - s_k) / s0
    ss = sn[None, :] + sn[:, None]
    with np.errstate(divide="ignore", invalid="ignore"):
        if broaden == "squares":
            q = ds * ss
            f = q / (q * q + eps_f) / (s0 * s0)
        elif broaden == "difference":
            f = np.where(ss > 0.0, ds / (ds * ds + eps_f) / np.where(ss > 0.0, ss, 1.0), 0.0) / (s0 * s0)
        else:
            raise ValueError(f"unknown broadening {broaden!r}")
    np.fill_diagonal(f, 0.0)
    jm = u.conj().T @ ubar
    km = v.conj().T @ vbar
    inv = np.zeros(r)
    nz = ubar.any(axis=0) | vbar.any(axis=0) | (sbar != 0)
    inv[nz] = 1.0 / s[nz]                      # only kept triplets carry adjoints
    inner = (f * (jm - jm.conj().T)) * s[None, :] + s[:, None] * (f * (km - km.conj().T))
    inner = inner + np.diag(sbar + 0.5j * (np.imag(np.diag(jm)) - np.imag(np.diag(km))) * inv)
    abar = u @ inner @ vh
    abar += (ubar - u @ (u.conj().T @ ubar)) @ np.diag(inv) @ vh
    abar += u @ np.diag(inv) @ (vbar.conj().T - (vbar.conj().T @ v) @ vh)
    return abar


def _gate_backward(peps: su.PEPS, rec: _GateRecord, theta_j: float, adj_g: List[np.ndarray],
                   adj_l: List[np.ndarray], eps_f: float, broaden: str = "difference") -> float:
    """Reverse of one gate.  adj_g / adj_l hold the adjoints of the post-gate state on entry and
    of the pre-gate state on exit.  Returns the contribution to dL/dtheta_J."""
    e, i, j, chi = rec.e, rec.i, rec.j, rec.chi
    g, dg = _gate_and_derivative(theta_j)
    mi, mj = rec.a_i.shape[0], rec.a_j.shape[0]
    # adjoints of the post-gate tensors as row arrays (the state still has the post-gate shapes)
    gbar_i, _, _, _ = _rows(peps, i, e, adj_g[i])
    gbar_j, _, _, _ = _rows(peps, j, e, adj_g[j])
    wbar_i = -np.real(np.sum(np.conj(gbar_i) * rec.new_i, axis=(1, 2))) / rec.w_i
    wbar_j = -np.real(np.sum(np.conj(gbar_j) * rec.new_j, axis=(1, 2))) / rec.w_j
    r = rec.s.shape[0]
    ubar = np.zeros((2 * mi, r), dtype=np.complex128)
    vbar = np.zeros((2 * mj, r), dtype=np.complex128)
    ubar[:, :chi] = (gbar_i / rec.w_i[:, None, None]).reshape(2 * mi, chi)
    # Gamma_j'[b, t, k] = conj(V[(t, b), k]) / w_j[b]
    vbar[:, :chi] = np.conj(gbar_j / rec.w_j[:, None, None]).transpose(1, 0, 2).reshape(2 * mj, chi)
    # lambda_e' = s[:chi] / ||s[:chi]||
    sk = rec.s[:chi]
    nrm = np.linalg.norm(sk)
    lbar = adj_l[e]
    sbar = np.zeros(r)
    sbar[:chi] = lbar / nrm - sk * float(np.dot(lbar, sk)) / nrm ** 3
    phibar = _svd_backward(rec.u, rec.s, rec.vh, ubar, vbar, sbar, eps_f, broaden).reshape(mi, 2, 2, mj)
    ai = rec.a_i * rec.w_i[:, None, None]
    aj = rec.a_j * rec.w_j[:, None, None]
    lam = rec.lam_e
    # Phi[a,s,t,b] = g(s,t) sum_k ai[a,s,k] lam_k aj[b,t,k]
    abar_i = np.einsum("astb,st,k,btk->ask", phibar, np.conj(g), lam, np.conj(aj))
    abar_j = np.einsum("astb,st,k,ask->btk", phibar, np.conj(g), lam, np.conj(ai))
    lambar_e = np.real(np.einsum("astb,st,ask,btk->k", np.conj(phibar), g, ai, aj))
    dtheta_j = float(np.real(np.einsum("astb,st,ask,k,btk->", np.conj(phibar), dg, ai, lam, aj)))
    # A = Gamma rows * w
    wbar_i = wbar_i + np.real(np.sum(np.conj(abar_i) * rec.a_i, axis=(1, 2)))
    wbar_j = wbar_j + np.real(np.sum(np.conj(abar_j) * rec.a_j, axis=(1, 2)))
    gpre_i = abar_i * rec.w_i[:, None, None]
    gpre_j = abar_j * rec.w_j[:, None, None]
    # restore the pre-gate shapes before writing the pre-gate adjoints
    peps.gammas[i], peps.gammas[j] = rec.gam_i, rec.gam_j
    peps.lambdas[e] = lam
    adj_g[i] = _unrows(peps, i, e, gpre_i, rec.oth_i, rec.dims_i)
    adj_g[j] = _unrows(peps, j, e, gpre_j, rec.oth_j, rec.dims_j)
    adj_l[e] = lambar_e
    # w = product of the other legs' lambdas
    for wbar, oth, dims in ((wbar_i, rec.oth_i, rec.dims_i), (wbar_j, rec.oth_j, rec.dims_j)):
        if not oth:
            continue
        full = wbar.reshape(dims)
        lams = [peps.lambdas[f] for f in oth]
        for k, f in enumerate(oth):
            other = np.ones(dims)
            for k2, f2 in enumerate(oth):
                if k2 != k:
                    shape = [1] * len(dims)
                    shape[k2] = dims[k2]
                    other = other * lams[k2].reshape(shape)
            axes = tuple(a for a in range(len(dims)) if a != k)
            adj_l[f] = adj_l[f] + np.sum(full * other, axis=axes) if axes else adj_l[f] + full * other
    return dtheta_j


def _readout_adjoint(peps: su.PEPS, weights: np.ndarray):
    """Adjoints of L = sum_v weights[v] z_v with respect to every Gamma_v and lambda_e."""
    adj_g = []
    adj_l = [np.zeros_like(lam) for lam in peps.lambdas]
    for v in range(peps.n_nodes):
        gam = peps.gammas[v]
        w = np.ones(gam.shape[1:])
        for k, f in enumerate(peps.incident[v]):
            shape = [1] * (gam.ndim - 1)
            shape[k] = peps.lambdas[f].shape[0]
            w = w * (peps.lambdas[f] ** 2).reshape(shape)
        p = np.abs(gam) ** 2
        r0 = float(np.sum(p[0] * w))
        r1 = float(np.sum(p[1] * w))
        den = (r0 + r1) ** 2
        d0 = weights[v] * 2.0 * r1 / den    # dL/drho00
        d1 = -weights[v] * 2.0 * r0 / den   # dL/drho11
        a = np.empty_like(gam)
        a[0] = 2.0 * d0 * gam[0] * w
        a[1] = 2.0 * d1 * gam[1] * w
        adj_g.append(a)
        q = d0 * p[0] + d1 * p[1]          # dL/dW(x) with W = prod_l lambda_l^2
        for k, f in enumerate(peps.incident[v]):
            lamf = peps.lambdas[f]
            axes = tuple(ax for ax in range(gam.ndim - 1) if ax != k)
            tot = np.sum(q * w, axis=axes) if axes else q * w
            adj_l[f] = adj_l[f] + tot * 2.0 / lamf
    return adj_g, adj_l


@dataclasses.dataclass
class GradResult:
    loss: float
    dtheta_h: float
    dtheta_j: float
    z: np.ndarray  # <Z_v> after the last step


def loss_and_grad(n_nodes: int, edges: np.ndarray, colour: np.ndarray, theta_h: float, theta_j: float,
                  d_max: int, steps: int, eps: float = 1e-12, eps_f: float = 1e-12,
                  broaden: str = "difference") -> GradResult:
    """Mean <Z> after `steps` steps and its derivatives by the hand-written reverse sweep.

    broaden selects the Lorentzian of the SVD backward (see _svd_backward)."""
    edges = np.asarray(edges)
    colour = np.asarray(colour)
    n_col = int(colour.max()) + 1 if len(colour) else 0
    classes = [[int(e) for e in np.nonzero(colour == c)[0]] for c in range(n_col)]
    peps = su.product_state(n_nodes, edges)
    checkpoints = []
    for _ in range(steps):
        checkpoints.append(copy.deepcopy((peps.gammas, peps.lambdas)))
        su.apply_rx_layer(peps, theta_h)
        for cls in classes:
            for e in cls:
                _gate_forward(peps, e, theta_j, d_max, eps)
    z = su.site_z(peps)
    loss = float(np.mean(z))
    adj_g, adj_l = _readout_adjoint(peps, np.full(n_nodes, 1.0 / n_nodes))
    rx, drx = _rx_and_derivative(theta_h)
    dth, dtj = 0.0, 0.0
    for t in reversed(range(steps)):
        gam0, lam0 = copy.deepcopy(checkpoints[t])
        peps.gammas, peps.lambdas = gam0, lam0
        pre_rx = [x.copy() for x in peps.gammas]
        su.apply_rx_layer(peps, theta_h)
        recs = []
        for cls in classes:
            for e in cls:
                recs.append(_gate_forward(peps, e, theta_j, d_max, eps))
        for rec in reversed(recs):
            dtj += _gate_backward(peps, rec, theta_j, adj_g, adj_l, eps_f, broaden)
        # RX layer: Gamma' = RX Gamma on the physical index
        for v in range(n_nodes):
            dth += float(np.real(np.sum(np.conj(adj_g[v]) * np.tensordot(drx, pre_rx[v], axes=([1], [0])))))
            adj_g[v] = np.tensordot(rx.conj().T, adj_g[v], axes=([1], [0]))
        peps.gammas = pre_rx
    return GradResult(loss=loss, dtheta_h=dth, dtheta_j=dtj, z=z)


def loss_and_grad_graph(graph, theta_h, theta_j, d_max, steps, eps=1e-12, eps_f=1e-12,
                        broaden="difference") -> GradResult:
    return loss_and_grad(graph.n_nodes, graph.edges, graph.colour, theta_h, theta_j, d_max, steps, eps, eps_f,
                         broaden)


def mean_z(graph, theta_h, theta_j, d_max, steps, eps=1e-12) -> float:
    """The loss alone, from the simple-update oracle (used for finite differences)."""
    return float(np.mean(su.evolve_graph(graph, theta_h, theta_j, d_max, steps, eps).z[-1]))
