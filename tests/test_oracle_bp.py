"""The BP oracle pinned by brute-force state vectors and by the Vidal-gauge fixed point.

  * on a tree BP is exact after as many iterations as the diameter: its <Z> equals the
    state vector of the circuit, also after a random non-unitary change of gauge on every
    bond (which leaves the state unchanged but breaks the mean-field readout);
  * for the untruncated simple update on a tree (Vidal gauge) the fixed point is
    diag(lambda_e) / sum(lambda_e) on every directed edge;
  * a planted slip (lambda instead of sqrt(lambda) in the symmetric gauge) breaks the pins.
"""

import math

import numpy as np
import pytest

import oracle.bp as bp
import oracle.su as su
from exactref import statevector_z
from heavyhex import eagle127, tree_from_edges

TJ = -math.pi / 2
TREE11 = [(0, 1), (1, 2), (2, 3), (0, 4), (4, 5), (0, 6), (6, 7), (7, 8), (7, 9), (9, 10)]


def _tree_state(steps=4, theta_h=1.1):
    t = tree_from_edges("tree11", 11, TREE11)
    tr = su.evolve_graph(t, theta_h, TJ, 64, steps, keep_state=True)
    sv = statevector_z(11, t.edges.tolist(), theta_h, TJ, steps)[-1]
    return t, tr, sv


def _scrambled(peps, seed=3):
    """The same state with a random invertible X_e on every bond: A_u <- A_u X, A_w <- X^-1 A_w,
    carried as gammas with unit lambdas."""
    rng = np.random.default_rng(seed)
    a = bp.symmetric_tensors(peps)
    for e, (u, w) in enumerate(peps.edges):
        d = peps.lambdas[e].shape[0]
        x = np.eye(d) + 0.5 * (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d)))
        xi = np.linalg.inv(x)
        for v, m in ((int(u), x), (int(w), xi.T)):
            k = 1 + peps.incident[v].index(e)
            a[v] = np.moveaxis(np.tensordot(a[v], m, axes=([k], [0])), -1, k)
    lams = [np.ones(l.shape[0]) for l in peps.lambdas]
    return su.PEPS(peps.n_nodes, peps.edges, peps.incident, a, lams)


def test_bp_exact_on_tree():
    _, tr, sv = _tree_state()
    r = bp.run(tr.peps, 8)
    assert np.max(np.abs(r.z - sv)) < 1e-12
    assert r.residual < 1e-12


def test_bp_fixed_point_is_vidal_lambda():
    _, tr, _ = _tree_state()
    r = bp.run(tr.peps, 8)
    for (e, _), m in r.messages.items():
        lam = tr.peps.lambdas[e]
        assert np.max(np.abs(m - np.diag(lam / lam.sum()))) < 1e-12


def test_bp_gauge_invariant_on_tree():
    """A non-unitary gauge change leaves BP's readout exact and breaks the mean-field one."""
    _, tr, sv = _tree_state()
    sc = _scrambled(tr.peps)
    assert np.max(np.abs(bp.run(sc, 8).z - sv)) < 1e-10
    assert np.max(np.abs(su.site_z(sc) - sv)) > 1e-2


def test_bp_product_state():
    g = eagle127()
    r = bp.run(su.product_state(g.n_nodes, g.edges), 3)
    assert np.all(r.z == 1.0) and r.residual == 0.0


def test_planted_mistake_full_lambda(monkeypatch):
    _, tr, sv = _tree_state()

    def full_lambda(peps):
        out = []
        for v in range(peps.n_nodes):
            a = peps.gammas[v].copy()
            for k, e in enumerate(peps.incident[v]):
                shape = [1] * a.ndim
                shape[1 + k] = peps.lambdas[e].shape[0]
                a = a * peps.lambdas[e].reshape(shape)
            out.append(a)
        return out
    monkeypatch.setattr(bp, "symmetric_tensors", full_lambda)
    assert np.max(np.abs(bp.run(tr.peps, 8).z - sv)) > 1e-3


def _classes(g):
    return [[int(e) for e in np.nonzero(g.colour == c)[0]] for c in range(g.n_colours)]


def test_regauge_sweeps_reach_bp_fixed_point():
    """Identity-gate simple-update sweeps leave the state (its BP readout) unchanged and drive
    the mean-field readout onto the BP readout: their fixed point is BP's."""
    g = eagle127()
    tr = su.evolve_graph(g, 0.8, TJ, 16, 6, 1e-6, keep_state=True)
    p = tr.peps
    before = bp.run(p, 40).z
    assert np.max(np.abs(before - su.site_z(p))) > 1e-3
    for _ in range(20):
        su.regauge_sweep(p, _classes(g), 16, 1e-6)
    after = bp.run(p, 40).z
    assert np.max(np.abs(after - before)) < 1e-11
    assert np.max(np.abs(su.site_z(p) - after)) < 1e-10


def test_regauge_restores_vidal_gauge_on_tree():
    """From a random non-unitary gauge on a tree, regauge sweeps make the mean-field readout exact."""
    t, tr, sv = _tree_state()
    sc = _scrambled(tr.peps)
    for _ in range(15):
        su.regauge_sweep(sc, _classes(t), 64, 1e-12)
    assert np.max(np.abs(su.site_z(sc) - sv)) < 1e-10
