"""The FP64 oracle pinned to values fixed by the paper and by the mathematics.

Pins (each chosen so a plausible slip in the oracle fails at least one):
  * theta_h = 0: the state stays |0...0>, <Z_i> = 1 exactly (Eq. 2: RX(0) = I, RZZ diagonal);
  * theta_J = 0: free precession, <Z_i>_t = cos(t theta_h) (Eq. 2);
  * t = 1: <Z_i> = cos(theta_h) for any theta_J (ZZ commutes with Z_i);
  * symmetries of Eq. 2 that the simple update keeps exactly:
    theta_h -> -theta_h, (theta_h, theta_J) -> (-theta_h, -theta_J), theta_h -> pi - theta_h;
  * light-cone exactness: for t <= 5 the ball of radius t-1 on the heavy-hex lattice is a tree,
    so untruncated simple update with the mean-field readout is exact (Results A reports
    ~1e-15 at n = 5, chi = 32; Appendix C: no loops before the 5th neighbour);
  * brute-force state vectors on the 12-site ring and on loop-free graphs;
  * Clifford point theta_h = pi/2: <Z_i> = 0 while the bond is untruncated;
  * bond-rank bound: with D >= 2^t nothing is truncated, results do not depend on D;
  * weight-N observables (Appendix B): n inverse steps at the forward angle undo n forward
    steps exactly (<Z> = 1), and on a tree, <Z_q> after n inverse steps at pi/2 equals the
    state-vector expectation of the Pauli string U(pi/2)^n Z_q U(pi/2)^{dagger n}.
"""

import json
import math
import os

import numpy as np
import pytest

import oracle.su as su
from exactref import lightcone_z, pauli_expect, propagate_pauli, statevector, statevector_z
from heavyhex import eagle127, path, ring, tree_from_edges

TJ = -math.pi / 2
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def g127():
    return eagle127()


def test_theta_h_zero_is_exactly_one(g127):
    tr = su.evolve_graph(g127, 0.0, TJ, 4, 6)
    assert np.all(tr.z == 1.0)
    assert np.all(tr.bond_dims == 1)


def test_theta_j_zero_free_precession(g127):
    th = 0.37
    tr = su.evolve_graph(g127, th, 0.0, 4, 6)
    want = np.cos(th * np.arange(1, 7))[:, None]
    assert np.max(np.abs(tr.z - want)) < 1e-13


def test_first_step_is_cos_theta(g127):
    for th, tj in ((0.3, TJ), (1.1, 0.4), (2.0, -1.3)):
        tr = su.evolve_graph(g127, th, tj, 4, 1)
        assert np.max(np.abs(tr.z[0] - math.cos(th))) < 1e-14


@pytest.mark.parametrize("steps", [5])
def test_symmetries_under_truncation(g127, steps):
    th, tj, d = 0.61, TJ, 4
    base = su.evolve_graph(g127, th, tj, d, steps).z
    assert np.max(np.abs(su.evolve_graph(g127, -th, tj, d, steps).z - base)) < 1e-11
    assert np.max(np.abs(su.evolve_graph(g127, -th, -tj, d, steps).z - base)) < 1e-11
    flip = su.evolve_graph(g127, math.pi - th, tj, d, steps).z
    sign = (-1.0) ** np.arange(1, steps + 1)[:, None]
    assert np.max(np.abs(flip - sign * base)) < 1e-11


def test_lightcone_exact_all_sites_t4(g127):
    th = 0.7
    tr = su.evolve_graph(g127, th, TJ, 16, 4)
    for t in range(1, 5):
        ex = np.array([lightcone_z(g127.n_nodes, g127.edges, s, th, TJ, t) for s in range(g127.n_nodes)])
        assert np.max(np.abs(tr.z[t - 1] - ex)) < 1e-12, t


def test_lightcone_exact_t5_chi32(g127):
    """The paper's n = 5, chi = 32 accuracy claim (Results A), on sampled sites."""
    gold = json.load(open(os.path.join(GOLDEN, "paper_accuracy.json")))
    th = 0.9
    tr = su.evolve_graph(g127, th, TJ, gold["chi"], gold["n_steps"])
    for s in (62, 13, 58, 0, 14, 126):
        ex = lightcone_z(g127.n_nodes, g127.edges, s, th, TJ, 5)
        assert abs(tr.z[4, s] - ex) < 1e-12


def test_ring12_statevector():
    r = ring(12)
    sv = statevector_z(12, r.edges.tolist(), 0.5, TJ, 7)
    tr = su.evolve_graph(r, 0.5, TJ, 32, 7)
    # exact while the light cone is loop-free (ball radius t-1 < 6)
    assert np.max(np.abs(tr.z[:6] - sv[:6])) < 1e-12
    # the ring closes at t = 7: the lambda environment is no longer exact
    assert np.max(np.abs(tr.z[6] - sv[6])) > 1e-10


def test_ring12_d4_error_is_reported():
    """The 12-ring at D=4 truncates from t = 3; its error is a number, not a pin."""
    r = ring(12)
    sv = statevector_z(12, r.edges.tolist(), 0.5, TJ, 5)
    tr = su.evolve_graph(r, 0.5, TJ, 4, 5)
    err = np.max(np.abs(tr.z - sv), axis=1)
    assert np.all(err[:2] < 1e-12) and err[-1] < 1e-2


def test_loop_free_graphs_exact_all_steps():
    """Untruncated simple update is exact on trees for every t."""
    chain = path(10)
    sv = statevector_z(10, chain.edges.tolist(), 0.8, TJ, 9)
    tr = su.evolve_graph(chain, 0.8, TJ, 32, 9)
    assert np.max(np.abs(tr.z - sv)) < 1e-11
    # a heavy-hex-like tree: a degree-3 hub with three arms, one branched
    edges = [(0, 1), (1, 2), (2, 3), (0, 4), (4, 5), (0, 6), (6, 7), (7, 8), (7, 9), (9, 10)]
    t = tree_from_edges("tree11", 11, edges)
    sv = statevector_z(11, t.edges.tolist(), 1.1, TJ, 8)
    tr = su.evolve_graph(t, 1.1, TJ, 64, 8)
    assert np.max(np.abs(tr.z - sv)) < 1e-11


def test_clifford_point_zero(g127):
    tr = su.evolve_graph(g127, math.pi / 2, TJ, 8, 3)
    assert np.max(np.abs(tr.z)) < 1e-12
    r = ring(12)
    tr = su.evolve_graph(r, math.pi / 2, TJ, 64, 6)
    sv = statevector_z(12, r.edges.tolist(), math.pi / 2, TJ, 6)
    assert np.max(np.abs(sv)) < 1e-12 and np.max(np.abs(tr.z)) < 1e-12


def test_bond_dimension_independence(g127):
    a = su.evolve_graph(g127, 0.8, TJ, 16, 4)
    b = su.evolve_graph(g127, 0.8, TJ, 64, 4)
    assert np.max(np.abs(a.z - b.z)) < 1e-12
    # bond ranks never exceed 2^t (RZZ has operator-Schmidt rank 2); leaf bonds stay <= 2
    for t in range(4):
        assert b.bond_dims[t].max() <= 2 ** (t + 1)
    leaf = [e for e, (u, v) in enumerate(g127.edges) if min(g127.degrees()[u], g127.degrees()[v]) == 1]
    assert b.bond_dims[:, leaf].max() <= 2


# ----- planted mistakes: each must break a pin above -----------------------------------------

def _lightcone_error(g, fn_patch, monkeypatch, t=4, th=0.7):
    with monkeypatch.context() as m:
        fn_patch(m)
        tr = su.evolve_graph(g, th, TJ, 16, t)
    sites = (62, 13, 58, 0)
    return max(abs(tr.z[t - 1, s] - lightcone_z(g.n_nodes, g.edges, s, th, TJ, t)) for s in sites)


def test_planted_mistake_no_environment(g127, monkeypatch):
    orig = su._side_matrix

    def no_env(peps, v, e):
        saved = [lam.copy() for lam in peps.lambdas]
        for f in peps.incident[v]:
            if f != e:
                peps.lambdas[f] = np.ones_like(peps.lambdas[f])
        out = orig(peps, v, e)
        peps.lambdas[:] = saved
        return out
    assert _lightcone_error(g127, lambda m: m.setattr(su, "_side_matrix", no_env), monkeypatch) > 1e-4


def test_planted_mistake_no_inverse(g127, monkeypatch):
    orig = su._restore_site

    def keep_env(peps, v, e, x, others, other_dims, pos):
        saved = [lam.copy() for lam in peps.lambdas]
        for f in others:
            peps.lambdas[f] = np.ones_like(peps.lambdas[f])
        orig(peps, v, e, x, others, other_dims, pos)
        peps.lambdas[:] = saved
    assert _lightcone_error(g127, lambda m: m.setattr(su, "_restore_site", keep_env), monkeypatch) > 1e-4


def test_planted_mistake_conjugated_readout_weight(g127, monkeypatch):
    orig = su.site_z

    def lam_not_squared(peps):
        saved = [lam.copy() for lam in peps.lambdas]
        for f in range(len(peps.lambdas)):
            peps.lambdas[f] = np.sqrt(peps.lambdas[f])
        out = orig(peps)
        peps.lambdas[:] = saved
        return out
    assert _lightcone_error(g127, lambda m: m.setattr(su, "site_z", lam_not_squared), monkeypatch) > 1e-4


def test_planted_mistake_gate_on_wrong_pair(g127, monkeypatch):
    """A gate phase that is not z_s z_t (here z_s only) breaks the t = 2 light cone."""
    def bad_gate(theta_j):
        return np.exp(-0.5j * theta_j * np.outer(su.Z_SIGN, np.ones(2)))
    assert _lightcone_error(g127, lambda m: m.setattr(su, "rzz_diagonal", bad_gate), monkeypatch, t=2) > 1e-4


def test_planted_mistake_transposed_columns(g127, monkeypatch):
    """Site matrices with columns ordered (leg e, s) where (s, leg e) is assumed break the light cone."""
    orig = su._side_matrix

    def swapped(peps, v, e):
        a, others, dims, pos = orig(peps, v, e)
        de = peps.lambdas[e].shape[0]
        a = a.reshape(a.shape[0], 2, de).transpose(0, 2, 1).reshape(a.shape[0], 2 * de)
        return a, others, dims, pos
    assert _lightcone_error(g127, lambda m: m.setattr(su, "_side_matrix", swapped), monkeypatch, t=3) > 1e-4


def test_layer_order_and_ry_are_unobservable(g127, monkeypatch):
    """Two changes that <Z> cannot see, recorded so nobody mistakes them for missing pins:
    RY differs from RX by diag(1, i), which commutes with Z and ZZ; and the last ZZ layer
    commutes with every Z_i, so applying ZZ before RX in each step leaves <Z> unchanged."""
    a = su.evolve_graph(g127, 0.7, TJ, 16, 3).z
    with monkeypatch.context() as m:
        m.setattr(su, "rx_matrix", lambda th: np.array([[math.cos(th / 2), -math.sin(th / 2)],
                                                         [math.sin(th / 2), math.cos(th / 2)]],
                                                        dtype=np.complex128))
        b = su.evolve_graph(g127, 0.7, TJ, 16, 3).z
    assert np.max(np.abs(a - b)) < 1e-12

    def zz_first(peps, classes, theta_h, theta_j, d_max, eps):
        recs = [su.simple_update_edge(peps, e, theta_j, d_max, eps) for cls in classes for e in cls]
        su.apply_rx_layer(peps, theta_h)
        return recs
    with monkeypatch.context() as m:
        m.setattr(su, "trotter_step", zz_first)
        c = su.evolve_graph(g127, 0.7, TJ, 16, 3).z
    assert np.max(np.abs(a - c)) < 1e-12


TREE11 = [(0, 1), (1, 2), (2, 3), (0, 4), (4, 5), (0, 6), (6, 7), (7, 8), (7, 9), (9, 10)]


def _inverse_identity_error(g127):
    tr = su.evolve_graph(g127, 0.9, TJ, 16, 3, inverse_steps=3, theta_h_inverse=0.9)
    assert np.max(tr.discarded[:3]) < 1e-20  # bonds <= 8: the forward steps truncate nothing
    return float(np.max(np.abs(tr.z[-1] - 1.0)))


def _weight_tree_error(steps):
    t = tree_from_edges("tree11", 11, TREE11)
    psi = statevector(11, t.edges.tolist(), 1.1, TJ, steps)
    tr = su.evolve_graph(t, 1.1, TJ, 64, steps, inverse_steps=steps)
    err = 0.0
    for q in range(11):
        w = pauli_expect(psi, 11, *propagate_pauli(t.edges, {q: "Z"}, steps))
        assert abs(w.imag) < 1e-12
        err = max(err, abs(w.real - tr.z[-1][q]))
    return err


def test_inverse_steps_undo_forward_steps(g127):
    """U(theta)^{dagger 3} U(theta)^3 = 1 on the 127-qubit lattice: the state returns to |0...0>."""
    assert _inverse_identity_error(g127) < 1e-12


@pytest.mark.parametrize("steps", [1, 2, 3, 4])
def test_weight_observable_tree_exact(steps):
    """<omega| Z_q |omega> = <psi| U^n Z_q U^{dagger n} |psi> (Appendix B) on a tree, every q."""
    assert _weight_tree_error(steps) < 1e-10


def test_planted_mistake_inverse_layer_order_and_sign(g127, monkeypatch):
    """An inverse step with RX first, or with RZZ(+theta_J), breaks both Appendix B pins."""
    def rx_first(peps, classes, theta_h, theta_j, d_max, eps):
        su.apply_rx_layer(peps, -theta_h)
        return [su.simple_update_edge(peps, e, -theta_j, d_max, eps) for cls in classes for e in cls]

    def zz_sign(peps, classes, theta_h, theta_j, d_max, eps):
        recs = [su.simple_update_edge(peps, e, theta_j, d_max, eps) for cls in classes for e in cls]
        su.apply_rx_layer(peps, -theta_h)
        return recs
    for bad in (rx_first, zz_sign):
        with monkeypatch.context() as m:
            m.setattr(su, "inverse_trotter_step", bad)
            assert _inverse_identity_error(g127) > 0.1
            assert _weight_tree_error(3) > 0.1


@pytest.mark.parametrize("steps,d", [(4, 16), (5, 32)])
def test_cell10_equals_infinite_lattice_lightcone(steps, d):
    """The simple update on the 10-qubit periodic cell is exact for t <= 5 on the infinite
    lattice (girth 12: the cones are trees, Results A): <Z> of every cell qubit equals the
    brute-force light-cone value of a qubit of the same class deep inside the 1123-qubit patch."""
    from heavyhex import heavy_hex, heavy_hex_cell10
    cell = heavy_hex_cell10()
    big = heavy_hex(21, 43, False)
    co = big.coords
    # cell qubit -> (row, column) of a representative in the patch (row 10, columns 20..23)
    rep = {0: (20.0, 20.0), 1: (20.0, 21.0), 2: (20.0, 22.0), 3: (20.0, 23.0), 4: (21.0, 20.0),
           5: (22.0, 20.0), 6: (22.0, 21.0), 7: (22.0, 22.0), 8: (22.0, 23.0), 9: (19.0, 22.0)}
    tr = su.evolve_graph(cell, 0.9, TJ, d, steps, 1e-12)
    for q, (y, x) in rep.items():
        v = int(np.nonzero((co[:, 0] == y) & (co[:, 1] == x))[0][0])
        assert abs(tr.z[-1][q] - lightcone_z(big.n_nodes, big.edges, v, 0.9, TJ, steps)) < 1e-12, q



# ----- exact pin of one truncating gate (rows a6/a7) ----------------------------------------------
#
# On a tree, the untruncated simple update keeps the state in the Vidal gauge, so the two-site
# tensor of a gate on edge e, with the lambda environment absorbed, is the Schmidt decomposition of
# the post-gate state across the cut at e.  Keeping D values is then the best rank-D approximation
# across that cut, and the mean-field <Z> of the two gate sites is their exact expectation in the
# normalised truncated state.  Edge (0, 6) of the 11-qubit tree joins two degree-3 ends, so both
# QR reductions run.

SCHMIDT_EDGE, SCHMIDT_STEPS, SCHMIDT_TH = (0, 6), 3, 0.9


def _schmidt_oracle(d_keep, plant=None):
    """The oracle: 3 untruncated steps, the next RX layer, then one gate on (0, 6) kept to D.
    plant() (tests of planted mistakes) runs just before that gate."""
    t = tree_from_edges("tree11", 11, TREE11)
    e = t.edges.tolist().index(list(SCHMIDT_EDGE))
    tr = su.evolve_graph(t, SCHMIDT_TH, TJ, 64, SCHMIDT_STEPS, keep_state=True)
    peps = tr.peps
    su.apply_rx_layer(peps, SCHMIDT_TH)
    if plant is not None:
        plant()
    su.simple_update_edge(peps, e, TJ, d_keep, 1e-12)
    z = su.site_z(peps)
    i, j = SCHMIDT_EDGE
    return peps.lambdas[e], z[i], z[j]


def _schmidt_reference(d_keep):
    """The same circuit on 2^11 amplitudes, cut at (0, 6) by a numpy SVD: (normalised top-D
    Schmidt values, <Z_i>, <Z_j> of the normalised truncated state, relative gap at the cut)."""
    t = tree_from_edges("tree11", 11, TREE11)
    edges = [tuple(x) for x in t.edges.tolist()]
    i, j = SCHMIDT_EDGE
    psi = statevector(11, edges, SCHMIDT_TH, TJ, SCHMIDT_STEPS).reshape((2,) * 11)
    c, sn = math.cos(SCHMIDT_TH / 2), math.sin(SCHMIDT_TH / 2)
    rx = np.array([[c, -1j * sn], [-1j * sn, c]])
    for q in range(11):
        psi = np.moveaxis(np.tensordot(rx, psi, axes=([1], [q])), 0, q)
    zz = np.array([[1.0, -1.0], [-1.0, 1.0]])
    phase = np.exp(-0.5j * TJ * zz).reshape((2, 2) + (1,) * 9)
    psi = np.moveaxis(np.moveaxis(psi, (i, j), (0, 1)) * phase, (0, 1), (i, j))
    # the component of i once edge (i, j) is removed
    side, todo = {i}, [i]
    while todo:
        x = todo.pop()
        for a, b in edges:
            if (a, b) == SCHMIDT_EDGE:
                continue
            y = b if a == x else a if b == x else None
            if y is not None and y not in side:
                side.add(y)
                todo.append(y)
    left = sorted(side)
    right = [q for q in range(11) if q not in side]
    mat = np.transpose(psi, left + right).reshape(2 ** len(left), 2 ** len(right))
    u, s, vh = np.linalg.svd(mat, full_matrices=False)
    kept = (u[:, :d_keep] * s[:d_keep]) @ vh[:d_keep]
    kept = np.transpose(kept.reshape((2,) * 11), np.argsort(left + right))
    p = np.abs(kept) ** 2 / np.sum(np.abs(kept) ** 2)
    zi = float(np.sum(p.take(0, axis=i)) - np.sum(p.take(1, axis=i)))
    zj = float(np.sum(p.take(0, axis=j)) - np.sum(p.take(1, axis=j)))
    return s[:d_keep] / np.linalg.norm(s[:d_keep]), zi, zj, float((s[d_keep - 1] - s[d_keep]) / s[0])


def _schmidt_error(d_keep, plant=None):
    lam_ref, ri, rj, gap = _schmidt_reference(d_keep)  # before any planted change
    lam, zi, zj = _schmidt_oracle(d_keep, plant)
    assert gap > 1e-4  # the kept set is unique
    lam_err = float(np.max(np.abs(lam - lam_ref))) if lam.shape == lam_ref.shape else math.inf
    return max(lam_err, abs(zi - ri), abs(zj - rj)), abs(zi - ri) + abs(zj - rj)


@pytest.mark.parametrize("d_keep", [2, 3, 5])
def test_truncation_is_the_schmidt_truncation(d_keep):
    """Rows a6/a7 pinned exactly: lambda_e equals the top-D normalised Schmidt values across the
    cut, and <Z> at both gate sites equals the state vector's after projecting onto the top-D
    Schmidt vectors."""
    err, _ = _schmidt_error(d_keep)
    assert err < 1e-12


def test_planted_mistake_truncation_keeps_smallest(monkeypatch):
    """Nonzero singular values taken in ascending order (the D smallest kept) fail the pin."""
    real_svd = np.linalg.svd

    def ascending(a, full_matrices=True, **kw):
        u, s, vh = real_svd(a, full_matrices=full_matrices, **kw)
        n = int(np.count_nonzero(s > 1e-12 * s[0]))
        return u[:, :n][:, ::-1], s[:n][::-1], vh[:n][::-1]
    err, zerr = _schmidt_error(3, lambda: monkeypatch.setattr(su.np.linalg, "svd", ascending))
    assert err > 1e-3 and zerr > 1e-3


def test_planted_mistake_truncation_rank_off_by_one(monkeypatch):
    """chi = D - 1 fails the Schmidt pin in lambda and in <Z> of the gate sites."""
    real = su.kept_rank
    err, zerr = _schmidt_error(3, lambda: monkeypatch.setattr(
        su, "kept_rank", lambda s, d, eps: max(1, real(s, d, eps) - 1)))
    assert err > 1e-3 and zerr > 1e-4
