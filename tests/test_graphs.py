"""Workload graphs: sizes, degrees, colouring, labelling (pinned by the paper's Appendix B)."""

import collections
import json
import os

import numpy as np

from heavyhex import bfs_ball, check_proper_colouring, eagle127, heavy_hex, make_workload, ring
from exactref import propagate_pauli

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _girth(g):
    adj = g.adjacency()
    best = 10 ** 9
    for s in range(g.n_nodes):
        dist = {s: 0}
        par = {s: -1}
        q = [s]
        for x in q:
            for y in adj[x]:
                if y not in dist:
                    dist[y] = dist[x] + 1
                    par[y] = x
                    q.append(y)
                elif par[x] != y:
                    best = min(best, dist[x] + dist[y] + 1)
    return best


def test_eagle127_structure():
    g = eagle127()
    assert g.n_nodes == 127 and g.n_edges == 144
    assert dict(collections.Counter(g.degrees().tolist())) == {1: 2, 2: 89, 3: 36}
    deg = g.degrees()
    types = collections.Counter(tuple(sorted((int(deg[u]), int(deg[v])))) for u, v in g.edges)
    assert types == {(2, 3): 106, (2, 2): 36, (1, 3): 2}
    assert check_proper_colouring(g.n_nodes, g.edges, g.colour)
    assert [len(c) for c in g.colour_classes()] == [54, 54, 36]
    assert _girth(g) == 12
    # 180-degree rotation i -> 126 - i is an automorphism of the labelled lattice
    es = {tuple(e) for e in g.edges.tolist()}
    assert {tuple(sorted((126 - u, 126 - v))) for u, v in es} == es


def test_edges_sorted_and_unique():
    g = eagle127()
    e = g.edges.tolist()
    assert e == sorted(e)
    assert all(u < v for u, v in e)
    assert len(set(map(tuple, e))) == len(e)


def test_large_patches():
    for (r, l), (n, m, cls) in {(13, 27): (435, 506, [181, 181, 144]),
                                (21, 43): (1123, 1322, [461, 461, 400])}.items():
        g = heavy_hex(r, l, False)
        assert (g.n_nodes, g.n_edges) == (n, m)
        assert g.degrees().max() == 3
        assert check_proper_colouring(g.n_nodes, g.edges, g.colour)
        assert [len(c) for c in g.colour_classes()] == cls


def test_ring12_two_colours():
    g = ring(12)
    assert g.n_edges == 12 and g.n_colours == 2
    assert check_proper_colouring(g.n_nodes, g.edges, g.colour)


def test_bfs_ball_sizes():
    # largest light-cone balls on the 127 lattice, radius 1..5
    g = eagle127()
    adj = g.adjacency()
    sizes = [max(len(bfs_ball(adj, s, r)) for s in range(g.n_nodes)) for r in range(1, 6)]
    assert sizes == [4, 7, 13, 19, 31]


def test_appendix_b_weight_operators():
    """Z_13 and Z_58 pushed through five Clifford steps give the paper's W10 and W17."""
    gold = json.load(open(os.path.join(GOLDEN, "appendix_b_weight_operators.json")))
    g = eagle127()
    for key, sign in (("W10", 1), ("W17", -1)):
        w = gold[key]
        phase, ops = propagate_pauli(g.edges, {w["q"]: "Z"}, 5)
        got = {p: sorted(q for q, x in ops.items() if x == p) for p in "XYZ"}
        assert got == {p: w[p] for p in "XYZ"}
        # the paper prints no sign; the propagated operator carries +1 (W10) and -1 (W17)
        assert phase == sign


def test_opposite_orientation_does_not_match():
    """U^dag Z U (the other conjugation order) gives different operators: the orientation is pinned."""
    gold = json.load(open(os.path.join(GOLDEN, "appendix_b_weight_operators.json")))
    g = eagle127()
    # reversing the roles: conjugate by U^dag = RX^dag . ZZ^dag, i.e. the ZZ layer first
    from exactref import _mul
    phase, cur = 1, {13: "Z"}
    for _ in range(5):
        for u, v in g.edges:
            anti = sum(1 for q in (int(u), int(v)) if cur.get(q, "I") in ("X", "Y")) % 2
            if anti:
                phase, cur = _mul(phase * (1j), cur, {int(u): "Z", int(v): "Z"})
        cur = {q: ("Y" if p == "Z" else "Z" if p == "Y" else p) for q, p in cur.items()}
    got = {p: sorted(q for q, x in cur.items() if x == p) for p in "XYZ"}
    assert got != {p: gold["W10"][p] for p in "XYZ"}


def test_workload_recipes():
    w = make_workload("eagle127_sweep_d32")
    assert len(w.instances) == 32
    assert w.instances[0].theta_h == 0.0 and abs(w.instances[-1].theta_h - np.pi / 2) < 1e-15
    assert w.edge_updates == 32 * 144 * 20
    m = make_workload("mixed_d32")
    assert [m.graphs[i.graph].n_nodes for i in m.instances] == [435, 1123] + [127] * 8
    assert sum(m.graphs[i.graph].n_edges for i in m.instances) == 2980
    ths = [i.theta_h for i in m.instances]
    assert np.allclose(ths, np.random.default_rng(0).uniform(0.1, 1.0, 10))
    assert make_workload("eagle127_d16").edge_updates == 2880
    s16 = make_workload("eagle127_sweep_d16")
    assert len(s16.instances) == 256 and s16.d_max == 16 and s16.edge_updates == 256 * 144 * 20
    assert s16.instances[0].theta_h == 0.0 and abs(s16.instances[-1].theta_h - np.pi / 2) < 1e-15
    g32 = make_workload("eagle127_grad_d32")
    assert g32.d_max == 32 and g32.steps == 20 and g32.instances[0].theta_h == 0.6


def _cell_label(big, v):
    """Unit-cell label of a vertex of a large patch: chain qubits by (row mod 2, column mod 4),
    bridges by the parity of the gap they sit in."""
    y, x = big.coords[v]
    if int(y) % 2 == 0:
        r = int(y) // 2
        return (r % 2) * 5 + int(x) % 4
    return 4 if (int(y) // 2) % 2 == 0 else 9


def test_cell10_is_the_quotient_of_the_lattice():
    """Every vertex of a large patch maps onto the 10-qubit cell, edges onto edges, and every
    vertex away from the boundary has the degree of its image: the cell with its wrapped links
    is the infinite heavy-hex lattice modulo its translations."""
    from heavyhex import heavy_hex_cell10
    cell = heavy_hex_cell10()
    assert cell.n_nodes == 10 and cell.n_edges == 12
    assert sorted(collections.Counter(cell.degrees().tolist()).items()) == [(2, 6), (3, 4)]
    assert check_proper_colouring(cell.n_nodes, cell.edges, cell.colour) and cell.n_colours == 3
    cell_edges = {tuple(e) for e in cell.edges.tolist()}
    big = heavy_hex(21, 43, False)
    hit = set()
    for u, v in big.edges.tolist():
        a, b = sorted((_cell_label(big, u), _cell_label(big, v)))
        assert (a, b) in cell_edges
        hit.add((a, b))
    assert hit == cell_edges
    deg = big.degrees()
    interior = [v for v in range(big.n_nodes) if 4 <= big.coords[v][0] <= 36 and 4 <= big.coords[v][1] <= 38]
    assert all(deg[v] == cell.degrees()[_cell_label(big, v)] for v in interior)


def test_cell10_weights_after_five_clifford_steps():
    """On the infinite lattice U(pi/2)^5 Z_q U(pi/2)^{dagger 5} has weight 19 on the degree-3
    qubits and 21 on the degree-2 qubits (an interior qubit of the 1123-qubit patch, whose
    five-step cone stays away from the boundary); qubit 2 of the cell (Table I's Q on the
    infinite lattice) is a degree-3 qubit."""
    from heavyhex import heavy_hex_cell10
    cell = heavy_hex_cell10()
    big = heavy_hex(21, 43, False)
    for q in range(10):
        v = next(v for v in range(big.n_nodes)
                 if _cell_label(big, v) == q and 18 <= big.coords[v][0] <= 23 and 18 <= big.coords[v][1] <= 23)
        _, ops = propagate_pauli(big.edges, {v: "Z"}, 5)
        assert len(ops) == (19 if cell.degrees()[q] == 3 else 21), q
    assert cell.degrees()[2] == 3
