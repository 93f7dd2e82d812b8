"""Qubit graphs of the kicked-Ising workloads and their gate schedule.

Heavy-hexagon patches (Fig. 1 and the Method section of the paper): rows of
qubit chains joined by single "bridge" qubits, open boundaries.  Qubits are
labelled sequentially, left to right and top to bottom, starting at 0 (caption
of Fig. 2 and Appendix B); bridge qubits sit between the two rows they join,
so they are labelled after the upper row and before the lower one.

Construction used here (R rows of L columns):
  * row r holds qubits at columns x = 0..L-1; with ``trim`` the first row
    drops its last column and the last row drops its first column (this is
    the 127-qubit Eagle shape: row lengths 14, 15, 15, 15, 15, 15, 14);
  * the gap between rows g and g+1 holds one bridge qubit at every column
    x = 0 (mod 4) for even g and x = 2 (mod 4) for odd g, provided the column
    exists in both rows; alternating the offset keeps every degree <= 3 and
    the lattice a subdivided hexagonal lattice (every face has 12 qubits);
  * edges are the chain links of every row plus two links per bridge.

Edges are numbered in lexicographic order of (min endpoint, max endpoint).
The gate order inside one Trotter layer is fixed by a proper edge colouring
computed deterministically in that edge order (König / Kempe alternating-path
method for bipartite graphs): all gates of colour class 0 act first, then class
1, and so on.  The paper does not state an order; since truncation does not
commute between overlapping gates, the colouring is part of the workload and
both the oracle and the GPU path consume the same one.
"""

from __future__ import annotations

import dataclasses
from collections import deque
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class Graph:
    """An undirected simple qubit graph with a gate colouring.

    ``edges`` is an int32 array [n_edges, 2] with edges[e, 0] < edges[e, 1],
    sorted lexicographically; ``colour`` is an int32 array [n_edges] with
    values 0..n_colours-1 forming a proper edge colouring.
    """

    name: str
    n_nodes: int
    edges: np.ndarray
    colour: np.ndarray
    coords: Optional[np.ndarray] = None  # [n_nodes, 2] (row-ish y, column x), for layouts only

    @property
    def n_edges(self) -> int:
        return int(self.edges.shape[0])

    @property
    def n_colours(self) -> int:
        return int(self.colour.max()) + 1 if self.n_edges else 0

    def degrees(self) -> np.ndarray:
        deg = np.zeros(self.n_nodes, dtype=np.int64)
        for u, v in self.edges:
            deg[u] += 1
            deg[v] += 1
        return deg

    def incident_edges(self) -> List[List[int]]:
        """Incident edge ids of every vertex, in ascending edge id order."""
        inc: List[List[int]] = [[] for _ in range(self.n_nodes)]
        for e, (u, v) in enumerate(self.edges):
            inc[u].append(e)
            inc[v].append(e)
        return inc

    def adjacency(self) -> List[List[int]]:
        adj: List[List[int]] = [[] for _ in range(self.n_nodes)]
        for u, v in self.edges:
            adj[u].append(int(v))
            adj[v].append(int(u))
        return adj

    def colour_classes(self) -> List[List[int]]:
        """Edge ids of each colour class, ascending."""
        return [[int(e) for e in np.nonzero(self.colour == c)[0]] for c in range(self.n_colours)]


def _normalise_edges(edges: Sequence[Tuple[int, int]]) -> np.ndarray:
    seen = set()
    out = []
    for u, v in edges:
        u, v = int(u), int(v)
        if u == v:
            raise ValueError(f"self-loop at {u}")
        a, b = (u, v) if u < v else (v, u)
        if (a, b) in seen:
            raise ValueError(f"duplicate edge {(a, b)}")
        seen.add((a, b))
        out.append((a, b))
    out.sort()
    return np.asarray(out, dtype=np.int32).reshape(-1, 2)


def kempe_edge_colouring(n_nodes: int, edges: np.ndarray) -> np.ndarray:
    """Proper edge colouring with max-degree colours for a bipartite graph.

    Edges are coloured one at a time in the given order.  For edge (u, v) let
    a be the smallest colour free at u and b the smallest colour free at v.
    If a is also free at v the edge takes a; else if b is free at u it takes
    b; otherwise the a/b alternating path that starts at v with its a-edge is
    recoloured (a <-> b) -- in a bipartite graph that path cannot reach u --
    after which a is free at both ends.  Raises ValueError on a non-bipartite
    conflict (path reaching u).
    """
    n_e = int(edges.shape[0])
    deg = np.zeros(n_nodes, dtype=np.int64)
    for u, v in edges:
        deg[u] += 1
        deg[v] += 1
    k = int(deg.max()) if n_e else 0
    colour = -np.ones(n_e, dtype=np.int32)
    at: List[Dict[int, int]] = [dict() for _ in range(n_nodes)]

    def free(x: int) -> int:
        for c in range(k):
            if c not in at[x]:
                return c
        raise ValueError("no free colour (degree bound violated)")

    for e in range(n_e):
        u, v = int(edges[e, 0]), int(edges[e, 1])
        a = free(u)
        b = free(v)
        if a not in at[v]:
            c = a
        elif b not in at[u]:
            c = b
        else:
            # alternating a/b path from v, starting with v's a-edge
            path: List[int] = []
            x, cur = v, a
            while cur in at[x]:
                f = at[x][cur]
                path.append(f)
                p, q = int(edges[f, 0]), int(edges[f, 1])
                y = q if p == x else p
                if y == u:
                    raise ValueError("graph is not bipartite: Kempe path reached the other end")
                x = y
                cur = b if cur == a else a
            for f in path:
                p, q = int(edges[f, 0]), int(edges[f, 1])
                del at[p][int(colour[f])]
                del at[q][int(colour[f])]
            for f in path:
                p, q = int(edges[f, 0]), int(edges[f, 1])
                colour[f] = b if colour[f] == a else a
                at[p][int(colour[f])] = f
                at[q][int(colour[f])] = f
            c = a
        colour[e] = c
        at[u][c] = e
        at[v][c] = e
    return colour


def check_proper_colouring(n_nodes: int, edges: np.ndarray, colour: np.ndarray) -> bool:
    """True when no two edges sharing a vertex have the same colour."""
    used = [set() for _ in range(n_nodes)]
    for (u, v), c in zip(edges, colour):
        c = int(c)
        if c < 0 or c in used[u] or c in used[v]:
            return False
        used[u].add(c)
        used[v].add(c)
    return True


def _make(name: str, n_nodes: int, raw_edges, coords=None) -> Graph:
    edges = _normalise_edges(raw_edges)
    colour = kempe_edge_colouring(n_nodes, edges)
    return Graph(name=name, n_nodes=n_nodes, edges=edges, colour=colour, coords=coords)


def heavy_hex(rows: int, cols: int, trim: bool, name: Optional[str] = None) -> Graph:
    """Heavy-hexagon patch with ``rows`` qubit chains of ``cols`` columns.

    See the module docstring for the construction.  heavy_hex(7, 15, True) is
    the 127-qubit Eagle graph; heavy_hex(13, 27, False) has 435 qubits and
    heavy_hex(21, 43, False) has 1123 qubits.
    """
    if rows < 1 or cols < 1:
        raise ValueError("rows and cols must be positive")

    def row_cols(r: int) -> List[int]:
        xs = list(range(cols))
        if trim and rows > 1:
            if r == 0:
                xs = xs[:-1]
            if r == rows - 1:
                xs = xs[1:]
        return xs

    label: Dict[Tuple[str, int, int], int] = {}
    coords: List[Tuple[float, float]] = []
    nxt = 0
    for r in range(rows):
        for x in row_cols(r):
            label[("q", r, x)] = nxt
            coords.append((2.0 * r, float(x)))
            nxt += 1
        if r < rows - 1:
            off = 0 if r % 2 == 0 else 2
            upper, lower = set(row_cols(r)), set(row_cols(r + 1))
            for x in range(off, cols, 4):
                if x in upper and x in lower:
                    label[("b", r, x)] = nxt
                    coords.append((2.0 * r + 1.0, float(x)))
                    nxt += 1
    raw = []
    for r in range(rows):
        xs = row_cols(r)
        for x0, x1 in zip(xs[:-1], xs[1:]):
            raw.append((label[("q", r, x0)], label[("q", r, x1)]))
    for key, b in label.items():
        if key[0] != "b":
            continue
        _, r, x = key
        raw.append((label[("q", r, x)], b))
        raw.append((b, label[("q", r + 1, x)]))
    nm = name or f"heavyhex_{rows}x{cols}{'_trim' if trim else ''}"
    return _make(nm, nxt, raw, coords=np.asarray(coords))


def eagle127() -> Graph:
    """The 127-qubit heavy-hexagon graph (7 rows, 15 columns, trimmed corners)."""
    return heavy_hex(7, 15, True, name="eagle127")


def heavy_hex_cell10() -> Graph:
    """The infinite heavy-hexagon lattice as a 10-qubit periodic unit cell (Method and Results).

    The construction of heavy_hex repeats with period 4 in the column and 2 in the row (bridges at
    x = 0 (mod 4) below even rows, x = 2 (mod 4) below odd rows), so one period holds two rows of
    four chain qubits and two bridges.  Labels follow the finite patches (left to right, top to
    bottom, bridges between the rows they join):
        0 1 2 3      row 0 (x = 0..3), chain link 3-0 wraps around
        4            bridge below row 0 at x = 0, joins 0 and 5
        5 6 7 8      row 1, chain link 8-5 wraps around
        9            bridge below row 1 at x = 2, joins 7 and row 0's x = 2, i.e. qubit 2
    Qubits 0, 2, 5, 7 have degree 3 and the other six degree 2.  A graph PEPS on this cell with
    these wrapped links is the translation-invariant state on the infinite lattice: every gate
    sees the same neighbouring tensors and weights as its translates do.
    """
    raw = [(0, 1), (1, 2), (2, 3), (3, 0), (5, 6), (6, 7), (7, 8), (8, 5), (0, 4), (4, 5), (7, 9), (9, 2)]
    coords = np.array([(0.0, 0.0), (0.0, 1.0), (0.0, 2.0), (0.0, 3.0), (1.0, 0.0),
                       (2.0, 0.0), (2.0, 1.0), (2.0, 2.0), (2.0, 3.0), (3.0, 2.0)])
    return _make("heavyhex_cell10", 10, raw, coords=coords)


def ring(n: int) -> Graph:
    """An n-cycle: one heavy-hexagon face when n = 12."""
    return _make(f"ring{n}", n, [(i, (i + 1) % n) for i in range(n)])


def path(n: int) -> Graph:
    """An open chain of n qubits."""
    return _make(f"path{n}", n, [(i, i + 1) for i in range(n - 1)])


def tree_from_edges(name: str, n_nodes: int, edges: Sequence[Tuple[int, int]]) -> Graph:
    """A graph from an explicit edge list (used for small loop-free fragments)."""
    return _make(name, n_nodes, edges)


def bfs_ball(adj: List[List[int]], centre: int, radius: int) -> List[int]:
    """Vertices at graph distance <= radius from ``centre``, sorted."""
    dist = {centre: 0}
    dq = deque([centre])
    while dq:
        x = dq.popleft()
        if dist[x] == radius:
            continue
        for y in adj[x]:
            if y not in dist:
                dist[y] = dist[x] + 1
                dq.append(y)
    return sorted(dist)
