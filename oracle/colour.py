"""Colour classes for the Gauss-Seidel smoother.

The paper smooths with Gauss-Seidel (Section 5; and the scaling study's V(2,2) cycles) but
does not fix an ordering.  The reading taken here: a forward sweep that first updates every
node interior to a macro element, colour class by colour class, and then every node on the
macro vertices/edges/faces (the interface), again class by class.  Every colour class is an
independent set of the fine-mesh graph, so updating a class simultaneously equals updating
its nodes one after the other.

Colours:
* interior nodes, red-black rule: parity of the sum of the node's integer grid coordinates
  (coordinates times 2^(p+l), 2^p the smallest power of two making every macro vertex
  integral); classes 0 and 1.  Exact Gauss-Seidel only on meshes whose off-axis couplings
  vanish (right-isosceles triangles, Kuhn tetrahedra); ``is_proper_for`` checks that.
* interior nodes, multicolour rule: with integer barycentrics (c_0..c_d) in the macro's vertex
  order, (c_1 + 2 c_2) mod 3 in 2D and (c_1 + 2 c_2 + 3 c_3) mod 4 in 3D; classes 0..C-1.
* interface nodes come after all interior classes.
  - 3D: red-black gives C + parity; multicolour colours them greedily, first fit, in
    canonical DoF order, avoiding already coloured interface neighbours, and numbers those
    classes from C on.
  - 2D (both Gauss-Seidel smoothers): a node interior to a macro edge at lattice distance a
    from the edge's lower-id vertex, with 2 <= a <= n - 2, gets class C + (a mod 2): the
    points of every edge alternate between two classes, and no point of one edge with
    2 <= a <= n - 2 touches another edge.  The remaining interface nodes (macro vertices and
    the edge points next to them, a = 1 and a = n - 1) follow in classes from C + 2 on:
    red-black C + 2 + parity, multicolour greedy first fit in canonical order among these
    nodes.  (Ordering the two edge classes before the vertex neighbourhoods lets one
    wavefront sweep both classes of an edge segment without waiting on any other.)
Nodes on the Dirichlet boundary are never updated and get colour -1.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _dyadic_power(coords: np.ndarray) -> int:
    for p in range(0, 40):
        s = coords * (2.0 ** p)
        if np.all(s == np.round(s)):
            return p
    raise ValueError("coarse coordinates are not dyadic")


def _interior_mask(h, l):
    return (h.levels[l].node_bary > 0).sum(axis=1) == h.d + 1


def edge_position_2d(h, l: int) -> np.ndarray:
    """2D: for every node of level l interior to a macro edge, its lattice distance a from the
    edge's lower-id vertex (the barycentric weight of the higher-id vertex); -1 elsewhere."""
    lv = h.levels[l]
    gv = h.coarse_cells[lv.node_macro]
    bary = lv.node_bary
    on_edge = (bary > 0).sum(axis=1) == 2
    pos = np.full(lv.n, -1, dtype=np.int64)
    for i in np.nonzero(on_edge)[0]:
        sup = np.nonzero(bary[i] > 0)[0]
        vs, cs = gv[i][sup], bary[i][sup]
        pos[i] = cs[int(np.argmax(vs))]
    return pos


def _edge_classes_2d(h, l: int, C: int):
    """2D interface split: class C + (a mod 2) for edge points with 2 <= a <= n - 2; returns
    the colours and the mask of the remaining interface nodes (vertex neighbourhoods)."""
    lv = h.levels[l]
    n = 2 ** l
    inner = _interior_mask(h, l)
    a = edge_position_2d(h, l)
    col = np.full(lv.n, -1, dtype=np.int64)
    edge = (a >= 2) & (a <= n - 2) & ~lv.boundary
    col[edge] = C + a[edge] % 2
    rest = ~inner & ~edge & ~lv.boundary
    return col, rest


def red_black(h, l: int) -> np.ndarray:
    lv = h.levels[l]
    p = _dyadic_power(h.coarse_coords)
    ic = np.round(lv.X * (2.0 ** (p + l))).astype(np.int64)
    par = (ic.sum(axis=1) % 2).astype(np.int64)
    inner = _interior_mask(h, l)
    if h.d == 2:
        col, rest = _edge_classes_2d(h, l, 2)
        col[inner] = par[inner]
        col[rest] = 4 + par[rest]
    else:
        col = par.copy()
        col[~inner] += 2
    col[lv.boundary] = -1
    return col


def mesh_graph(lv) -> sp.csr_matrix:
    E = lv.E
    d1 = E.shape[1]
    r, c = [], []
    for i in range(d1):
        for j in range(d1):
            if i != j:
                r.append(E[:, i]); c.append(E[:, j])
    r = np.concatenate(r); c = np.concatenate(c)
    G = sp.coo_matrix((np.ones(r.size, dtype=np.int8), (r, c)), shape=(lv.n, lv.n)).tocsr()
    G.data[:] = 1
    return G


def multicolour(h, l: int) -> np.ndarray:
    lv = h.levels[l]
    d = h.d
    bary = lv.node_bary
    inner = _interior_mask(h, l)
    C = 3 if d == 2 else 4
    col = np.full(lv.n, -1, dtype=np.int64)
    if d == 2:
        ci = (bary[:, 1] + 2 * bary[:, 2]) % 3
    else:
        ci = (bary[:, 1] + 2 * bary[:, 2] + 3 * bary[:, 3]) % 4
    if d == 2:
        col, rest = _edge_classes_2d(h, l, C)
        first = C + 2
    else:
        rest = ~inner & ~lv.boundary
        first = C
    col[inner] = ci[inner]
    G = mesh_graph(lv)
    order = h.canonical_order(l)
    for i in order:
        if not rest[i]:
            continue
        nb = G.indices[G.indptr[i]:G.indptr[i + 1]]
        used = set(int(col[q]) for q in nb if rest[q] and col[q] >= 0)
        c = first
        while c in used:
            c += 1
        col[i] = c
    return col


def classes(col: np.ndarray) -> list[np.ndarray]:
    """Non-empty colour classes in sweep order."""
    C = int(col.max()) + 1 if col.size and col.max() >= 0 else 0
    out = [np.nonzero(col == c)[0] for c in range(C)]
    return [c for c in out if c.size]


def is_proper_for(col: np.ndarray, A: sp.csr_matrix, tol: float = 0.0) -> bool:
    """True if no two distinct nodes of the same colour are coupled by A (|A_ij| > tol)."""
    Acoo = A.tocoo()
    m = (Acoo.row != Acoo.col) & (np.abs(Acoo.data) > tol)
    r, c = Acoo.row[m], Acoo.col[m]
    same = (col[r] == col[c]) & (col[r] >= 0)
    return not bool(np.any(same))
