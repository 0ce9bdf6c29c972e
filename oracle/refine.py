"""Uniform refinement of the macro mesh into the nested hierarchy T_0, ..., T_L (Section 2,
"Hybrid tetrahedral grids": the coarse triangulation is refined uniformly L times by Bey's
rule, giving nested meshes and therefore a geometric multigrid hierarchy).

Each level is a *global* unstructured mesh.  Refinement is done recursively element by
element, never through a lattice formula:
  2D: a triangle (x0,x1,x2) is split at its edge midpoints into (x0,x01,x02), (x01,x1,x12),
      (x02,x12,x2), (x01,x12,x02);
  3D: a tetrahedron (x0,x1,x2,x3) is split into Bey's eight children (x0,x01,x02,x03),
      (x01,x1,x12,x13), (x02,x12,x2,x23), (x03,x13,x23,x3), (x01,x02,x03,x13),
      (x01,x02,x12,x13), (x02,x03,x13,x23), (x02,x12,x13,x23).
Nodes of level l are the first N_l nodes of level l+1; every new node is the midpoint of one
edge of level l, recorded in ``parents`` (this is the refinement relation the prolongation
uses).

Each element also carries the integer barycentric coordinates of its vertices with respect
to the macro element it lies in (scaled by 2^l), so every node knows which macro primitive
(vertex, edge, face or volume) it belongs to and its integer position there.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# local edges of a simplex, in the order their midpoints are numbered (after the corners)
EDGES = {2: [(0, 1), (0, 2), (1, 2)],
         3: [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]}
# children in terms of local node numbers: corners 0..d, then one midpoint per EDGES entry
CHILDREN = {2: [(0, 3, 4), (3, 1, 5), (4, 5, 2), (3, 5, 4)],
            3: [(0, 4, 5, 6), (4, 1, 7, 8), (5, 7, 2, 9), (6, 8, 9, 3),
                (4, 5, 6, 8), (4, 5, 7, 8), (5, 6, 8, 9), (5, 7, 8, 9)]}


@dataclass
class MeshLevel:
    level: int
    X: np.ndarray              # (N, d) node coordinates
    E: np.ndarray              # (ne, d+1) element node ids
    emacro: np.ndarray         # (ne,) macro element of each element
    ebary: np.ndarray          # (ne, d+1, d+1) integer barycentrics of element vertices in its macro
    parents: np.ndarray | None = None   # (N_{l+1} - N_l, 2): endpoints of the edge whose midpoint is node N_l + i
    node_macro: np.ndarray = field(default=None)   # (N,) one macro containing the node
    node_bary: np.ndarray = field(default=None)    # (N, d+1) integer barycentrics in node_macro

    @property
    def n(self) -> int:
        return self.X.shape[0]


def _refine(lv: MeshLevel, d: int) -> tuple[MeshLevel, np.ndarray]:
    E = lv.E
    ne = E.shape[0]
    N = lv.X.shape[0]
    edges = EDGES[d]
    a = np.stack([E[:, i] for i, _ in edges], axis=1)
    b = np.stack([E[:, j] for _, j in edges], axis=1)
    lo = np.minimum(a, b).astype(np.int64)
    hi = np.maximum(a, b).astype(np.int64)
    key = lo * N + hi
    ukey, inv = np.unique(key.ravel(), return_inverse=True)
    inv = inv.reshape(key.shape)
    par = np.stack([ukey // N, ukey % N], axis=1)
    Xnew = 0.5 * (lv.X[par[:, 0]] + lv.X[par[:, 1]])
    X = np.concatenate([lv.X, Xnew], axis=0)
    local = np.concatenate([E.astype(np.int64), N + inv], axis=1)       # (ne, d+1+nedges)
    # barycentrics of the local nodes at the next level's scale
    bary_local = np.concatenate(
        [2 * lv.ebary] + [(lv.ebary[:, i] + lv.ebary[:, j])[:, None] for i, j in edges], axis=1)
    kids = CHILDREN[d]
    Ec = np.stack([local[:, list(c)] for c in kids], axis=1).reshape(-1, d + 1)
    Bc = np.stack([bary_local[:, list(c)] for c in kids], axis=1).reshape(-1, d + 1, d + 1)
    Mc = np.repeat(lv.emacro, len(kids))
    nxt = MeshLevel(lv.level + 1, X, Ec, Mc, Bc)
    return nxt, par


def _node_info(lv: MeshLevel, d: int):
    N = lv.X.shape[0]
    nm = np.empty(N, dtype=np.int64)
    nb = np.empty((N, d + 1), dtype=np.int64)
    for a in range(d + 1):
        nm[lv.E[:, a]] = lv.emacro
        nb[lv.E[:, a]] = lv.ebary[:, a, :]
    lv.node_macro, lv.node_bary = nm, nb


def boundary_nodes(lv: MeshLevel, d: int) -> np.ndarray:
    """Boolean mask of nodes on the domain boundary: vertices of facets that belong to exactly
    one element of this level."""
    E = lv.E
    facets = []
    for skip in range(d + 1):
        cols = [c for c in range(d + 1) if c != skip]
        facets.append(np.sort(E[:, cols], axis=1))
    F = np.concatenate(facets, axis=0).astype(np.int64)
    N = lv.X.shape[0]
    if d == 2:
        key = F[:, 0] * N + F[:, 1]
    else:
        key = (F[:, 0] * N + F[:, 1]) * N + F[:, 2]
    uk, idx, cnt = np.unique(key, return_index=True, return_counts=True)
    bf = F[idx[cnt == 1]]
    mask = np.zeros(N, dtype=bool)
    mask[bf.ravel()] = True
    return mask


class Hierarchy:
    """Nested meshes T_0..T_L of a macro mesh, plus per-node primitive information."""

    def __init__(self, coords, cells, L: int):
        coords = np.asarray(coords, dtype=np.float64)
        cells = np.asarray(cells, dtype=np.int64)
        self.d = d = coords.shape[1]
        self.L = L
        self.coarse_coords = coords
        self.coarse_cells = cells
        nc = cells.shape[0]
        eb = np.broadcast_to(np.eye(d + 1, dtype=np.int64), (nc, d + 1, d + 1)).copy()
        lv = MeshLevel(0, coords.copy(), cells.copy(), np.arange(nc), eb)
        self.levels = [lv]
        for _ in range(L):
            nxt, par = _refine(lv, d)
            lv.parents = par
            self.levels.append(nxt)
            lv = nxt
        for lv in self.levels:
            _node_info(lv, d)
            lv.boundary = boundary_nodes(lv, d)
        self._coarse_primitives()

    # ---------------------------------------------------------------------------------------
    def _coarse_primitives(self):
        d, cells = self.d, self.coarse_cells
        pairs = set()
        tris = set()
        for c in cells:
            c = [int(v) for v in c]
            for i in range(d + 1):
                for j in range(i + 1, d + 1):
                    pairs.add(tuple(sorted((c[i], c[j]))))
            if d == 3:
                for skip in range(4):
                    tris.add(tuple(sorted(c[k] for k in range(4) if k != skip)))
        self.coarse_edges = sorted(pairs)
        self.coarse_faces = sorted(tris)
        self.edge_id = {e: i for i, e in enumerate(self.coarse_edges)}
        self.face_id = {f: i for i, f in enumerate(self.coarse_faces)}

    def canonical_keys(self, l: int) -> np.ndarray:
        """Sort keys (rows) that define the canonical DoF order on level l:
        (class, primitive id, c_p, ..., c_1) with class 0=vertex, 1=edge, 2=face (3D),
        d=macro interior; vertex/edge/face coordinates are taken in the frame of the
        primitive's vertices sorted by global id, interior coordinates in the macro's own
        vertex order; the trailing coordinates are compared last-coordinate first."""
        lv = self.levels[l]
        d = self.d
        N = lv.n
        keys = np.zeros((N, 2 + d), dtype=np.int64)
        cells = self.coarse_cells
        gv = cells[lv.node_macro]                 # (N, d+1) global ids of node's macro vertices
        bary = lv.node_bary
        support = bary > 0
        cls = support.sum(axis=1)                 # 1..d+1
        inner = cls == d + 1
        keys[inner, 0] = d
        keys[inner, 1] = lv.node_macro[inner]
        keys[inner, 2:2 + d] = bary[inner][:, d:0:-1]     # macro frame: c_d, ..., c_1
        for i in np.nonzero(~inner)[0]:
            s = cls[i]
            vs = gv[i][support[i]]
            cs = bary[i][support[i]]
            order = np.argsort(vs)
            vs, cs = vs[order], cs[order]
            keys[i, 0] = s - 1
            if s == 1:
                keys[i, 1] = vs[0]
            elif s == 2:
                keys[i, 1] = self.edge_id[(int(vs[0]), int(vs[1]))]
            else:
                keys[i, 1] = self.face_id[(int(vs[0]), int(vs[1]), int(vs[2]))]
            rev = cs[:0:-1]                        # c_{s-1}, ..., c_1
            keys[i, 2:2 + len(rev)] = rev
        return keys

    def canonical_order(self, l: int) -> np.ndarray:
        """Permutation perm such that node perm[r] is the r-th DoF in canonical order."""
        k = self.canonical_keys(l)
        return np.lexsort(k.T[::-1])

    def support_size(self, l: int) -> np.ndarray:
        return (self.levels[l].node_bary > 0).sum(axis=1)


def build_hierarchy(coords, cells, L: int) -> Hierarchy:
    return Hierarchy(coords, cells, L)
