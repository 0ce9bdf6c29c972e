"""Host-side k-refinement of the macro mesh (Section 3): fixed-fraction marking and red-green
refinement of the coarse triangulation.  The macro mesh is small, so this runs serially on
the host, as the paper does.

2D red-green (Section 3): a marked triangle is split regularly (red, 4 children at the edge
midpoints); a triangle with more than one hanging node is split red as well, repeatedly;
triangles with exactly one hanging node are bisected towards it (green).  Green triangles
are transient: the state kept between steps holds only red leaves, so greens are reverted
before the next step, and marking a green triangle refines its red parent instead.
Coarsening (named as future work in the conclusion, Section 6) merges the four red children
of a parent back into it when all four are leaves and marked, as long as the parent is left
with at most one hanging node.

3D red-green (Algorithm 3): red-refine marked cells; repeatedly red-refine every face that
has more than one hanging node on its boundary; cells with more than three hanging nodes
become red; finally every cell with hanging nodes is closed by one of three green types
(one, two or three new vertices on its faces, each face following the 2D rule).  Coarsening
merges the eight red children of a parent back when all are marked leaves, drops the
midpoints no leaf uses any more, and runs the same closure again.
"""
from __future__ import annotations

import itertools
import math
import numpy as np

from workloads.meshes import CoarseMesh


def mark_fraction(eta: np.ndarray, frac: float) -> np.ndarray:
    """Indices of the ceil(frac * n) macros with the largest indicator; ties go to the lower
    index (marking fraction of Section 5: 10 % in 2D, 12.5 % in the 3D scaling study)."""
    eta = np.asarray(eta, dtype=np.float64)
    k = int(math.ceil(frac * eta.size))
    order = sorted(range(eta.size), key=lambda i: (-eta[i], i))
    return np.array(sorted(order[:k]), dtype=np.int64)


class RedGreen2D:
    """Red-green refinement of a triangle mesh with green revert."""

    def __init__(self, mesh: CoarseMesh):
        if mesh.dim != 2:
            raise ValueError("RedGreen2D needs a triangle mesh")
        self.X = [tuple(float(v) for v in p) for p in mesh.coords]
        self.tris = [tuple(int(v) for v in t) for t in mesh.cells]   # red leaves
        self.mid = {}                                                 # edge -> midpoint vertex
        self.children = {}                                            # red parent -> its 4 children
        self._last_parent = None
        self._act = None                                              # vertices of the leaves

    def _active(self):
        if self._act is None:
            self._act = {v for t in self.tris for v in t}
        return self._act

    def _midpoint(self, a, b):
        e = (min(a, b), max(a, b))
        if e not in self.mid:
            pa, pb = self.X[a], self.X[b]
            self.X.append(tuple(0.5 * (x + y) for x, y in zip(pa, pb)))
            self.mid[e] = len(self.X) - 1
        return self.mid[e]

    def _red(self, t):
        a, b, c = t
        ab, ac, bc = self._midpoint(a, b), self._midpoint(a, c), self._midpoint(b, c)
        ch = [(a, ab, ac), (ab, b, bc), (ac, bc, c), (ab, bc, ac)]
        self.children[t] = ch
        return ch

    def _mid_active(self, p, q):
        """Midpoint of edge (p, q) if it is a vertex of the current leaves (else None)."""
        m = self.mid.get((min(p, q), max(p, q)))
        return m if m is not None and m in self._active() else None

    def _hanging(self, t):
        """Edges of leaf t whose midpoint is a vertex of the leaves (refined from the other side)."""
        a, b, c = t
        out = []
        for i, (p, q) in enumerate(((b, c), (a, c), (a, b))):     # edge opposite vertex i
            m = self._mid_active(p, q)
            if m is not None:
                out.append((i, m))
        return out

    def _edge_nodes(self, a, b):
        """Number of leaf vertices in the open edge (a, b): midpoints, recursively."""
        m = self._mid_active(a, b)
        return 0 if m is None else 1 + self._edge_nodes(a, m) + self._edge_nodes(m, b)

    def _n_hanging(self, t):
        a, b, c = t
        return self._edge_nodes(b, c) + self._edge_nodes(a, c) + self._edge_nodes(a, b)

    def conforming(self):
        """Red leaves plus green bisections: (cells, parent red leaf of every cell)."""
        cells, parent = [], []
        for ti, t in enumerate(self.tris):
            h = self._hanging(t)
            if not h:
                cells.append(t); parent.append(ti)
            elif len(h) == 1:
                i, m = h[0]
                v = t[i]
                p, q = [t[j] for j in range(3) if j != i]
                cells.append((v, p, m)); parent.append(ti)
                cells.append((v, m, q)); parent.append(ti)
            else:
                raise RuntimeError("closure left a triangle with two hanging nodes")
        self._last_parent = parent
        return cells, parent

    def refine(self, marked_cells) -> None:
        """Refine the cells (indices into the last conforming() output) marked red."""
        if self._last_parent is None:
            self.conforming()
        red = {self._last_parent[i] for i in marked_cells}
        tris = []
        for ti, t in enumerate(self.tris):
            tris.extend(self._red(t) if ti in red else [t])
        self.tris = tris
        self._act = None
        changed = True
        while changed:                       # red closure: more than one hanging node
            changed = False
            nxt = []
            for t in self.tris:
                if self._n_hanging(t) > 1:
                    nxt.extend(self._red(t)); changed = True
                else:
                    nxt.append(t)
            self.tris = nxt
            self._act = None
        self._last_parent = None

    def coarsen(self, marked_cells) -> int:
        """Merge red sibling groups back into their parents (cells: indices into the last
        conforming() output; a marked green cell marks its red parent leaf).  All groups whose
        four children are marked leaves merge at once; the red closure then splits again every
        merged parent left with more than one hanging node (merging removes vertices, so no
        other leaf gains one).  Merged parents count as marked, so coarsening repeats upwards
        while it makes progress.  Returns the number of merged groups."""
        if self._last_parent is None:
            self.conforming()
        marked = {self.tris[self._last_parent[i]] for i in marked_cells}
        merged = 0
        while True:
            leaves = set(self.tris)
            groups = [P for P, ch in self.children.items() if all(c in leaves and c in marked for c in ch)]
            if not groups:
                break
            drop = {c for P in groups for c in self.children[P]}
            self.tris = [t for t in self.tris if t not in drop] + groups
            self._act = None
            changed = True
            while changed:                   # red closure
                changed = False
                nxt = []
                for t in self.tris:
                    if self._n_hanging(t) > 1:
                        nxt.extend(self._red(t)); changed = True
                    else:
                        nxt.append(t)
                self.tris = nxt
                self._act = None
            leaves = set(self.tris)
            kept = [P for P in groups if P in leaves]
            if not kept:
                break
            for P in kept:
                del self.children[P]
                marked.add(P)
            merged += len(kept)
        self._last_parent = None
        return merged

    def mesh(self, name="") -> CoarseMesh:
        cells, _ = self.conforming()
        used = sorted({v for c in cells for v in c})
        remap = {v: i for i, v in enumerate(used)}
        coords = np.array([self.X[v] for v in used])
        cc = np.array([[remap[v] for v in c] for c in cells], dtype=np.int32)
        return CoarseMesh(coords, cc, name)


def lshape_corner_refined(steps: int = 6) -> CoarseMesh:
    """L-shape macro mesh k-refined `steps` times towards the re-entrant corner: each step
    marks every macro triangle that has the origin as a vertex (red), then closes with greens
    (reverted before the next step)."""
    from workloads.meshes import lshape_6tri
    rg = RedGreen2D(lshape_6tri())
    for _ in range(steps):
        cells, _ = rg.conforming()
        origin = [v for v, p in enumerate(rg.X) if p == (0.0, 0.0)][0]
        rg.refine([i for i, c in enumerate(cells) if origin in c])
    return rg.mesh(f"lshape_corner{steps}")


# -------------------------------------------------------------------------------------------
# 3D red-green (Algorithm 3)
_TET_EDGES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
_BEY = [(0, 4, 5, 6), (4, 1, 7, 8), (5, 7, 2, 9), (6, 8, 9, 3),
        (4, 5, 6, 8), (4, 5, 7, 8), (5, 6, 8, 9), (5, 7, 8, 9)]


class RedGreen3D:
    """Red-green refinement of a tetrahedral mesh following Algorithm 3, greens reverted
    between steps.  Red cells use Bey's children; a face is 'red' once all three of its edge
    midpoints exist.  After the face rule, a cell's hanging nodes lie on one edge, on two
    opposite edges, or on the three edges of one face; the green closure splits it so that
    each of its faces follows the 2D rule: one bisected edge (2 cells), two bisected opposite
    edges (4 cells) or one red face joined to the opposite vertex (4 cells)."""

    def __init__(self, mesh: CoarseMesh):
        if mesh.dim != 3:
            raise ValueError("RedGreen3D needs a tetrahedral mesh")
        self.X = [tuple(float(v) for v in p) for p in mesh.coords]
        self.tets = [tuple(int(v) for v in t) for t in mesh.cells]
        self.mid = {}          # edge -> midpoint vertex, for the midpoints that currently exist
        self._mid_all = {}     # edge -> midpoint vertex ever created (reused after coarsening)
        self.children = {}     # red parent -> its 8 children
        self._last_parent = None

    def _midpoint(self, a, b, create=True):
        e = (min(a, b), max(a, b))
        if e not in self.mid:
            if not create:
                return None
            if e not in self._mid_all:
                pa, pb = self.X[a], self.X[b]
                self.X.append(tuple(0.5 * (x + y) for x, y in zip(pa, pb)))
                self._mid_all[e] = len(self.X) - 1
            self.mid[e] = self._mid_all[e]
        return self.mid[e]

    def _red(self, t):
        loc = list(t) + [self._midpoint(t[a], t[b]) for a, b in _TET_EDGES]
        ch = [tuple(loc[i] for i in c) for c in _BEY]
        self.children[t] = ch
        return ch

    def _hanging_edges(self, t):
        return [k for k, (a, b) in enumerate(_TET_EDGES) if (min(t[a], t[b]), max(t[a], t[b])) in self.mid]

    def _mid(self, a, b):
        return self.mid.get((min(a, b), max(a, b)))

    def _edge_nodes(self, a, b):
        m = self._mid(a, b)
        return 0 if m is None else 1 + self._edge_nodes(a, m) + self._edge_nodes(m, b)

    def _face_inner_nodes(self, a, b, c):
        """Vertices strictly inside triangle (a, b, c): only present once all three edge
        midpoints exist, then inside the four sub-triangles and on their inner edges."""
        ab, ac, bc = self._mid(a, b), self._mid(a, c), self._mid(b, c)
        if ab is None or ac is None or bc is None:
            return 0
        n = self._edge_nodes(ab, ac) + self._edge_nodes(ab, bc) + self._edge_nodes(ac, bc)
        for tri in ((a, ab, ac), (ab, b, bc), (ac, bc, c), (ab, bc, ac)):
            n += self._face_inner_nodes(*tri)
        return n

    def _n_hanging_face_boundary(self, t, skip):
        vs = [t[v] for v in range(4) if v != skip]
        return sum(self._edge_nodes(x, y) for x, y in itertools.combinations(vs, 2))

    def _n_hanging(self, t):
        n = sum(self._edge_nodes(t[a], t[b]) for a, b in _TET_EDGES)
        for skip in range(4):
            vs = [t[v] for v in range(4) if v != skip]
            n += self._face_inner_nodes(*vs)
        return n

    @staticmethod
    def _face_edges(skip):
        vs = [v for v in range(4) if v != skip]
        return [_TET_EDGES.index((a, b)) for a, b in itertools.combinations(vs, 2)]

    def refine(self, marked_cells) -> None:
        if self._last_parent is None:
            self.conforming()
        self._closure({self._last_parent[i] for i in marked_cells})
        self._last_parent = None

    def _closure(self, red):
        """Red-refine the leaves `red` (indices into self.tets), then close: faces with more
        than one hanging node on their boundary get all three edge midpoints, and cells with
        more than three hanging nodes are refined red, until nothing changes."""
        while True:
            tets = []
            for ti, t in enumerate(self.tets):
                tets.extend(self._red(t) if ti in red else [t])
            self.tets = tets
            # faces with more than one hanging node on their boundary are refined red
            while True:
                added = False
                for t in self.tets:
                    for skip in range(4):
                        if self._n_hanging_face_boundary(t, skip) > 1:
                            for k in self._face_edges(skip):
                                a, b = _TET_EDGES[k]
                                if self._mid(t[a], t[b]) is None:
                                    self._midpoint(t[a], t[b]); added = True
                if not added:
                    break
            red = {ti for ti, t in enumerate(self.tets) if self._n_hanging(t) > 3}
            if not red:
                break

    def coarsen(self, marked_cells) -> int:
        """Merge red sibling groups back into their parents, the inverse of red refinement
        (cells: indices into the last conforming() output; a marked green cell marks its red
        parent leaf).  All groups whose eight children are marked leaves merge at once; the
        midpoints that no remaining leaf has as a vertex are dropped, and the closure of
        Algorithm 3 (face rule, red for more than three hanging nodes) runs again, which
        re-splits a merged parent that the surrounding refinement does not allow.  Merged
        parents count as marked, so coarsening repeats upwards while it makes progress.
        Returns the number of merged groups."""
        if self._last_parent is None:
            self.conforming()
        marked = {self.tets[self._last_parent[i]] for i in marked_cells}
        merged = 0
        while True:
            leaves = set(self.tets)
            groups = [P for P, ch in self.children.items() if all(c in leaves and c in marked for c in ch)]
            if not groups:
                break
            drop = {c for P in groups for c in self.children[P]}
            self.tets = [t for t in self.tets if t not in drop] + groups
            used = {v for t in self.tets for v in t}
            self.mid = {e: m for e, m in self.mid.items() if m in used}
            self._closure(set())
            leaves = set(self.tets)
            kept = [P for P in groups if P in leaves]
            if not kept:
                break
            for P in kept:
                del self.children[P]
                marked.add(P)
            merged += len(kept)
        self._last_parent = None
        return merged

    def _green(self, t):
        he = self._hanging_edges(t)
        if len(he) == 1:                                  # one new vertex: bisect the edge
            a, b = _TET_EDGES[he[0]]
            m = self._midpoint(t[a], t[b], create=False)
            o = [t[v] for v in range(4) if v not in (a, b)]
            return [(t[a], m, o[0], o[1]), (m, t[b], o[0], o[1])]
        if len(he) == 3:                                  # three new vertices on one face: red face
            vs = set()
            for k in he:
                vs |= set(_TET_EDGES[k])
            if len(vs) != 3:
                raise RuntimeError("green closure: three hanging edges not on one face")
            apex = [v for v in range(4) if v not in vs][0]
            f = sorted(vs)
            a, b, c = (t[v] for v in f)
            ab, ac, bc = (self._midpoint(x, y, create=False) for x, y in ((a, b), (a, c), (b, c)))
            tris = [(a, ab, ac), (ab, b, bc), (ac, bc, c), (ab, bc, ac)]
            return [tr + (t[apex],) for tr in tris]
        if len(he) == 2:                                  # two new vertices on opposite edges
            (a, b), (c, d) = (_TET_EDGES[k] for k in he)
            if set((a, b)) & set((c, d)):
                raise RuntimeError("green closure: two hanging nodes on one face (face rule violated)")
            m1 = self._midpoint(t[a], t[b], create=False)
            m2 = self._midpoint(t[c], t[d], create=False)
            A, B, Cc, Dd = t[a], t[b], t[c], t[d]
            return [(A, m1, Cc, m2), (A, m1, m2, Dd), (m1, B, Cc, m2), (m1, B, m2, Dd)]
        raise RuntimeError(f"green closure: unsupported pattern {he}")

    def conforming(self):
        cells, parent = [], []
        for ti, t in enumerate(self.tets):
            if not self._hanging_edges(t):
                cells.append(t); parent.append(ti)
            else:
                for g in self._green(t):
                    cells.append(g); parent.append(ti)
        self._last_parent = parent
        return cells, parent

    def mesh(self, name="") -> CoarseMesh:
        cells, _ = self.conforming()
        used = sorted({v for c in cells for v in c})
        remap = {v: i for i, v in enumerate(used)}
        coords = np.array([self.X[v] for v in used])
        cc = np.array([[remap[v] for v in c] for c in cells], dtype=np.int32)
        return CoarseMesh(coords, cc, name)
