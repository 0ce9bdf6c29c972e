"""Coarse (macro) meshes used as inputs.

All coordinates are dyadic rationals, so every midpoint produced by uniform refinement is
exact in binary64 and fine-grid nodes can be matched across implementations by exact
coordinate equality.

Vertex order inside a cell matters: it fixes the local index frame of the macro element
(vertex x0 is the origin, x1-x0, x2-x0[, x3-x0] are the axes).  The cube generator lists each
tetrahedron in *path order* p, p+h e_a, p+h(e_a+e_b), p+h(1,1,1) (a Kuhn / Freudenthal
simplex), which is the order under which Bey's interior diagonal falls on the cube lattice.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np


@dataclass
class CoarseMesh:
    coords: np.ndarray          # (n_vertices, dim) float64
    cells: np.ndarray           # (n_cells, dim+1) int32, vertex ids
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def dim(self) -> int:
        return int(self.coords.shape[1])

    @property
    def n_cells(self) -> int:
        return int(self.cells.shape[0])

    @property
    def n_vertices(self) -> int:
        return int(self.coords.shape[0])

    def copy(self) -> "CoarseMesh":
        return CoarseMesh(self.coords.copy(), self.cells.copy(), self.name, dict(self.meta))


def unit_square_2tri() -> CoarseMesh:
    """(0,1)^2 split by the diagonal (0,0)-(1,1) into two right isosceles triangles."""
    coords = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    cells = np.array([[0, 1, 2], [0, 3, 2]], dtype=np.int32)
    return CoarseMesh(coords, cells, "unit_square_2tri")


def unit_square_grid(m: int) -> CoarseMesh:
    """(0,1)^2 as an m x m grid of squares, each split by its (1,1) diagonal: 2 m^2 triangles."""
    g = np.linspace(0.0, 1.0, m + 1)
    X, Y = np.meshgrid(g, g, indexing="ij")
    coords = np.stack([X.ravel(), Y.ravel()], axis=1)
    vid = lambda i, j: i * (m + 1) + j
    cells = []
    for i in range(m):
        for j in range(m):
            a, b, c, d = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            cells.append([a, b, c])
            cells.append([a, d, c])
    return CoarseMesh(coords, np.array(cells, dtype=np.int32), f"unit_square_grid{m}")


def rect_grid(mx: int, my: int, h: float) -> CoarseMesh:
    """(0, mx h) x (0, my h) as an mx x my grid of squares of side h, each split by its (1,1)
    diagonal: 2 mx my triangles.  With h a power of two every coordinate, and every midpoint of
    the refined levels, is exact in float64."""
    coords = np.array([[i * h, j * h] for i in range(mx + 1) for j in range(my + 1)], dtype=np.float64)
    vid = lambda i, j: i * (my + 1) + j
    cells = []
    for i in range(mx):
        for j in range(my):
            a, b, c, d = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            cells.append([a, b, c])
            cells.append([a, d, c])
    return CoarseMesh(coords, np.array(cells, dtype=np.int32), f"rect_grid{mx}x{my}")


def lshape_6tri() -> CoarseMesh:
    """L-shaped domain (-1,1)^2 without the quadrant x>0, y<0 (polar angle in (0, 3pi/2)).

    The three unit squares of quadrants I, II and III are each split by the diagonal that
    passes through the re-entrant corner at the origin; the origin is vertex x0 of every
    triangle.
    """
    coords = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0],
                       [-1.0, 1.0], [-1.0, 0.0], [-1.0, -1.0], [0.0, -1.0]])
    cells = np.array([[0, 1, 2], [0, 2, 3], [0, 3, 4], [0, 4, 5], [0, 5, 6], [0, 6, 7]],
                     dtype=np.int32)
    return CoarseMesh(coords, cells, "lshape_6tri")


def lshape_24tri() -> CoarseMesh:
    """The L-shaped domain of lshape_6tri as 12 squares of side 1/2, each split into two
    triangles by the diagonal whose line passes nearest the re-entrant corner ((1,1)
    direction in quadrants I and III, (-1,1) in quadrant II): 24 triangles, symmetric about
    the line y = -x."""
    pts = {}
    cells = []

    def vid(x, y):
        key = (round(2 * x), round(2 * y))
        if key not in pts:
            pts[key] = len(pts)
        return pts[key]

    for qx, qy in ((0.0, 0.0), (-1.0, 0.0), (-1.0, -1.0)):
        for i in range(2):
            for j in range(2):
                x0, y0 = qx + 0.5 * i, qy + 0.5 * j
                a, b, c, d = vid(x0, y0), vid(x0 + 0.5, y0), vid(x0 + 0.5, y0 + 0.5), vid(x0, y0 + 0.5)
                if qx < 0 <= qy:            # quadrant II: diagonal b-d
                    cells += [[a, b, d], [b, c, d]]
                else:                       # quadrants I and III: diagonal a-c
                    cells += [[a, b, c], [a, c, d]]
    coords = np.zeros((len(pts), 2))
    for (kx, ky), v in pts.items():
        coords[v] = (0.5 * kx, 0.5 * ky)
    return CoarseMesh(coords, np.array(cells, dtype=np.int32), "lshape_24tri")


def kuhn_cube(ns: int, lo: float = 0.0, hi: float = 1.0) -> CoarseMesh:
    """[lo,hi]^3 as ns^3 subcubes, each split into the 6 Kuhn tetrahedra (path order)."""
    g = np.linspace(lo, hi, ns + 1)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    coords = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)

    def vid(p):
        return (p[0] * (ns + 1) + p[1]) * (ns + 1) + p[2]

    cells = []
    for a, b, c in itertools.product(range(ns), repeat=3):
        p0 = np.array([a, b, c])
        for perm in itertools.permutations(range(3)):
            p1 = p0.copy(); p1[perm[0]] += 1
            p2 = p1.copy(); p2[perm[1]] += 1
            p3 = p0 + 1
            cells.append([vid(p0), vid(p1), vid(p2), vid(p3)])
    return CoarseMesh(coords, np.array(cells, dtype=np.int32), f"kuhn_cube{ns}")
