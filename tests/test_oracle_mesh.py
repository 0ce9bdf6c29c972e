"""Pins for the oracle's uniform refinement (Section 2: HHG construction)."""
import itertools

import numpy as np
import pytest

from oracle import refine
from oracle.assemble import element_geometry
from workloads import meshes


def _counts(mesh):
    cells = [tuple(int(v) for v in c) for c in mesh.cells]
    d = mesh.dim
    E = {tuple(sorted(p)) for c in cells for p in itertools.combinations(c, 2)}
    F = {tuple(sorted(p)) for c in cells for p in itertools.combinations(c, 3)} if d == 3 else set()
    return mesh.n_vertices, len(E), len(F), len(cells)


def dof_formula(mesh, L):
    """N_L = V + E(n-1) + F(n-1)(n-2)/2 [+ C(n-1)(n-2)(n-3)/6], n = 2^L."""
    V, E, F, C = _counts(mesh)
    n = 2 ** L
    if mesh.dim == 2:
        return V + E * (n - 1) + C * (n - 1) * (n - 2) // 2
    return V + E * (n - 1) + F * (n - 1) * (n - 2) // 2 + C * (n - 1) * (n - 2) * (n - 3) // 6


@pytest.mark.parametrize("mk,L,expect", [
    (meshes.unit_square_2tri, 5, 1089),
    (lambda: meshes.kuhn_cube(1), 4, 17 ** 3),
    (lambda: meshes.kuhn_cube(2), 3, 17 ** 3),
    (meshes.lshape_6tri, 4, None),
    (lambda: meshes.unit_square_grid(3), 3, 25 ** 2),
])
def test_dof_count(mk, L, expect):
    m = mk()
    h = refine.Hierarchy(m.coords, m.cells, L)
    for l in range(L + 1):
        assert h.levels[l].n == dof_formula(m, l)
    if expect is not None:
        assert h.levels[L].n == expect


def test_kuhn_cube_dof_formula_closed_form():
    # ns^3 Kuhn cubes refined L times is the (ns 2^L + 1)^3 grid: 129^3 and 257^3 for the
    # single cube at L=7 and the 4^3 cube at L=6
    assert dof_formula(meshes.kuhn_cube(1), 7) == 129 ** 3
    assert dof_formula(meshes.kuhn_cube(4), 6) == 257 ** 3


@pytest.mark.parametrize("mk,L,area", [
    (meshes.unit_square_2tri, 4, 1.0), (meshes.lshape_6tri, 3, 3.0),
    (lambda: meshes.kuhn_cube(2), 2, 1.0)])
def test_volume_sum(mk, L, area):
    m = mk()
    h = refine.Hierarchy(m.coords, m.cells, L)
    for lv in h.levels:
        _, vol = element_geometry(lv.X, lv.E)
        assert abs(vol.sum() - area) < 1e-13
        assert vol.min() > 0


def test_nested_numbering():
    m = meshes.kuhn_cube(1)
    h = refine.Hierarchy(m.coords, m.cells, 3)
    for l in range(3):
        a, b = h.levels[l], h.levels[l + 1]
        assert np.array_equal(a.X, b.X[:a.n])
        mid = 0.5 * (a.X[a.parents[:, 0]] + a.X[a.parents[:, 1]])
        assert np.array_equal(mid, b.X[a.n:])


def _lattice_tets(n):
    """Kuhn triangulation of the simplex {0 <= p1 <= p2 <= p3 <= n} in p-space, returned in
    barycentric-index coordinates (i, j, k) = (p1, p2 - p1, p3 - p2)."""
    out = set()
    for c in itertools.product(range(n), repeat=3):
        for perm in itertools.permutations(range(3)):
            vs = [np.array(c)]
            for a in perm:
                v = vs[-1].copy(); v[a] += 1; vs.append(v)
            if all(0 <= v[0] <= v[1] <= v[2] <= n for v in vs):
                out.add(frozenset((int(v[0]), int(v[1] - v[0]), int(v[2] - v[1])) for v in vs))
    return out


def test_bey_recursion_equals_kuhn_lattice():
    # one tetrahedron with non-special vertices; Bey's recursive rule must produce the lattice
    coords = np.array([[0.0, 0.0, 0.0], [1.0, 0.25, 0.0], [0.5, 1.0, 0.125], [0.25, 0.5, 1.0]])
    h = refine.Hierarchy(coords, np.array([[0, 1, 2, 3]]), 3)
    for l in range(4):
        lv = h.levels[l]
        got = {frozenset(tuple(int(x) for x in b[1:]) for b in eb) for eb in lv.ebary}
        assert got == _lattice_tets(2 ** l)
        assert len(got) == 8 ** l


def test_triangle_recursion_equals_lattice():
    coords = np.array([[0.0, 0.0], [1.0, 0.25], [0.375, 1.0]])
    h = refine.Hierarchy(coords, np.array([[0, 1, 2]]), 4)
    n = 16
    want = set()
    for i in range(n):
        for j in range(n - i):
            want.add(frozenset([(i, j), (i + 1, j), (i, j + 1)]))
            if i + j + 2 <= n:
                want.add(frozenset([(i + 1, j), (i, j + 1), (i + 1, j + 1)]))
    got = {frozenset(tuple(int(x) for x in b[1:]) for b in eb) for eb in h.levels[4].ebary}
    assert got == want


def test_kuhn_macro_micro_tets_congruent():
    m = meshes.kuhn_cube(1)
    h = refine.Hierarchy(m.coords, m.cells[:1], 3)
    lv = h.levels[3]
    P = lv.X[lv.E]
    lens = []
    for e in P:
        d = sorted(round(float(np.linalg.norm(e[a] - e[b])) * 8, 12)
                   for a, b in itertools.combinations(range(4), 2))
        lens.append(tuple(d))
    assert len(set(lens)) == 1


def test_boundary_nodes_unit_square():
    m = meshes.unit_square_2tri()
    h = refine.Hierarchy(m.coords, m.cells, 3)
    lv = h.levels[3]
    on = (lv.X[:, 0] == 0) | (lv.X[:, 0] == 1) | (lv.X[:, 1] == 0) | (lv.X[:, 1] == 1)
    assert np.array_equal(on, lv.boundary)


def test_canonical_order_is_a_permutation_with_primitives_first():
    m = meshes.kuhn_cube(1)
    h = refine.Hierarchy(m.coords, m.cells, 2)
    perm = h.canonical_order(2)
    assert np.array_equal(np.sort(perm), np.arange(h.levels[2].n))
    s = h.support_size(2)[perm]
    assert np.all(np.diff(s) >= 0)          # vertices, then edges, faces, cell interiors
