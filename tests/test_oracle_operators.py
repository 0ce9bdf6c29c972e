"""Pins for the oracle's level operators: stiffness, mass, prolongation, right-hand side and
colouring (Section 4.4 linear systems; Section 5 Poisson form)."""
import numpy as np
import pytest

from oracle import assemble, colour, fmg, refine
from workloads import meshes


def _h(mk, L):
    m = mk()
    return refine.Hierarchy(m.coords, m.cells, L)


MESHES = [(meshes.unit_square_2tri, 3), (meshes.lshape_6tri, 3), (lambda: meshes.kuhn_cube(1), 3),
          (lambda: meshes.kuhn_cube(2), 2)]


@pytest.mark.parametrize("mk,L", MESHES)
def test_stiffness_symmetric_zero_rowsum_affine_kernel(mk, L):
    h = _h(mk, L)
    lv = h.levels[L]
    A = assemble.stiffness(lv)
    assert abs(A - A.T).max() < 1e-13
    assert np.abs(A @ np.ones(lv.n)).max() < 1e-12
    inner = ~lv.boundary
    rng = np.random.default_rng(1)
    for _ in range(3):
        c = rng.standard_normal(h.d + 1)
        aff = c[0] + lv.X @ c[1:]
        assert np.abs((A @ aff)[inner]).max() < 1e-11
    # positive definite on inner block
    I = np.nonzero(inner)[0]
    if I.size:
        ev = np.linalg.eigvalsh(A[I][:, I].toarray())
        assert ev.min() > 0


def test_closed_form_stencils():
    # right-isosceles lattice: [4, -1, -1, -1, -1] (independent of h)
    h = _h(meshes.unit_square_2tri, 4)
    lv = h.levels[4]
    A = assemble.stiffness(lv)
    i = int(np.argmin(np.abs(lv.X - [0.5, 0.25]).sum(1)))
    row = A[i].toarray().ravel()
    nz = np.sort(row[np.abs(row) > 1e-14])
    assert np.allclose(nz, [-1, -1, -1, -1, 4], atol=1e-13)
    # Kuhn lattice: h [6, -1 x 6] with h the micro mesh width
    h3 = _h(lambda: meshes.kuhn_cube(1), 4)
    lv = h3.levels[4]
    A = assemble.stiffness(lv)
    i = int(np.argmin(np.abs(lv.X - [0.5, 0.25, 0.75]).sum(1)))
    row = A[i].toarray().ravel() * 16
    nz = np.sort(row[np.abs(row) > 1e-12])
    assert np.allclose(nz, [-1] * 6 + [6], atol=1e-12)


@pytest.mark.parametrize("mk,L", MESHES)
def test_galerkin_identities(mk, L):
    h = _h(mk, L)
    rng = np.random.default_rng(3)
    kc = rng.uniform(0.5, 2.0, h.coarse_cells.shape[0])
    for l in range(1, L + 1):
        P = assemble.prolongation(h, l - 1)
        Af, Ac = assemble.stiffness(h.levels[l], kc), assemble.stiffness(h.levels[l - 1], kc)
        assert abs(P.T @ Af @ P - Ac).max() < 1e-12
        Mf, Mc = assemble.mass(h.levels[l]), assemble.mass(h.levels[l - 1])
        assert abs(P.T @ Mf @ P - Mc).max() < 1e-14


@pytest.mark.parametrize("mk,L,vol", [(meshes.unit_square_2tri, 3, 1.0), (meshes.lshape_6tri, 3, 3.0),
                                      (lambda: meshes.kuhn_cube(2), 2, 1.0)])
def test_mass_total_and_load_vector(mk, L, vol):
    h = _h(mk, L)
    lv = h.levels[L]
    M = assemble.mass(lv)
    one = np.ones(lv.n)
    assert abs(one @ M @ one - vol) < 1e-13
    # int x_0 over the domain via b = M f with f = x_0 (P1 integrates affine exactly)
    ref = (one @ M @ lv.X[:, 0])
    _, v = assemble.element_geometry(lv.X, lv.E)
    cen = lv.X[lv.E].mean(axis=1)[:, 0]
    assert abs(ref - float(v @ cen)) < 1e-13


@pytest.mark.parametrize("mk,L", MESHES)
def test_prolongation_reproduces_affine(mk, L):
    h = _h(mk, L)
    rng = np.random.default_rng(5)
    c = rng.standard_normal(h.d + 1)
    for l in range(L):
        P = assemble.prolongation(h, l)
        ac = c[0] + h.levels[l].X @ c[1:]
        af = c[0] + h.levels[l + 1].X @ c[1:]
        assert np.abs(P @ ac - af).max() < 1e-13
        assert np.allclose(np.asarray(P.sum(axis=1)).ravel(), 1.0)


@pytest.mark.parametrize("mk,L,rule", [
    (meshes.unit_square_2tri, 4, "redblack"), (lambda: meshes.kuhn_cube(1), 3, "redblack"),
    (lambda: meshes.kuhn_cube(2), 2, "redblack"), (meshes.lshape_6tri, 4, "multicolour"),
    (lambda: meshes.kuhn_cube(1), 3, "multicolour")])
def test_colouring_is_proper(mk, L, rule):
    h = _h(mk, L)
    for l in range(L + 1):
        lv = h.levels[l]
        col = colour.red_black(h, l) if rule == "redblack" else colour.multicolour(h, l)
        A = assemble.stiffness(lv)
        assert colour.is_proper_for(col, A, tol=1e-12)
        assert np.all(col[lv.boundary] == -1) and np.all(col[~lv.boundary] >= 0)
        if rule == "multicolour":
            # proper on the full mesh graph, not only on nonzero couplings
            G = colour.mesh_graph(lv)
            assert colour.is_proper_for(col, G)


def test_red_black_not_exact_on_generic_triangles():
    # a non-right triangle couples same-parity nodes: red-black must be rejected there
    coords = np.array([[0.0, 0.0], [1.0, 0.0], [0.5, 1.0]])
    h = refine.Hierarchy(coords, np.array([[0, 1, 2]]), 3)
    A = assemble.stiffness(h.levels[3])
    assert not colour.is_proper_for(colour.red_black(h, 3), A, tol=1e-12)


def test_colour_sweep_equals_pointwise_gauss_seidel():
    # the simultaneous update of a colour class equals a point-by-point Gauss-Seidel sweep
    h = _h(meshes.lshape_6tri, 3)
    S = fmg.FMGSolver(h, smoother="multicolour")
    s = S.sys[3]
    rng = np.random.default_rng(11)
    u0 = rng.standard_normal(s.N)
    b = rng.standard_normal(s.N)
    u1 = u0.copy()
    S.smooth(3, u1, b, 1)
    A = s.A.toarray()
    u2 = u0.copy()
    for c in np.unique(s.col[s.col >= 0]):
        for i in np.nonzero(s.col == c)[0]:
            u2[i] = (b[i] - A[i] @ u2 + A[i, i] * u2[i]) / A[i, i]
    assert np.abs(u1 - u2).max() < 1e-12


@pytest.mark.parametrize("mk,L,rule", [(meshes.unit_square_2tri, 5, "redblack"), (meshes.lshape_6tri, 5, "multicolour"),
                                       (lambda: meshes.unit_square_grid(4), 4, "multicolour"),
                                       (lambda: meshes.unit_square_grid(4), 3, "redblack")])
def test_2d_edge_classes_touch_only_their_own_edge(mk, L, rule):
    # the reading that lets one wavefront sweep both edge classes of an edge segment: a node of
    # the two edge classes (C, C + 1) lies on a macro edge at distance 2 <= a <= n - 2 from its
    # lower-id vertex, its class is C + (a mod 2), and each of its mesh neighbours is interior,
    # on the same macro edge, or in a later (vertex) class
    h = _h(mk, L)
    C = 2 if rule == "redblack" else 3
    for l in range(L + 1):
        lv = h.levels[l]
        n = 2 ** l
        col = colour.red_black(h, l) if rule == "redblack" else colour.multicolour(h, l)
        a = colour.edge_position_2d(h, l)
        gv = h.coarse_cells[lv.node_macro]
        sup = lv.node_bary > 0
        def edge_of(i):
            return tuple(sorted(int(v) for v in gv[i][sup[i]])) if sup[i].sum() == 2 else None
        G = colour.mesh_graph(lv)
        inner = sup.sum(axis=1) == 3
        E = np.nonzero((col == C) | (col == C + 1))[0]
        assert np.all((a[E] >= 2) & (a[E] <= n - 2))
        assert np.all(col[E] == C + a[E] % 2)
        for i in E:
            for q in G.indices[G.indptr[i]:G.indptr[i + 1]]:
                assert inner[q] or edge_of(q) == edge_of(i) or col[q] >= C + 2 or col[q] == -1
        # every edge point with 2 <= a <= n - 2 off the Dirichlet boundary is in them
        want = (a >= 2) & (a <= n - 2) & ~lv.boundary
        assert np.array_equal(np.sort(E), np.nonzero(want)[0])
