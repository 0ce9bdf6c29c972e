"""CPU tests of the host-side k-refinement: marking and red-green refinement (Section 3,
Algorithm 3)."""
import itertools

import numpy as np
import pytest

from paper_2508_06049_amd import mesh as M
from oracle.assemble import element_geometry
from workloads import meshes


def _facets(cells, d):
    out = {}
    for ci, c in enumerate(cells):
        for f in itertools.combinations(sorted(int(v) for v in c), d):
            out.setdefault(f, []).append(ci)
    return out


def _check_conforming(mesh, volume):
    d = mesh.dim
    _, vol = element_geometry(mesh.coords, mesh.cells)
    assert vol.min() > 0
    assert abs(vol.sum() - volume) < 1e-12
    fac = _facets(mesh.cells, d)
    assert max(len(v) for v in fac.values()) <= 2
    # no hanging node: no vertex lies in the interior of another cell's edge
    X = mesh.coords
    edges = {tuple(sorted(e)) for c in mesh.cells for e in itertools.combinations(c, 2)}
    mids = {tuple(0.5 * (X[a] + X[b])) for a, b in edges}
    for p in map(tuple, X):
        if p in mids:
            # a vertex at an edge midpoint must be a vertex of every cell containing that edge
            for a, b in edges:
                if tuple(0.5 * (X[a] + X[b])) == p:
                    raise AssertionError("hanging node")
    # boundary facets lie on the domain boundary: total boundary measure
    return fac


def test_mark_fraction_ceil_and_ties():
    eta = np.array([1.0, 3.0, 3.0, 2.0, 0.5, 3.0, 0.1, 0.2, 0.3, 0.4, 0.45])
    assert list(M.mark_fraction(eta, 0.1)) == [1, 2]          # ceil(1.1) = 2, ties -> lower ids
    assert list(M.mark_fraction(eta, 0.125)) == [1, 2]
    assert len(M.mark_fraction(eta, 1.0)) == eta.size


def test_lshape_corner_refinement_is_conforming():
    m = M.lshape_corner_refined(6)
    assert m.n_cells == 144
    fac = _check_conforming(m, 3.0)
    # the smallest macros touch the corner and have edge length 2^-6
    o = int(np.nonzero((m.coords == 0).all(1))[0][0])
    touching = [c for c in m.cells if o in c]
    lens = [np.linalg.norm(m.coords[a] - m.coords[b]) for c in touching for a, b in itertools.combinations(c, 2)]
    assert min(lens) == 2.0 ** -6


def test_green_triangles_are_reverted():
    rg = M.RedGreen2D(meshes.unit_square_grid(2))
    cells, _ = rg.conforming()
    rg.refine([0])
    c1, p1 = rg.conforming()
    n_red_leaves = len(rg.tris)
    # an empty refinement step keeps the mesh, and greens are never stored
    rg.refine([])
    c2, _ = rg.conforming()
    assert sorted(map(tuple, c1)) == sorted(map(tuple, c2))
    assert len(rg.tris) == n_red_leaves
    assert len(c1) > len(rg.tris)   # greens present in the output only
    # marking a green cell refines its red parent
    green = [i for i in range(len(c1)) if sum(1 for q in p1 if q == p1[i]) == 2][0]
    rg.refine([green])
    m = rg.mesh()
    _check_conforming(m, 1.0)


@pytest.mark.parametrize("steps", [1, 2, 3])
def test_red_green_3d_conforming(steps):
    rg = M.RedGreen3D(meshes.kuhn_cube(2))
    cells, _ = rg.conforming()
    rng = np.random.default_rng(steps)
    for _ in range(steps):
        marked = rng.choice(len(cells), max(1, len(cells) // 8), replace=False)
        rg.refine(marked)
        cells, _ = rg.conforming()
    m = rg.mesh()
    fac = _check_conforming(m, 1.0)
    # boundary faces cover the cube surface (area 6)
    area = 0.0
    for f, cs in fac.items():
        if len(cs) == 1:
            P = m.coords[list(f)]
            area += 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))
    assert abs(area - 6.0) < 1e-12


def test_green_types_3d_only_three():
    # after closure every irregular cell has hanging nodes on one edge, two opposite edges or one face
    rg = M.RedGreen3D(meshes.kuhn_cube(2))
    cells, _ = rg.conforming()
    rg.refine([0, 5, 17])
    for t in rg.tets:
        he = rg._hanging_edges(t)
        assert len(he) in (0, 1, 2, 3)


def test_lshape_24tri_is_conforming_and_symmetric():
    m = meshes.lshape_24tri()
    assert m.n_cells == 24 and m.n_vertices == 21
    _check_conforming(m, 3.0)
    # symmetric about y = -x: the mirror image of every cell is a cell
    key = lambda pts: tuple(sorted(tuple(np.round(p, 12)) for p in pts))
    cells = {key(m.coords[c]) for c in m.cells}
    mirror = {key(-m.coords[c][:, ::-1]) for c in m.cells}
    assert cells == mirror


def test_waves_right_hand_side_is_minus_laplacian():
    # f = -Laplace(u) for the waves solution of Section 5.1, checked by a fourth-order
    # central difference; u vanishes on the boundary of the unit square
    from workloads import problems
    rng = np.random.default_rng(41)
    X = rng.uniform(0.05, 0.95, (200, 2))
    h = 2e-4
    lap = np.zeros(len(X))
    for d in range(2):
        e = np.zeros(2); e[d] = h
        u = lambda Y: problems.waves_u(Y)
        lap += (-u(X + 2 * e) + 16 * u(X + e) - 30 * u(X) + 16 * u(X - e) - u(X - 2 * e)) / (12 * h * h)
    f = problems.waves_f(X)
    assert np.max(np.abs(-lap - f)) <= 1e-5 * np.max(np.abs(f))
    t = np.linspace(0, 1, 11)
    B = np.concatenate([np.stack([t, 0 * t], 1), np.stack([t, 1 + 0 * t], 1), np.stack([0 * t, t], 1),
                        np.stack([1 + 0 * t, t], 1)])
    assert np.max(np.abs(problems.waves_u(B))) < 1e-12


def test_error_ratio_and_mean_width():
    # rho = Hbar^2 e_h / (hbar^2 e_H): an error sequence e = C hbar^2 through the coarse-grid
    # error gives rho = 1 on every step, a sequence at half that error gives 1/2
    from paper_2508_06049_amd import kl
    m0 = meshes.unit_square_grid(4)
    assert abs(kl.domain_measure(m0) - 1.0) < 1e-15
    assert abs(kl.domain_measure(meshes.lshape_24tri()) - 3.0) < 1e-15
    assert abs(kl.mean_width(m0, 0) - (1 / 32) ** 0.5) < 1e-15
    assert abs(kl.mean_width(m0, 3) - (1 / (32 * 64)) ** 0.5) < 1e-15
    H = kl.mean_width(m0, 0)
    eH = 0.3
    steps = []
    for k, L in enumerate((2, 4, 6)):
        hb = kl.mean_width(m0, L)
        steps.append(kl.KStep(k, m0, 0, hb, (0.5 if k else 1.0) * eH * (hb / H) ** 2, eH, 0.0, 0.0,
                              np.zeros(32), None, 0, 0, 0, 0, 0))
    rho = kl.error_ratio(steps)
    assert abs(rho[0] - 1.0) < 1e-12 and abs(rho[1] - 0.5) < 1e-12 and abs(rho[2] - 0.5) < 1e-12


def test_coarsening_round_trip_and_conformity():
    # coarsening (future work in the conclusion): marking every cell after two kl-steps merges
    # all red groups back to the coarse mesh; a partial marking leaves a conforming mesh of the
    # same area with fewer cells; nothing marked changes nothing
    m0 = meshes.lshape_24tri()
    rg = M.RedGreen2D(m0)
    cen = m0.coords[m0.cells].mean(axis=1)
    rg.refine(M.mark_fraction(-np.hypot(cen[:, 0], cen[:, 1]), 0.25))
    m1 = rg.mesh()
    rg.refine(list(range(0, m1.n_cells, 3)))
    m2 = rg.mesh()
    _check_conforming(m2, 3.0)
    assert rg.coarsen([]) == 0 and rg.mesh().n_cells == m2.n_cells
    # partial: the cells away from the re-entrant corner
    c2 = m2.coords[m2.cells].mean(axis=1)
    far = np.nonzero(np.hypot(c2[:, 0], c2[:, 1]) > 0.6)[0]
    n = rg.coarsen(far)
    m3 = rg.mesh()
    _check_conforming(m3, 3.0)
    assert n > 0 and m0.n_cells < m3.n_cells < m2.n_cells
    # everything: back to the coarse mesh
    rg.coarsen(list(range(m3.n_cells)))
    m4 = rg.mesh()
    key = lambda m: sorted(tuple(sorted(map(tuple, np.round(m.coords[c], 12).tolist()))) for c in m.cells)
    assert key(m4) == key(m0)
    # and refining again reproduces the first step
    c4 = m4.coords[m4.cells].mean(axis=1)
    rg.refine(M.mark_fraction(-np.hypot(c4[:, 0], c4[:, 1]), 0.25))
    assert key(rg.mesh()) == key(m1)


def test_coarsening_3d_round_trip_and_conformity():
    # 3D coarsening (the inverse of red refinement, closed again by Algorithm 3): marking
    # every cell after two steps merges all red groups back to the coarse mesh; a partial
    # marking leaves a conforming mesh of the same volume with fewer cells; nothing marked
    # changes nothing; refining the coarsened mesh again reproduces the first step
    m0 = meshes.kuhn_cube(2)
    rg = M.RedGreen3D(m0)
    cen = m0.coords[m0.cells].mean(axis=1)
    rg.refine(M.mark_fraction(-np.linalg.norm(cen, axis=1), 0.125))
    m1 = rg.mesh()
    c1 = m1.coords[m1.cells].mean(axis=1)
    rg.refine(M.mark_fraction(-np.linalg.norm(c1, axis=1), 0.125))
    m2 = rg.mesh()
    _check_conforming(m2, 1.0)
    assert rg.coarsen([]) == 0 and rg.mesh().n_cells == m2.n_cells
    # partial: cells away from the refined corner
    c2 = m2.coords[m2.cells].mean(axis=1)
    far = np.nonzero(np.linalg.norm(c2, axis=1) > 0.3)[0]
    n = rg.coarsen(far)
    m3 = rg.mesh()
    _check_conforming(m3, 1.0)
    assert n > 0 and m3.n_cells < m2.n_cells
    # everything: back to the coarse mesh
    rg.coarsen(list(range(m3.n_cells)))
    m4 = rg.mesh()
    key = lambda m: sorted(tuple(sorted(map(tuple, np.round(m.coords[c], 12).tolist()))) for c in m.cells)
    assert key(m4) == key(m0)
    c4 = m4.coords[m4.cells].mean(axis=1)
    rg.refine(M.mark_fraction(-np.linalg.norm(c4, axis=1), 0.125))
    assert key(rg.mesh()) == key(m1)
