"""Pins for the oracle's solution transfer between macro meshes (the transfer T_L^k ->
T_L^(k+1) that the conclusion lists as missing)."""
import numpy as np

from oracle import assemble, refine, transfer
from paper_2508_06049_amd import mesh as hostmesh
from workloads import meshes


def test_affine_functions_transfer_exactly():
    # P1 reproduces affine functions: any transfer of an affine nodal vector is affine
    m0 = meshes.lshape_24tri()
    rg = hostmesh.RedGreen2D(m0)
    rg.conforming()
    rg.refine([0, 5, 11])
    m1 = rg.mesh()
    h0 = refine.Hierarchy(m0.coords, m0.cells, 2)
    h1 = refine.Hierarchy(m1.coords, m1.cells, 2)
    aff = lambda X: 0.3 - 1.7 * X[:, 0] + 0.6 * X[:, 1]
    got = transfer.transfer(h0, aff(h0.levels[2].X), h1.levels[2].X)
    assert np.all(np.isfinite(got))
    assert np.abs(got - aff(h1.levels[2].X)).max() < 1e-13


def test_nested_transfer_is_the_prolongation():
    # from level l to level l+1 of the same hierarchy the transfer is the prolongation P_l
    # (built from the refinement's parent relation, not from point location)
    m = meshes.lshape_6tri()
    h = refine.Hierarchy(m.coords, m.cells, 3)
    u = np.random.default_rng(3).standard_normal(h.levels[2].n)
    got = transfer.transfer(h, u, h.levels[3].X, level=2)
    P = assemble.prolongation(h, 2)
    assert np.abs(got - P @ u).max() < 1e-13


def test_identity_on_the_same_mesh_and_nan_outside():
    m = meshes.unit_square_grid(2)
    h = refine.Hierarchy(m.coords, m.cells, 2)
    X = h.levels[2].X
    u = np.sin(X[:, 0]) + X[:, 1] ** 2
    assert np.abs(transfer.transfer(h, u, X) - u).max() < 1e-14
    out = transfer.evaluate_p1(X, h.levels[2].E, u, np.array([[1.5, 0.5], [-0.1, 0.2]]))
    assert np.all(np.isnan(out))


def test_affine_and_nested_transfer_in_3d():
    # tetrahedra: affine functions are reproduced across a red-green step of the Kuhn cube, and
    # from level 1 to level 2 of one hierarchy (Bey's children) the transfer is P_1
    m0 = meshes.kuhn_cube(1)
    rg = hostmesh.RedGreen3D(m0)
    rg.refine([0, 3])
    m1 = rg.mesh()
    h0 = refine.Hierarchy(m0.coords, m0.cells, 2)
    h1 = refine.Hierarchy(m1.coords, m1.cells, 2)
    aff = lambda X: 0.3 - 1.7 * X[:, 0] + 0.6 * X[:, 1] + 0.45 * X[:, 2]
    got = transfer.transfer(h0, aff(h0.levels[2].X), h1.levels[2].X)
    assert np.all(np.isfinite(got))
    assert np.abs(got - aff(h1.levels[2].X)).max() < 1e-13
    u = np.random.default_rng(4).standard_normal(h0.levels[1].n)
    got = transfer.transfer(h0, u, h0.levels[2].X, level=1)
    assert np.abs(got - assemble.prolongation(h0, 1) @ u).max() < 1e-13
