"""Pins of the oracle's interpolation to a node set T_G (Sec. 3.1)."""
import numpy as np
import pytest

import workloads as W
from oracle import interp as oi


def meshes():
    return [W.uniform_mesh(8), W.jittered_mesh(8, 7, 3)]


@pytest.mark.parametrize("m", [0, 1])
def test_linear_functions_are_reproduced(m):
    mesh = meshes()[m]
    xy, tri, bnd = mesh["mesh_xy"], mesh["mesh_tri"], mesh["mesh_boundary"]
    pts = W.random_points(200, 5)
    A = oi.interpolation_matrix(xy, tri, np.zeros(len(xy), bool), pts)  # every vertex carries a value
    for a, b, c in [(1.0, 0.0, 0.0), (0.3, -1.7, 2.2), (-2.0, 0.5, 0.25)]:
        f = a + b * xy[:, 0] + c * xy[:, 1]
        assert np.abs(A @ f - (a + b * pts[:, 0] + c * pts[:, 1])).max() <= 1e-13
    # partition of unity and non-negative coordinates inside the domain
    assert np.abs(A.sum(axis=1) - 1.0).max() <= 1e-13
    assert A.min() >= -1e-12


@pytest.mark.parametrize("m", [0, 1])
def test_vertices_reproduce_nodal_values(m):
    mesh = meshes()[m]
    xy, tri, bnd = mesh["mesh_xy"], mesh["mesh_tri"], np.asarray(mesh["mesh_boundary"], bool)
    inner = np.nonzero(~bnd)[0]
    pick = inner[::3]
    A = oi.interpolation_matrix(xy, tri, bnd, xy[pick])
    u = np.random.default_rng(1).standard_normal(len(inner))
    gid = {v: g for g, v in enumerate(inner)}
    assert np.abs(A @ u - u[[gid[v] for v in pick]]).max() <= 1e-13
    # boundary vertices carry the Dirichlet value 0
    bpts = xy[np.nonzero(bnd)[0][:5]]
    assert np.abs(oi.interpolation_matrix(xy, tri, bnd, bpts) @ u).max() <= 1e-13


def test_points_outside_are_rejected():
    mesh = W.uniform_mesh(4)
    with pytest.raises(ValueError):
        oi.interpolation_matrix(mesh["mesh_xy"], mesh["mesh_tri"], mesh["mesh_boundary"], np.array([[1.2, 0.5]]))
