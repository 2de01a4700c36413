"""Pins of the general-triangulation P1 sampler (oracle side)."""
import numpy as np
from scipy.sparse import coo_matrix

import workloads as W
from oracle import fem, fem_mesh
from oracle import periodization as per


def test_uniform_mesh_reproduces_the_structured_oracle():
    # the same discrete system written as a general triangulation
    n, d = 12, 4
    prob = W.pde_problem(n, d, 4)
    u = W.uniform_mesh(n)
    g = np.random.default_rng(1)
    for model in (per.PERIODIC, per.AFFINE, per.LOGNORMAL):
        a0 = 0.5 if model == per.LOGNORMAL else 1.0
        S1 = fem.PDESampler(n, a0, prob["amp"], prob["mode1"], prob["mode2"], model=model, delta=0.01)
        S2 = fem_mesh.MeshSampler(u["mesh_xy"], u["mesh_tri"], u["mesh_boundary"], a0, prob["amp"], prob["mode1"],
                                  prob["mode2"], model=model, delta=0.01)
        for t in g.random((3, d)):
            ref = S1.solve_one(t)
            assert np.allclose(S2.solve_one(t), ref, rtol=1e-12, atol=0)


def _full_matrix(mesh, a_tri):
    rows, cols, vals = [], [], []
    for a in range(3):
        for b in range(3):
            rows.append(mesh.tri[:, a])
            cols.append(mesh.tri[:, b])
            vals.append(a_tri * mesh.kgeo[:, a, b])
    nv = len(mesh.xy)
    return coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nv, nv)).toarray()


def test_patch_test_and_definiteness_on_a_jittered_mesh():
    m = W.jittered_mesh(8, 9, seed=3)
    mesh = fem_mesh.TriMesh(m["mesh_xy"], m["mesh_tri"], m["mesh_boundary"])
    K = _full_matrix(mesh, np.ones(len(mesh.tri)))
    # every row annihilates constants, interior rows annihilate linear
    # functions (P1 reproduces linears): sum_j K_ij l(x_j) = 0
    assert np.abs(K.sum(axis=1)).max() < 1e-12
    for c in ((1.0, 0.0), (0.0, 1.0), (0.7, -2.0)):
        lin = m["mesh_xy"] @ np.array(c) + 0.3
        assert np.abs((K @ lin)[mesh.interior]).max() < 1e-12
    A = mesh.stiffness(np.random.default_rng(0).uniform(0.5, 2.0, len(mesh.tri))).toarray()
    assert np.allclose(A, A.T, rtol=0, atol=1e-14)
    assert np.linalg.eigvalsh(A).min() > 0
    # the load vector integrates f = 1 over the domain
    assert abs(mesh.load_all.sum() - 1.0) < 1e-14


def test_manufactured_discrete_solution():
    m = W.jittered_mesh(10, 11, seed=4)
    prob = W.pde_problem(8, 3, 4)
    S = fem_mesh.MeshSampler(m["mesh_xy"], m["mesh_tri"], m["mesh_boundary"], 1.0, prob["amp"], prob["mode1"],
                             prob["mode2"])
    y = np.array([0.1, 0.7, 0.35])
    a = fem.coefficient_on_triangles(S.mesh, 1.0, prob["amp"], prob["mode1"], prob["mode2"], y)
    A = S.mesh.stiffness(a)
    ustar = np.random.default_rng(2).standard_normal(S.G)
    from scipy.sparse.linalg import spsolve
    assert np.allclose(spsolve(A.tocsc(), A @ ustar), ustar, rtol=0, atol=1e-11)
    # the sampler solves A u = load
    u = S.solve_param(y)
    assert np.abs(A @ u - S.mesh.load).max() < 1e-14 * S.G
