"""Pins of the FEM oracle against facts that do not come from its own code."""
import math

import numpy as np
import pytest

from oracle import fem
import workloads as W


def grid(u, n):
    return u.reshape(n - 1, n - 1)  # [j-1, i-1]


def test_constant_coefficient_closed_form():
    # a = 1: stiffness = 5-point Laplacian; sine eigenbasis gives the exact solution
    n = 12
    S = fem.PDESampler(n, 1.0, [0.0], [1], [1])
    u = S.solve_one([0.3])
    h = 1.0 / n
    idx = np.arange(1, n)
    Sm = np.sin(np.pi * np.outer(idx, idx) * h)  # Sm[p, i] = sin(p pi i h)
    lam = 4 - 2 * np.cos(np.pi * idx * h)[:, None] - 2 * np.cos(np.pi * idx * h)[None, :]
    b = np.full((n - 1, n - 1), h * h)
    # expand b in the basis (Sm is orthogonal up to n/2)
    bh = (Sm @ b @ Sm.T) * (2.0 / n) ** 2
    uh = bh / lam.T
    ref = Sm.T @ uh @ Sm
    assert np.allclose(grid(u, n), ref, rtol=1e-12, atol=1e-15)


def test_bilinear_form_from_gradients():
    # v^T A u = sum_T a_T |T| grad u_T . grad v_T, gradients by differences of the
    # linear interpolant on each right triangle (independent of the element matrices)
    n = 7
    h = 1.0 / n
    prob = W.pde_problem(n, 3, 4)
    y = np.array([0.11, 0.52, 0.83])
    mesh = fem.Mesh(n)
    a_tri = fem.coefficient_on_triangles(mesh, 1.0, prob["amp"], prob["mode1"], prob["mode2"], y)
    A = fem.dense_stiffness(mesh, a_tri)
    g = np.random.default_rng(0)
    U = np.zeros((n + 1, n + 1))
    V = np.zeros((n + 1, n + 1))
    U[1:n, 1:n] = g.standard_normal((n - 1, n - 1))
    V[1:n, 1:n] = g.standard_normal((n - 1, n - 1))

    def coef(cx, cy):
        s = 1.0
        for j in range(3):
            s += prob["amp"][j] * math.sin(2 * math.pi * y[j]) * math.sin(prob["mode1"][j] * math.pi * cx) * math.sin(prob["mode2"][j] * math.pi * cy)
        return s

    form = 0.0
    for i in range(n):
        for j in range(n):
            # lower triangle (i,j),(i+1,j),(i+1,j+1)
            a = coef((i + 2 / 3) * h, (j + 1 / 3) * h)
            gu = ((U[i + 1, j] - U[i, j]) / h, (U[i + 1, j + 1] - U[i + 1, j]) / h)
            gv = ((V[i + 1, j] - V[i, j]) / h, (V[i + 1, j + 1] - V[i + 1, j]) / h)
            form += a * 0.5 * h * h * (gu[0] * gv[0] + gu[1] * gv[1])
            # upper triangle (i,j),(i,j+1),(i+1,j+1)
            a = coef((i + 1 / 3) * h, (j + 2 / 3) * h)
            gu = ((U[i + 1, j + 1] - U[i, j + 1]) / h, (U[i, j + 1] - U[i, j]) / h)
            gv = ((V[i + 1, j + 1] - V[i, j + 1]) / h, (V[i, j + 1] - V[i, j]) / h)
            form += a * 0.5 * h * h * (gu[0] * gv[0] + gu[1] * gv[1])
    # node g = (j-1)(n-1)+(i-1) <-> U[i, j]
    u = U[1:n, 1:n].T.reshape(-1)
    v = V[1:n, 1:n].T.reshape(-1)
    assert abs(v @ A @ u - form) <= 1e-12 * abs(form)


def test_manufactured_discrete_solution():
    n = 16
    prob = W.pde_problem(n, 4, 8, modes="diagonal")
    S = fem.PDESampler(n, 1.0, prob["amp"], prob["mode1"], prob["mode2"])
    y = np.array([0.1, 0.7, 0.25, 0.9])
    a_tri = fem.coefficient_on_triangles(S.mesh, 1.0, S.amp, S.mode1, S.mode2, y)
    A = fem.dense_stiffness(S.mesh, a_tri)
    ustar = np.random.default_rng(1).standard_normal(S.G)
    ab = fem.banded_stiffness(S.mesh, a_tri)
    u = fem.solve_banded(ab, A @ ustar)
    assert np.linalg.norm(u - ustar) <= 1e-12 * np.linalg.norm(ustar)


def poisson_center_value():
    # -Lap u = 1 on the unit square, u = 0 on the boundary: double sine series at (1/2, 1/2)
    s = 0.0
    for m in range(1, 400, 2):
        for k in range(1, 400, 2):
            s += 16.0 / (math.pi ** 4 * m * k * (m * m + k * k)) * math.sin(m * math.pi / 2) * math.sin(k * math.pi / 2)
    return s


def test_poisson_convergence_second_order():
    ref = poisson_center_value()
    errs = []
    for n in (8, 16, 32):
        S = fem.PDESampler(n, 1.0, [0.0], [1], [1])
        u = grid(S.solve_one([0.0]), n)
        errs.append(abs(u[n // 2 - 1, n // 2 - 1] - ref))
    assert 3.5 < errs[0] / errs[1] < 4.5
    assert 3.5 < errs[1] / errs[2] < 4.5


def test_variable_coefficient_second_order():
    # centroid quadrature keeps O(h^2): successive differences at shared nodes shrink ~4x
    prob = W.pde_problem(64, 4, 8, modes="diagonal")
    y = np.array([0.2, 0.4, 0.6, 0.8])
    vals = []
    for n in (8, 16, 32, 64):
        S = fem.PDESampler(n, 1.0, prob["amp"], prob["mode1"], prob["mode2"])
        u = grid(S.solve_one(y), n)
        vals.append(u[n // 4 - 1 :: n // 4, n // 4 - 1 :: n // 4][:3, :3])
    d1 = np.abs(vals[1] - vals[0]).max()
    d2 = np.abs(vals[2] - vals[1]).max()
    d3 = np.abs(vals[3] - vals[2]).max()
    assert 3.0 < d1 / d2 < 5.0 and 3.0 < d2 / d3 < 5.0


def test_symmetries_of_diagonal_modes():
    n = 16
    prob = W.pde_problem(n, 4, 16, modes="diagonal")
    S = fem.PDESampler(n, 1.0, prob["amp"], prob["mode1"], prob["mode2"])
    y = np.array([0.13, 0.41, 0.77, 0.05])
    u = grid(S.solve_one(y), n)
    assert np.allclose(u, u.T, rtol=1e-12, atol=0)          # x1 <-> x2
    assert np.allclose(u, u[::-1, ::-1], rtol=1e-12, atol=0)  # x -> 1 - x
    # sin(2 pi (1/2 - y)) = sin(2 pi y): u is invariant under y_j -> 1/2 - y_j
    y2 = y.copy()
    y2[2] = 0.5 - y2[2]
    assert np.allclose(S.solve_one(y), S.solve_one(y2), rtol=1e-13, atol=0)


def test_banded_equals_dense():
    n = 9
    prob = W.pde_problem(n, 5, 8)
    mesh = fem.Mesh(n)
    a_tri = fem.coefficient_on_triangles(mesh, 1.0, prob["amp"], prob["mode1"], prob["mode2"], np.linspace(0.1, 0.9, 5))
    A = fem.dense_stiffness(mesh, a_tri)
    ab = fem.banded_stiffness(mesh, a_tri)
    B = np.zeros_like(A)
    for r in range(ab.shape[0]):
        off = mesh.bw - r
        for j in range(off, mesh.G):
            B[j - off, j] = ab[r, j]
            B[j, j - off] = ab[r, j]
    assert np.allclose(A, B, rtol=0, atol=1e-14)
