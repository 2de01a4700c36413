"""P1 finite-element sampler of the parametric diffusion problem (oracle side).

What is computed (Sec. 1, eq. (1.1) and (1.2); weak form in Sec. 2.1):
    -div(a(x, y) grad u) = f on D = (0,1)^2, u = 0 on the boundary,
    a(x, y) = a0 + sum_j amp_j * sin(2 pi y_j) * sin(m1_j pi x1) * sin(m2_j pi x2),
for one parameter vector y per solve.  The paper treats the solver as a black
box (Sec. 2.1); this build freezes one discretisation so that both sides solve
the same discrete system:
  * uniform grid, h = 1/n, interior nodes x_g = (i h, j h), 1 <= i, j <= n-1,
    numbered g = (j-1)(n-1) + (i-1);
  * every cell [ih,(i+1)h] x [jh,(j+1)h] is split by the diagonal from (i,j)
    to (i+1,j+1) into a lower triangle {(i,j),(i+1,j),(i+1,j+1)} and an upper
    triangle {(i,j),(i,j+1),(i+1,j+1)};
  * a is taken constant on each triangle, equal to its value at the centroid
    (one-point rule); f = 1 is integrated exactly.

The stiffness matrix is assembled triangle by triangle from the textbook
P1 element matrix  K_T[a,b] = a_T * |T| * grad(phi_a) . grad(phi_b)  and the
system is solved by a banded Cholesky factorisation (LAPACK via scipy).

Coefficient models (Sec. 1 and 3.2): periodic (the default above), affine
a = a0 + sum_j amp_j y_j psi_j and lognormal a = a0 + exp(sum_j amp_j y_j
psi_j), with the parameter y = phi(t) of the usFFT node t given by the
periodizations in oracle/periodization.py; psi_j = B1(m1 pi x1) B2(m2 pi x2)
with B = sin or cos per axis.

Pins (tests/test_oracle_fem.py, tests/test_oracle_periodization.py): a = 1 against the discrete sine eigenbasis
closed form; manufactured discrete solutions; O(h^2) convergence to a smooth
continuous solution; reflection symmetries of the mesh and coefficient.
"""
import numpy as np
from scipy.linalg import solveh_banded

from .periodization import LOGNORMAL, PERIODIC, to_parameter


def triangles(n):
    """Vertex grid coordinates (i, j) of all 2 n^2 triangles, shape (2n^2, 3, 2)."""
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    i = i.ravel()
    j = j.ravel()
    lower = np.stack([np.stack([i, j], -1), np.stack([i + 1, j], -1), np.stack([i + 1, j + 1], -1)], 1)
    upper = np.stack([np.stack([i, j], -1), np.stack([i, j + 1], -1), np.stack([i + 1, j + 1], -1)], 1)
    return np.concatenate([lower, upper], 0)


class Mesh:
    """Geometry of the uniform triangulation; independent of y."""

    def __init__(self, n):
        self.n = n
        self.h = 1.0 / n
        self.G = (n - 1) * (n - 1)
        tri = triangles(n)
        xy = tri.astype(np.float64) * self.h  # (T, 3, 2)
        self.centroid = xy.mean(axis=1)
        # gradients of the three barycentric functions on each triangle
        e1 = xy[:, 1] - xy[:, 0]
        e2 = xy[:, 2] - xy[:, 0]
        det = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
        self.area = 0.5 * np.abs(det)
        # inverse of [[e1x, e2x], [e1y, e2y]]; rows give grad(phi1), grad(phi2)
        inv = np.empty((len(xy), 2, 2))
        inv[:, 0, 0] = e2[:, 1] / det
        inv[:, 0, 1] = -e2[:, 0] / det
        inv[:, 1, 0] = -e1[:, 1] / det
        inv[:, 1, 1] = e1[:, 0] / det
        g1 = inv[:, 0, :]
        g2 = inv[:, 1, :]
        g0 = -(g1 + g2)
        grads = np.stack([g0, g1, g2], 1)  # (T, 3, 2)
        # geometric element matrices |T| grad phi_a . grad phi_b
        self.kgeo = self.area[:, None, None] * np.einsum("tad,tbd->tab", grads, grads)
        # global node ids, -1 for boundary vertices
        ii = tri[..., 0]
        jj = tri[..., 1]
        interior = (ii >= 1) & (ii <= n - 1) & (jj >= 1) & (jj <= n - 1)
        self.node = np.where(interior, (jj - 1) * (n - 1) + (ii - 1), -1)
        # load vector for f = 1: each vertex of T receives |T| / 3 (exact)
        load = np.zeros(self.G)
        for a in range(3):
            m = self.node[:, a] >= 0
            np.add.at(load, self.node[m, a], self.area[m] / 3.0)
        self.load = load
        # flattened scatter pattern into LAPACK upper banded storage
        # a triangle couples nodes up to (n-1)+1 apart in this numbering
        bw = n
        rows, cols, src = [], [], []
        for a in range(3):
            for b in range(3):
                na = self.node[:, a]
                nb = self.node[:, b]
                m = (na >= 0) & (nb >= 0) & (na <= nb)
                rows.append(bw + na[m] - nb[m])
                cols.append(nb[m])
                src.append(np.nonzero(m)[0] * 9 + a * 3 + b)
        self.band_rows = np.concatenate(rows)
        self.band_cols = np.concatenate(cols)
        self.band_src = np.concatenate(src)
        self.bw = bw

    def node_xy(self):
        g = np.arange(self.G)
        i = g % (self.n - 1) + 1
        j = g // (self.n - 1) + 1
        return i * self.h, j * self.h


def _axis(basis, m, x):
    """sin(m pi x) (basis 0) or cos(m pi x) (basis 1)."""
    return np.cos(m * np.pi * x) if basis == 1 else np.sin(m * np.pi * x)


def coefficient_on_triangles(mesh, a0, amp, mode1, mode2, y, model=PERIODIC, basis=(0, 0)):
    """Centroid values of a(x, y) for the parameter y, with
    psi_j(x) = B1(m1_j pi x1) B2(m2_j pi x2), B = sin or cos (eq. (1.2) and
    the models of Sec. 1):
      periodic:  a = a0 + sum_j amp_j sin(2 pi y_j) psi_j(x)
      affine:    a = a0 + sum_j amp_j y_j psi_j(x)
      lognormal: a = a0 + exp(sum_j amp_j y_j psi_j(x))."""
    cx = mesh.centroid[:, 0]
    cy = mesh.centroid[:, 1]
    b = np.zeros(len(cx))
    for j in range(len(amp)):
        theta = np.sin(2.0 * np.pi * y[j]) if model == PERIODIC else y[j]
        b += amp[j] * theta * _axis(basis[0], mode1[j], cx) * _axis(basis[1], mode2[j], cy)
    return float(a0) + (np.exp(b) if model == LOGNORMAL else b)


def banded_stiffness(mesh, a_tri):
    """Upper banded form (bw+1, G) of the assembled P1 stiffness matrix."""
    vals = (a_tri[:, None, None] * mesh.kgeo).reshape(-1)[mesh.band_src]
    ab = np.zeros((mesh.bw + 1, mesh.G))
    flat = mesh.band_rows * mesh.G + mesh.band_cols
    ab.ravel()[:] = np.bincount(flat, weights=vals, minlength=ab.size)
    return ab


def dense_stiffness(mesh, a_tri):
    """Dense assembled matrix (small meshes only)."""
    A = np.zeros((mesh.G, mesh.G))
    K = a_tri[:, None, None] * mesh.kgeo
    for a in range(3):
        for b in range(3):
            na = mesh.node[:, a]
            nb = mesh.node[:, b]
            m = (na >= 0) & (nb >= 0)
            np.add.at(A, (na[m], nb[m]), K[m, a, b])
    return A


def solve_banded(ab, rhs):
    return solveh_banded(ab, rhs, lower=False, check_finite=False)


class PDESampler:
    """Black-box sampler of Sec. 2.1: one solve per y gives u(x_g, y) for all g."""

    def __init__(self, n, a0, amp, mode1, mode2, model=PERIODIC, alpha=-1.0, beta=1.0, delta=0.0, basis=(0, 0)):
        self.mesh = Mesh(n)
        self.n = n
        self.a0 = float(a0)
        self.amp = np.asarray(amp, dtype=np.float64)
        self.mode1 = np.asarray(mode1)
        self.mode2 = np.asarray(mode2)
        self.G = self.mesh.G
        self.model, self.alpha, self.beta, self.delta, self.basis = model, alpha, beta, delta, tuple(basis)

    def solve_one(self, t):
        """One solve at the sampling node t in T^d (Sec. 3.2: y = phi(t))."""
        y = to_parameter(self.model, t, self.alpha, self.beta, self.delta)
        a = coefficient_on_triangles(self.mesh, self.a0, self.amp, self.mode1, self.mode2, y, self.model, self.basis)
        return solve_banded(banded_stiffness(self.mesh, a), self.mesh.load)

    def solve_param(self, y):
        """One solve at the parameter y itself (the test solves of Sec. 4)."""
        a = coefficient_on_triangles(self.mesh, self.a0, self.amp, self.mode1, self.mode2,
                                     np.asarray(y, dtype=np.float64), self.model, self.basis)
        return solve_banded(banded_stiffness(self.mesh, a), self.mesh.load)

    def __call__(self, Y):
        Y = np.atleast_2d(np.asarray(Y, dtype=np.float64))
        out = np.empty((len(Y), self.G))
        for s in range(len(Y)):
            out[s] = self.solve_one(Y[s])
        return out
