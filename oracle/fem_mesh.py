"""P1 finite-element sampler on a general triangulation (oracle side).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline, never by the library.

The paper samples the parametric problem of Sec. 1 (eq. (1.1), (1.2)) with a
finite element solver on an unstructured mesh of D = [0,1]^2 (Sec. 4: maximal
edge length 0.075, 737 inner and 104 boundary nodes); the spatial nodes T_G
are the inner mesh vertices.  What is computed here, for a triangulation
given by its vertices, triangles and boundary flags:
  * T_G = the vertices not flagged as boundary, in vertex order;
  * a constant on each triangle, its value at the centroid (the same one-point
    rule as the uniform mesh), from the coefficient models of fem.py;
  * the stiffness matrix from the textbook P1 element matrix
    K_T[a, b] = a_T |T| grad(phi_a) . grad(phi_b), restricted to T_G (zero
    Dirichlet data), and the load b_i = sum_{T containing i} |T| / 3 (f = 1,
    exact);
  * one sparse direct solve per parameter (scipy's SuperLU).

Pins (tests/test_oracle_fem_mesh.py): on the uniform right-triangle mesh given
as a general triangulation it reproduces the structured oracle fem.py; the
stiffness matrix annihilates linear functions at vertices whose patch is
interior (patch test) and is symmetric positive definite; manufactured
discrete solutions; the load sums to the area of the domain.
"""
import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.linalg import spsolve

from .fem import coefficient_on_triangles
from .periodization import PERIODIC, to_parameter


class TriMesh:
    """Geometry of a triangulation; independent of the parameter."""

    def __init__(self, xy, tri, boundary):
        self.xy = np.asarray(xy, dtype=np.float64)
        self.tri = np.asarray(tri, dtype=np.int64)
        bnd = np.asarray(boundary, dtype=bool)
        self.interior = np.nonzero(~bnd)[0]
        self.G = len(self.interior)
        gid = -np.ones(len(self.xy), dtype=np.int64)
        gid[self.interior] = np.arange(self.G)
        self.node = gid[self.tri]  # (T, 3), -1 for boundary vertices
        P = self.xy[self.tri]  # (T, 3, 2)
        self.centroid = P.mean(axis=1)
        e1 = P[:, 1] - P[:, 0]
        e2 = P[:, 2] - P[:, 0]
        det = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
        self.area = 0.5 * np.abs(det)
        # gradients of the barycentric functions: rows of the inverse Jacobian
        g1 = np.stack([e2[:, 1] / det, -e2[:, 0] / det], -1)
        g2 = np.stack([-e1[:, 1] / det, e1[:, 0] / det], -1)
        grads = np.stack([-(g1 + g2), g1, g2], 1)
        self.kgeo = self.area[:, None, None] * np.einsum("tad,tbd->tab", grads, grads)
        load = np.zeros(self.G)
        for a in range(3):
            m = self.node[:, a] >= 0
            np.add.at(load, self.node[m, a], self.area[m] / 3.0)
        self.load = load
        self.load_all = np.zeros(len(self.xy))
        for a in range(3):
            np.add.at(self.load_all, self.tri[:, a], self.area / 3.0)

    def stiffness(self, a_tri):
        """Interior stiffness matrix (CSR) for triangle coefficients a_tri."""
        rows, cols, vals = [], [], []
        for a in range(3):
            for b in range(3):
                na, nb = self.node[:, a], self.node[:, b]
                m = (na >= 0) & (nb >= 0)
                rows.append(na[m])
                cols.append(nb[m])
                vals.append(a_tri[m] * self.kgeo[m, a, b])
        A = coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(self.G, self.G))
        return A.tocsr()


class MeshSampler:
    """Black-box sampler of Sec. 2.1 on a general triangulation."""

    def __init__(self, xy, tri, boundary, a0, amp, mode1, mode2, model=PERIODIC, alpha=-1.0, beta=1.0,
                 delta=0.0, basis=(0, 0)):
        self.mesh = TriMesh(xy, tri, boundary)
        self.G = self.mesh.G
        self.a0 = float(a0)
        self.amp = np.asarray(amp, dtype=np.float64)
        self.mode1 = np.asarray(mode1)
        self.mode2 = np.asarray(mode2)
        self.model, self.alpha, self.beta, self.delta, self.basis = model, alpha, beta, delta, tuple(basis)

    def solve_param(self, y):
        a = coefficient_on_triangles(self.mesh, self.a0, self.amp, self.mode1, self.mode2,
                                     np.asarray(y, dtype=np.float64), self.model, self.basis)
        return spsolve(self.mesh.stiffness(a).tocsc(), self.mesh.load)

    def solve_one(self, t):
        """One solve at the sampling node t in T^d (y = phi(t), Sec. 3.2)."""
        return self.solve_param(to_parameter(self.model, t, self.alpha, self.beta, self.delta))

    def __call__(self, Y):
        Y = np.atleast_2d(np.asarray(Y, dtype=np.float64))
        out = np.empty((len(Y), self.G))
        for s in range(len(Y)):
            out[s] = self.solve_one(Y[s])
        return out
