"""Finite-element solutions at a node set T_G that is not the mesh's vertex
set (oracle side; Sec. 3.1: the sampler's values at the nodes x_g may have
to be interpolated from the discretisation).

TEST INFRASTRUCTURE ONLY: imported by tests/, never by the library.

The P1 solution is the piecewise linear function with the computed values at
the inner vertices and 0 at the boundary vertices, so its value at a point x
of triangle T is sum_a lambda_a(x) u(v_a) over T's vertices, lambda the
barycentric coordinates of x in T.  Here every point is located by brute
force: the barycentric coordinates of x in every triangle, and the first
triangle (lowest index) in which none is below -1e-12 contains it.  Points on
a shared edge may take either triangle: the P1 function is continuous there.

Pins (tests/test_oracle_interp.py): linear functions are reproduced exactly
at arbitrary points on both meshes; points at vertices reproduce the nodal
values; the coordinates are a partition of unity; points outside the
domain are rejected.
"""
import numpy as np


def barycentric(xy, tri, pts):
    """(npts, ntri, 3) barycentric coordinates of every point in every triangle."""
    P = np.asarray(xy, dtype=np.float64)[np.asarray(tri)]  # (T, 3, 2)
    x = np.asarray(pts, dtype=np.float64)[:, None, :]      # (n, 1, 2)
    e1 = P[:, 1] - P[:, 0]
    e2 = P[:, 2] - P[:, 0]
    det = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
    r = x - P[None, :, 0]                                   # (n, T, 2)
    l1 = (r[..., 0] * e2[:, 1] - r[..., 1] * e2[:, 0]) / det
    l2 = (e1[:, 0] * r[..., 1] - e1[:, 1] * r[..., 0]) / det
    return np.stack([1.0 - l1 - l2, l1, l2], -1)


def locate(xy, tri, pts, tol=1e-12):
    """First containing triangle of every point and its barycentric coordinates."""
    lam = barycentric(xy, tri, pts)
    inside = lam.min(axis=2) >= -tol
    if not inside.any(axis=1).all():
        raise ValueError("a node lies outside the triangulation")
    t = inside.argmax(axis=1)
    return t, lam[np.arange(len(t)), t]


def interpolation_matrix(xy, tri, boundary, pts):
    """(npts, G) matrix taking the inner-vertex values (vertex order) to the points."""
    boundary = np.asarray(boundary, dtype=bool)
    inner = np.nonzero(~boundary)[0]
    gid = -np.ones(len(boundary), dtype=np.int64)
    gid[inner] = np.arange(len(inner))
    t, lam = locate(xy, tri, pts)
    A = np.zeros((len(pts), len(inner)))
    for p in range(len(pts)):
        for a in range(3):
            g = gid[tri[t[p]][a]]
            if g >= 0:
                A[p, g] += lam[p, a]
    return A


class InterpolatingSampler:
    """A mesh-vertex sampler followed by interpolation to the points."""

    def __init__(self, sampler, xy, tri, boundary, pts):
        self.sampler = sampler
        self.A = interpolation_matrix(xy, tri, boundary, pts)
        self.G = len(self.A)

    def __call__(self, Y):
        return self.sampler(Y) @ self.A.T

    def solve_one(self, t):
        return self.A @ self.sampler.solve_one(t)

    def solve_param(self, y):
        return self.A @ self.sampler.solve_param(y)
