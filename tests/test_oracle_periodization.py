"""Pins of the oracle's periodizations (Sec. 3.2, Lemma 3.1) and coefficient models."""
import numpy as np
from scipy.stats import norm

from oracle import fem
from oracle import periodization as P
from oracle.lattice import lattice_nodes


def test_tent_conditions_and_inverse():
    # (A1)-(A4) of Sec. 3.2 and the inverse against bisection on phi itself
    for alpha, beta in ((-1.0, 1.0), (-0.5, 0.5), (0.2, 3.0)):
        t = np.linspace(0.0, 1.0, 4001)
        f = P.tent(t, alpha, beta)
        assert abs(f[0] - alpha) < 1e-14 and abs(f[-1] - alpha) < 1e-14 and abs(P.tent(0.5, alpha, beta) - beta) < 1e-14
        assert np.max(np.abs(np.diff(f))) <= 2.0 * (beta - alpha) * (t[1] - t[0]) * (1 + 1e-12)
        h = t[t <= 0.5]
        assert np.allclose(P.tent(0.5 - h, alpha, beta), P.tent(0.5 + h, alpha, beta), rtol=0, atol=1e-15)
        assert np.all(np.diff(P.tent(h, alpha, beta)) > 0)
        ys = np.linspace(alpha, beta, 97)
        lo, hi = np.zeros_like(ys), np.full_like(ys, 0.5)
        for _ in range(60):  # bisection for phi(t) = y on [0, 1/2]
            mid = 0.5 * (lo + hi)
            up = P.tent(mid, alpha, beta) < ys
            lo, hi = np.where(up, mid, lo), np.where(up, hi, mid)
        assert np.allclose(P.tent_inv(ys, alpha, beta), 0.5 * (lo + hi), rtol=0, atol=1e-14)
        assert np.allclose(P.tent(P.tent_inv(ys, alpha, beta), alpha, beta), ys, rtol=0, atol=1e-14)


def test_shifted_tent_continuity_and_inverse():
    for delta in (0.1, 1e-3, P.delta_opt(9601)):
        eps = 1e-12
        for k in (delta, 0.5 + delta):  # the kinks
            assert abs(P.tau2(k - eps, delta) - P.tau2(k + eps, delta)) < 1e-10
        assert P.tau2(delta, delta) == -0.5 and abs(P.tau2(0.5 + delta, delta) - 0.5) < 1e-15
        t = np.linspace(0.0, 1.0 - 1e-9, 5001)
        v = P.tau2(t, delta)
        assert v.min() >= -0.5 - 1e-15 and v.max() <= 0.5 + 1e-15
        assert abs(P.tau2(0.0, delta) - P.tau2(1.0, delta)) < 1e-12  # 1-periodic
        s = np.linspace(delta, 0.5 + delta, 101)
        assert np.allclose(P.tau2_inv(P.tau2(s, delta), delta), s, rtol=0, atol=1e-15)


def test_tau1_is_the_normal_quantile():
    # tau_1 maps U(-1/2, 1/2) to N(0, 1): Phi(tau_1(v)) = v + 1/2 with the
    # normal CDF from scipy.stats, and tau_1^{-1} inverts it
    v = np.linspace(-0.499, 0.499, 999)
    assert np.allclose(norm.cdf(P.tau1(v)), v + 0.5, rtol=0, atol=1e-13)
    y = np.linspace(-4, 4, 81)  # erf saturates beyond: the round trip loses digits there
    assert np.allclose(P.tau1(P.tau1_inv(y)), y, rtol=0, atol=1e-8)
    assert P.tau1(0.0) == 0.0
    t = np.linspace(0.0, 1.0, 2001)[:-1] + 0.5 / 2000
    delta = 0.013
    y = P.lognormal_map(t, delta)
    s = t[(t > delta + 1e-9) & (t < 0.5 + delta - 1e-9)]
    assert np.allclose(P.lognormal_inv(P.lognormal_map(s, delta), delta), s, rtol=0, atol=1e-12)
    assert np.all(np.isfinite(y))


def test_lemma_delta_opt_by_brute_force():
    # min over the lattice nodes of the distances to Delta and Delta + 1/2 is
    # largest at Delta = 1/(4M) among 0 < Delta < 1/(2M) (Lemma 3.1)
    g = np.random.default_rng(4)
    for M in (5, 7, 11, 13, 31):
        z = g.integers(1, M, size=3)
        nodes = lattice_nodes(M, z).ravel()
        ds = np.linspace(0.0, 1.0 / (2 * M), 2001)[1:-1]
        f = [min(np.min(np.abs(nodes - d)), np.min(np.abs(nodes - (d + 0.5)))) for d in ds]
        best = ds[int(np.argmax(f))]
        assert abs(best - P.delta_opt(M)) <= (ds[1] - ds[0])
        assert abs(max(f) - P.delta_opt(M)) < 1e-12


def test_models_reduce_to_constant_coefficient():
    # tent: t = 1/4 gives y = (alpha + beta)/2 = 0 on [-1, 1]; lognormal:
    # t = 1/4 + Delta gives y = 0, so a = a0 + 1; both solves equal the
    # constant-coefficient ones
    n, d = 12, 4
    amp, m1, m2 = [0.3, 0.2, 0.1, 0.05], [1, 2, 1, 3], [1, 1, 2, 2]
    const = fem.PDESampler(n, 1.0, [0.0] * d, m1, m2)
    aff = fem.PDESampler(n, 1.0, amp, m1, m2, model=P.AFFINE, alpha=-1.0, beta=1.0)
    assert np.allclose(aff.solve_one(np.full(d, 0.25)), const.solve_one(np.zeros(d)), rtol=1e-13, atol=0)
    delta = 0.01
    logn = fem.PDESampler(n, 0.5, amp, m1, m2, model=P.LOGNORMAL, delta=delta, basis=(0, 1))
    const2 = fem.PDESampler(n, 1.5, [0.0] * d, m1, m2)
    assert np.allclose(logn.solve_one(np.full(d, 0.25 + delta)), const2.solve_one(np.zeros(d)), rtol=1e-13, atol=0)


def test_lognormal_coefficient_positive_and_affine_linear():
    mesh = fem.Mesh(8)
    amp, m1, m2 = np.array([2.0, 1.5]), [1, 2], [3, 1]
    y = np.array([3.0, -4.0])
    a = fem.coefficient_on_triangles(mesh, 0.0, amp, m1, m2, y, model=P.LOGNORMAL, basis=(1, 0))
    assert np.all(a > 0)
    b = np.log(a)
    cx, cy = mesh.centroid[:, 0], mesh.centroid[:, 1]
    ref = 2.0 * 3.0 * np.cos(np.pi * cx) * np.sin(3 * np.pi * cy) - 1.5 * 4.0 * np.cos(2 * np.pi * cx) * np.sin(np.pi * cy)
    assert np.allclose(b, ref, rtol=0, atol=1e-12)
    # affine: a - a0 is linear in y
    a1 = fem.coefficient_on_triangles(mesh, 1.0, amp, m1, m2, y, model=P.AFFINE)
    a2 = fem.coefficient_on_triangles(mesh, 1.0, amp, m1, m2, 2 * y, model=P.AFFINE)
    assert np.allclose(a2 - 1.0, 2 * (a1 - 1.0), rtol=1e-14, atol=1e-14)
