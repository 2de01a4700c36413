"""Pins of the oracle's post-processing (Sec. 4, Sec. 4.1)."""
import itertools

import numpy as np
from numpy.polynomial.hermite_e import hermegauss
from numpy.polynomial.legendre import leggauss

from oracle import evaluation as ev
from oracle import periodization as per


def _gauss_legendre(a, b, n):
    x, w = leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def _gauss_normal(n):
    # nodes and weights of E[f(Y)], Y ~ N(0, 1)
    x, w = hermegauss(n)
    return x, w / np.sqrt(2 * np.pi)


def test_affine_d_factor_is_the_uniform_mean_of_the_mode():
    # D_k = E e^{2 pi i k phi^{-1}(y)}, y ~ U[alpha, beta] (Sec. 4.1), by quadrature
    for alpha, beta in ((-1.0, 1.0), (0.2, 3.0)):
        y, w = _gauss_legendre(alpha, beta, 80)
        for k in range(-7, 8):
            quad = np.sum(w * np.exp(2j * np.pi * k * per.tent_inv(y, alpha, beta))) / (beta - alpha)
            assert abs(ev.d_factors([[k]], per.AFFINE)[0] - quad) < 1e-13, (alpha, beta, k)


def test_lognormal_d_factor_is_the_gaussian_mean_of_the_mode():
    y, w = _gauss_normal(300)
    for delta in (0.0, 1.0 / (4 * 9601), 0.013):
        for k in range(-7, 8):
            quad = np.sum(w * np.exp(2j * np.pi * k * per.lognormal_inv(y, delta)))
            assert abs(ev.d_factors([[k]], per.LOGNORMAL, delta)[0] - quad) < 1e-13, (delta, k, quad)


def test_expectation_matches_tensor_quadrature_of_the_approximation():
    g = np.random.default_rng(3)
    I = np.array(list(itertools.product(range(-3, 4), repeat=2)))
    C = g.standard_normal((len(I), 3)) + 1j * g.standard_normal((len(I), 3))
    # periodic: the mean over an aliasing-free grid of the torus
    t = (np.arange(9) + 0.25) / 9
    T = np.array(list(itertools.product(t, t)))
    ref = ev.approximation(I, C, T).mean(axis=0) + 1j * ev.approximation(I, -1j * C, T).mean(axis=0)
    assert np.allclose(ev.expectation(I, C, per.PERIODIC), ref, rtol=0, atol=1e-13)
    # affine on [alpha, beta]^2: Gauss-Legendre tensor rule
    alpha, beta = -1.0, 2.0
    y, w = _gauss_legendre(alpha, beta, 40)
    Y = np.array(list(itertools.product(y, y)))
    W = np.outer(w, w).ravel() / (beta - alpha) ** 2
    re = W @ ev.approximation(I, C, Y, per.AFFINE, alpha, beta)
    im = W @ ev.approximation(I, -1j * C, Y, per.AFFINE, alpha, beta)
    assert np.allclose(ev.expectation(I, C, per.AFFINE), re + 1j * im, rtol=0, atol=1e-12)
    # lognormal, N(0, I_2): Gauss-Hermite tensor rule
    delta = 0.01
    y, w = _gauss_normal(120)
    Y = np.array(list(itertools.product(y, y)))
    W = np.outer(w, w).ravel()
    re = W @ ev.approximation(I, C, Y, per.LOGNORMAL, delta=delta)
    im = W @ ev.approximation(I, -1j * C, Y, per.LOGNORMAL, delta=delta)
    assert np.allclose(ev.expectation(I, C, per.LOGNORMAL, delta), re + 1j * im, rtol=0, atol=1e-9)


def _grid_function(I, C, N):
    # u~(t) = sum_k c_k e^{2 pi i k.t} on the full N^d grid, axes in order
    d = I.shape[1]
    t = np.arange(N) / N
    T = np.array(list(itertools.product(*([t] * d))))
    F = np.exp(2j * np.pi * (T @ I.T)) @ C
    return F.reshape((N,) * d + (C.shape[1],))


def test_variance_is_the_mean_square_minus_the_squared_mean():
    g = np.random.default_rng(5)
    I = np.array(list(itertools.product(range(-3, 4), repeat=3)))
    I = I[g.random(len(I)) < 0.3]
    I = np.vstack([np.zeros((1, 3), dtype=int), I[np.any(I != 0, axis=1)]])
    C = g.standard_normal((len(I), 2)) + 1j * g.standard_normal((len(I), 2))
    F = _grid_function(I, C, 8)  # |u~|^2 has frequencies in [-6, 6]^3: 8 points are exact
    ref = np.mean(np.abs(F) ** 2, axis=(0, 1, 2)) - np.abs(np.mean(F, axis=(0, 1, 2))) ** 2
    assert np.allclose(ev.variance(I, C), ref, rtol=1e-13, atol=0)


def test_sensitivity_indices_are_the_anova_variance_shares():
    # ANOVA terms by brute force on the grid: f_u = sum_{v in u} (-1)^{|u|-|v|} P_v f,
    # P_v = mean over the coordinates outside v; rho(J_l) = sum_{|u| = l} var(f_u) / var(f)
    g = np.random.default_rng(6)
    d, N = 3, 8
    I = np.array(list(itertools.product(range(-3, 4), repeat=d)))
    I = I[g.random(len(I)) < 0.35]
    C = g.standard_normal((len(I), 2)) + 1j * g.standard_normal((len(I), 2))
    F = _grid_function(I, C, N)

    def proj(v):
        out = F
        for ax in range(d):
            if ax not in v:
                out = out.mean(axis=ax, keepdims=True)
        return out

    total = np.mean(np.abs(F - proj(())) ** 2, axis=tuple(range(d)))
    share = np.zeros((d, 2))
    for l in range(1, d + 1):
        for u in itertools.combinations(range(d), l):
            fu = sum((-1) ** (l - len(v)) * proj(v) for m in range(l + 1) for v in itertools.combinations(u, m))
            share[l - 1] += np.mean(np.abs(np.broadcast_to(fu, F.shape)) ** 2, axis=tuple(range(d)))
    rho = ev.sensitivity_indices(I, C)
    assert np.allclose(rho, share / total, rtol=0, atol=1e-12)
    assert np.allclose(rho.sum(axis=0), 1.0, rtol=0, atol=1e-12)
    # an additive function has all of its variance in J_1
    I1 = np.array([[0, 0, 0], [2, 0, 0], [0, -1, 0], [0, 0, 3]])
    rho1 = ev.sensitivity_indices(I1, np.ones((4, 1)))
    assert np.array_equal(rho1[:, 0], [1.0, 0.0, 0.0])
    # no variance: every index is 0
    assert np.array_equal(ev.sensitivity_indices(np.zeros((1, 3), dtype=int), np.ones((1, 1))), np.zeros((3, 1)))


def test_error_measures():
    n, G = 7, 3
    U = np.random.default_rng(1).standard_normal((n, G))
    for c in (0.0, 0.25, -3.0):
        for p in (1.0, 2.0, 3.5):
            ep, ei = ev.errors(U + c, U, p)
            assert np.allclose(ep, abs(c), rtol=1e-14, atol=0) and np.allclose(ei, abs(c), rtol=1e-14, atol=0)
    D = np.array([1.0, -2.0, 3.0, 4.0])[:, None]
    e1, ei = ev.errors(D, np.zeros_like(D), 1.0)
    e2, _ = ev.errors(D, np.zeros_like(D), 2.0)
    assert e1[0] == 2.5 and ei[0] == 4.0 and abs(e2[0] - np.sqrt(7.5)) < 1e-15
