"""Whole-driver pins: exact recovery of seeded sparse trigonometric polynomials
(the event of Theorem 1.1), the PDE run against the Fourier coefficients it
approximates (full-grid DFT of the solves), and invariants of the PDE run."""
import numpy as np
import pytest

from oracle import fem
from oracle.usfft import TrigPolySampler, evaluate, usfft
import workloads as W


@pytest.mark.parametrize("seed,d,N,G,nf", [(1, 3, 8, 5, 21), (2, 5, 16, 12, 41), (3, 8, 32, 7, 61)])
def test_exact_recovery_of_trig_polynomials(seed, d, N, G, nf):
    K, P = W.trig_poly(seed, d, N, G, nf, cmin=1e-2)
    S = TrigPolySampler(K, P)
    theta = 1e-6
    res = usfft(S, d, [-N] * d, [N] * d, 2 * nf, 2 * nf, 4, theta, False, seed)
    support = {tuple(k) for k, row in zip(K.tolist(), P) if np.abs(row).max() > 0}
    found = {tuple(k) for k in res.I.tolist()}
    assert found == support
    idx = {tuple(k): a for a, k in enumerate(K.tolist())}
    for a, k in enumerate(res.I.tolist()):
        assert np.allclose(res.C[a], P[idx[tuple(k)]], rtol=0, atol=1e-12)
    # evaluation reproduces the polynomial
    Y = np.random.default_rng(seed).random((7, d))
    assert np.allclose(evaluate(res.I, res.C, Y), S(Y), atol=1e-11)


def test_sets_are_lexicographic_and_symmetric_pde():
    prob, par = W.WORKLOADS["cpu16_d4"]
    S = fem.PDESampler(prob["mesh_n"], prob["a0"], prob["amp"], prob["mode1"], prob["mode2"])
    res = usfft(S, prob["d"], prob["k_lo"], prob["k_hi"], par["s"], par["s_local"], par["r"], par["theta"], True, 11)
    I = res.I.tolist()
    assert I == sorted(I)
    assert {tuple(k) for k in I} == {tuple(-v for v in k) for k in I}  # real u: +-closed
    # coefficients of -k are conjugates of those of k, bitwise
    idx = {tuple(k): a for a, k in enumerate(I)}
    for a, k in enumerate(I):
        b = idx[tuple(-v for v in k)]
        assert np.array_equal(res.C[b], np.conj(res.C[a]))
    # the mean coefficient is the largest and positive (u > 0 for f = 1)
    z = idx[tuple([0] * prob["d"])]
    assert (res.C[z].real > 0).all()


def test_step3_on_a_given_superset_recovers_the_polynomial():
    # Sec. 4.5: step 3 alone on an a-priori set.  On any set containing the
    # support (here with extra frequencies, in shuffled order) the lattice
    # family reconstructs the polynomial exactly: its coefficients, and zero
    # on the frequencies it does not use
    from oracle.usfft import coefficients
    d, N = 4, 8
    K, P = W.trig_poly(11, d, N, 6, 31, cmin=1e-2)
    extra = W.hyperbolic_cross(d, N, [4] * d)
    I = np.unique(np.vstack([K, extra]), axis=0)
    I = I[np.random.default_rng(2).permutation(len(I))]
    C, fam, ns = coefficients(TrigPolySampler(K, P), I, seed=5)
    idx = {tuple(k): a for a, k in enumerate(K.tolist())}
    for a, k in enumerate(I.tolist()):
        want = P[idx[tuple(k)]] if tuple(k) in idx else 0.0
        assert np.allclose(C[a], want, rtol=0, atol=1e-12)
    assert ns == sum(fam.M)
    C0, fam0, ns0 = coefficients(TrigPolySampler(K, P), np.zeros((0, d), dtype=int), seed=5)
    assert C0.shape == (0, 6) and ns0 == 0


def test_a_priori_sets_match_their_definitions():
    # Sec. 4.5 index sets against brute-force enumeration of the box
    import itertools
    d, N = 3, 6
    box = list(itertools.product(range(-N, N + 1), repeat=d))
    mult = [1, 2, 3]
    cases = [
        (W.axis_cross(d, N), lambda k: sum(1 for v in k if v) <= 1 and sum(map(abs, k)) <= N),
        (W.hyperbolic_cross(d, N, [4] * d), lambda k: np.prod([max(1, 4 * abs(v)) for v in k]) <= N),
        (W.hyperbolic_cross(d, N, mult), lambda k: np.prod([max(1, m * abs(v)) for m, v in zip(mult, k)]) <= N),
        (W.weighted_l1_ball(d, N, mult), lambda k: sum(m * abs(v) for m, v in zip(mult, k)) <= N),
    ]
    for got, test in cases:
        assert got.tolist() == sorted([list(k) for k in box if test(k)])


@pytest.mark.parametrize("case", range(3))
def test_degenerate_runs(case):
    name, K, P, lo, hi, theta, r = W.degenerate_trig_cases()[case]
    d = K.shape[1]
    res = usfft(TrigPolySampler(K, P), d, lo, hi, 40, 40, r, theta, False, 7)
    support = {tuple(k) for k, row in zip(K.tolist(), P) if np.abs(row).max() > 0}
    if name == "empty":
        assert res.I.shape == (0, d) and res.C.shape == (0, P.shape[1])
        assert res.samples == d * r * 17  # step 1 only
        return
    assert {tuple(k) for k in res.I.tolist()} == support
    idx = {tuple(k): a for a, k in enumerate(K.tolist())}
    for a, k in enumerate(res.I.tolist()):
        assert np.allclose(res.C[a], P[idx[tuple(k)]], rtol=0, atol=1e-12)


def _full_grid_coefficients(S, d, P):
    """c_k(x_g) of t -> u(x_g, t) by the plain d-dimensional DFT of the solves
    on the full grid (j / P)^d: exact up to aliasing from |k|_inf >= P / 2."""
    ax = np.arange(P) / P
    grid = np.stack(np.meshgrid(*([ax] * d), indexing="ij"), -1).reshape(-1, d)
    U = S(grid)
    return np.fft.fftn(U.reshape((P,) * d + (S.G,)), axes=tuple(range(d))) / P ** d


@pytest.mark.parametrize("d,N,P,theta", [(2, 12, 64, 1e-5), (2, 12, 64, 1e-7), (3, 10, 32, 1e-5)])
def test_pde_run_against_full_grid_fourier_coefficients(d, N, P, theta):
    # What the PDE run approximates, by its definition: the Fourier
    # coefficients of the parametric solution (Sec. 1), here from a full
    # tensor grid (for this smooth coefficient they fall below 1e-11 at
    # |k|_inf = P / 2, so the grid values stand for the true ones to ~1e-11).
    #  - step 3 reads c_k from a lattice on which k aliases with no other
    #    frequency of I, so its error is at most the l1 norm T_g of the
    #    coefficients outside I;
    #  - the final selection keeps a frequency only where its computed value
    #    reaches theta, so its true value is at least theta - T_g there;
    #  - every frequency of the box whose coefficient is ten times theta is
    #    detected.
    # A conjugated transform, a lost 1/M, a shifted node or a dropped stage
    # breaks the first bound by orders of magnitude.
    prob = W.pde_problem(8, d, N)
    S = fem.PDESampler(prob["mesh_n"], prob["a0"], prob["amp"], prob["mode1"], prob["mode2"])
    res = usfft(S, d, prob["k_lo"], prob["k_hi"], 100, 100, 3, theta, True, 5)
    F = _full_grid_coefficients(S, d, P)
    slack = 1e-10
    I = [tuple(k) for k in res.I.tolist()]
    cell = lambda k: tuple(v % P for v in k)
    outside = np.ones((P,) * d, dtype=bool)
    for k in I:
        outside[cell(k)] = False
    T = np.abs(F)[outside].sum(axis=0)  # (G,)
    th = np.sqrt(res.theta2)
    for a, k in enumerate(I):
        ck = F[cell(k)]
        assert (np.abs(res.C[a] - ck) <= T + slack).all(), k
        assert (np.abs(ck) + T + slack).max() >= th, k
    big = [k for k in np.ndindex(*([2 * N + 1] * d))
           if np.abs(F[cell([v - N for v in k])]).max() >= 10 * th]
    assert {tuple(v - N for v in k) for k in big} <= set(I)
    assert len(big) > 10


def test_relative_threshold_reading_first_stage():
    # Reading of the relative threshold: theta_abs = theta_rel * max |u^_k(x_g)|
    # over the first detection stage (coordinate 1, iteration 1).  Rebuilt
    # here from the stage's definition (nodes l / K in coordinate 1, the
    # iteration's seeded tail elsewhere) with numpy's FFT in place of the
    # oracle's DFT, over every node and all K bins.
    from oracle import rng
    prob = W.pde_problem(8, 3, 4)
    S = fem.PDESampler(prob["mesh_n"], prob["a0"], prob["amp"], prob["mode1"], prob["mode2"])
    d, theta, seed = prob["d"], 1e-3, 7
    res = usfft(S, d, prob["k_lo"], prob["k_hi"], 20, 20, 2, theta, True, seed)
    K = prob["k_hi"][0] - prob["k_lo"][0] + 1
    code = rng.stream_code(rng.KIND_TAIL1, 1, 1)
    Y = np.array([[l / K if j == 0 else rng.uniform01(seed, code, j) for j in range(d)] for l in range(K)])
    F = np.fft.fft(S(Y), axis=0) / K
    want = theta ** 2 * (np.abs(F) ** 2).max()
    assert abs(res.theta2 - want) <= 1e-12 * want
    # a later stage's maximum gives a different threshold
    code2 = rng.stream_code(rng.KIND_TAIL1, 2, 1)
    Y2 = np.array([[l / K if j == 1 else rng.uniform01(seed, code2, j) for j in range(d)] for l in range(K)])
    F2 = np.fft.fft(S(Y2), axis=0) / K
    assert abs(theta ** 2 * (np.abs(F2) ** 2).max() - want) > 1e-9 * want
