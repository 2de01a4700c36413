"""Whole-driver pins: exact recovery of seeded sparse trigonometric polynomials
(the event of Theorem 1.1) and invariants of the PDE run."""
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
