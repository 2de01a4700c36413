"""Pins of the oracle's DFT, lattice planner and selection/join."""
import itertools

import numpy as np
import pytest

from oracle import dft, lattice, rng, select
import workloads as W


def test_pure_tone_one_hot_on_lattice():
    M, z = 31, [1, 7]
    Y = lattice.lattice_nodes(M, z)
    k = np.array([2, -3])
    u = np.cos(2 * np.pi * Y @ k)  # = (e^{ik.y} + e^{-ik.y}) / 2
    F = dft.dft_bins(u[:, None], np.arange(M))[:, 0]
    b = (k @ np.array(z)) % M
    expect = np.zeros(M, complex)
    expect[b] += 0.5
    expect[(-b) % M] += 0.5
    assert np.allclose(F, expect, atol=1e-14)


def test_tensor_grid_dft_brute_force():
    # on the full grid (2N+1)^2 every k in [-N,N]^2 is its own bin: coefficients exact
    N = 3
    K = 2 * N + 1
    gen = np.random.default_rng(3)
    freqs = list(itertools.product(range(-N, N + 1), repeat=2))
    c = {f: gen.standard_normal() + 1j * gen.standard_normal() for f in freqs}
    for f in freqs:  # real signal
        if f > tuple(-v for v in f):
            c[f] = np.conj(c[tuple(-v for v in f)])
    c[(0, 0)] = c[(0, 0)].real
    pts = [(a / K, b / K) for a in range(K) for b in range(K)]
    u = np.array([sum((c[f] * np.exp(2j * np.pi * (f[0] * y0 + f[1] * y1))).real for f in freqs) for (y0, y1) in pts])
    # brute force 2-D DFT
    for f in freqs:
        brute = sum(u[a * K + b] * np.exp(-2j * np.pi * (f[0] * a + f[1] * b) / K) for a in range(K) for b in range(K)) / K ** 2
        assert abs(brute - c[f]) < 1e-12
    # the same coefficients through a rank-1 lattice z = (1, K) of size K^2 (tensor grid as a lattice)
    M = K * K
    Y = lattice.lattice_nodes(M, [1, K])
    uu = np.array([sum((c[f] * np.exp(2j * np.pi * (f[0] * y[0] + f[1] * y[1]))).real for f in freqs) for y in Y])
    Fb = dft.dft_bins(uu[:, None], [(f[0] + K * f[1]) % M for f in freqs])[:, 0]
    assert np.allclose(Fb, [c[f] for f in freqs], atol=1e-12)


def test_parseval_and_conjugate_bins():
    M = 29
    u = np.random.default_rng(2).standard_normal((M, 3))
    F = dft.dft_bins(u, np.arange(M))
    assert np.allclose((np.abs(F) ** 2).sum(0), (u ** 2).sum(0) / M, rtol=1e-12)
    # canonical half-spectrum: bins b and M-b are exact conjugates, bitwise
    for b in range(1, M):
        assert np.array_equal(F[b], np.conj(F[M - b]))


def sieve(n):
    s = np.ones(n + 1, bool)
    s[:2] = False
    for p in range(2, int(n ** 0.5) + 1):
        if s[p]:
            s[p * p :: p] = False
    return s


def test_prime_and_smooth_predicates():
    s = sieve(5000)
    for m in range(5000):
        assert lattice.is_prime(m) == bool(s[m])
    smooth = {a * b * c * d for a in [2 ** i for i in range(13)] for b in [3 ** i for i in range(8)]
              for c in [5 ** i for i in range(6)] for d in [7 ** i for i in range(5)]}
    for m in range(1, 5000):
        assert lattice.is_7smooth(m) == (m in smooth)


@pytest.mark.parametrize("seed,npar,t,nch", [(1, 60, 3, 9), (2, 80, 5, 9), (3, 9, 2, 33), (4, 1, 2, 1)])
def test_family_alias_free_by_brute_force(seed, npar, t, nch):
    parent, child = W.candidate_set(seed, npar, t, nch)
    J = select.product(parent, child)
    fam = lattice.plan_family(J, 2.0, 9601, 8, 64, seed, rng.KIND_LAT2, t)
    assert (fam.assign >= 0).all()
    for l, (M, z) in enumerate(zip(fam.M, fam.z)):
        assert lattice.admissible(M)
        members = np.nonzero(fam.assign == l)[0]
        for a in members:
            b = int(sum(int(J[a, j]) * z[j] for j in range(t))) % M
            assert b == fam.bins[a]
            for c in range(len(J)):
                if c != a:
                    assert int(sum(int(J[c, j]) * z[j] for j in range(t))) % M != b


def test_family_is_deterministic_and_first_cover():
    parent, child = W.candidate_set(9, 120, 4, 9)
    J = select.product(parent, child)
    f1 = lattice.plan_family(J, 2.0, 9601, 8, 64, 5, rng.KIND_LAT2, 4)
    f2 = lattice.plan_family(J, 2.0, 9601, 8, 64, 5, rng.KIND_LAT2, 4)
    assert f1.M == f2.M and f1.z == f2.z and np.array_equal(f1.assign, f2.assign)
    # a candidate assigned to lattice l was not alias-free in any earlier lattice of the family
    for a in range(len(J)):
        for l in range(fam_l := f1.assign[a]):
            M, z = f1.M[l], np.array(f1.z[l])
            bins = (J @ z) % M
            assert (bins == bins[a]).sum() > 1


def test_selection_ranks_ties_threshold():
    V = np.array([[9.0, 1.0], [4.0, 1.0], [4.0, 1.0], [1.0, 1e-9], [0.5, 0.0]])
    # s~ = 2: column 0 tau^2 = 4 -> rows 0,1,2 (tie kept); column 1 all-equal ones kept
    m, thr, keep = select.detect_mask(V, 2, 0.0)
    assert keep[:, 0].tolist() == [True, True, True, False, False]
    assert keep[:, 1].tolist() == [True, True, True, False, False]
    # threshold dominates
    m, thr, keep = select.detect_mask(V, 5, 2.0)
    assert keep[:, 0].tolist() == [True, True, True, False, False]
    # fewer candidates than s~: only theta applies
    m, thr, keep = select.detect_mask(V[:2], 10, 0.0)
    assert keep.all()
    # values within the tie band of tau^2 count as ties
    V2 = np.array([[1.0], [1.0 - 1e-12], [0.9]])
    m, thr, keep = select.detect_mask(V2, 1, 0.0)
    assert keep[:, 0].tolist() == [True, True, False]


def test_product_order_and_size():
    parent = np.array([[-1, 0], [0, 0], [2, -1]])
    child = np.array([-1, 0, 3])
    J = select.product(parent, child)
    brute = [list(p) + [c] for p in parent.tolist() for c in child.tolist()]
    assert J.tolist() == brute
    assert select.is_lex_sorted(J)
