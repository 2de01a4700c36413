"""Rank-1 lattices and the multiple-lattice family used as Algorithm A (oracle).

A rank-1 lattice is {(m z mod M)/M : m = 0..M-1} (App. A).  Sampling a
function along it turns its Fourier coefficient c_k into DFT bin k.z mod M,
so a candidate k can be read off the length-M DFT without error from the
other candidates exactly when no other candidate of the set falls into the
same bin ("alias-free").  The paper runs Algorithm A as a random rank-1
lattice method [KaKrVo20] and step 3 as a multiple rank-1 lattice method
[Kae17]; neither construction is given in the text.  This build's reading
(for both places) is a greedy multiple rank-1 lattice family:

  sizes   admissible primes M (prime, M-1 has no prime factor above 7) taken
          in increasing order from lo = min(max(3, ceil(c |J|)), M_max // 2)
          up to M_max, cycling when the list is exhausted; c = 2 as in the
          multiple-lattice bound quoted in Remark 4.2.  Prime sizes follow
          the remark after the proof of Lemma 3.1.
  choice  for attempt a, T candidate generators z (rng kind 3/4, try b);
          keep the one that makes the most still-uncovered candidates
          alias-free (ties: the lowest try index); a lattice that covers
          nothing new is dropped; fail after L_max attempts.
  assign  every candidate k is read from the first lattice in which it is
          alias-free.

Pins: tests/test_oracle_lattice.py checks the alias-free property of every
assignment by brute force and the prime/smoothness predicates against
a sieve.
"""
import numpy as np

from . import rng


def is_prime(m: int) -> bool:
    if m < 2:
        return False
    if m % 2 == 0:
        return m == 2
    f = 3
    while f * f <= m:
        if m % f == 0:
            return False
        f += 2
    return True


def is_7smooth(m: int) -> bool:
    if m < 1:
        return False
    for p in (2, 3, 5, 7):
        while m % p == 0:
            m //= p
    return m == 1


def admissible(m: int) -> bool:
    return m >= 3 and is_prime(m) and is_7smooth(m - 1)


def admissible_sizes(lo: int, hi: int):
    return [m for m in range(max(lo, 3), hi + 1) if admissible(m)]


class LatticeFamily:
    def __init__(self, sizes, gens, assign, bins):
        self.M = list(sizes)          # lattice sizes
        self.z = list(gens)           # generating vectors (lists of ints)
        self.assign = assign          # (n,) lattice index of each candidate
        self.bins = bins              # (n,) bin k.z mod M in its lattice

    @property
    def total_samples(self):
        return int(sum(self.M))


class LatticeError(RuntimeError):
    pass


def plan_family(J, c, m_max, tries, l_max, seed, kind, t_code):
    """Greedy multiple rank-1 lattice family for candidate set J (n x t)."""
    J = np.asarray(J, dtype=np.int64)
    n = len(J)
    if n == 0:
        return LatticeFamily([], [], np.zeros(0, np.int64), np.zeros(0, np.int64))
    t = J.shape[1]
    lo = max(3, int(np.ceil(c * n)))
    lo = min(lo, m_max // 2)
    sizes = admissible_sizes(lo, m_max)
    if not sizes:
        raise LatticeError("no admissible lattice size in [%d, %d]" % (lo, m_max))
    uncovered = np.ones(n, dtype=bool)
    assign = np.full(n, -1, dtype=np.int64)
    bins_out = np.full(n, -1, dtype=np.int64)
    Ms, Zs = [], []
    attempt = 0
    while uncovered.any():
        if attempt >= l_max:
            raise LatticeError("lattice family incomplete after %d attempts" % l_max)
        M = sizes[attempt % len(sizes)]
        best = None
        for b in range(tries):
            stream = rng.stream_code(kind, t_code, attempt, b)
            z = np.array(rng.lattice_generator(seed, stream, t, M), dtype=np.int64)
            bins = (J @ z) % M
            counts = np.bincount(bins, minlength=M)
            free = (counts[bins] == 1) & uncovered
            score = int(free.sum())
            if best is None or score > best[0]:
                best = (score, z, free, bins)
        attempt += 1
        if best[0] == 0:
            continue
        _, z, free, bins = best
        assign[free] = len(Ms)
        bins_out[free] = bins[free]
        uncovered &= ~free
        Ms.append(M)
        Zs.append([int(v) for v in z])
    return LatticeFamily(Ms, Zs, assign, bins_out)


def lattice_nodes(M, z):
    """Nodes (m z mod M)/M, m = 0..M-1, of a rank-1 lattice (App. A), shape (M, t)."""
    m = np.arange(M, dtype=np.int64)[:, None]
    return ((m * np.asarray(z, dtype=np.int64)[None, :]) % M) / float(M)
