"""Alg. 1 (the usFFT on a node set T_G), run step by step in float64 (oracle).

Follows Alg. 1 of the paper in its own order:
  step 1 & 2a  for t = 1..d and i = 1..r: K_t equispaced nodes l/K_t in
               coordinate t, random tail y' elsewhere, one sampler call per
               node, length-K_t DFT per node x_g, select, union over g and i;
  step 2       for t = 2..d: J_t = I^(1..t-1) x I^(t); sampling set from the
               lattice family of J_t (Algorithm A, reading in lattice.py);
               for i = 1..r~ a fresh random tail y'_(t+1..d); sample; DFT
               at each candidate's assigned bin; select with s~; union;
               r~ = r, s~ = s_local for t < d and r~ = 1, s~ = s for t = d;
  step 3       lattice family for I = I^(1..d) (no tail), sample, all
               coefficients c_k, k in I, for every node.
The relative threshold of the workloads is read as an absolute one,
theta_abs = theta_rel * max_{k,g} |c| over the first detection stage
(t = 1, i = 1).

The sampler is any callable Y (n x d) -> U (n x G); fem.PDESampler and
TrigPolySampler below are the two used here.

Parity: the whole driver is pinned by exact recovery of seeded sparse
trigonometric polynomials (the event of Theorem 1.1; tests/test_oracle_usfft.py).
The paper prints no detected sets for its PDE runs; on the PDE sampler
(d = 2, 3) the run is pinned to the Fourier coefficients it approximates, taken
from the DFT of solves on a full tensor grid: step-3 coefficients within the
l1 norm of the coefficients outside I, no kept frequency below theta by more
than that norm, every frequency above ten times theta detected.
"""
import numpy as np

from . import rng
from .dft import dft_bins
from .lattice import lattice_nodes, plan_family
from .select import TIE_REL, detect_mask, product


class TrigPolySampler:
    """u_g(y) = Re sum_k P[k, g] exp(2 pi i k.y) for a fixed frequency list."""

    def __init__(self, K, P):
        self.K = np.asarray(K, dtype=np.float64)
        self.P = np.asarray(P, dtype=np.complex128)
        self.G = self.P.shape[1]

    def __call__(self, Y):
        Y = np.atleast_2d(np.asarray(Y, dtype=np.float64))
        E = np.exp(2j * np.pi * (Y @ self.K.T))
        return (E @ self.P).real


def evaluate(I, C, Y):
    """Approximant of Sec. 3.1 / eq. (3.1) for the periodic model: Re sum_k c_k e^{2 pi i k.y}."""
    I = np.asarray(I, dtype=np.float64)
    Y = np.atleast_2d(np.asarray(Y, dtype=np.float64))
    return (np.exp(2j * np.pi * (Y @ I.T)) @ np.asarray(C)).real


def tail(seed, kind, t, i, d):
    stream = rng.stream_code(kind, t, i)
    return np.array([rng.uniform01(seed, stream, j) for j in range(d)])


class Result:
    def __init__(self):
        self.I = None
        self.C = None
        self.stages = []
        self.samples = 0
        self.theta2 = None


def usfft(sampler, d, k_lo, k_hi, s, s_local, r, theta, theta_relative, seed,
          lattice_c=2.0, lattice_tries=8, lattice_max=64, lattice_mmax=9601,
          tie_rel=TIE_REL, keep_values=False):
    res = Result()
    theta2 = None if theta_relative else float(theta) ** 2

    def record(**kw):
        # keep ratio of every candidate: max over nodes of |c|^2 over the
        # node's keep threshold (kept exactly when >= 1); a diagnostic that
        # locates decisions close to the threshold, not part of the method
        with np.errstate(divide="ignore", invalid="ignore"):
            kw["ratio"] = (kw["V"] / kw["thr"][None, :]).max(axis=1) if kw["V"].size else np.zeros(0)
        if not keep_values:
            kw.pop("V", None)
        res.stages.append(kw)

    # ---- step 1 & 2a: one-dimensional detection in every coordinate ----
    I1 = []
    for t in range(d):
        K = k_hi[t] - k_lo[t] + 1
        ks = np.arange(k_lo[t], k_hi[t] + 1, dtype=np.int64)
        mask = np.zeros(K, dtype=bool)
        for i in range(r):
            Y = np.tile(tail(seed, rng.KIND_TAIL1, t + 1, i + 1, d), (K, 1))
            Y[:, t] = np.arange(K) / K
            U = sampler(Y)
            res.samples += K
            F = dft_bins(U, ks % K)
            V = (F.real ** 2 + F.imag ** 2)
            if theta2 is None:
                theta2 = float(theta) ** 2 * float(V.max())
                res.theta2 = theta2
            m, thr, _ = detect_mask(V, s_local, theta2, tie_rel)
            mask |= m
            record(step=1, t=t + 1, i=i + 1, cand=ks.copy(), mask=m, thr=thr, V=V)
        I1.append(ks[mask])
    if res.theta2 is None:
        res.theta2 = theta2

    # ---- step 2: coupling increments ----
    Iprev = I1[0][:, None]
    for t in range(1, d):
        last = t == d - 1
        r_t = 1 if last else r
        s_t = s if last else s_local
        J = product(Iprev, I1[t])
        fam = plan_family(J, lattice_c, lattice_mmax, lattice_tries, lattice_max,
                          seed, rng.KIND_LAT2, t + 1)
        mask = np.zeros(len(J), dtype=bool)
        for i in range(r_t):
            y_tail = tail(seed, rng.KIND_TAIL2, t + 1, i + 1, d)
            V = np.zeros((len(J), sampler.G))
            for l, (M, z) in enumerate(zip(fam.M, fam.z)):
                Y = np.tile(y_tail, (M, 1))
                Y[:, : t + 1] = lattice_nodes(M, z)
                U = sampler(Y)
                res.samples += M
                sel = fam.assign == l
                F = dft_bins(U, fam.bins[sel])
                V[sel] = F.real ** 2 + F.imag ** 2
            m, thr, _ = detect_mask(V, s_t, theta2, tie_rel)
            mask |= m
            record(step=2, t=t + 1, i=i + 1, cand=J, family=fam, mask=m, thr=thr, V=V)
        Iprev = J[mask]

    # ---- step 3: coefficients on the detected set ----
    I = Iprev
    C, fam, ns = coefficients(sampler, I, seed, lattice_c, lattice_tries, lattice_max, lattice_mmax)
    res.samples += ns
    res.stages.append(dict(step=3, t=d, i=1, cand=I, family=fam))
    res.I = I
    res.C = C
    return res


def coefficients(sampler, I, seed, lattice_c=2.0, lattice_tries=8, lattice_max=64, lattice_mmax=9601):
    """Step 3 of Alg. 1 on the frequency set I (n x d): the lattice family of
    I (Algorithm A, reading in lattice.py), one sample per lattice node, and
    c_k read from k's bin of its assigned lattice.  Used on the detected set
    and, as in Sec. 4.5, on an a-priori set.  Returns (C, family, samples)."""
    I = np.asarray(I, dtype=np.int64)
    C = np.zeros((len(I), sampler.G), dtype=np.complex128)
    if len(I) == 0:
        return C, None, 0
    fam = plan_family(I, lattice_c, lattice_mmax, lattice_tries, lattice_max, seed, rng.KIND_LAT3, 0)
    ns = 0
    for l, (M, z) in enumerate(zip(fam.M, fam.z)):
        U = sampler(lattice_nodes(M, z))
        ns += M
        sel = fam.assign == l
        C[sel] = dft_bins(U, fam.bins[sel])
    return C, fam, ns
