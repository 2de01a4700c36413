"""Periodizations of the affine and lognormal coefficient models (oracle side).

Test infrastructure only: imported by tests/, the smoke check and the CPU
baseline, never by the library.

What is computed (Sec. 3.2):
  * affine model, y ~ U([alpha, beta]^d): the tent transformation of
    eq. (3.2), phi(t) = beta - |(beta - alpha)(1 - 2 t)| on T = [0, 1), with
    inverse phi^{-1}(y) = (y - alpha) / (2 (beta - alpha)) onto [0, 1/2];
  * lognormal model, y ~ N(0, 1)^d: phi_Delta = tau_1 o tau_{2,Delta} of
    eq. (3.3), where tau_{2,Delta} is the tent shifted by Delta onto
    [-1/2, 1/2] and tau_1(v) = sqrt(2) erf^{-1}(2 v) maps U(-1/2, 1/2) to
    N(0, 1); inverse phi_Delta^{-1}(y) = erf(y / sqrt(2)) / 4 + Delta + 1/4;
  * the shift of Lemma 3.1: Delta_opt = 1 / (4 M) for a rank-1 lattice of
    size M.
The usFFT then samples u(x_g, phi(t)) at its nodes t and evaluates its
approximation at phi^{-1}(y) (eq. (3.1) with phi^{-1}).

Pins (tests/test_oracle_periodization.py): the endpoint, symmetry and
monotonicity conditions (A1)-(A4) of Sec. 3.2, phi(phi^{-1}(y)) = y, the
normal pushforward of tau_1, and Lemma 3.1 by brute force over the nodes of
random lattices.
"""
import numpy as np
from scipy.special import erf, erfinv

PERIODIC, AFFINE, LOGNORMAL = 0, 1, 2


def tent(t, alpha, beta):
    """phi(t) = beta - |(beta - alpha)(1 - 2 t)|, eq. (3.2)."""
    t = np.asarray(t, dtype=np.float64)
    return beta - np.abs((beta - alpha) * (1.0 - 2.0 * t))


def tent_inv(y, alpha, beta):
    """phi^{-1}(y) = (y - alpha) / (2 (beta - alpha)), onto [0, 1/2]."""
    return (np.asarray(y, dtype=np.float64) - alpha) / (2.0 * (beta - alpha))


def tau2(t, delta):
    """Tent shifted by delta, onto [-1/2, 1/2], piecewise as in Sec. 3.2."""
    t = np.asarray(t, dtype=np.float64)
    return np.where(t < delta, -0.5 - 2.0 * (t - delta),
                    np.where(t < 0.5 + delta, -0.5 + 2.0 * (t - delta), 1.5 - 2.0 * (t - delta)))


def tau2_inv(v, delta):
    """Inverse on [delta, 1/2 + delta]: v / 2 + delta + 1/4."""
    return np.asarray(v, dtype=np.float64) / 2.0 + delta + 0.25


def tau1(v):
    """sqrt(2) erf^{-1}(2 v): U(-1/2, 1/2) -> N(0, 1)."""
    return np.sqrt(2.0) * erfinv(2.0 * np.asarray(v, dtype=np.float64))


def tau1_inv(y):
    """erf(y / sqrt(2)) / 2."""
    return 0.5 * erf(np.asarray(y, dtype=np.float64) / np.sqrt(2.0))


def lognormal_map(t, delta):
    """phi_Delta = tau_1 o tau_{2,Delta}."""
    return tau1(tau2(t, delta))


def lognormal_inv(y, delta):
    """phi_Delta^{-1} = tau_{2,Delta}^{-1} o tau_1^{-1}."""
    return tau2_inv(tau1_inv(y), delta)


def delta_opt(M):
    """Lemma 3.1: the shift farthest from every lattice node, 1 / (4 M)."""
    return 1.0 / (4.0 * M)


def to_parameter(model, t, alpha=-1.0, beta=1.0, delta=0.0):
    """Sampling node t in [0, 1)^d -> parameter y of the model."""
    if model == PERIODIC:
        return np.asarray(t, dtype=np.float64)
    if model == AFFINE:
        return tent(t, alpha, beta)
    if model == LOGNORMAL:
        return lognormal_map(t, delta)
    raise ValueError("unknown model")


def to_node(model, y, alpha=-1.0, beta=1.0, delta=0.0):
    """Parameter y -> point of T^d at which the Fourier approximation is evaluated."""
    if model == PERIODIC:
        return np.asarray(y, dtype=np.float64)
    if model == AFFINE:
        return tent_inv(y, alpha, beta)
    if model == LOGNORMAL:
        return lognormal_inv(y, delta)
    raise ValueError("unknown model")
