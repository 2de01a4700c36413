"""Post-processing of the usFFT approximation (Sec. 4 and Sec. 4.1), oracle side.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline, never by the library.

For every spatial node x_g the usFFT returns coefficients c_{k,g}, k in I,
of the periodized solution u~(x_g, t) = sum_k c_{k,g} e^{2 pi i k.t}; the
approximation of u(x_g, y) is u~(x_g, phi^{-1}(y)) (Sec. 3.2).  Computed here,
per node:
  * the error measures of Sec. 4 over n_test parameters y^(j) drawn from
    the model's distribution:
        err_p   = ( (1/n_test) sum_j |u_FE(x_g, y^(j)) - u_usFFT(x_g, y^(j))|^p )^(1/p),
        err_inf = max_j |u_FE(x_g, y^(j)) - u_usFFT(x_g, y^(j))|;
  * the variance of the approximation (Sec. 4),
        sigma^2 = ||u~||^2_{L2(T^d)} - |c_0|^2 = sum_{k in I, k != 0} |c_k|^2;
  * the global sensitivity index of a subset J of I (Sec. 4), the share of
    sigma^2 carried by the nonzero frequencies of J, for the sets
        J_l = {k in I : ||k||_0 = l},  l = 1..d,
    where ||k||_0 counts the nonzero components of k;
  * the expectation of the approximation under the model's distribution
    (Sec. 4.1), E = sum_k c_k D_k with D_k = prod_j D_{k_j}:
        periodic  (y uniform on the torus):   D_k = 1 if k = 0, else 0;
        affine    (y ~ U[alpha, beta]^d):     D_{k_j} = 2i / (pi k_j) for odd k_j,
                                              1 for k_j = 0, 0 for even k_j != 0;
        lognormal (y ~ N(0, I_d), shift Delta): the affine factor times
                                              e^{2 pi i k_j Delta}.

Readings: for a node with sigma^2 = 0 every index is reported as 0.  The
expectation is complex in general (real when I is closed under k -> -k with
conjugate coefficients); it is returned as a complex number.

Pins (tests/test_oracle_evaluation.py): the D factors against the integral
that defines them (Gauss-Legendre for the affine model, Gauss-Hermite for the
lognormal one); the expectation of a trigonometric polynomial against tensor
quadrature of its evaluation; sigma^2 against the mean of |u~|^2 over a full
grid (discrete orthogonality); the J_l indices against a brute-force ANOVA
decomposition on a grid; err_p / err_inf against constant and scaled
differences.
"""
import numpy as np

from . import periodization as per


def approximation(I, C, Y, model=per.PERIODIC, alpha=-1.0, beta=1.0, delta=0.0):
    """u_usFFT(x_g, y) = Re sum_k c_{k,g} e^{2 pi i k . phi^{-1}(y)} for parameters Y (n x d): n x G."""
    T = per.to_node(model, np.atleast_2d(np.asarray(Y, dtype=np.float64)), alpha, beta, delta)
    E = np.exp(2j * np.pi * (T @ np.asarray(I, dtype=np.float64).T))
    return (E @ np.asarray(C, dtype=np.complex128)).real


def errors(U_fe, U_approx, p):
    """err_p and err_inf of Sec. 4 per node; U_fe, U_approx are n_test x G."""
    D = np.abs(np.asarray(U_fe, dtype=np.float64) - np.asarray(U_approx, dtype=np.float64))
    return np.mean(D ** p, axis=0) ** (1.0 / p), np.max(D, axis=0)


def variance(I, C):
    """sigma^2 per node: the squared coefficients of every nonzero frequency (Sec. 4)."""
    nz = np.any(np.asarray(I) != 0, axis=1)
    return np.sum(np.abs(np.asarray(C)[nz]) ** 2, axis=0)


def sensitivity_indices(I, C):
    """rho(J_l) for l = 1..d (rows), per node (columns) (Sec. 4)."""
    I = np.asarray(I)
    C = np.asarray(C)
    d = I.shape[1]
    order = np.count_nonzero(I, axis=1)
    var = variance(I, C)
    out = np.zeros((d, C.shape[1]))
    for l in range(1, d + 1):
        part = np.sum(np.abs(C[order == l]) ** 2, axis=0)
        out[l - 1] = np.where(var > 0, part / np.where(var > 0, var, 1.0), 0.0)
    return out


def d_factors(I, model=per.PERIODIC, delta=0.0):
    """D_k of Sec. 4.1 for every k in I (complex)."""
    I = np.asarray(I, dtype=np.int64)
    if model == per.PERIODIC:
        return np.where(np.all(I == 0, axis=1), 1.0 + 0j, 0.0 + 0j)
    out = np.ones(I.shape[0], dtype=np.complex128)
    for j in range(I.shape[1]):
        k = I[:, j]
        f = np.zeros(k.shape, dtype=np.complex128)
        f[k == 0] = 1.0
        odd = (k % 2) != 0
        f[odd] = 2j / (np.pi * k[odd])
        if model == per.LOGNORMAL:
            f[odd] *= np.exp(2j * np.pi * k[odd] * delta)
        elif model != per.AFFINE:
            raise ValueError("unknown model")
        out *= f
    return out


def expectation(I, C, model=per.PERIODIC, delta=0.0):
    """E(u_usFFT(x_g, .)) = sum_k c_{k,g} D_k per node (Sec. 4.1), complex."""
    return d_factors(I, model, delta) @ np.asarray(C, dtype=np.complex128)
