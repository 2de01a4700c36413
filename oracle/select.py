"""Per-node selection, uniform union over nodes and the set join (oracle side).

Selection (Alg. 1, step 1&2a and step 2d): for every node x_g keep the
candidates whose coefficient is among the s~ largest in absolute value and at
least theta; the detected set is the union over g (and over the detection
iterations i).  Readings of this build:
  * ranks count with multiplicity; tau_g is the s~-th largest |coefficient|
    of column g (no rank limit when the column has fewer than s~ entries);
  * "larger than theta" and ">= theta" are both read as >=;
  * values within a relative TIE band of tau_g^2 count as ties with it and
    are kept, so that exact mathematical ties (symmetries of the problem in
    y) do not depend on rounding;
  * all comparisons use squared magnitudes in float64.
Join (Alg. 1, step 2): J_t = I^(1..t-1) x I^(t), parent-major, which keeps
lexicographic order when both factors are sorted; the box Gamma needs no
intersection because every product element already lies in P_(1..t)(Gamma).

Pins: hand-built columns with known ranks and ties, brute-force product and
order checks (tests/test_oracle_select.py).
"""
import numpy as np

TIE_REL = 2.0 ** -30


def column_thresholds(V, s_tilde, theta2, tie_rel=TIE_REL):
    """V: (n, G) squared magnitudes.  Returns the per-column keep threshold."""
    n, G = V.shape
    if n >= s_tilde and s_tilde > 0:
        tau2 = -np.sort(-V, axis=0)[s_tilde - 1]
    else:
        tau2 = np.zeros(G)
    return np.maximum(theta2, (1.0 - tie_rel) * tau2), tau2


def detect_mask(V, s_tilde, theta2, tie_rel=TIE_REL):
    thr, tau2 = column_thresholds(V, s_tilde, theta2, tie_rel)
    keep = V >= thr[None, :]
    return keep.any(axis=1), thr, keep


def product(parent, child):
    """Parent-major Cartesian product of an (p x (t-1)) and a (c,) set."""
    parent = np.asarray(parent, dtype=np.int64)
    if parent.ndim == 1:
        parent = parent[:, None]
    child = np.asarray(child, dtype=np.int64)
    P = np.repeat(parent, len(child), axis=0)
    C = np.tile(child, len(parent))[:, None]
    return np.concatenate([P, C], axis=1)


def is_lex_sorted(S):
    S = np.asarray(S)
    for a in range(1, len(S)):
        if tuple(S[a - 1]) >= tuple(S[a]):
            return False
    return True
