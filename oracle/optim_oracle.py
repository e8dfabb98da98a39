"""FP64 oracle of the batched L-BFGS steps (an optimiser beside the paper's GRAPE
gradient steps; test infrastructure only, see the package docstring).

lbfgs_direction(g, pairs, gamma0) is the direction d = H g of the limited-memory
BFGS inverse-curvature estimate for an ascent on F (equivalently a descent on -F):
pairs are (s, y) with s = x_{k+1} - x_k and y = g_k - g_{k+1}, oldest first; H is
the BFGS inverse update applied to each pair in turn starting from gamma I with
gamma = s.y / y.y of the newest pair, evaluated by the two-loop recursion.  With
no pair, or when g.d <= 0, d = gamma0 g / max|g|.

Pinned (tests/test_oracle_pins.py) against bfgs_inverse_matrix, the same estimate
formed as an explicit matrix by the textbook update
H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T, and by the secant condition
H y = s of the newest pair.
"""
import numpy as np


def bfgs_inverse_matrix(pairs, gamma):
    n = pairs[0][0].shape[0]
    H = gamma * np.eye(n)
    for s, y in pairs:
        rho = 1.0 / (y @ s)
        E = np.eye(n) - rho * np.outer(s, y)
        H = E @ H @ E.T + rho * np.outer(s, s)
    return H


def lbfgs_direction(g, pairs, gamma0):
    g = np.asarray(g, dtype=np.float64)
    fallback = gamma0 / np.abs(g).max() * g
    if not pairs:
        return fallback
    q = g.copy()
    al = []
    for s, y in reversed(pairs):
        rho = 1.0 / (y @ s)
        a = rho * (s @ q)
        q -= a * y
        al.append((a, rho))
    al.reverse()
    s_new, y_new = pairs[-1]
    r = (s_new @ y_new) / (y_new @ y_new) * q
    for (s, y), (a, rho) in zip(pairs, al):
        beta = rho * (y @ r)
        r += s * (a - beta)
    return r if g @ r > 0 else fallback
