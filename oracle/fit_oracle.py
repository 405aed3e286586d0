"""Plain FP64 CPU oracle of the linear POD fit.

Test infrastructure, not product code.  Only the test suite, the smoke check
and the benchmark's CPU leg import this module; the HIP library and its
binding never call it, and it shares no code with them.

The fit follows arXiv:2212.14446, Sec. IV.A: the energy is linear in the
coefficients, E = c . G (eq. (58a)), so forces are linear too,
F_n = -sum_m c_m dG_m/dr_n, and the coefficients solve the regularised
least-squares problem of eq. (63a),

    min_c  || A c - b ||^2 + gamma || c ||^2 ,

where every configuration contributes one energy row (G, E_ref) and 3 N_c
force rows (-dG/dr_n,d, F_ref_n,d).  Reading of the weights (the paper sets
them to 100 for energies and 1 for forces without saying where they enter):
as in the loss of eq. (63b) they multiply the squared residuals, i.e. the
energy rows of A and b are scaled by sqrt(w_e) and the force rows by
sqrt(w_f).

The solution is taken by an orthogonal least-squares solve of the stacked
system [A; sqrt(gamma) I] c = [b; 0] (numpy.linalg.lstsq), which is the plain
definition of the ridge problem and does not form the normal equations.
"""
from __future__ import annotations

import numpy as np


def design_matrix(G, dGdR, E_ref, F_ref, w_e: float, w_f: float):
    """Weighted rows of eq. (63a).

    G      : [n_cfg, M] global descriptors G_c = sum_{i in c} D_i (eq. (58a))
    dGdR   : [R_f, M] derivative rows dG/dr_{n,d} (all cells stacked)
    E_ref  : [n_cfg] reference energies
    F_ref  : [R_f] reference forces, in the row order of dGdR
    Returns (A, b) with the energy rows first, then the force rows."""
    G = np.asarray(G, dtype=np.float64).reshape(-1, np.shape(G)[-1])
    M = G.shape[1]
    dGdR = np.asarray(dGdR, dtype=np.float64).reshape(-1, M)
    se, sf = np.sqrt(float(w_e)), np.sqrt(float(w_f))
    A = np.vstack([se * G, -sf * dGdR])
    b = np.concatenate([se * np.asarray(E_ref, dtype=np.float64).ravel(),
                        sf * np.asarray(F_ref, dtype=np.float64).ravel()])
    return A, b


def ridge_solve(A, b, gamma: float):
    """argmin_c ||A c - b||^2 + gamma ||c||^2 by a least-squares solve of the
    stacked system (eq. (63a))."""
    A = np.asarray(A, dtype=np.float64)
    M = A.shape[1]
    As = np.vstack([A, np.sqrt(float(gamma)) * np.eye(M)])
    bs = np.concatenate([np.asarray(b, dtype=np.float64), np.zeros(M)])
    c, *_ = np.linalg.lstsq(As, bs, rcond=None)
    return c


def objective(A, b, c, gamma: float) -> float:
    """Value of eq. (63a) at c."""
    r = np.asarray(A) @ np.asarray(c) - np.asarray(b)
    return float(r @ r + gamma * np.asarray(c) @ np.asarray(c))


def weighted_loss(G, dGdR, E_ref, F_ref, c, w_e: float, w_f: float, gamma: float) -> float:
    """The same objective written per configuration as in eq. (63b):
    sum_k w_e (E_k - E_ref_k)^2 + w_f ||F_k - F_ref_k||^2 + gamma ||c||^2,
    with E_k = c . G_k and F_k = -dG_k/dR c, summed by explicit loops."""
    c = np.asarray(c, dtype=np.float64)
    total = 0.0
    for k in range(len(E_ref)):
        e = float(np.dot(G[k], c)) - float(E_ref[k])
        total += w_e * e * e
    for r in range(len(F_ref)):
        f = -float(np.dot(dGdR[r], c)) - float(F_ref[r])
        total += w_f * f * f
    return total + gamma * float(c @ c)


def gram(A, b):
    """[A b]^T [A b]: the normal-equation blocks A^T A, A^T b and b^T b in one
    (M+1) x (M+1) matrix (the quantities the device accumulates)."""
    X = np.hstack([np.asarray(A, dtype=np.float64), np.asarray(b, dtype=np.float64)[:, None]])
    return X.T @ X
