"""Plain FP64 CPU oracle of the exclusive-sum descriptors (the earlier POD
form that the paper compares its fast descriptors with).

Test infrastructure, not product code.  Only the test suite, the smoke check
and the benchmark's CPU leg import this module; the HIP library and its
binding never call it, and it shares no code with them.  It reuses the
radial basis and pair geometry of the POD oracle (pod_oracle).

Following arXiv:2212.14446:
  * exclusive 3-body descriptors   Sec. II.C, eq. (15b): sum over j, k > j
  * symmetric angular functions    Sec. II.D, eq. (19a), Table 2
  * exclusive 4-body descriptors   Sec. II.D, eq. (20a): sum over j < k < l
  * the 2/3-body exclusive model (OPOD of Sec. V, Table 6): linear energy
    c . [1 | D2 | D3] and its forces by the chain rule

Readings (listed with the others in the design notes):
  * g_p holds the distinct members of the cyclic orbit {(a,b,c), (c,a,b),
    (b,c,a)} of the exponents of (w_ijk, w_ijl, w_ikl), each once: this is
    how Table 2 prints g_1 = 1 and g_7 = w_ijk w_ijl w_ikl, where the
    three-term sum of eq. (19a) would give three times those.
  * For (a, b, c) with three distinct exponents (g_6, g_9 at P <= 4) the
    cyclic sum is invariant under cyclic permutations of (j, k, l) only, so
    eq. (20a) depends on the order of the neighbour list for those p; the
    sum runs over j < k < l in list order.
"""
from __future__ import annotations

import numpy as np

from oracle import pod_oracle as po


def symmetric_terms(a: int, b: int, c: int):
    """Exponent triples of g_p for (a, b, c): the cyclic orbit of eq. (19a),
    each distinct member once (Table 2)."""
    out = []
    for t in ((a, b, c), (c, a, b), (b, c, a)):
        if t not in out:
            out.append(t)
    return out


def g_value(abc, w1, w2, w3):
    """g_p(w_ijk, w_ijl, w_ikl) for the triple abc (eq. (19a), Table 2)."""
    s = 0.0
    for (x, y, z) in symmetric_terms(*abc):
        s = s + w1 ** x * w2 ** y * w3 ** z
    return s


def descriptors_env(Rn, U, p: po.PodParams):
    """Exclusive descriptors of one atom from its neighbours' radial values
    Rn [n_i, K] and unit vectors U [n_i, 3], in the order of the list:
    [1 | D2 (k < K2) | D3 (m < K3, n = 0..P3) | D4 (m < K4, Table-1 order)]."""
    Rn = np.asarray(Rn, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    ni = Rn.shape[0]
    W = U @ U.T
    out = [1.0]
    for k in range(p.K2):                                     # eq. (12b)
        out.append(Rn[:, k].sum())
    for m in range(p.K3):                                     # eq. (15b)
        for n in range(p.P3 + 1):
            s = 0.0
            for j in range(ni):
                for k in range(j + 1, ni):
                    s += Rn[j, m] * Rn[k, m] * W[j, k] ** n
            out.append(s)
    trip = po.four_body_triples(p.P4) if p.K4 > 0 else []
    for m in range(p.K4):                                     # eq. (20a)
        for abc in trip:
            s = 0.0
            for j in range(ni):
                for k in range(j + 1, ni):
                    for l in range(k + 1, ni):
                        s += Rn[j, m] * Rn[k, m] * Rn[l, m] * g_value(abc, W[j, k], W[j, l], W[k, l])
            out.append(s)
    return np.array(out)


def descriptors(pos, cell, offsets, nbr_j, shift, p: po.PodParams, Q, atoms=None):
    """Per-atom exclusive descriptors [n_atoms, M] (small systems)."""
    pos = np.asarray(pos, dtype=np.float64)
    if atoms is None:
        atoms = np.arange(pos.shape[0])
    M, _ = po.num_descriptors(p)
    D = np.zeros((len(atoms), M))
    for ii, a in enumerate(atoms):
        _, _, d = po.pair_vectors(pos, cell, offsets, nbr_j, shift, [a])
        if d.shape[0] == 0:
            D[ii] = descriptors_env(np.zeros((0, p.K)), np.zeros((0, 3)), p)
            continue
        r = np.sqrt((d * d).sum(1))
        Rn, _ = po.radial_basis(r, p, Q)
        D[ii] = descriptors_env(Rn, d / r[:, None], p)
    return D


def energy_forces(pos, cell, offsets, nbr_j, shift, p: po.PodParams, Q, c):
    """Energies, forces and virial of the 2/3-body exclusive model
    E_i = c . [1 | D2_i | D3_i] (K4 = 0).

    Per atom: E_i = c_0 + sum_k c2_k sum_j R_k(r_ij)
                  + sum_{j<k} sum_m R_m(r_ij) R_m(r_ik) P_m(w_ijk),
    P_m(w) = sum_n c3_mn w^n.  The gradient with respect to r_ij (chain rule
    through r = |r_ij| and w = rhat_ij . rhat_ik, dw/dr_ij = (rhat_ik - w
    rhat_ij) / r_ij) gives F_i += g_ij, F_j -= g_ij and
    W_ab = -sum_pairs r_ij,a g_ij,b."""
    if p.K4 != 0:
        raise ValueError("the exclusive energy model here is 2/3-body only")
    pos = np.asarray(pos, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    N = pos.shape[0]
    c2 = c[1:1 + p.K2]
    c3 = c[1 + p.K2:].reshape(p.K3, p.P3 + 1) if p.K3 > 0 else np.zeros((0, p.P3 + 1))
    E_atom = np.zeros(N)
    F = np.zeros((N, 3))
    W = np.zeros((3, 3))
    offsets = np.asarray(offsets)
    nbr_j = np.asarray(nbr_j)
    for i in range(N):
        _, pidx, d = po.pair_vectors(pos, cell, offsets, nbr_j, shift, [i])
        e = c[0]
        ni = d.shape[0]
        if ni == 0:
            E_atom[i] = e
            continue
        r = np.sqrt((d * d).sum(1))
        U = d / r[:, None]
        R, dR = po.radial_basis(r, p, Q)
        g = np.zeros((ni, 3))
        # 2-body
        e += float((R[:, :p.K2] @ c2).sum())
        g += ((dR[:, :p.K2] @ c2))[:, None] * U
        # 3-body, exclusive pairs j < k
        for j in range(ni):
            for k in range(j + 1, ni):
                w = float(U[j] @ U[k])
                for m in range(p.K3):
                    Pm = sum(c3[m, n] * w ** n for n in range(p.P3 + 1))
                    dPm = sum(n * c3[m, n] * w ** (n - 1) for n in range(1, p.P3 + 1))
                    Rj, Rk = R[j, m], R[k, m]
                    e += Rj * Rk * Pm
                    g[j] += dR[j, m] * Rk * Pm * U[j] + Rj * Rk * dPm * (U[k] - w * U[j]) / r[j]
                    g[k] += Rj * dR[k, m] * Pm * U[k] + Rj * Rk * dPm * (U[j] - w * U[k]) / r[k]
        E_atom[i] = e
        F[i] += g.sum(0)
        np.add.at(F, nbr_j[pidx], -g)
        W -= d.T @ g
    return {"E_atom": E_atom, "E": float(E_atom.sum()), "F": F, "W": W}


def total_energy(pos, cell, offsets, nbr_j, shift, p, Q, c):
    return energy_forces(pos, cell, offsets, nbr_j, shift, p, Q, c)["E"]
