"""Plain FP64 CPU oracle for fast proper orthogonal descriptors (POD).

Test infrastructure, not product code.  Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark import this module; the product
path (the HIP library and its Python binding) never calls it, and it shares
no code, tables or helpers with that path.

It follows N.-C. Nguyen, "Fast proper orthogonal descriptors for many-body
interatomic potentials" (arXiv:2212.14446), Section II, step by step:

  * radial snapshots and cut-off            Sec. II.B, eqs. (3)-(8), (11)
  * POD radial basis R_k = sum_l Q_lk Phi_l  Sec. II.B, eq. (12)
  * 2-body descriptors                       Sec. II.B, eq. (12b)
  * 3-body descriptors (full double sum)     Sec. II.C, eqs. (14)-(15)
  * exclusive 3-body descriptors             Sec. II.C, eq. (15b)
  * 4-body descriptors (full triple sum)     Sec. II.D, eqs. (16a), (17a), (18a), Table 1
  * angular monomials / atomic basis         Sec. II.E, eq. (23b), eq. (24b), Table 3
  * fast 2/3/4-body contractions             Sec. II.E, eqs. (25)-(30a), Table 4
  * linear energy model                      Sec. IV.A, eqs. (57a), (58a)
  * derivatives / forces                     Sec. II.G, eqs. (26c), (24c); product rule
                                             for the 2- and 4-body terms

Everything is float64 NumPy.  The naive forms are the paper's sums written
out over every ordered neighbour pair/triple; the fast forms take the atom
density route.  Readings where the paper is silent (the snapshot family, the
eigenvector normalisation, the descriptor ordering, the virial sign) are
listed in the design notes and restated next to the code that takes them.

Parity status of each function is pinned by tests/test_oracle_*.py; the POD
eigenbasis and everything downstream of it carry no printed numeric value in
the paper ("parity unpinned" against printed numbers) and are pinned instead
by closed forms, identities, symmetry and finite differences.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from math import factorial, pi

import numpy as np

EPS_FC = 1e-6  # epsilon inside the cut-off function, Sec. II.B eq. (8)


# --------------------------------------------------------------------------
# Parameters
# --------------------------------------------------------------------------
@dataclass
class PodParams:
    """Radial, angular and body-order parameters of Sec. II.

    rin, rcut         inner / outer cut-off (Sec. II.B)
    alpha, beta,      one snapshot tuple mu_l = (rin, rcut, alpha, beta,
    gamma, kappa      gamma, kappa) per entry, l = 1..L (Sec. II.B, eq. (11))
    K2, K3, K4        radial functions per body order (eqs. (12b), (14), (17a));
                      0 switches that body order off
    P3, P4            highest angular degree of 3- and 4-body terms
    """
    rin: float
    rcut: float
    alpha: np.ndarray
    beta: np.ndarray
    gamma: np.ndarray
    kappa: np.ndarray
    K2: int
    K3: int
    K4: int
    P3: int
    P4: int

    @property
    def L(self) -> int:
        return len(self.alpha)

    @property
    def K(self) -> int:
        return max(self.K2, self.K3, self.K4)

    @property
    def PA(self) -> int:
        """Highest angular degree P_a = max(P3, P4) (Sec. II.E); 0 with no 3/4-body."""
        p = 0
        if self.K3 > 0:
            p = max(p, self.P3)
        if self.K4 > 0:
            p = max(p, self.P4)
        return p


def default_snapshot_family(L: int, beta: float = 3.0):
    """Snapshot tuples used throughout (a reading: Sec. II.B defers the choice).

    Bessel-type snapshots (kappa = 1) with alpha = 1..L-2 at one beta, and
    inverse-power snapshots (kappa = 0) with gamma = 1, 2.
    """
    if L < 3:
        raise ValueError("need L >= 3")
    nb = L - 2
    alpha = np.concatenate([np.arange(1, nb + 1, dtype=float), np.zeros(2)])
    betas = np.concatenate([np.full(nb, beta), np.zeros(2)])
    gamma = np.concatenate([np.zeros(nb), np.array([1.0, 2.0])])
    kappa = np.concatenate([np.ones(nb), np.zeros(2)])
    return alpha, betas, gamma, kappa


def make_params(rin, rcut, L, K2, K3, K4, P3, P4, beta=3.0) -> PodParams:
    a, b, g, k = default_snapshot_family(L, beta)
    return PodParams(rin, rcut, a, b, g, k, K2, K3, K4, P3, P4)


# --------------------------------------------------------------------------
# Radial snapshots, Sec. II.B
# --------------------------------------------------------------------------
def _check_domain(r, rin, rcut):
    r = np.asarray(r, dtype=np.float64)
    if np.any(~np.isfinite(r)):
        raise ValueError("non-finite distance")
    if np.any(r <= rin) or np.any(r >= rcut):
        raise ValueError("distance outside the open interval (rin, rcut)")
    return r


def scaled_distance(r, rin, rcut, beta):
    """Scaled distance x(r) of Sec. II.B and dx/dr.

    x = (exp(-beta t) - 1) / (exp(-beta) - 1), t = (r - rin)/(rcut - rin);
    written with expm1 so that it stays accurate for small beta t.  beta = 0
    is the limit x = t.
    """
    r = np.asarray(r, dtype=np.float64)
    h = rcut - rin
    t = (r - rin) / h
    if beta == 0.0:
        return t, np.full_like(t, 1.0 / h)
    den = np.expm1(-beta)
    x = np.expm1(-beta * t) / den
    dxdr = -beta * np.exp(-beta * t) / den / h
    return x, dxdr


def cutoff(r, rin, rcut):
    """Cut-off function f_c of Sec. II.B eq. (8) and its r-derivative."""
    r = np.asarray(r, dtype=np.float64)
    h = rcut - rin
    t = (r - rin) / h
    y = 1.0 - t ** 3
    s = y * y + EPS_FC
    fc = np.exp(1.0 - 1.0 / np.sqrt(s))
    # d/dr [1 - s^(-1/2)] = (1/2) s^(-3/2) ds/dr,  ds/dr = 2 y dy/dr,  dy/dr = -3 t^2 / h
    dfc = fc * (y * s ** -1.5) * (-3.0 * t * t / h)
    return fc, dfc


def snapshots(r, p: PodParams):
    """Snapshots Phi_l(r) = f_c(r) psi(r; mu_l), l = 1..L (eqs. (3)-(6), (11)).

    psi = kappa * sin(alpha pi x)/(r - rin) + (1 - kappa) * r^(-gamma).
    Returns (Phi, dPhi/dr), each of shape (n, L).
    """
    r = _check_domain(np.atleast_1d(r), p.rin, p.rcut)
    fc, dfc = cutoff(r, p.rin, p.rcut)
    d = r - p.rin
    n, L = r.shape[0], p.L
    Phi = np.empty((n, L))
    dPhi = np.empty((n, L))
    for l in range(L):
        kap = p.kappa[l]
        psi = np.zeros(n)
        dpsi = np.zeros(n)
        if kap != 0.0:
            x, dx = scaled_distance(r, p.rin, p.rcut, p.beta[l])
            w = p.alpha[l] * pi
            s, c = np.sin(w * x), np.cos(w * x)
            phi = s / d
            dphi = (w * c * dx * d - s) / (d * d)
            psi += kap * phi
            dpsi += kap * dphi
        if kap != 1.0:
            g = p.gamma[l]
            psi += (1.0 - kap) * r ** (-g)
            dpsi += (1.0 - kap) * (-g) * r ** (-g - 1.0)
        Phi[:, l] = fc * psi
        dPhi[:, l] = dfc * psi + fc * dpsi
    return Phi, dPhi


def quadrature_nodes(p: PodParams, n_quad: int = 2000):
    """Midpoint nodes on (rin, rcut) used to sample the snapshots."""
    h = (p.rcut - p.rin) / n_quad
    return p.rin + (np.arange(n_quad) + 0.5) * h


def pod_basis(p: PodParams, n_quad: int = 2000):
    """POD of the snapshot family (Sec. II.B, eq. (12)); method of snapshots.

    Reading: the correlation matrix C = Phi^T Phi / n_quad of the snapshots
    sampled at midpoint nodes is diagonalised; Q holds its unit eigenvectors
    ordered by decreasing eigenvalue, each signed so that its entry of
    largest magnitude is positive.  Returns (Q [L x L], eigenvalues [L]).
    """
    rs = quadrature_nodes(p, n_quad)
    Phi, _ = snapshots(rs, p)
    C = Phi.T @ Phi / n_quad
    lam, V = np.linalg.eigh(C)
    order = np.argsort(lam)[::-1]
    lam, V = lam[order], V[:, order].copy()
    for k in range(V.shape[1]):
        i = int(np.argmax(np.abs(V[:, k])))
        if V[i, k] < 0:
            V[:, k] = -V[:, k]
    return V, lam


def radial_basis(r, p: PodParams, Q):
    """Orthogonal radial functions R_k(r) = sum_l Q_lk Phi_l(r), k < K (eq. (12))."""
    Phi, dPhi = snapshots(r, p)
    Qk = np.asarray(Q)[:, : p.K]
    return Phi @ Qk, dPhi @ Qk


# --------------------------------------------------------------------------
# Index tables, Sec. II.D-II.F
# --------------------------------------------------------------------------
def monomial_exponents(P: int):
    """Exponents (a, b, c) of the angular monomials x^a y^b z^c, a+b+c = n,
    n = 0..P (eq. (23b), Table 3).  Within a degree the order is
    lexicographically descending; any order gives the same descriptors."""
    out = []
    for n in range(P + 1):
        for a in range(n, -1, -1):
            for b in range(n - a, -1, -1):
                out.append((a, b, n - a - b))
    return out


def monomial_degree(P: int):
    return np.array([sum(e) for e in monomial_exponents(P)], dtype=int)


def multinomial(e) -> int:
    """c = n!/(a! b! c!): coefficient of the multinomial expansion of
    (x + y + z)^n (Sec. II.E, Table 4)."""
    a, b, c = e
    return factorial(a + b + c) // (factorial(a) * factorial(b) * factorial(c))


def four_body_triples(P4: int):
    """(a, b, c), a >= b >= c >= 0, a+b+c = n <= P4, in the order of Table 1:
    n ascending, then (a, b, c) lexicographically descending (eq. (16a))."""
    out = []
    for n in range(P4 + 1):
        for a in range(n, -1, -1):
            for b in range(min(a, n - a), -1, -1):
                c = n - a - b
                if 0 <= c <= b:
                    out.append((a, b, c))
    return out


def n_four_body(P4: int) -> int:
    return len(four_body_triples(P4))


def num_descriptors(p: PodParams):
    """M = 1 + K2 + K3 (1 + P3) + K4 K_a(P4) (caption of Table 6), and the
    per-body-order counts (1-, 2-, 3-, 4-body)."""
    m2 = p.K2
    m3 = p.K3 * (p.P3 + 1) if p.K3 > 0 else 0
    m4 = p.K4 * n_four_body(p.P4) if p.K4 > 0 else 0
    return 1 + m2 + m3 + m4, (1, m2, m3, m4)


# --------------------------------------------------------------------------
# Geometry and neighbours, Sec. II.A
# --------------------------------------------------------------------------
def neighbors_bruteforce(pos, cell, rcut):
    """All (i, j, n) with d = r_j + n.cell - r_i, 0 < |d| < rcut, n in Z^3
    (periodic images are distinct neighbours, i == j allowed for n != 0).
    cell: 3x3 with the lattice vectors as rows, or None for an open system.
    Returns CSR (offsets, nbr_j, shift[P,3]) sorted by i, then j, then n."""
    pos = np.asarray(pos, dtype=np.float64)
    N = pos.shape[0]
    if cell is None:
        images = [np.zeros(3, dtype=int)]
        cellm = np.zeros((3, 3))
    else:
        cellm = np.asarray(cell, dtype=np.float64)
        # number of images needed along each lattice vector: rcut over the
        # spacing of the lattice planes, plus one for atoms anywhere in the cell
        inv = np.linalg.inv(cellm)
        spacing = 1.0 / np.linalg.norm(inv, axis=0)
        nimg = np.ceil(rcut / spacing).astype(int) + 1
        rng = [np.arange(-k, k + 1) for k in nimg]
        images = [np.array([a, b, c]) for a in rng[0] for b in rng[1] for c in rng[2]]
    rows = []
    for i in range(N):
        for j in range(N):
            for n in images:
                d = pos[j] + n @ cellm - pos[i]
                r = np.sqrt(d @ d)
                if 0.0 < r < rcut:
                    rows.append((i, j, int(n[0]), int(n[1]), int(n[2])))
    rows.sort()
    offsets = np.zeros(N + 1, dtype=np.int64)
    for row in rows:
        offsets[row[0] + 1] += 1
    offsets = np.cumsum(offsets)
    nbr_j = np.array([row[1] for row in rows], dtype=np.int64)
    shift = np.array([row[2:] for row in rows], dtype=np.int64).reshape(-1, 3)
    return offsets, nbr_j, shift


def pair_vectors(pos, cell, offsets, nbr_j, shift, atoms=None):
    """r_ij = r_j + n.cell - r_i for the pairs of the given centre atoms.
    Returns (centre index per pair, pair index, r_ij [P,3])."""
    pos = np.asarray(pos, dtype=np.float64)
    offsets = np.asarray(offsets)
    if atoms is None:
        atoms = np.arange(pos.shape[0])
    atoms = np.asarray(atoms)
    counts = offsets[atoms + 1] - offsets[atoms]
    centre = np.repeat(atoms, counts)
    pidx = np.concatenate([np.arange(offsets[a], offsets[a + 1]) for a in atoms]) \
        if len(atoms) else np.zeros(0, dtype=int)
    pidx = pidx.astype(np.int64)
    j = np.asarray(nbr_j)[pidx]
    sh = np.asarray(shift, dtype=np.float64)[pidx]
    cellm = np.zeros((3, 3)) if cell is None else np.asarray(cell, dtype=np.float64)
    d = pos[j] + sh @ cellm - pos[centre]
    return centre, pidx, d


# --------------------------------------------------------------------------
# Naive descriptors: the sums of eqs. (12b), (15), (15b), (18a) written out
# --------------------------------------------------------------------------
def descriptors_naive_env(Rn, U, p: PodParams):
    """Descriptor vector of one atom from its neighbour radial values
    Rn [n_i, K] and unit vectors U [n_i, 3], by the full sums.

    Layout: [1 | D2 (k < K2) | D3 (m < K3, n = 0..P3) | D4 (m < K4, Table-1 p)].
    """
    Rn = np.asarray(Rn, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    ni = Rn.shape[0]
    W = U @ U.T  # W[j, k] = w_ijk = rhat_ij . rhat_ik
    out = [1.0]
    for k in range(p.K2):                                     # eq. (12b)
        out.append(Rn[:, k].sum())
    for m in range(p.K3):                                     # eqs. (14)-(15)
        for n in range(p.P3 + 1):
            s = 0.0
            for j in range(ni):
                for k in range(ni):
                    s += Rn[j, m] * Rn[k, m] * W[j, k] ** n
            out.append(s)
    trip = four_body_triples(p.P4) if p.K4 > 0 else []
    for m in range(p.K4):                                     # eqs. (16a), (17a), (18a)
        R = Rn[:, m]
        for (a, b, c) in trip:
            # sum over all ordered (j, k, l): R_j R_k R_l w_jk^a w_jl^b w_kl^c
            t = np.einsum("j,k,l,jk,jl,kl->", R, R, R, W ** a, W ** b, W ** c)
            out.append(float(t))
    return np.array(out)


def three_body_exclusive_env(Rn, U, K3, P3):
    """Exclusive 3-body descriptors of eq. (15b): sum over j and k > j."""
    W = U @ U.T
    ni = Rn.shape[0]
    D = np.zeros((K3, P3 + 1))
    for m in range(K3):
        for n in range(P3 + 1):
            s = 0.0
            for j in range(ni):
                for k in range(j + 1, ni):
                    s += Rn[j, m] * Rn[k, m] * W[j, k] ** n
            D[m, n] = s
    return D


def descriptors_naive(pos, cell, offsets, nbr_j, shift, p: PodParams, Q, atoms=None):
    """Naive per-atom descriptors D [n_atoms, M] (small systems only)."""
    pos = np.asarray(pos, dtype=np.float64)
    if atoms is None:
        atoms = np.arange(pos.shape[0])
    M, _ = num_descriptors(p)
    D = np.zeros((len(atoms), M))
    for ii, a in enumerate(atoms):
        _, _, d = pair_vectors(pos, cell, offsets, nbr_j, shift, [a])
        if d.shape[0] == 0:
            D[ii] = descriptors_naive_env(np.zeros((0, p.K)), np.zeros((0, 3)), p)
            continue
        r = np.sqrt((d * d).sum(1))
        Rn, _ = radial_basis(r, p, Q)
        D[ii] = descriptors_naive_env(Rn, d / r[:, None], p)
    return D


# --------------------------------------------------------------------------
# Fast form: atom density representation, Sec. II.E
# --------------------------------------------------------------------------
def monomials(U, P):
    """A_{n l}(u) = x^a y^b z^c for every exponent of monomial_exponents(P),
    evaluated at the rows of U [n, 3] (eq. (23b)).  Returns [n, N_a]."""
    E = monomial_exponents(P)
    U = np.asarray(U, dtype=np.float64)
    A = np.empty((U.shape[0], len(E)))
    for mu, (a, b, c) in enumerate(E):
        A[:, mu] = U[:, 0] ** a * U[:, 1] ** b * U[:, 2] ** c
    return A


def monomial_gradients(U, P):
    """Gradient of each monomial with respect to u = (x, y, z) taken as
    independent variables.  Returns [n, N_a, 3]."""
    E = monomial_exponents(P)
    U = np.asarray(U, dtype=np.float64)
    x, y, z = U[:, 0], U[:, 1], U[:, 2]
    G = np.zeros((U.shape[0], len(E), 3))
    for mu, (a, b, c) in enumerate(E):
        if a > 0:
            G[:, mu, 0] = a * x ** (a - 1) * y ** b * z ** c
        if b > 0:
            G[:, mu, 1] = b * x ** a * y ** (b - 1) * z ** c
        if c > 0:
            G[:, mu, 2] = c * x ** a * y ** b * z ** (c - 1)
    return G


def atomic_basis(centre, R, A, n_atoms, atom_index):
    """B_{i m mu} = sum_j R_m(r_ij) A_mu(rhat_ij) (eq. (24b)).
    centre: centre atom of each pair; atom_index maps atom id -> row."""
    B = np.zeros((n_atoms, R.shape[1], A.shape[1]))
    rows = atom_index[centre]
    np.add.at(B, rows, R[:, :, None] * A[:, None, :])
    return B


def _mono_lookup(P):
    return {e: mu for mu, e in enumerate(monomial_exponents(P))}


def fast_descriptors_from_B(B, p: PodParams):
    """Descriptors from the atomic basis B [n, K, N_a]:
    D2_m = B_{m,0} (eq. (25)); D3_mn = sum_l c_nl B_{mnl}^2 (eq. (26a));
    D4 by eq. (27a) for b = c = 0 and by eq. (30a) otherwise."""
    PA = p.PA
    E = monomial_exponents(PA)
    deg = np.array([sum(e) for e in E])
    cmu = np.array([multinomial(e) for e in E], dtype=np.float64)
    look = _mono_lookup(PA)
    n = B.shape[0]
    M, _ = num_descriptors(p)
    D = np.zeros((n, M))
    D[:, 0] = 1.0
    col = 1
    D[:, col:col + p.K2] = B[:, : p.K2, 0]
    col += p.K2
    # 3-body: for every degree up to PA (the 4-body (a,0,0) terms reuse them)
    D3all = np.zeros((n, p.K, PA + 1))
    for nn in range(PA + 1):
        sel = deg == nn
        D3all[:, :, nn] = (cmu[sel][None, None, :] * B[:, :, sel] ** 2).sum(-1)
    for m in range(p.K3):
        D[:, col:col + p.P3 + 1] = D3all[:, m, : p.P3 + 1]
        col += p.P3 + 1
    if p.K4 > 0:
        trip = four_body_triples(p.P4)
        for m in range(p.K4):
            for (a, b, c) in trip:
                if b == 0 and c == 0:                         # eq. (27a)
                    D[:, col] = B[:, m, 0] * D3all[:, m, a]
                else:                                          # eq. (30a)
                    s = np.zeros(n)
                    for ea in monomial_exponents(a)[_deg_start(a):]:
                        for eb in monomial_exponents(b)[_deg_start(b):]:
                            for ec in monomial_exponents(c)[_deg_start(c):]:
                                coef = multinomial(ea) * multinomial(eb) * multinomial(ec)
                                ij = look[_add(ea, eb)]
                                ik = look[_add(ea, ec)]
                                il = look[_add(eb, ec)]
                                s += coef * B[:, m, ij] * B[:, m, ik] * B[:, m, il]
                    D[:, col] = s
                col += 1
    return D


def _deg_start(n):
    """Index of the first degree-n exponent in monomial_exponents(n)."""
    return n * (n + 1) * (n + 2) // 6


def _add(e, f):
    return (e[0] + f[0], e[1] + f[1], e[2] + f[2])


def descriptors_fast(pos, cell, offsets, nbr_j, shift, p: PodParams, Q, atoms=None):
    """Per-atom descriptors [n_atoms, M] by the fast (atom density) form."""
    pos = np.asarray(pos, dtype=np.float64)
    if atoms is None:
        atoms = np.arange(pos.shape[0])
    atoms = np.asarray(atoms)
    B, _ = _basis_for_atoms(pos, cell, offsets, nbr_j, shift, p, Q, atoms)
    return fast_descriptors_from_B(B, p)


def _basis_for_atoms(pos, cell, offsets, nbr_j, shift, p, Q, atoms):
    centre, pidx, d = pair_vectors(pos, cell, offsets, nbr_j, shift, atoms)
    index = np.full(pos.shape[0], -1, dtype=np.int64)
    index[atoms] = np.arange(len(atoms))
    K, PA = p.K, p.PA
    Na = (PA + 1) * (PA + 2) * (PA + 3) // 6
    if d.shape[0] == 0:
        return np.zeros((len(atoms), K, Na)), None
    r = np.sqrt((d * d).sum(1))
    U = d / r[:, None]
    R, dR = radial_basis(r, p, Q)
    A = monomials(U, PA)
    B = atomic_basis(centre, R, A, len(atoms), index)
    return B, (centre, pidx, d, r, U, R, dR, A, index)


# --------------------------------------------------------------------------
# Linear energy model, Sec. IV.A, and its derivatives, Sec. II.G
# --------------------------------------------------------------------------
def energy_from_descriptors(D, c):
    """E_i = sum_m c_m D_im (eq. (57a)); E = sum_i E_i; G = sum_i D_i (eq. (58a))."""
    Ei = D @ np.asarray(c, dtype=np.float64)
    return Ei, Ei.sum(), D.sum(0)


def descriptor_jacobian_B(B, p: PodParams):
    """dD_i/dB_i for every descriptor: J [n, M, K, N_a], by the product rule
    applied to eqs. (25), (26a), (27a), (30a) (eq. (26c) for the 3-body)."""
    PA = p.PA
    E = monomial_exponents(PA)
    deg = np.array([sum(e) for e in E])
    cmu = np.array([multinomial(e) for e in E], dtype=np.float64)
    look = _mono_lookup(PA)
    n, K, Na = B.shape
    M, _ = num_descriptors(p)
    J = np.zeros((n, M, K, Na))
    col = 1
    for k in range(p.K2):
        J[:, col, k, 0] = 1.0
        col += 1
    for m in range(p.K3):
        for nn in range(p.P3 + 1):
            sel = np.where(deg == nn)[0]
            J[:, col, m, sel] = 2.0 * cmu[sel][None, :] * B[:, m, sel]
            col += 1
    if p.K4 > 0:
        trip = four_body_triples(p.P4)
        for m in range(p.K4):
            for (a, b, c) in trip:
                if b == 0 and c == 0:
                    sel = np.where(deg == a)[0]
                    d3 = (cmu[sel][None, :] * B[:, m, sel] ** 2).sum(-1)
                    J[:, col, m, 0] += d3
                    J[:, col, m, sel] += B[:, m, 0][:, None] * 2.0 * cmu[sel][None, :] * B[:, m, sel]
                else:
                    for ea in monomial_exponents(a)[_deg_start(a):]:
                        for eb in monomial_exponents(b)[_deg_start(b):]:
                            for ec in monomial_exponents(c)[_deg_start(c):]:
                                coef = multinomial(ea) * multinomial(eb) * multinomial(ec)
                                x = look[_add(ea, eb)]
                                y = look[_add(ea, ec)]
                                z = look[_add(eb, ec)]
                                J[:, col, m, x] += coef * B[:, m, y] * B[:, m, z]
                                J[:, col, m, y] += coef * B[:, m, x] * B[:, m, z]
                                J[:, col, m, z] += coef * B[:, m, x] * B[:, m, y]
                col += 1
    return J


def basis_pair_derivative(R, dR, A, U, r, PA):
    """dB_{m mu}/dr_ij contributed by one pair (eq. (24c)):
    dR_m/dr_ij A_mu + R_m dA_mu/dr_ij, with dR_m/dr_ij = R'_m rhat and
    dA_mu/dr_ij = (I - rhat rhat^T) grad_u A_mu / r (chain rule through
    rhat = r_ij/|r_ij|).  Returns [P, K, N_a, 3]."""
    G = monomial_gradients(U, PA)                                # [P, Na, 3]
    proj = G - (G * U[:, None, :]).sum(-1, keepdims=True) * U[:, None, :]
    dA = proj / r[:, None, None]                                 # [P, Na, 3]
    return (dR[:, :, None, None] * A[:, None, :, None] * U[:, None, None, :]
            + R[:, :, None, None] * dA[:, None, :, :])


def energy_forces(pos, cell, offsets, nbr_j, shift, p: PodParams, Q, c,
                  chunk_atoms: int = 1024, force_atoms=None):
    """Energies and forces of the linear POD model.

    Returns dict with E_atom [N], E, G [M], F [N,3] (F_n = -dE/dr_n) and the
    virial W_ab = -sum_pairs r_ij,a dE_i/dr_ij,b (reading: equals -dE/d(strain)
    for a symmetric strain).  Atoms are processed independently in chunks;
    this only bounds memory.  With force_atoms given, F is computed only for
    those atoms (others are left zero) and W is not computed.
    """
    pos = np.asarray(pos, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    N = pos.shape[0]
    offsets = np.asarray(offsets)
    nbr_j = np.asarray(nbr_j)
    M, _ = num_descriptors(p)
    E_atom = np.zeros(N)
    G = np.zeros(M)
    F = np.zeros((N, 3))
    W = np.zeros((3, 3))
    if force_atoms is None:
        centres = np.arange(N)
        want_F = None
    else:
        force_atoms = np.asarray(force_atoms)
        # every centre whose energy depends on a force atom: the force atoms
        # themselves and every atom that has one of them as a neighbour
        mask = np.zeros(N, dtype=bool)
        mask[force_atoms] = True
        centre_all = np.repeat(np.arange(N), np.diff(offsets))
        hit = mask[nbr_j]
        mask[np.unique(centre_all[hit])] = True
        centres = np.where(mask)[0]
        want_F = np.zeros(N, dtype=bool)
        want_F[force_atoms] = True
    for s in range(0, len(centres), chunk_atoms):
        atoms = centres[s:s + chunk_atoms]
        B, geo = _basis_for_atoms(pos, cell, offsets, nbr_j, shift, p, Q, atoms)
        D = fast_descriptors_from_B(B, p)
        Ei = D @ c
        E_atom[atoms] = Ei
        G += D.sum(0)
        if geo is None:
            continue
        centre, pidx, d, r, U, R, dR, A, index = geo
        J = descriptor_jacobian_B(B, p)                         # [n, M, K, Na]
        Abar = np.einsum("m,nmka->nka", c, J)                   # dE_i/dB_i
        dB = basis_pair_derivative(R, dR, A, U, r, p.PA)        # [P, K, Na, 3]
        g = np.einsum("pka,pkad->pd", Abar[index[centre]], dB)  # dE_i/dr_ij
        np.add.at(F, centre, g)
        np.add.at(F, nbr_j[pidx], -g)
        if want_F is None:
            W -= d.T @ g
    if want_F is not None:
        F[~want_F] = 0.0
        W = None
        E = None
    else:
        E = E_atom.sum()
    return {"E_atom": E_atom, "E": E, "G": G if want_F is None else None, "F": F, "W": W}


def descriptor_derivatives(pos, cell, offsets, nbr_j, shift, p: PodParams, Q, atoms=None):
    """dD_i/dr_ij for every pair of the given centres: [P_sel, M, 3], plus the
    centre and pair index of each row (eq. (26c), (24c); product rule)."""
    pos = np.asarray(pos, dtype=np.float64)
    if atoms is None:
        atoms = np.arange(pos.shape[0])
    atoms = np.asarray(atoms)
    B, geo = _basis_for_atoms(pos, cell, offsets, nbr_j, shift, p, Q, atoms)
    M, _ = num_descriptors(p)
    if geo is None:
        return np.zeros((0, M, 3)), np.zeros(0, int), np.zeros(0, int)
    centre, pidx, d, r, U, R, dR, A, index = geo
    J = descriptor_jacobian_B(B, p)
    dB = basis_pair_derivative(R, dR, A, U, r, p.PA)
    dD = np.einsum("pmka,pkad->pmd", J[index[centre]], dB)
    return dD, centre, pidx


def global_descriptor_derivatives(pos, cell, offsets, nbr_j, shift, p: PodParams, Q):
    """dG_m/dr_n for the whole configuration: [N, 3, M] with
    G_m = sum_i D_im and r_ij = r_j + n.cell - r_i."""
    N = np.asarray(pos).shape[0]
    M, _ = num_descriptors(p)
    dD, centre, pidx = descriptor_derivatives(pos, cell, offsets, nbr_j, shift, p, Q)
    out = np.zeros((N, M, 3))
    np.add.at(out, np.asarray(nbr_j)[pidx], dD)
    np.add.at(out, centre, -dD)
    return out.transpose(0, 2, 1).copy()


# --------------------------------------------------------------------------
# Finite-difference helpers
# --------------------------------------------------------------------------
def total_energy(pos, cell, offsets, nbr_j, shift, p, Q, c):
    D = descriptors_fast(pos, cell, offsets, nbr_j, shift, p, Q)
    return float((D @ np.asarray(c, dtype=np.float64)).sum())


def fd_forces(pos, cell, offsets, nbr_j, shift, p, Q, c, atoms, h=1e-5):
    """Central differences F_n = -(E(r_n + h e) - E(r_n - h e)) / 2h with the
    neighbour list held fixed (valid while no pair crosses rcut)."""
    pos = np.asarray(pos, dtype=np.float64)
    F = np.zeros((len(atoms), 3))
    for ii, a in enumerate(atoms):
        for d in range(3):
            pp = pos.copy(); pp[a, d] += h
            pm = pos.copy(); pm[a, d] -= h
            F[ii, d] = -(total_energy(pp, cell, offsets, nbr_j, shift, p, Q, c)
                         - total_energy(pm, cell, offsets, nbr_j, shift, p, Q, c)) / (2 * h)
    return F


def fd_virial(pos, cell, offsets, nbr_j, shift, p, Q, c, h=1e-6):
    """W_ab = -dE/d eps_ab for a symmetric homogeneous strain applied to the
    positions and the cell (central differences)."""
    pos = np.asarray(pos, dtype=np.float64)
    cellm = np.asarray(cell, dtype=np.float64)
    W = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            eps = np.zeros((3, 3)); eps[a, b] += 0.5 * h; eps[b, a] += 0.5 * h
            Ep = total_energy(pos @ (np.eye(3) + eps).T, cellm @ (np.eye(3) + eps).T,
                              offsets, nbr_j, shift, p, Q, c)
            Em = total_energy(pos @ (np.eye(3) - eps).T, cellm @ (np.eye(3) - eps).T,
                              offsets, nbr_j, shift, p, Q, c)
            W[a, b] = -(Ep - Em) / (2 * h)
    return W
