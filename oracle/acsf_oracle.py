"""Plain FP64 CPU oracle of atom-centred symmetry functions (ACSF).

Test infrastructure, not product code.  Only the test suite, the smoke check
and the benchmark's CPU leg import this module; the HIP library and its
binding never call it, and it shares no code with them.

The functions are the ones of Sec. III.B, evaluated by their defining sums
over neighbours, pairs and triples of neighbours:

    G2_i = sum_j exp(-eta (r_ij - r_s)^2) f_c(r_ij)                  eq. (21c)
    G3_i = 2^(1-zeta) sum_{j,k} (1 + lambda w_ijk)^zeta
           exp(-eta (r_ij^2 + r_ik^2)) f_c(r_ij) f_c(r_ik)            eq. (22c)
    G4_i = sum_{j,k,l} (1 + alpha w_ijk)^a (1 + beta w_ijl)^b
           (1 + gamma w_ikl)^c exp(-eta (r_ij^2 + r_ik^2 + r_il^2))
           f_c(r_ij) f_c(r_ik) f_c(r_il)                              eq. (22d)

with w_ijk = rhat_ij . rhat_ik (Sec. II.A) and f_c the cut-off function of
eq. (8).  Readings: the sums run over all ordered tuples of neighbours,
repeated indices included, as the POD sums of eqs. (15) and (18) do; the
exponents zeta, a, b, c are non-negative integers.

Forces of a weighted sum E = sum_i W_i . G_i come from PyTorch's reverse-mode
differentiation of these same sums (CPU, float64), so values and gradients
have one definition.
"""
from __future__ import annotations

import numpy as np
import torch

EPS_FC = 1e-6


def cutoff_t(r, rin, rcut):
    """f_c of eq. (8) on a torch tensor of distances."""
    t = (r - rin) / (rcut - rin)
    y = 1.0 - t * t * t
    return torch.exp(1.0 - 1.0 / torch.sqrt(y * y + EPS_FC))


def _ipow(x, n: int):
    """x^n for an integer n >= 0 by repeated products (x^0 = 1, also at 0)."""
    out = torch.ones_like(x)
    for _ in range(n):
        out = out * x
    return out


def env_functions(d, spec, rin, rcut):
    """All functions of one atom from its neighbour vectors d [n, 3] (torch,
    float64): a tensor of length spec.n in the order G2, G3, G4."""
    out = []
    r = torch.sqrt((d * d).sum(1))
    fc = cutoff_t(r, rin, rcut)
    u = d / r[:, None]
    w = u @ u.T                                    # w[j, k] = cos(theta_ijk)
    for eta, rs in spec.g2:
        out.append((torch.exp(-eta * (r - rs) ** 2) * fc).sum())
    for eta, zeta, lam in spec.g3:
        g = torch.exp(-eta * r * r) * fc
        ang = _ipow(1.0 + lam * w, int(zeta))
        out.append(2.0 ** (1 - int(zeta)) * (ang * g[:, None] * g[None, :]).sum())
    for eta, a, b, c, al, be, ga in spec.g4:
        g = torch.exp(-eta * r * r) * fc
        t_jk = _ipow(1.0 + al * w, int(a))[:, :, None]     # (j, k, .)
        t_jl = _ipow(1.0 + be * w, int(b))[:, None, :]     # (j, ., l)
        t_kl = _ipow(1.0 + ga * w, int(c))[None, :, :]     # (., k, l)
        gg = g[:, None, None] * g[None, :, None] * g[None, None, :]
        out.append((t_jk * t_jl * t_kl * gg).sum())
    if not out:
        return torch.zeros(0, dtype=d.dtype)
    return torch.stack(out)


def _pair_vectors_t(x, cell, offsets, nbr_j, shift3, i):
    """r_ij = x_j + n.cell - x_i of the pairs of atom i (torch)."""
    p0, p1 = int(offsets[i]), int(offsets[i + 1])
    j = torch.as_tensor(np.asarray(nbr_j[p0:p1], dtype=np.int64))
    sh = np.asarray(shift3[p0:p1], dtype=np.float64).reshape(-1, 3)
    cellm = np.zeros((3, 3)) if cell is None else np.asarray(cell, dtype=np.float64).reshape(3, 3)
    return x[j] + torch.as_tensor(sh @ cellm) - x[i]


def _keep_within(d, rcut):
    """Pairs at or beyond rcut are not neighbours (a skin list may hold them)."""
    r = torch.sqrt((d * d).sum(1))
    return d[r.detach() < rcut]


def descriptors(pos, cell, offsets, nbr_j, shift3, rin, rcut, spec, atoms=None):
    """G [len(atoms), spec.n] (numpy float64); shift3 is [P, 3] integer."""
    x = torch.as_tensor(np.asarray(pos, dtype=np.float64))
    N = x.shape[0]
    atoms = range(N) if atoms is None else atoms
    rows = []
    for i in atoms:
        d = _keep_within(_pair_vectors_t(x, cell, offsets, nbr_j, shift3, i), rcut)
        rows.append(env_functions(d, spec, rin, rcut).numpy())
    return np.array(rows, dtype=np.float64).reshape(len(rows), spec.n)


def energy_forces(pos, cell, offsets, nbr_j, shift3, rin, rcut, spec, W, atoms=None):
    """E = sum_i W_i . G_i and F = -dE/dx (numpy, float64).

    W: [N, spec.n] per-atom weights or [spec.n] shared by all atoms.  With
    `atoms`, only the forces on those atoms are returned ([len(atoms), 3]),
    computed from the centres whose energy depends on them: each atom itself
    and its neighbours (a full list is symmetric); E is then the partial sum
    over those centres."""
    x = torch.tensor(np.asarray(pos, dtype=np.float64), requires_grad=True)
    N = x.shape[0]
    Wt = torch.as_tensor(np.asarray(W, dtype=np.float64))
    if atoms is None:
        centres = range(N)
    else:
        cs = set(int(a) for a in atoms)
        for a in atoms:
            cs.update(int(j) for j in nbr_j[int(offsets[a]):int(offsets[a + 1])])
        centres = sorted(cs)
    E = torch.zeros((), dtype=torch.float64)
    for i in centres:
        d = _keep_within(_pair_vectors_t(x, cell, offsets, nbr_j, shift3, i), rcut)
        if d.shape[0] == 0:
            continue
        w = Wt if Wt.dim() == 1 else Wt[i]
        E = E + (w * env_functions(d, spec, rin, rcut)).sum()
    if E.requires_grad:
        (g,) = torch.autograd.grad(E, x)
    else:
        g = torch.zeros_like(x)
    F = -g.numpy()
    if atoms is not None:
        F = F[np.asarray(atoms, dtype=np.int64)]
    return float(E.detach()), F
