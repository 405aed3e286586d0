"""Plain FP64 CPU oracle of five-body POD descriptors.

Test infrastructure, not product code.  Only the test suite, the smoke check
and the benchmark's CPU leg import this module; the HIP library and its
binding never call it, and it shares no code with them.

Sec. II.F closes by extending the construction to any body order: a
five-body descriptor uses the four distances r_ij, r_ik, r_il, r_in and the
six angles between the four neighbours, built like the four-body descriptors
of eqs. (16a)-(18a).  Reading taken here (the paper gives no formula):

    D5_{i m e} = sum_{j,k,l,n} R_m(r_ij) R_m(r_ik) R_m(r_il) R_m(r_in)
                 w_ijk^e1 w_ijl^e2 w_ijn^e3 w_ikl^e4 w_ikn^e5 w_iln^e6

for exponent tuples e = (e1, ..., e6) of non-negative integers with
|e| <= P5, the same radial function m in every factor (as in eq. (17a)), all
ordered neighbour tuples with repeated indices (as in eq. (18a)).  Relabelling
(j, k, l, n) permutes the six angle positions without changing the sum, so
there is one descriptor per orbit of the 24 relabellings -- the analogue of
the a >= b >= c ordering of Table 1 for the three angles of the four-body
term.  Order: |e| ascending; within a degree, the orbits by their
lexicographically largest tuple, descending.

The energy E_i = sum_{m,e} c5_{m e} D5_{i m e} and its forces come from
PyTorch's reverse-mode differentiation (CPU, float64) of the same sums, with
R_m and R'_m taken from the POD oracle's radial basis.
"""
from __future__ import annotations

import itertools

import numpy as np

from oracle import pod_oracle as po

# angle positions: (j,k), (j,l), (j,n), (k,l), (k,n), (l,n) with j,k,l,n = 0,1,2,3
EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def relabel(perm, e):
    """The tuple e after renaming neighbour slot v to perm[v]."""
    out = [0] * 6
    for t, (a, b) in enumerate(EDGES):
        u, v = sorted((perm[a], perm[b]))
        out[EDGES.index((u, v))] = e[t]
    return tuple(out)


def orbit(e):
    return {relabel(p, e) for p in itertools.permutations(range(4))}


def orbits(P5: int):
    """One representative (the largest tuple) per orbit, in descriptor order."""
    out = []
    for n in range(P5 + 1):
        reps = set()
        for e in itertools.product(range(n + 1), repeat=6):
            if sum(e) == n:
                reps.add(max(orbit(e)))
        out.extend(sorted(reps, reverse=True))
    return out


def five_body_sum(R, W, e):
    """The defining quadruple sum for one radial vector R [n] and the cosine
    matrix W [n, n] at exponent tuple e."""
    return float(np.einsum("j,k,l,n,jk,jl,jn,kl,kn,ln->", R, R, R, R,
                           W ** e[0], W ** e[1], W ** e[2], W ** e[3], W ** e[4], W ** e[5],
                           optimize=True))


def descriptors5_env(Rn, U, K5: int, P5: int):
    """[K5 * n_orbits] for one atom (m-major) from its neighbours' radial
    values Rn [n, >= K5] and unit vectors U [n, 3]."""
    W = np.asarray(U) @ np.asarray(U).T
    reps = orbits(P5)
    return np.array([five_body_sum(np.asarray(Rn)[:, m], W, e) for m in range(K5) for e in reps])


def descriptors5(pos, cell, offsets, nbr_j, shift3, p: po.PodParams, Q, K5: int, P5: int, atoms=None):
    """[len(atoms), K5 * n_orbits] with the radial basis of eq. (12); pairs at
    or beyond rcut are not neighbours."""
    pos = np.asarray(pos, dtype=np.float64)
    atoms = np.arange(pos.shape[0]) if atoms is None else np.asarray(atoms)
    rows = []
    for a in atoms:
        _, _, d = po.pair_vectors(pos, cell, offsets, nbr_j, shift3, atoms=[int(a)])
        r = np.sqrt((d * d).sum(1))
        keep = r < p.rcut
        d, r = d[keep], r[keep]
        Rn = po.radial_basis(r, p, Q)[0] if r.size else np.zeros((0, p.K))
        rows.append(descriptors5_env(Rn, d / r[:, None] if r.size else np.zeros((0, 3)), K5, P5))
    return np.array(rows).reshape(len(atoms), K5 * len(orbits(P5)))


# --------------------------------------------------------------------------
# Energy c5 . D5 and forces (PyTorch CPU float64 autograd of the same sums)
# --------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _ipow(x, n: int):
    """x^n by repeated products (x^0 = 1 with a zero derivative everywhere)."""
    out = _torch().ones_like(x)
    for _ in range(n):
        out = out * x
    return out


def _radial_fn(p, Q, K5):
    """R_m(r), m < K5, as a differentiable function of r: values and
    derivatives from the POD oracle's radial basis (eq. (12))."""
    torch = _torch()

    class Radial(torch.autograd.Function):
        @staticmethod
        def forward(ctx, r):
            R, dR = po.radial_basis(r.detach().numpy(), p, Q)
            ctx.save_for_backward(torch.as_tensor(dR[:, :K5]))
            return torch.as_tensor(R[:, :K5])

        @staticmethod
        def backward(ctx, g):
            (dR,) = ctx.saved_tensors
            return (g * dR).sum(1)

    return Radial.apply


def energy_forces5(pos, cell, offsets, nbr_j, shift3, p: po.PodParams, Q, K5: int, P5: int, c5):
    """E_i = sum_{m, e} c5[m, e] D5_{i m e} (c5: K5 x n_orbits, m-major as D5)
    and F = -dE/dx with E = sum_i E_i.  Returns (E_atom [N], F [N, 3])."""
    torch = _torch()
    pos = np.asarray(pos, dtype=np.float64)
    N = pos.shape[0]
    reps = orbits(P5)
    c5 = np.asarray(c5, dtype=np.float64).reshape(K5, len(reps))
    x = torch.tensor(pos, requires_grad=True)
    cellm = torch.zeros((3, 3), dtype=torch.float64) if cell is None else torch.as_tensor(np.asarray(cell, float))
    radial = _radial_fn(p, Q, K5)
    E_atom = np.zeros(N)
    for i in range(N):
        p0, p1 = int(offsets[i]), int(offsets[i + 1])
        j = torch.as_tensor(np.asarray(nbr_j[p0:p1], dtype=np.int64))
        sh = torch.as_tensor(np.asarray(shift3[p0:p1], dtype=np.float64).reshape(-1, 3))
        with torch.no_grad():
            rr = torch.sqrt(((x[j] + sh @ cellm - x[i]) ** 2).sum(1))
        keep = rr < p.rcut
        if not bool(keep.any()):
            continue
        d = (x[j] + sh @ cellm - x[i])[keep]
        r = torch.sqrt((d * d).sum(1))
        u = d / r[:, None]
        W = u @ u.T
        R = radial(r)
        for m in range(K5):
            Rm = R[:, m]
            # the angular factor of every orbit, weighted and summed, then one
            # quadruple contraction with the radial values
            ang = 0.0
            for t, e in enumerate(reps):
                ang = ang + c5[m, t] * (_ipow(W, e[0])[:, :, None, None] * _ipow(W, e[1])[:, None, :, None]
                                        * _ipow(W, e[2])[:, None, None, :] * _ipow(W, e[3])[None, :, :, None]
                                        * _ipow(W, e[4])[None, :, None, :] * _ipow(W, e[5])[None, None, :, :])
            Em = torch.einsum("j,k,l,n,jkln->", Rm, Rm, Rm, Rm, ang)
            E_atom[i] += float(Em.detach())
            Em.backward(retain_graph=m < K5 - 1)
    g = x.grad if x.grad is not None else torch.zeros_like(x)
    return E_atom, -g.numpy()
