"""Pins of the ACSF oracle (eqs. (21c), (22c), (22d)).

Environments with one, two and three neighbours whose sums can be written out
by hand (every ordered tuple enumerated), the special exponents that reduce
the functions to powers of the radial sum, invariance under rotation and
neighbour permutation, the cut-off contract, forces against central
finite differences of the weighted energy, and the invariant expansion the
device uses against the defining sums."""
import math

import numpy as np
import pytest
import torch

from oracle import acsf_oracle as ao
from oracle import pod_oracle as po
from paper_2212_14446_amd import workloads as wl

RIN, RCUT = 0.5, 5.0


def _fc(r):
    return float(po.cutoff(r, RIN, RCUT)[0])


def _env(vectors, spec):
    d = torch.as_tensor(np.asarray(vectors, dtype=np.float64))
    return ao.env_functions(d, spec, RIN, RCUT).numpy()


def _dir(theta):
    return np.array([math.cos(theta), math.sin(theta), 0.0])


def test_cutoff_matches_pod_oracle():
    r = np.linspace(0.6, 4.99, 57)
    got = ao.cutoff_t(torch.as_tensor(r), RIN, RCUT).numpy()
    assert np.abs(got - po.cutoff(r, RIN, RCUT)[0]).max() <= 1e-15


def test_single_neighbour_closed_forms():
    r = 2.7
    spec = wl.AcsfSpec(g2=((1.3, 2.0),), g3=((0.1, 3, -1.0), (0.1, 2, 1.0)),
                       g4=((0.07, 2, 1, 1, 0.5, -0.25, 1.0),))
    G = _env([[0.0, 0.0, r]], spec)
    fc = _fc(r)
    g3 = math.exp(-0.1 * r * r) * fc
    g4 = math.exp(-0.07 * r * r) * fc
    want = [math.exp(-1.3 * (r - 2.0) ** 2) * fc,
            2.0 ** -2 * 0.0 ** 3 * g3 * g3,                 # (1 - 1)^3
            2.0 ** -1 * 2.0 ** 2 * g3 * g3,
            1.5 ** 2 * 0.75 * 2.0 * g4 ** 3]
    assert np.allclose(G, want, rtol=1e-14, atol=1e-300)


@pytest.mark.parametrize("zeta,lam", [(1, 1.0), (2, -1.0), (4, 1.0), (5, -0.6)])
def test_two_neighbours_g3(zeta, lam):
    th, r1, r2, eta = 1.2, 2.2, 3.1, 0.3
    spec = wl.AcsfSpec(g3=((eta, zeta, lam),))
    G = _env([r1 * _dir(0.0), r2 * _dir(th)], spec)
    g1 = math.exp(-eta * r1 * r1) * _fc(r1)
    g2 = math.exp(-eta * r2 * r2) * _fc(r2)
    c = math.cos(th)
    # ordered pairs (1,1), (2,2) at w = 1; (1,2), (2,1) at w = cos(theta)
    want = 2.0 ** (1 - zeta) * ((1 + lam) ** zeta * (g1 * g1 + g2 * g2) + 2 * (1 + lam * c) ** zeta * g1 * g2)
    assert abs(G[0] - want) <= 1e-14 * abs(want)


def test_two_neighbours_g4_all_eight_tuples():
    th, r1, r2, eta = 1.22, 2.4, 3.3, 0.05
    a, b, c, al, be, ga = 2, 1, 3, 0.5, -0.3, 0.8
    spec = wl.AcsfSpec(g4=((eta, a, b, c, al, be, ga),))
    G = _env([r1 * _dir(0.0), r2 * _dir(th)], spec)
    g = [math.exp(-eta * r * r) * _fc(r) for r in (r1, r2)]
    cs = math.cos(th)
    want = 0.0
    for j in range(2):
        for k in range(2):
            for l in range(2):
                w = lambda p, q: 1.0 if p == q else cs
                want += ((1 + al * w(j, k)) ** a * (1 + be * w(j, l)) ** b * (1 + ga * w(k, l)) ** c
                         * g[j] * g[k] * g[l])
    # the same sum grouped by hand: (1,1,1), (2,2,2) | j = k != l | j = l != k | k = l != j
    P = (1 + al) ** a * (1 + be) ** b * (1 + ga) ** c
    X = (1 + al) ** a * (1 + be * cs) ** b * (1 + ga * cs) ** c
    Y = (1 + al * cs) ** a * (1 + be) ** b * (1 + ga * cs) ** c
    Z = (1 + al * cs) ** a * (1 + be * cs) ** b * (1 + ga) ** c
    grouped = P * (g[0] ** 3 + g[1] ** 3) + (X + Y + Z) * (g[0] ** 2 * g[1] + g[0] * g[1] ** 2)
    assert abs(want - grouped) <= 1e-14 * abs(grouped)
    assert abs(G[0] - want) <= 1e-14 * abs(want)


@pytest.mark.parametrize("zeta,lam", [(1, 1.0), (3, -1.0), (6, 1.0)])
def test_equilateral_triangle_g3(zeta, lam):
    r, eta = 2.9, 0.2
    spec = wl.AcsfSpec(g3=((eta, zeta, lam),))
    G = _env([r * _dir(2 * math.pi * k / 3) for k in range(3)], spec)
    g = math.exp(-eta * r * r) * _fc(r)
    # 3 diagonal pairs at w = 1, 6 off-diagonal at w = -1/2
    want = 2.0 ** (1 - zeta) * g * g * (3 * (1 + lam) ** zeta + 6 * (1 - lam / 2) ** zeta)
    assert abs(G[0] - want) <= 1e-14 * abs(want)


def test_zero_exponents_reduce_to_radial_powers():
    rng = np.random.default_rng(3)
    d = rng.normal(size=(9, 3))
    d *= (rng.uniform(1.0, 4.8, size=9) / np.linalg.norm(d, axis=1))[:, None]
    eta = 0.11
    spec = wl.AcsfSpec(g2=((eta, 0.0),), g3=((eta, 0, 1.0), (eta, 0, -1.0)),
                       g4=((eta, 0, 0, 0, 0.7, 0.2, -0.4), (eta, 3, 2, 1, 0.0, 0.0, 0.0)))
    G = _env(d, spec)
    s = G[0]            # G2 with r_s = 0 is the radial sum sum_j g_j
    assert np.allclose(G[1:3], 2 * s * s, rtol=1e-13)
    assert np.allclose(G[3:5], s ** 3, rtol=1e-13)


def test_invariance_and_cutoff_contract():
    rng = np.random.default_rng(8)
    d = rng.normal(size=(12, 3))
    d *= (rng.uniform(1.0, 4.8, size=12) / np.linalg.norm(d, axis=1))[:, None]
    spec = wl.acsf_standard()
    G = _env(d, spec)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    assert np.abs(_env(d @ q.T, spec) - G).max() <= 1e-12 * np.abs(G).max()
    assert np.abs(_env(d[rng.permutation(12)], spec) - G).max() <= 1e-12 * np.abs(G).max()
    # a list entry at or beyond rcut is not a neighbour
    pos = np.vstack([np.zeros(3), d, [[RCUT + 0.2, 0.0, 0.0]]])
    n = pos.shape[0]
    offsets = np.array([0] + [n - 1] * n)
    nbr_j = np.arange(1, n)
    shift3 = np.zeros((n - 1, 3), dtype=int)
    got = ao.descriptors(pos, None, offsets, nbr_j, shift3, RIN, RCUT, spec, atoms=[0])
    assert np.abs(got[0] - G).max() <= 1e-12 * np.abs(G).max()


def _small_system(seed=4):
    pos, cell = wl.bcc(2)
    pos = wl.displace(pos, 0.12, seed)
    nl = wl.neighbor_list(pos, cell, RCUT)
    return pos, cell, nl


def test_forces_match_finite_differences():
    pos, cell, nl = _small_system()
    spec = wl.AcsfSpec(g2=((2.0, 2.5),), g3=((0.05, 2, -1.0),), g4=((0.05, 2, 1, 1, 1.0, -1.0, 0.5),))
    W = np.random.default_rng(5).normal(size=(pos.shape[0], spec.n))
    E, F = ao.energy_forces(pos, cell, nl.offsets, nl.nbr_j, nl.shift3, RIN, RCUT, spec, W)
    G = ao.descriptors(pos, cell, nl.offsets, nl.nbr_j, nl.shift3, RIN, RCUT, spec)
    assert abs(E - (W * G).sum()) <= 1e-12 * abs(E)
    assert np.abs(F.sum(0)).max() <= 1e-10 * np.abs(F).max()        # translation invariance
    h = 1e-5
    for a, e in ((0, 0), (5, 1), (11, 2)):
        xp, xm = pos.copy(), pos.copy()
        xp[a, e] += h
        xm[a, e] -= h
        # displacements of 1e-5 A keep the list valid (no pair crosses rcut)
        Ep = (W * ao.descriptors(xp, cell, nl.offsets, nl.nbr_j, nl.shift3, RIN, RCUT, spec)).sum()
        Em = (W * ao.descriptors(xm, cell, nl.offsets, nl.nbr_j, nl.shift3, RIN, RCUT, spec)).sum()
        fd = -(Ep - Em) / (2 * h)
        assert abs(F[a, e] - fd) <= 1e-6 * max(1.0, np.abs(F).max())


def test_forces_of_a_subset_equal_the_full_evaluation():
    pos, cell, nl = _small_system(6)
    spec = wl.acsf_standard()
    W = np.random.default_rng(2).normal(size=spec.n)
    _, F = ao.energy_forces(pos, cell, nl.offsets, nl.nbr_j, nl.shift3, RIN, RCUT, spec, W)
    atoms = [1, 7, 12]
    _, Fs = ao.energy_forces(pos, cell, nl.offsets, nl.nbr_j, nl.shift3, RIN, RCUT, spec, W, atoms=atoms)
    assert np.abs(Fs - F[atoms]).max() <= 1e-12 * np.abs(F).max()


def test_defining_sums_equal_the_invariant_expansion():
    """The expansion the device evaluates (Sec. II.E applied to eqs. (22c),
    (22d)): G3 = 2^(1-zeta) sum_n C(zeta, n) lambda^n S_n with
    S_n = sum_jk g_j g_k w_jk^n, and G4 = sum C(a,n1) C(b,n2) C(c,n3)
    alpha^n1 beta^n2 gamma^n3 T(sorted(n1, n2, n3)) with T the symmetric
    four-body sum -- checked here against the defining sums, on the CPU."""
    rng = np.random.default_rng(12)
    d = rng.normal(size=(8, 3))
    d *= (rng.uniform(1.0, 4.8, size=8) / np.linalg.norm(d, axis=1))[:, None]
    r = np.linalg.norm(d, axis=1)
    u = d / r[:, None]
    w = u @ u.T
    fc = po.cutoff(r, RIN, RCUT)[0]
    spec = wl.AcsfSpec(g3=((0.1, 3, -0.7), (0.2, 0, 1.0), (0.05, 6, 1.0)),
                       g4=((0.05, 2, 1, 3, 0.5, -0.3, 0.8), (0.1, 1, 1, 1, 1.0, 1.0, 1.0)))
    G = _env(d, spec)

    def S(eta, n):
        g = np.exp(-eta * r * r) * fc
        return float(np.einsum("jk,j,k->", w ** n, g, g))

    def T(eta, n1, n2, n3):
        g = np.exp(-eta * r * r) * fc
        return float(np.einsum("jk,jl,kl,j,k,l->", w ** n1, w ** n2, w ** n3, g, g, g))

    want = []
    for eta, z, lam in spec.g3:
        want.append(sum(2.0 ** (1 - z) * math.comb(z, n) * lam ** n * S(eta, n) for n in range(z + 1)))
    for eta, a, b, c, al, be, ga in spec.g4:
        v = 0.0
        for n1 in range(a + 1):
            for n2 in range(b + 1):
                for n3 in range(c + 1):
                    wgt = math.comb(a, n1) * al ** n1 * math.comb(b, n2) * be ** n2 * math.comb(c, n3) * ga ** n3
                    v += wgt * T(eta, *sorted((n1, n2, n3), reverse=True))
        want.append(v)
    assert np.abs(G - np.array(want)).max() <= 1e-12 * np.abs(G).max()
