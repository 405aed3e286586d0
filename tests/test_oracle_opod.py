"""Pins of the exclusive-sum oracle (eqs. (15b), (19a), (20a), Table 2).

Table 2 is a golden fixture; eq. (15c) ties the exclusive 3-body
descriptors to the full ones of the fast oracle (an independent route); the
paper's statement that two neighbours give no exclusive 4-body descriptor,
a three-neighbour closed form from the printed Table 2 terms, a brute force
over ordered distinct triples for the fully symmetric g_p, permutation
invariance, and central differences of the energy pin the rest."""
import itertools
import os

import numpy as np
import pytest

from oracle import opod_oracle as oo
from oracle import pod_oracle as po
from paper_2212_14446_amd import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _table2():
    rows = {}
    with open(os.path.join(GOLD, "table2_symmetric_angular.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p, terms = line.split(":")
            rows[int(p)] = [tuple(int(x) for x in t.split()) for t in terms.split(";")]
    return rows


def _table1():
    rows = {}
    with open(os.path.join(GOLD, "table1_four_body.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p, a, b, c = (int(x) for x in line.split())
            rows[p] = (a, b, c)
    return rows


def _env(rng, n, K):
    U = rng.normal(size=(n, 3))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    return rng.normal(size=(n, K)), U


def _params(K2, K3, K4, P3, P4):
    return po.make_params(0.5, 5.0, 8, K2, K3, K4, P3, P4)


def test_table2_terms():
    t1, t2 = _table1(), _table2()
    assert sorted(t2) == list(range(1, 12))
    for p in range(1, 12):
        assert set(oo.symmetric_terms(*t1[p])) == set(t2[p]), p
        assert len(oo.symmetric_terms(*t1[p])) == len(t2[p])


def test_eq15c_against_the_full_sums():
    rng = np.random.default_rng(1)
    p = _params(3, 4, 0, 4, 0)
    M2 = 1 + p.K2
    for n in (1, 2, 6, 11):
        Rn, U = _env(rng, n, p.K)
        full = po.descriptors_naive_env(Rn, U, p)[M2:].reshape(p.K3, p.P3 + 1)
        excl = oo.descriptors_env(Rn, U, p)[M2:].reshape(p.K3, p.P3 + 1)
        two = (Rn[:, :p.K3] ** 2).sum(0)
        assert np.allclose(full, 2 * excl + two[:, None], rtol=1e-12, atol=1e-12 * np.abs(full).max())


def test_two_neighbours_give_no_four_body():
    rng = np.random.default_rng(2)
    p = _params(1, 1, 3, 1, 4)
    M = po.num_descriptors(p)[0]
    for n in (0, 1, 2):
        Rn, U = _env(rng, n, p.K)
        D = oo.descriptors_env(Rn, U, p)
        assert np.all(D[M - p.K4 * po.n_four_body(p.P4):] == 0.0)


def test_three_neighbours_closed_form():
    rng = np.random.default_rng(3)
    p = _params(1, 1, 2, 1, 4)
    t1, t2 = _table1(), _table2()
    Rn, U = _env(rng, 3, p.K)
    D = oo.descriptors_env(Rn, U, p)
    w12, w13, w23 = U[0] @ U[1], U[0] @ U[2], U[1] @ U[2]
    base = 1 + p.K2 + p.K3 * (p.P3 + 1)
    for m in range(p.K4):
        for q in range(1, 12):
            g = sum(w12 ** a * w13 ** b * w23 ** c for (a, b, c) in t2[q])
            want = Rn[0, m] * Rn[1, m] * Rn[2, m] * g
            got = D[base + m * 11 + (q - 1)]
            assert abs(got - want) <= 1e-13 * max(1.0, abs(want)), (m, q)
    assert [t1[q] for q in range(1, 12)] == po.four_body_triples(4)


def test_symmetric_gp_against_distinct_ordered_triples():
    """For g_p with a repeated exponent, every ordering of a triple is one of
    its terms: sum over ordered distinct (j, k, l) of f_p = (6 / #terms) D4."""
    rng = np.random.default_rng(4)
    p = _params(1, 1, 2, 1, 4)
    base = 1 + p.K2 + p.K3 * (p.P3 + 1)
    Rn, U = _env(rng, 6, p.K)
    W = U @ U.T
    D = oo.descriptors_env(Rn, U, p)
    for m in range(p.K4):
        for q, (a, b, c) in enumerate(po.four_body_triples(4)):
            if len({a, b, c}) == 3:
                continue
            s = 0.0
            for j, k, l in itertools.permutations(range(6), 3):
                s += Rn[j, m] * Rn[k, m] * Rn[l, m] * W[j, k] ** a * W[j, l] ** b * W[k, l] ** c
            nterms = len(oo.symmetric_terms(a, b, c))
            assert abs(s - 6 / nterms * D[base + m * 11 + q]) <= 1e-12 * max(1.0, abs(s)), (a, b, c)


def test_permutation_invariance():
    rng = np.random.default_rng(5)
    p = _params(2, 3, 2, 3, 4)
    Rn, U = _env(rng, 7, p.K)
    D = oo.descriptors_env(Rn, U, p)
    perm = rng.permutation(7)
    Dp = oo.descriptors_env(Rn[perm], U[perm], p)
    base = 1 + p.K2 + p.K3 * (p.P3 + 1)
    trip = po.four_body_triples(4)
    sym = np.ones(D.size, dtype=bool)
    for m in range(p.K4):
        for q, abc in enumerate(trip):
            sym[base + m * len(trip) + q] = len(set(abc)) < 3
    assert np.allclose(D[sym], Dp[sym], rtol=1e-12, atol=1e-12)
    # the cyclic-only g_p (three distinct exponents) follow the list order
    assert not np.allclose(D[~sym], Dp[~sym], rtol=1e-6)


def _small(seed, n=2):
    s = wl.PodSetup(0.5, 5.0, 8, 3, 4, 0, 3, 0)
    w = wl.small_bcc(n, sigma=0.15, seed=seed, setup=s)
    p = po.PodParams(s.rin, s.rcut, *s.snapshot_family(), s.K2, s.K3, s.K4, s.P3, s.P4)
    Q, _ = po.pod_basis(p)
    return w, p, Q


def test_energy_matches_descriptors_and_differences():
    w, p, Q = _small(21)
    c = wl.coefficients(po.num_descriptors(p)[0], 4)
    args = (w.pos, w.cell, w.nl.offsets.astype(np.int64), w.nl.nbr_j, w.nl.shift3, p, Q)
    out = oo.energy_forces(*args, c)
    D = oo.descriptors(*args)
    assert np.allclose(out["E_atom"], D @ c, rtol=1e-12, atol=1e-12 * np.abs(D @ c).max())
    assert np.abs(out["F"].sum(0)).max() <= 1e-10 * np.abs(out["F"]).max()
    h = 1e-5
    for a in (0, 5):
        for d in range(3):
            pp, pm = w.pos.copy(), w.pos.copy()
            pp[a, d] += h
            pm[a, d] -= h
            fd = -(oo.total_energy(pp, *args[1:], c) - oo.total_energy(pm, *args[1:], c)) / (2 * h)
            assert abs(fd - out["F"][a, d]) <= 1e-6 * max(1.0, np.abs(out["F"]).max()), (a, d)


def test_virial_against_strain_differences():
    w, p, Q = _small(22)
    c = wl.coefficients(po.num_descriptors(p)[0], 5)
    nl = w.nl
    args = (nl.offsets.astype(np.int64), nl.nbr_j, nl.shift3, p, Q)
    W = oo.energy_forces(w.pos, w.cell, *args, c)["W"]
    h = 1e-6
    for a, b in ((0, 0), (0, 1), (2, 1)):
        eps = np.zeros((3, 3))
        eps[a, b] = eps[b, a] = h / 2 if a != b else h
        Ep = oo.total_energy(w.pos @ (np.eye(3) + eps).T, w.cell @ (np.eye(3) + eps).T, *args, c)
        Em = oo.total_energy(w.pos @ (np.eye(3) - eps).T, w.cell @ (np.eye(3) - eps).T, *args, c)
        dEde = (Ep - Em) / (2 * h)
        sym = (W[a, b] + W[b, a]) / 2 if a != b else W[a, a]
        assert abs(-dEde - sym) <= 1e-6 * max(1.0, np.abs(W).max()), (a, b)
