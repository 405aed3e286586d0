"""Pins of the five-body oracle.

The orbit count against Burnside's lemma; the invariance that defines the
orbits; the exponent tuples whose angle graph splits or leaves a neighbour
free, which reduce the quadruple sum to products of the POD oracle's own two-,
three- and four-body descriptors (eqs. (12b), (15), (18a)); and geometric
closed forms for environments with cosines 0 and -1; the energy c5 . D5 and
its forces against central finite differences; and the atomic-basis
expansion the device uses against the defining sums."""
import itertools
import math

import numpy as np
import pytest

from oracle import five_oracle as fo
from oracle import pod_oracle as po
from paper_2212_14446_amd import workloads as wl


def _burnside(P5):
    """Orbits of tuples with |e| <= P5: the mean over the 24 relabellings of
    the tuples each one fixes (constant on the relabelling's cycles of
    angle positions)."""
    total = 0
    for perm in itertools.permutations(range(4)):
        # cycles of the induced permutation of the six positions
        img = [fo.EDGES.index(tuple(sorted((perm[a], perm[b])))) for (a, b) in fo.EDGES]
        seen, lens = set(), []
        for s in range(6):
            if s in seen:
                continue
            L, t = 0, s
            while t not in seen:
                seen.add(t)
                t = img[t]
                L += 1
            lens.append(L)
        # fixed tuples: one value per cycle, sum of value * cycle length <= P5
        cnt = 0
        for vals in itertools.product(range(P5 + 1), repeat=len(lens)):
            if sum(v * L for v, L in zip(vals, lens)) <= P5:
                cnt += 1
        total += cnt
    assert total % 24 == 0
    return total // 24


@pytest.mark.parametrize("P5", range(0, 5))
def test_orbit_count_matches_burnside(P5):
    reps = fo.orbits(P5)
    assert len(reps) == _burnside(P5)
    assert len(set(reps)) == len(reps)
    assert [sum(e) for e in reps] == sorted(sum(e) for e in reps)


def test_orbit_counts_per_degree():
    # loopless multigraphs on four unlabelled vertices with n edges: 1, 1, 3, 6, 11
    counts = [len(fo.orbits(n)) - (len(fo.orbits(n - 1)) if n else 0) for n in range(5)]
    assert counts == [1, 1, 3, 6, 11]


def _env(n=9, seed=2):
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n, 3))
    r = rng.uniform(1.2, 4.8, size=n)
    d *= (r / np.linalg.norm(d, axis=1))[:, None]
    return d, r


def _pod_params(K=3, P=4):
    s = wl.PodSetup(0.5, 5.0, 6, K, K, K, P, P)
    p = po.PodParams(s.rin, s.rcut, *s.snapshot_family(), s.K2, s.K3, s.K4, s.P3, s.P4)
    Q, _ = po.pod_basis(p)
    return p, Q


def test_tuples_in_one_orbit_give_equal_sums():
    d, r = _env()
    p, Q = _pod_params()
    R = po.radial_basis(r, p, Q)[0][:, 1]
    U = d / r[:, None]
    W = U @ U.T
    for e in [(2, 1, 0, 0, 1, 0), (1, 1, 1, 1, 0, 0), (3, 0, 0, 0, 0, 1)]:
        vals = [fo.five_body_sum(R, W, f) for f in fo.orbit(e)]
        assert np.ptp(vals) <= 1e-12 * np.abs(vals).max()


def test_reducible_tuples_equal_products_of_lower_orders():
    d, r = _env(8, 5)
    p, Q = _pod_params()
    Rn = po.radial_basis(r, p, Q)[0]
    U = d / r[:, None]
    W = U @ U.T
    D = po.descriptors_naive_env(Rn, U, p)
    K = p.K2
    trip = po.four_body_triples(p.P4)

    def d2(m):
        return D[1 + m]

    def d3(m, n):
        return D[1 + K + m * (p.P3 + 1) + n]

    def d4(m, abc):
        return D[1 + K + K * (p.P3 + 1) + m * len(trip) + trip.index(tuple(sorted(abc, reverse=True)))]

    for m in range(K):
        R = Rn[:, m]
        f = lambda e: fo.five_body_sum(R, W, e)
        assert np.isclose(f((0,) * 6), d2(m) ** 4, rtol=1e-12)
        for a in range(1, 4):
            assert np.isclose(f((a, 0, 0, 0, 0, 0)), d3(m, a) * d2(m) ** 2, rtol=1e-12)
        for a, b in [(1, 1), (2, 1), (1, 3), (2, 2)]:
            # (j,k) and (l,n) disjoint: two independent pair sums
            assert np.isclose(f((a, 0, 0, 0, 0, b)), d3(m, a) * d3(m, b), rtol=1e-12)
            # (j,k) and (j,l) share j, n free: a four-body sum times the radial sum
            assert np.isclose(f((a, b, 0, 0, 0, 0)), d4(m, (a, b, 0)) * d2(m), rtol=1e-12)
        for abc in [(1, 1, 1), (2, 1, 1)]:
            # a triangle on (j, k, l), n free
            assert np.isclose(f((abc[0], abc[1], 0, abc[2], 0, 0)), d4(m, abc) * d2(m), rtol=1e-12)


def test_geometric_closed_forms():
    cycle = (1, 0, 1, 1, 0, 1)        # j-k, k-l, l-n, n-j
    R = np.array([0.7, 1.3])
    # two antiparallel neighbours: every cosine is +-1 and a cycle has an even
    # number of unlike edges, so each of the 16 tuples contributes R^4
    U = np.array([[1.0, 0.0, 0.0], [-1.0, 0.0, 0.0]])
    assert np.isclose(fo.five_body_sum(R, U @ U.T, cycle), R.sum() ** 4, rtol=1e-14)
    # two perpendicular neighbours: only j = k = l = n survives
    U = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    assert np.isclose(fo.five_body_sum(R, U @ U.T, cycle), (R ** 4).sum(), rtol=1e-14)
    # a star on j with exponents 1: sum_j R_j (sum_k R_k u_j.u_k)^3; perpendicular
    # neighbours leave only k = j
    assert np.isclose(fo.five_body_sum(R, U @ U.T, (1, 1, 1, 0, 0, 0)), (R ** 4).sum(), rtol=1e-14)


def test_rotation_and_permutation_invariance():
    d, r = _env(10, 7)
    p, Q = _pod_params()
    Rn = po.radial_basis(r, p, Q)[0]
    rng = np.random.default_rng(1)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    U = d / r[:, None]
    ref = fo.descriptors5_env(Rn, U, 2, 3)
    assert np.abs(fo.descriptors5_env(Rn, U @ q.T, 2, 3) - ref).max() <= 1e-12 * np.abs(ref).max()
    perm = rng.permutation(10)
    assert np.abs(fo.descriptors5_env(Rn[perm], U[perm], 2, 3) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_list_entries_beyond_rcut_are_ignored():
    p, Q = _pod_params()
    d, r = _env(6, 9)
    pos = np.vstack([np.zeros(3), d, [[5.3, 0.0, 0.0]]])
    n = pos.shape[0]
    offsets = np.array([0] + [n - 1] * n)
    got = fo.descriptors5(pos, None, offsets, np.arange(1, n), np.zeros((n - 1, 3), int), p, Q, 2, 2, atoms=[0])
    Rn = po.radial_basis(r, p, Q)[0]
    ref = fo.descriptors5_env(Rn, d / r[:, None], 2, 2)
    assert np.abs(got[0] - ref).max() <= 1e-12 * np.abs(ref).max()
    assert math.isclose(got.shape[1], 2 * 5)


def test_energy_and_forces_of_the_oracle():
    """E_i = c5 . D5_i with D5 from the quadruple sums; forces against
    central finite differences of that energy; sum F = 0."""
    p, Q = _pod_params(K=2, P=2)
    pos, cell = wl.bcc(1)
    pos = wl.displace(pos, 0.15, 3)
    nl = wl.neighbor_list(pos, cell, p.rcut)
    K5, P5 = 2, 3
    n5 = len(fo.orbits(P5))
    c5 = np.random.default_rng(6).normal(size=(K5, n5)) * 1e-3
    E_atom, F = fo.energy_forces5(pos, cell, nl.offsets, nl.nbr_j, nl.shift3, p, Q, K5, P5, c5)
    D = fo.descriptors5(pos, cell, nl.offsets, nl.nbr_j, nl.shift3, p, Q, K5, P5)
    assert np.allclose(E_atom, D @ c5.reshape(-1), rtol=1e-12)
    assert np.abs(F.sum(0)).max() <= 1e-10 * np.abs(F).max()
    h = 1e-5
    for a, e in ((0, 0), (1, 2)):
        xp, xm = pos.copy(), pos.copy()
        xp[a, e] += h
        xm[a, e] -= h
        Ep = (fo.descriptors5(xp, cell, nl.offsets, nl.nbr_j, nl.shift3, p, Q, K5, P5) @ c5.reshape(-1)).sum()
        Em = (fo.descriptors5(xm, cell, nl.offsets, nl.nbr_j, nl.shift3, p, Q, K5, P5) @ c5.reshape(-1)).sum()
        assert abs(F[a, e] + (Ep - Em) / (2 * h)) <= 1e-6 * np.abs(F).max()


def test_quadruple_sums_equal_the_atomic_basis_expansion():
    """The expansion the device evaluates: with B_mu = sum_j R_j u_j^mu,
    D5_e = sum over multi-indices alpha_t (|alpha_t| = e_t) of
    prod_t mult(alpha_t) times B at the monomial of each neighbour slot (the
    sum of the alpha_t of its three angles) -- against the defining sums."""
    d, r = _env(6, 13)
    p, Q = _pod_params()
    R = po.radial_basis(r, p, Q)[0][:, 0]
    U = d / r[:, None]
    W = U @ U.T

    def B(ex):
        return float((R * np.prod(U ** np.asarray(ex), axis=1)).sum())

    def monos(n):
        return [(a, b, n - a - b) for a in range(n + 1) for b in range(n + 1 - a)]

    def mult(al):
        return math.factorial(sum(al)) // (math.factorial(al[0]) * math.factorial(al[1]) * math.factorial(al[2]))

    slots = [[t for t, (a, b) in enumerate(fo.EDGES) if v in (a, b)] for v in range(4)]
    for e in fo.orbits(3) + [(2, 1, 0, 0, 1, 0), (1, 0, 1, 1, 0, 1)]:
        total = 0.0
        for als in itertools.product(*[monos(n) for n in e]):
            wgt = np.prod([mult(al) for al in als])
            prod = 1.0
            for v in range(4):
                ex = tuple(sum(als[t][k] for t in slots[v]) for k in range(3))
                prod *= B(ex)
            total += wgt * prod
        ref = fo.five_body_sum(R, W, e)
        assert abs(total - ref) <= 1e-12 * max(1.0, abs(ref)), e
