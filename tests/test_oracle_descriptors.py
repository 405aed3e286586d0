"""Oracle descriptors: naive sums (eqs. (12b), (15), (18a)) against the fast
atom-density form (eqs. (25)-(30a)), closed forms, the identities (15c) and
(27a), and invariance under the symmetries of Sec. I."""
import numpy as np
import pytest

from oracle import pod_oracle as po
from paper_2212_14446_amd import workloads as wl


def rand_params(K2, K3, K4, P3, P4, L=8):
    return po.make_params(0.5, 5.0, L, K2, K3, K4, P3, P4)


def rand_env(rng, n):
    U = rng.normal(size=(n, 3))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    return U


def fast_env(Rn, U, p):
    A = po.monomials(U, p.PA)
    B = (Rn[:, :, None] * A[:, None, :]).sum(0)[None]
    return po.fast_descriptors_from_B(B, p)[0]


@pytest.mark.parametrize("P3,P4", [(0, 0), (1, 1), (2, 3), (3, 2), (4, 4), (2, 5)])
def test_naive_equals_fast_random_radial(P3, P4):
    # eqs. (26a) and (30a) are identities: any radial values and directions
    rng = np.random.default_rng(100 + 10 * P3 + P4)
    p = rand_params(3, 3, 3, P3, P4)
    for n in (1, 2, 5, 7):
        Rn = rng.normal(size=(n, p.K))
        U = rand_env(rng, n)
        dn = po.descriptors_naive_env(Rn, U, p)
        df = fast_env(Rn, U, p)
        assert np.allclose(dn, df, rtol=1e-11, atol=1e-11 * np.max(np.abs(dn)))


def test_one_neighbor_closed_form():
    rng = np.random.default_rng(3)
    p = rand_params(4, 4, 4, 4, 4)
    Rn = rng.normal(size=(1, p.K))
    U = rand_env(rng, 1)
    D = fast_env(Rn, U, p)
    M, (m1, m2, m3, m4) = po.num_descriptors(p)
    R = Rn[0]
    assert D[0] == 1.0
    assert np.allclose(D[1:1 + m2], R[:4])
    assert np.allclose(D[1 + m2:1 + m2 + m3].reshape(4, 5), (R[:4] ** 2)[:, None])
    assert np.allclose(D[1 + m2 + m3:].reshape(4, -1), (R[:4] ** 3)[:, None])


def test_two_neighbor_closed_form():
    rng = np.random.default_rng(4)
    p = rand_params(2, 2, 2, 4, 4)
    Rn = rng.normal(size=(2, p.K))
    U = rand_env(rng, 2)
    cos = U[0] @ U[1]
    D = fast_env(Rn, U, p)
    M, (m1, m2, m3, m4) = po.num_descriptors(p)
    D3 = D[1 + m2:1 + m2 + m3].reshape(2, 5)
    D4 = D[1 + m2 + m3:].reshape(2, -1)
    for m in range(2):
        R1, R2 = Rn[0, m], Rn[1, m]
        for n in range(5):
            assert D3[m, n] == pytest.approx(R1 ** 2 + R2 ** 2 + 2 * R1 * R2 * cos ** n, rel=1e-12)
        for q, (a, b, c) in enumerate(po.four_body_triples(4)):
            want = R1 ** 3 + R2 ** 3 + R1 * R2 * (R1 + R2) * (cos ** (a + b) + cos ** (a + c) + cos ** (b + c))
            assert D4[m, q] == pytest.approx(want, rel=1e-12)
        # exactly two neighbours: the 4-body descriptors do not vanish (Sec. II.D)
        assert np.all(np.abs(D4[m]) > 0)


def test_identities_15c_and_27a_on_naive_sums():
    rng = np.random.default_rng(5)
    p = rand_params(3, 3, 3, 3, 3)
    Rn = rng.normal(size=(6, p.K))
    U = rand_env(rng, 6)
    D = po.descriptors_naive_env(Rn, U, p)
    M, (m1, m2, m3, m4) = po.num_descriptors(p)
    D2 = D[1:1 + m2]
    D3 = D[1 + m2:1 + m2 + m3].reshape(3, 4)
    D4 = D[1 + m2 + m3:].reshape(3, -1)
    excl = po.three_body_exclusive_env(Rn, U, 3, 3)
    for m in range(3):
        # eq. (15c): full = 2 x exclusive + sum_j R_m^2
        assert np.allclose(D3[m], 2 * excl[m] + np.sum(Rn[:, m] ** 2), rtol=1e-12)
        assert D3[m, 0] == pytest.approx(D2[m] ** 2, rel=1e-12)
        for q, (a, b, c) in enumerate(po.four_body_triples(3)):
            if b == 0 and c == 0:                         # eq. (27a)
                assert D4[m, q] == pytest.approx(D2[m] * D3[m, a], rel=1e-11)
        assert D4[m, 0] == pytest.approx(D2[m] ** 3, rel=1e-12)


def _small_system(n=2, sigma=0.15, seed=21, rcut=5.0):
    pos, cell = wl.bcc(n)
    pos = wl.displace(pos, sigma, seed)
    return pos, cell


def test_generator_neighbor_list_matches_bruteforce():
    p = rand_params(2, 2, 0, 2, 0)
    for n, rc in ((2, 5.0), (1, 4.0), (3, 5.0)):
        pos, cell = _small_system(n)
        off, nj, sh = po.neighbors_bruteforce(pos, cell, rc)
        nl = wl.neighbor_list(pos, cell, rc)
        assert np.array_equal(np.asarray(nl.offsets), off)
        assert np.array_equal(np.asarray(nl.nbr_j), nj)
        assert np.array_equal(np.asarray(nl.shift3), sh)


def test_full_pipeline_naive_equals_fast():
    p = rand_params(4, 4, 4, 3, 3)
    pos, cell = _small_system(2)
    off, nj, sh = po.neighbors_bruteforce(pos, cell, p.rcut)
    Q, _ = po.pod_basis(p)
    atoms = [0, 5, 11]
    Dn = po.descriptors_naive(pos, cell, off, nj, sh, p, Q, atoms)
    Df = po.descriptors_fast(pos, cell, off, nj, sh, p, Q, atoms)
    assert np.allclose(Dn, Df, rtol=1e-11, atol=1e-11 * np.abs(Dn).max())


def _descr(pos, cell, p, Q):
    off, nj, sh = po.neighbors_bruteforce(pos, cell, p.rcut)
    return po.descriptors_fast(pos, cell, off, nj, sh, p, Q)


def test_invariances():
    rng = np.random.default_rng(9)
    p = rand_params(3, 3, 3, 4, 4)
    Q, _ = po.pod_basis(p)
    pos, cell = _small_system(2, seed=31)
    D0 = _descr(pos, cell, p, Q)
    tol = dict(rtol=1e-10, atol=1e-10 * np.abs(D0).max())
    # rotation (+ reflection): rotate positions and lattice vectors together
    Rm, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    for Rot in (Rm, -Rm):
        assert np.allclose(_descr(pos @ Rot.T, cell @ Rot.T, p, Q), D0, **tol)
    # translation
    assert np.allclose(_descr(pos + np.array([0.3, -1.7, 2.2]), cell, p, Q), D0, **tol)
    # permutation of atom labels
    perm = rng.permutation(pos.shape[0])
    assert np.allclose(_descr(pos[perm], cell, p, Q), D0[perm], **tol)
    # permutation of the neighbour order inside each atom's list
    off, nj, sh = po.neighbors_bruteforce(pos, cell, p.rcut)
    nj2, sh2 = nj.copy(), sh.copy()
    for a in range(pos.shape[0]):
        s, e = off[a], off[a + 1]
        q = s + rng.permutation(e - s)
        nj2[s:e], sh2[s:e] = nj[q], sh[q]
    assert np.allclose(po.descriptors_fast(pos, cell, off, nj2, sh2, p, Q), D0, **tol)


def test_perfect_bcc_inversion_symmetry_and_extensivity():
    p = rand_params(3, 3, 3, 4, 4)
    Q, _ = po.pod_basis(p)
    c = np.random.default_rng(2).normal(size=po.num_descriptors(p)[0])
    Es = []
    for n in (2, 3):
        pos, cell = wl.bcc(n)
        D = _descr(pos, cell, p, Q)
        # every site is equivalent
        assert np.allclose(D, D[0], rtol=1e-11, atol=1e-11 * np.abs(D).max())
        # inversion centre: odd-degree 3-body descriptors vanish
        M, (m1, m2, m3, m4) = po.num_descriptors(p)
        D3 = D[0, 1 + m2:1 + m2 + m3].reshape(3, 5)
        assert np.all(np.abs(D3[:, 1::2]) < 1e-10 * np.abs(D3).max())
        Es.append((D @ c).sum() / pos.shape[0])
    assert Es[0] == pytest.approx(Es[1], rel=1e-11)
