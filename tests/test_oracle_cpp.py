"""The compiled FP64 oracle (oracle/oracle.cpp) against the NumPy oracle: the
same energies, global descriptors, forces and virial to 1e-12 on periodic
boxes (2/3-body and 2/3/4-body, angular degree up to 5), an open cluster,
a general snapshot family and a cell smaller than the cut-off (self-images),
for one and several threads; and the domain check."""
import numpy as np
import pytest

from oracle import oracle_c, pod_oracle as po
from paper_2212_14446_amd import workloads as wl


def _compare(pos, cell, off, nj, sh, p, Q, c, threads=(1, 3)):
    ref = po.energy_forces(pos, cell, off, nj, sh, p, Q, c)
    for th in threads:
        got = oracle_c.energy_forces(pos, cell, off, nj, sh, p, Q, c, threads=th)
        assert got["E"] == pytest.approx(ref["E"], rel=1e-12)
        for k in ("E_atom", "G", "F", "W"):
            den = max(np.abs(ref[k]).max(), 1e-300)
            assert np.abs(got[k] - ref[k]).max() < 1e-12 * den, (k, th)


@pytest.mark.parametrize("K2,K3,K4,P3,P4", [(4, 4, 0, 3, 0), (4, 4, 4, 3, 3), (3, 2, 3, 2, 5), (2, 0, 2, 0, 4)])
def test_periodic_boxes(K2, K3, K4, P3, P4):
    p = po.make_params(0.5, 5.0, 8, K2, K3, K4, P3, P4)
    Q, _ = po.pod_basis(p)
    pos, cell = wl.bcc(2)
    pos = wl.displace(pos, 0.15, 41)
    off, nj, sh = po.neighbors_bruteforce(pos, cell, p.rcut)
    c = np.random.default_rng(42).normal(size=po.num_descriptors(p)[0])
    _compare(pos, cell, off, nj, sh, p, Q, c)


def test_open_cluster_and_isolated_atom():
    p = po.make_params(0.5, 5.0, 8, 3, 3, 3, 4, 4)
    Q, _ = po.pod_basis(p)
    rng = np.random.default_rng(5)
    pos, _ = wl.lattice("bcc", 2, 2, 1, 3.31)
    pos = pos + rng.normal(0, 0.2, pos.shape)
    pos = np.vstack([pos, [[40.0, 40.0, 40.0]]])     # an atom with no neighbours
    off, nj, sh = po.neighbors_bruteforce(pos, None, p.rcut)
    c = rng.normal(size=po.num_descriptors(p)[0])
    _compare(pos, None, off, nj, sh, p, Q, c)


def test_general_snapshot_family_and_small_cell():
    # non-integer gamma, mixed kappa, two betas; a sheared cell thinner than
    # the cut-off, so an atom sees several images of itself
    alpha = np.array([1.0, 2.5, 3.0, 0.0, 1.5])
    beta = np.array([3.0, 3.0, 0.0, 0.0, 1.0])
    gamma = np.array([0.0, 0.0, 0.0, 1.7, 2.0])
    kappa = np.array([1.0, 1.0, 1.0, 0.0, 0.4])
    p = po.PodParams(0.5, 4.5, alpha, beta, gamma, kappa, 3, 3, 2, 3, 2)
    Q, _ = po.pod_basis(p)
    cell = np.array([[3.4, 0.0, 0.0], [0.9, 3.2, 0.0], [0.4, 0.6, 3.6]])
    rng = np.random.default_rng(3)
    pos = rng.uniform(0, 1, (3, 3)) @ cell
    off, nj, sh = po.neighbors_bruteforce(pos, cell, p.rcut)
    assert np.any(nj == np.repeat(np.arange(3), np.diff(off)))   # self-images present
    c = rng.normal(size=po.num_descriptors(p)[0])
    _compare(pos, cell, off, nj, sh, p, Q, c)


def test_pair_outside_domain_is_refused():
    p = po.make_params(0.5, 5.0, 6, 2, 2, 0, 2, 0)
    Q, _ = po.pod_basis(p)
    pos = np.array([[0.0, 0.0, 0.0], [0.3, 0.0, 0.0]])   # r = 0.3 <= rin
    off = np.array([0, 1, 2])
    nj = np.array([1, 0])
    sh = np.zeros((2, 3), dtype=int)
    c = np.ones(po.num_descriptors(p)[0])
    with pytest.raises(ValueError):
        oracle_c.energy_forces(pos, None, off, nj, sh, p, Q, c)
