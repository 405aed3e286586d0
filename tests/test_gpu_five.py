"""Five-body descriptors on the device (pod_five_body_descriptors) against the
five-body oracle, which evaluates the defining quadruple sums with the POD
oracle's radial basis (the same Q is passed to the library).

Energies and forces of c5 . D5 against the oracle's autograd of the same
sums.  FP64 at 1e-10 normwise per descriptor column and per array.  FP32: products of four basis
values summed with multinomial weights, where the columns with odd exponents
cancel between terms; measured 6e-6 normwise per column, checked at the FP32
energy bar of the POD path, 2e-5."""
import numpy as np
import pytest
import torch

from gpu_common import colerr, oracle_params, relerr, say
from oracle import five_oracle as fo
from oracle import pod_oracle as po
from paper_2212_14446_amd import pod, workloads as wl

pytestmark = pytest.mark.gpu

S = wl.PodSetup(0.5, 5.0, 6, 3, 3, 3, 2, 2)


def _model(s=S, dtype="f64"):
    p = oracle_params(s)
    Q, _ = po.pod_basis(p)
    K = max(s.K2, s.K3, s.K4)
    return pod.PodModel(pod.setup_from_workload(s), dtype, Q=Q[:, :K]), p, Q


def _oracle(pos, cell, nl, p, Q, K5, P5, atoms=None):
    return fo.descriptors5(pos, cell, nl.offsets, nl.nbr_j, nl.shift3, p, Q, K5, P5, atoms)


@pytest.mark.parametrize("n,K5,P5", [(2, 3, 4), (3, 2, 3), (2, 1, 0), (2, 3, 1)])
def test_descriptors_match_oracle(n, K5, P5):
    pos, cell = wl.bcc(n)
    pos = wl.displace(pos, 0.12, 40 + n)
    nl = wl.neighbor_list(pos, cell, S.rcut)
    say(f"[gpu] five-body N={pos.shape[0]} K5={K5} P5={P5}")
    m, p, Q = _model()
    D = m.five_body_descriptors(pos, cell, pod.DeviceNeighbors.from_list(nl), K5, P5).cpu().numpy()
    assert D.shape == (pos.shape[0], K5 * pod.pod_five_body_count(P5))
    assert colerr(D, _oracle(pos, cell, nl, p, Q, K5, P5)) <= 1e-10


def test_liquid_several_tiles_sampled():
    box = (300 * wl.V_ATOM) ** (1.0 / 3.0)
    pos, cell = wl.random_liquid(300, box, 2.2, 12)     # 64-atom tiles: four full, one ragged
    nl = wl.neighbor_list(pos, cell, S.rcut)
    m, p, Q = _model()
    D = m.five_body_descriptors(pos, cell, pod.DeviceNeighbors.from_list(nl), 3, 2).cpu().numpy()
    atoms = np.r_[0:8, 250:256, 292:300, np.random.default_rng(4).choice(300, 12, replace=False)]
    assert colerr(D[atoms], _oracle(pos, cell, nl, p, Q, 3, 2, atoms)) <= 1e-10


def test_fp32_follows_oracle():
    pos, cell = wl.bcc(2)
    pos = wl.displace(pos, 0.12, 42)
    nl = wl.neighbor_list(pos, cell, S.rcut)
    m, p, Q = _model(dtype="f32")
    D = m.five_body_descriptors(pos, cell, pod.DeviceNeighbors.from_list(nl), 3, 4).double().cpu().numpy()
    e = colerr(D, _oracle(pos.astype(np.float32).astype(np.float64), cell, nl, p, Q, 3, 4))
    say(f"[gpu] five-body fp32 colerr {e:.2e}")
    assert e <= 2e-5


def test_open_cluster_isolated_atom_and_skin_list():
    rng = np.random.default_rng(5)
    pos, _ = wl.lattice("bcc", 2, 2, 1, 3.31)
    pos = np.vstack([pos + rng.normal(0, 0.1, pos.shape), [[40.0, 40.0, 40.0]]])
    nl = wl.neighbor_list(pos, None, S.rcut)
    skin = wl.neighbor_list(pos, None, S.rcut + 0.6)
    assert skin.n_pairs > nl.n_pairs
    m, p, Q = _model()
    D = m.five_body_descriptors(pos, None, pod.DeviceNeighbors.from_list(nl), 3, 3).cpu().numpy()
    Ds = m.five_body_descriptors(pos, None, pod.DeviceNeighbors.from_list(skin), 3, 3).cpu().numpy()
    ref = _oracle(pos, None, nl, p, Q, 3, 3)
    assert colerr(D, ref) <= 1e-10 and colerr(Ds, ref) <= 1e-10
    assert np.all(D[-1] == 0.0)


def test_arguments_and_data_errors():
    m, p, Q = _model()
    pos, cell = wl.bcc(2)
    nl = wl.neighbor_list(pos, cell, S.rcut)
    nb = pod.DeviceNeighbors.from_list(nl)
    x = m._pos(pos)
    D = torch.empty((nb.N, 4 * 22), dtype=torch.float64, device="cuda")
    for K5, P5, code in ((4, 2, "POD_EINVAL"), (0, 2, "POD_EINVAL"), (2, 5, "POD_ENOTSUP"), (2, -1, "POD_EINVAL")):
        with pytest.raises(pod.PodError) as e:
            pod.pod_five_body_descriptors(m.h, nb.N, nb.P, x, cell, nb.offsets, nb.nbr_j, nb.shift, K5, P5, D)
        assert pod.ERRORS[e.value.code] == code
    z = torch.zeros(0, dtype=torch.float64, device="cuda")
    zi = torch.zeros(1, dtype=torch.int32, device="cuda")
    pod.pod_five_body_descriptors(m.h, 0, 0, z, None, zi, None, None, 2, 2, z)
    pod.pod_check(m.h)
    close = pos.copy()
    close[1] = close[0] + np.array([0.0, 0.4, 0.0])      # inside rin
    nl2 = wl.neighbor_list(close, cell, S.rcut)
    with pytest.raises(pod.PodError) as e:
        m.five_body_descriptors(close, cell, pod.DeviceNeighbors.from_list(nl2), 2, 2)
    assert pod.ERRORS[e.value.code] == "POD_ERANGE"


def test_bcc_15840_sampled():
    """The 15,840-atom box with its own radial basis (K = 6), P5 = 4: sampled
    atoms against the oracle."""
    w = wl.config2()
    m, p, Q = _model(w.setup)
    D = m.five_body_descriptors(w.pos, w.cell, pod.DeviceNeighbors.from_list(w.nl), 6, 4).cpu().numpy()
    assert D.shape == (w.N, 6 * 22) and np.all(np.isfinite(D))
    atoms = np.sort(np.random.default_rng(8).choice(w.N, 5, replace=False))
    assert colerr(D[atoms], _oracle(w.pos, w.cell, w.nl, p, Q, 6, 4, atoms)) <= 1e-10


def _c5(K5, P5, seed):
    return np.random.default_rng(seed).normal(size=(K5, pod.pod_five_body_count(P5)))


@pytest.mark.parametrize("n,K5,P5", [(2, 2, 4), (3, 3, 2), (2, 3, 0), (2, 1, 3)])
def test_energy_forces_match_oracle(n, K5, P5):
    pos, cell = wl.bcc(n)
    pos = wl.displace(pos, 0.12, 50 + n)
    nl = wl.neighbor_list(pos, cell, S.rcut)
    say(f"[gpu] five-body energy/forces N={pos.shape[0]} K5={K5} P5={P5}")
    m, p, Q = _model()
    c5 = _c5(K5, P5, 7)
    o = m.five_body_energy_forces(pos, cell, pod.DeviceNeighbors.from_list(nl), K5, P5, c5)
    E_ref, F_ref = fo.energy_forces5(pos, cell, nl.offsets, nl.nbr_j, nl.shift3, p, Q, K5, P5, c5)
    assert relerr(o["E_atom"].cpu().numpy(), E_ref) <= 1e-10
    assert relerr(o["F"].cpu().numpy(), F_ref) <= 1e-10


def test_energy_forces_fp32_reproducible_and_skin():
    pos, cell = wl.bcc(2)
    pos = wl.displace(pos, 0.12, 61)
    nl = wl.neighbor_list(pos, cell, S.rcut)
    skin = wl.neighbor_list(pos, cell, S.rcut + 0.5)
    c5 = _c5(2, 4, 8)
    m32, p, Q = _model(dtype="f32")
    nb = pod.DeviceNeighbors.from_list(skin)
    a = m32.five_body_energy_forces(pos, cell, nb, 2, 4, c5)
    b = m32.five_body_energy_forces(pos, cell, nb, 2, 4, c5)
    assert torch.equal(a["F"], b["F"]) and torch.equal(a["E_atom"], b["E_atom"])   # no atomics
    E_ref, F_ref = fo.energy_forces5(pos.astype(np.float32).astype(np.float64), cell, nl.offsets, nl.nbr_j,
                                     nl.shift3, p, Q, 2, 4, c5.astype(np.float32).astype(np.float64))
    eE = relerr(a["E_atom"].double().cpu().numpy(), E_ref)
    eF = relerr(a["F"].double().cpu().numpy(), F_ref)
    say(f"[gpu] five-body fp32 energy {eE:.2e} forces {eF:.2e}")
    assert eE <= 2e-5 and eF <= 1e-4
    F = a["F"].double().cpu().numpy()
    assert np.abs(F.sum(0)).max() <= 1e-5 * np.abs(F).max() * pos.shape[0]


def test_energy_forces_arguments():
    m, p, Q = _model()
    pos, cell = wl.bcc(2)
    nl = wl.neighbor_list(pos, cell, S.rcut)
    nb = pod.DeviceNeighbors.from_list(nl)
    nb.build_reverse(m)
    x = m._pos(pos)
    c5 = torch.ones(2 * 5, dtype=torch.float64, device="cuda")
    E = torch.empty(nb.N, dtype=torch.float64, device="cuda")
    F = torch.empty((nb.N, 3), dtype=torch.float64, device="cuda")
    args = (m.h, nb.N, nb.P, x, cell, nb.offsets, nb.nbr_j, nb.shift)
    for rev, c, e, f in ((None, c5, E, F), (nb.rev, None, E, F), (nb.rev, c5, None, None)):
        with pytest.raises(pod.PodError) as err:
            pod.pod_five_body_energy_forces(*args, rev, 2, 2, c, e, f)
        assert pod.ERRORS[err.value.code] == "POD_EINVAL"
    pod.pod_five_body_energy_forces(*args, None, 2, 2, c5, E, None)    # energies alone need no reverse index
    m.check()
    D = m.five_body_descriptors(pos, cell, nb, 2, 2).cpu().numpy()
    assert relerr(E.cpu().numpy(), D @ c5.cpu().numpy()) <= 1e-12


def test_energy_forces_open_cluster_with_isolated_atom():
    rng = np.random.default_rng(9)
    pos, _ = wl.lattice("bcc", 2, 1, 1, 3.31)
    pos = np.vstack([pos + rng.normal(0, 0.1, pos.shape), [[30.0, 30.0, 30.0]]])
    nl = wl.neighbor_list(pos, None, S.rcut)
    m, p, Q = _model()
    c5 = _c5(3, 3, 4)
    o = m.five_body_energy_forces(pos, None, pod.DeviceNeighbors.from_list(nl), 3, 3, c5)
    E_ref, F_ref = fo.energy_forces5(pos, None, nl.offsets, nl.nbr_j, nl.shift3, p, Q, 3, 3, c5)
    assert relerr(o["E_atom"].cpu().numpy(), E_ref) <= 1e-10
    assert relerr(o["F"].cpu().numpy(), F_ref) <= 1e-10
    assert o["E_atom"][-1].item() == 0.0 and torch.count_nonzero(o["F"][-1]).item() == 0
