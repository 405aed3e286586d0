"""Exclusive-sum descriptors and the 2/3-body exclusive model on the device
(pod_opod_descriptors, pod_opod_energy_forces) against the exclusive-sum
oracle (eqs. (15b), (19a), (20a)), FP64 at 1e-10 normwise per column or
array; forces accumulate with atomics, so only rounding order differs."""
import numpy as np
import pytest

from gpu_common import colerr, oracle_params, relerr, say
from oracle import opod_oracle as oo
from oracle import pod_oracle as po
from paper_2212_14446_amd import pod, workloads as wl

pytestmark = pytest.mark.gpu


def _model(s):
    p = oracle_params(s)
    Q, _ = po.pod_basis(p)
    m = pod.PodModel(pod.setup_from_workload(s), "f64", Q=Q[:, :max(s.K2, s.K3, s.K4)])
    return m, p, Q


def _args(w, p, Q):
    nl = w.nl
    return (w.pos, w.cell, nl.offsets.astype(np.int64), nl.nbr_j, nl.shift3, p, Q)


@pytest.mark.parametrize("setup", [wl.PodSetup(0.5, 5.0, 8, 4, 4, 4, 3, 3), wl.PodSetup(0.5, 5.0, 8, 3, 5, 6, 6, 4),
                                   wl.SETUP_CFG1, wl.PodSetup(0.5, 5.0, 6, 2, 1, 1, 2, 1)])
def test_descriptors_match_oracle(setup):
    w = wl.small_bcc(2, sigma=0.15, seed=31, setup=setup)
    say(f"[gpu] opod descriptors K={setup.K2},{setup.K3},{setup.K4} P={setup.P3},{setup.P4} N={w.N}")
    m, p, Q = _model(setup)
    D = m.opod_descriptors(w.pos, w.cell, pod.DeviceNeighbors.from_list(w.nl)).cpu().numpy()
    ref = oo.descriptors(*_args(w, p, Q), atoms=np.arange(w.N))
    assert colerr(D, ref) <= 1e-10


def test_descriptors_open_cluster_and_isolated_atoms():
    s = wl.PodSetup(0.5, 5.0, 8, 4, 4, 4, 3, 4)
    rng = np.random.default_rng(3)
    pos, _ = wl.lattice("bcc", 2, 2, 1, 3.31)
    pos = pos + rng.normal(0, 0.1, pos.shape)
    pos = np.vstack([pos, [[40.0, 40.0, 40.0]]])
    nl = wl.neighbor_list(pos, None, s.rcut)
    m, p, Q = _model(s)
    D = m.opod_descriptors(pos, None, pod.DeviceNeighbors.from_list(nl)).cpu().numpy()
    ref = oo.descriptors(pos, None, nl.offsets.astype(np.int64), nl.nbr_j, nl.shift3, p, Q)
    assert colerr(D, ref) <= 1e-10
    assert D[-1, 0] == 1.0 and np.all(D[-1, 1:] == 0.0)


@pytest.mark.parametrize("setup", [wl.SETUP_CFG1, wl.PodSetup(0.5, 5.0, 8, 6, 7, 0, 6, 0),
                                   wl.PodSetup(0.5, 5.0, 6, 2, 1, 0, 2, 0)])
def test_energy_forces_match_oracle(setup):
    w = wl.small_bcc(2, sigma=0.15, seed=32, setup=setup)
    say(f"[gpu] opod energy K2={setup.K2} K3={setup.K3} P3={setup.P3} N={w.N}")
    m, p, Q = _model(setup)
    c = wl.coefficients(setup.M, 6)
    o = m.opod_energy_forces(w.pos, w.cell, pod.DeviceNeighbors.from_list(w.nl), c)
    ref = oo.energy_forces(*_args(w, p, Q), c)
    assert relerr(o["E"].item(), ref["E"]) <= 1e-10
    assert relerr(o["E_atom"].cpu().numpy(), ref["E_atom"]) <= 1e-10
    assert relerr(o["F"].cpu().numpy(), ref["F"]) <= 1e-10
    assert relerr(o["W"].cpu().numpy(), ref["W"]) <= 1e-10
    # the exclusive energy is the descriptor row times c
    D = m.opod_descriptors(w.pos, w.cell, pod.DeviceNeighbors.from_list(w.nl)).cpu().numpy()
    assert relerr(o["E_atom"].cpu().numpy(), D @ c) <= 1e-12


def test_cfg2_box_sampled():
    """The 15,840-atom box at the Table 6 size M = 56 (K2 = 6, K3 = 7,
    P3 = 6): sampled atoms against the oracle."""
    s = wl.PodSetup(0.5, 5.0, 8, 6, 7, 0, 6, 0)
    w = wl.config2()
    m, p, Q = _model(s)
    nb = pod.DeviceNeighbors.from_list(w.nl)
    c = wl.coefficients(s.M, 7)
    o = m.opod_energy_forces(w.pos, w.cell, nb, c)
    D = m.opod_descriptors(w.pos, w.cell, nb).cpu().numpy()
    atoms = np.random.default_rng(2).choice(w.N, 24, replace=False)
    ref = oo.descriptors(*_args(w, p, Q), atoms=atoms)
    assert colerr(D[atoms], ref) <= 1e-10
    assert relerr(o["E_atom"].cpu().numpy()[atoms], ref @ c) <= 1e-10
    F = o["F"].cpu().numpy()
    assert np.abs(F.sum(0)).max() <= 1e-9 * np.abs(F).max()


def test_errors():
    m, p, Q = _model(wl.SETUP_CFG2)
    w = wl.small_bcc(2, sigma=0.1, seed=3)
    nb = pod.DeviceNeighbors.from_list(w.nl)
    with pytest.raises(pod.PodError) as e:   # 4-body handle: the exclusive energy model is 2/3-body
        m.opod_energy_forces(w.pos, w.cell, nb, np.zeros(m.M))
    assert pod.ERRORS[e.value.code] == "POD_ENOTSUP"
    m32 = pod.PodModel(pod.setup_from_workload(wl.SETUP_CFG1), "f32")
    with pytest.raises(pod.PodError) as e:
        m32.opod_descriptors(w.pos, w.cell, nb)
    assert pod.ERRORS[e.value.code] == "POD_ENOTSUP"



# The largest sizes of Table 6 (rows 5 and 6: K up to 12, 3-body degree 8
# and 10, 4-body degree 5 and 6, whose g_p of eq. (19a) go beyond Table 2),
# on a 16-atom box, against the exclusive-sum oracle.
@pytest.mark.parametrize("setup", [wl.PodSetup(0.5, 5.0, 14, 10, 9, 9, 8, 5),
                                   wl.PodSetup(0.5, 5.0, 14, 8, 12, 12, 10, 6),
                                   wl.PodSetup(0.5, 5.0, 8, 2, 2, 2, 2, 5)])
def test_descriptors_table6_large_rows(setup):
    w = wl.small_bcc(2, sigma=0.15, seed=33, setup=setup)
    say(f"[gpu] opod descriptors K={setup.K2},{setup.K3},{setup.K4} P={setup.P3},{setup.P4} N={w.N}")
    m, p, Q = _model(setup)
    D = m.opod_descriptors(w.pos, w.cell, pod.DeviceNeighbors.from_list(w.nl)).cpu().numpy()
    ref = oo.descriptors(*_args(w, p, Q), atoms=np.arange(w.N))
    assert colerr(D, ref) <= 1e-10


@pytest.mark.parametrize("setup", [wl.PodSetup(0.5, 5.0, 14, 10, 9, 0, 8, 0),
                                   wl.PodSetup(0.5, 5.0, 14, 8, 12, 0, 10, 0)])
def test_energy_forces_table6_large_rows(setup):
    w = wl.small_bcc(2, sigma=0.15, seed=34, setup=setup)
    say(f"[gpu] opod energy K2={setup.K2} K3={setup.K3} P3={setup.P3} N={w.N}")
    m, p, Q = _model(setup)
    c = wl.coefficients(setup.M, 8)
    o = m.opod_energy_forces(w.pos, w.cell, pod.DeviceNeighbors.from_list(w.nl), c)
    ref = oo.energy_forces(*_args(w, p, Q), c)
    assert relerr(o["E"].item(), ref["E"]) <= 1e-10
    assert relerr(o["E_atom"].cpu().numpy(), ref["E_atom"]) <= 1e-10
    assert relerr(o["F"].cpu().numpy(), ref["F"]) <= 1e-10
    assert relerr(o["W"].cpu().numpy(), ref["W"]) <= 1e-10
