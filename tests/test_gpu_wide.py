"""GPU parity of the wide-degree energy path (angular degree 7 to 10, or more
than 8 radial functions: the largest models of Table 6) against the FP64
oracle, through the C ABI.

Same tolerances as the main parity tests: FP64 1e-10 normwise for every
output (descriptors per column); FP32 2e-5 for energies and 1e-4 for forces,
virial and G.  Cases: the Table 6 rows 5 and 6 (2/3-body and with their
4-body terms), a degree-7 mixed model, K = 9 at degree 3 (wide by K alone), a
general snapshot family (generic radial code), an open cluster with an
isolated atom, a box with more atoms than persistent workgroups (sampled
against the oracle), the allocation-free entry point, and error reporting."""
import numpy as np
import pytest

from gpu_common import Case, colerr, oracle_params, relerr, say
from oracle import pod_oracle as po
from paper_2212_14446_amd import pod, workloads as wl

pytestmark = pytest.mark.gpu

TOL64 = 1e-10

WIDE = [
    # L, K2, K3, K4, P3, P4
    (14, 10, 9, 0, 8, 0),     # Table 6 row 5, OPOD/FPOD3 (M = 92)
    (14, 8, 12, 0, 10, 0),    # Table 6 row 6, OPOD/FPOD3 (M = 141)
    (14, 10, 9, 9, 8, 5),     # Table 6 row 5 with its 4-body terms (M = 236)
    (14, 8, 12, 12, 10, 6),   # Table 6 row 6 with its 4-body terms (M = 417)
    (12, 3, 4, 2, 7, 3),      # degree 7, mixed orders
    (12, 9, 2, 3, 3, 2),      # K = 9 at degree 3: wide by the radial count alone
    (10, 2, 2, 4, 2, 6),      # degree 6 at K = 4: the register path, as a control
]


@pytest.fixture(scope="module")
def box49():
    pos, cell = wl.bcc(3)
    pos = wl.remove_sites(pos, 5, seed=71)
    pos = wl.displace(pos, 0.12, seed=72)
    return pos, cell


def _compare(case, dtype):
    from test_gpu_parity import _compare as cmp
    return cmp(case, dtype)


@pytest.mark.parametrize("L,K2,K3,K4,P3,P4", WIDE)
def test_wide_f64(box49, L, K2, K3, K4, P3, P4):
    pos, cell = box49
    s = wl.PodSetup(0.5, 5.0, L, K2, K3, K4, P3, P4)
    nl = wl.neighbor_list(pos, cell, s.rcut)
    c = wl.coefficients(s.M, seed=300 + L + K2 + 3 * K3 + 5 * K4 + 7 * P3 + 11 * P4)
    errs = _compare(Case(pos, cell, nl, s, c, f"wide_L{L}_K{K2},{K3},{K4}_P{P3},{P4}"), "f64")
    for k, v in errs.items():
        assert v < TOL64, (k, v)


@pytest.mark.parametrize("L,K2,K3,K4,P3,P4", [WIDE[0], WIDE[3], WIDE[5]])
def test_wide_f32(box49, L, K2, K3, K4, P3, P4):
    pos, cell = box49
    s = wl.PodSetup(0.5, 5.0, L, K2, K3, K4, P3, P4)
    nl = wl.neighbor_list(pos, cell, s.rcut)
    c = wl.coefficients(s.M, seed=400 + L + K2 + 3 * K3 + 5 * K4 + 7 * P3 + 11 * P4)
    errs = _compare(Case(pos, cell, nl, s, c, f"wide32_L{L}_K{K2},{K3},{K4}_P{P3},{P4}"), "f32")
    assert errs["E"] < 2e-5 and errs["E_atom"] < 2e-5, errs
    assert errs["F"] < 1e-4 and errs["F_gather"] < 1e-4, errs
    assert errs["W"] < 1e-4 and errs["W_gather"] < 1e-4 and errs["G"] < 1e-4, errs
    assert errs["D"] < 1e-3, errs


def test_wide_general_snapshot_family(box49):
    # non-integer and unordered alpha, two betas, mixed kappa, non-integer
    # gamma: the generic radial code inside the wide kernel
    pos, cell = box49
    s = pod.Setup(0.4, 4.8,
                  np.array([1.0, 2.0, 1.5, 4.0, 3.0, 2.0, 0.0, 1.0, 5.0, 6.0]),
                  np.array([3.0, 3.0, 3.0, 3.0, 3.0, 1.0, 0.0, 0.0, 2.0, 2.0]),
                  np.array([0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 2.5, 1.0, 0.0, 0.0]),
                  np.array([1.0, 1.0, 1.0, 0.6, 1.0, 1.0, 0.0, 1.0, 1.0, 1.0]),
                  9, 4, 3, 8, 4)
    nl = wl.neighbor_list(pos, cell, s.rcut)
    M = po.num_descriptors(oracle_params(s))[0]
    errs = _compare(Case(pos, cell, nl, s, wl.coefficients(M, seed=15), "wide_general"), "f64")
    for k, v in errs.items():
        assert v < TOL64, (k, v)


def test_wide_open_cluster_with_isolated_atom():
    s = wl.PodSetup(0.5, 5.0, 14, 10, 9, 9, 8, 5)
    rng = np.random.default_rng(8)
    pos, _ = wl.lattice("bcc", 2, 2, 1, 3.31)
    pos = pos + rng.normal(0, 0.15, pos.shape)
    pos = np.vstack([pos, [[40.0, 40.0, 40.0]]])
    nl = wl.neighbor_list(pos, None, s.rcut)
    case = Case(pos, None, nl, s, wl.coefficients(s.M, seed=9), "wide_open")
    errs = _compare(case, "f64")
    for k, v in errs.items():
        assert v < TOL64, (k, v)
    got = case.run("f64")
    assert got["D"][-1, 0] == 1.0 and np.all(got["D"][-1, 1:] == 0.0)
    assert np.all(got["F"][-1] == 0.0)


def test_wide_many_atoms_per_workgroup_sampled():
    """4,394 atoms, more than the 2,048 persistent workgroups, so every
    workgroup walks two or three atoms: sampled descriptors, energies and
    forces against the oracle, plus the global checks (sum of forces, E =
    sum E_i, G = sum D_i)."""
    import torch
    s = wl.PodSetup(0.5, 5.0, 14, 10, 9, 9, 8, 5)
    pos, cell = wl.bcc(13)
    pos = wl.displace(pos, 0.1, seed=13)
    nl = wl.neighbor_list(pos, cell, s.rcut)
    case = Case(pos, cell, nl, s, wl.coefficients(s.M, seed=14), "wide_4394")
    say(f"[gpu] wide sampled N={len(pos)} P={nl.n_pairs}")
    m = case.model("f64")
    nb = pod.DeviceNeighbors.from_list(nl)
    D = m.descriptors(pos, cell, nb).cpu().numpy()
    nb.build_reverse(m)
    o = m.energy_forces(pos, cell, nb, case.c)
    torch.cuda.synchronize()
    E_atom = o["E_atom"].cpu().numpy()
    F = o["F"].cpu().numpy()
    rng = np.random.default_rng(5)
    atoms = np.sort(np.concatenate([[0, 1, 2047, 2048, 2049, 4095, 4096, len(pos) - 1],
                                    rng.choice(len(pos), 8, replace=False)]))
    Dref = case.oracle_descriptors(atoms=atoms)
    assert colerr(D[atoms], Dref) < TOL64
    assert relerr(E_atom[atoms], Dref @ case.c) < TOL64
    fat = atoms[:4]
    oref = po.energy_forces(pos, cell, nl.offsets.astype(np.int64), nl.nbr_j, nl.shift3, case.op, case.Q, case.c,
                            force_atoms=fat)
    assert relerr(F[fat], oref["F"][fat]) < TOL64
    assert abs(o["E"].item() - E_atom.sum()) <= 1e-12 * np.abs(E_atom).sum()
    assert relerr(o["G"].cpu().numpy(), D.sum(0)) < 1e-12
    assert np.abs(F.sum(0)).max() <= 1e-9 * np.abs(F).max()


def test_wide_noalloc_matches_energy_forces(box49):
    import torch
    from test_zz_no_alloc import _call
    pos, cell = box49
    s = wl.PodSetup(0.5, 5.0, 14, 8, 12, 12, 10, 6)
    nl = wl.neighbor_list(pos, cell, s.rcut)
    m = pod.PodModel(pod.setup_from_workload(s), "f64")
    nb = pod.DeviceNeighbors.from_list(nl)
    nb.build_reverse(m)
    x = m._pos(pos)
    c = torch.as_tensor(wl.coefficients(s.M, seed=21), dtype=torch.float64, device="cuda")
    ref = _call(pod.pod_energy_forces, m, nb, x, cell, c, nb.rev)
    got = _call(pod.pod_energy_forces_noalloc, m, nb, x, cell, c, nb.rev)
    for k in ref:
        assert np.array_equal(got[k], ref[k]), k


def test_wide_gather_forces_bitwise_reproducible(box49):
    pos, cell = box49
    s = wl.PodSetup(0.5, 5.0, 14, 10, 9, 9, 8, 5)
    nl = wl.neighbor_list(pos, cell, s.rcut)
    case = Case(pos, cell, nl, s, wl.coefficients(s.M, seed=22), "wide_repeat")
    a, b = case.run("f64"), case.run("f64")
    for k in ("E_atom", "F_gather", "W_gather", "G", "D"):
        assert np.array_equal(a[k], b[k]), k


def test_wide_error_pair_inside_rin():
    s = wl.PodSetup(0.5, 5.0, 14, 10, 9, 0, 8, 0)
    pos = np.array([[0.0, 0.0, 0.0], [0.3, 0.0, 0.0], [3.0, 0.0, 0.0]])
    nl = wl.neighbor_list(pos, None, s.rcut)
    m = pod.PodModel(pod.setup_from_workload(s), "f64")
    nb = pod.DeviceNeighbors.from_list(nl)
    with pytest.raises(pod.PodError) as e:
        m.energy_forces(pos, None, nb, wl.coefficients(s.M, seed=1))
    assert pod.ERRORS[e.value.code] == "POD_ERANGE"
    m.check()


def test_wide_refused_where_the_register_kernels_are_required():
    # batch assembly and the network surrogate keep the basis in registers:
    # a degree-8 model is refused before any launch
    s = wl.PodSetup(0.5, 5.0, 14, 10, 9, 0, 8, 0)
    m = pod.PodModel(pod.setup_from_workload(s), "f64")
    b = wl.make_batch(2, 11, s, n_min=2, n_max=20)
    with pytest.raises(pod.PodError) as e:
        pod.batch_assemble(m, pod.DeviceBatch.from_batch(b))
    assert pod.ERRORS[e.value.code] == "POD_ENOTSUP"
