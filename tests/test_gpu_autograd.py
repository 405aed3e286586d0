"""Differentiable POD energy (torch.autograd.Function over the adjoint kernel):
gradcheck in FP64, the 54,000-atom box against the compiled FP64 oracle on
every atom and its FP32 forces against central differences of the FP64 GPU
energy on 250 random atoms, dE/dc = G and the virial against a strain
difference."""
import numpy as np
import pytest
import torch

from gpu_common import Case, oracle_params, relerr, say
from oracle import pod_oracle as po
from paper_2212_14446_amd import pod, workloads as wl
from paper_2212_14446_amd.autograd import pod_energy

pytestmark = pytest.mark.gpu


def _setup_small():
    s = wl.PodSetup(0.5, 5.0, 8, 4, 4, 4, 3, 3)
    pos, cell = wl.bcc(2)
    pos = wl.displace(pos, 0.12, 13)
    nl = wl.neighbor_list(pos, cell, s.rcut)
    return s, pos, cell, nl


def test_gradcheck_fp64():
    s, pos, cell, nl = _setup_small()
    say("[gpu] autograd gradcheck")
    m = pod.PodModel(pod.setup_from_workload(s), "f64")
    nb = pod.DeviceNeighbors.from_list(nl)
    nb.build_reverse(m)
    x = torch.tensor(pos, dtype=torch.float64, device="cuda", requires_grad=True)
    c = torch.tensor(wl.coefficients(s.M, 3) * 1e-2, dtype=torch.float64, device="cuda", requires_grad=True)
    f = lambda xx, cc: pod_energy(xx, cc, m, nb, cell)[0]
    assert torch.autograd.gradcheck(f, (x, c), eps=1e-6, atol=1e-6, rtol=1e-5)


def test_grad_matches_oracle_forces():
    s, pos, cell, nl = _setup_small()
    case = Case(pos, cell, nl, s, wl.coefficients(s.M, 4), "autograd_small")
    m = case.model("f64")
    nb = pod.DeviceNeighbors.from_list(nl)
    x = torch.tensor(pos, dtype=torch.float64, device="cuda", requires_grad=True)
    c = torch.tensor(case.c, dtype=torch.float64, device="cuda", requires_grad=True)
    E, W = pod_energy(x, c, m, nb, cell)
    E.backward()
    o = case.oracle_ef()
    assert abs(E.item() - o["E"]) < 1e-10 * abs(o["E"])
    assert relerr(-x.grad.cpu().numpy(), o["F"]) < 1e-10
    assert relerr(c.grad.cpu().numpy(), o["G"]) < 1e-12
    assert relerr(W.cpu().numpy(), o["W"]) < 1e-10


@pytest.fixture(scope="module")
def box54k():
    w = wl.config4()
    return w


def test_cfg4_fp32_forces_vs_fp64_central_differences(box54k):
    w = box54k
    s = w.setup
    say(f"[gpu] cfg4 N={w.N} P={w.nl.n_pairs}")
    m64 = pod.PodModel(pod.setup_from_workload(s), "f64")
    nb = pod.DeviceNeighbors.from_list(w.nl)
    nb.build_reverse(m64)
    D = m64.descriptors(w.pos, w.cell, nb).cpu().numpy()
    c = wl.standardised_coefficients(D, s, seed=8)
    m32 = pod.PodModel(pod.setup_from_workload(s), "f32")
    x32 = torch.tensor(w.pos, dtype=torch.float32, device="cuda", requires_grad=True)
    c32 = torch.tensor(c, dtype=torch.float32, device="cuda")
    E32, W32 = pod_energy(x32, c32, m32, nb, w.cell)
    E32.backward()
    F32 = -x32.grad.double().cpu().numpy()
    # FP64 reference on the same (FP32-rounded) inputs
    pos_r = x32.detach().double().cpu().numpy()
    c_r = c32.double().cpu().numpy()
    o64 = m64.energy_forces(pos_r, w.cell, nb, c_r)
    F64 = o64["F"].cpu().numpy()
    E64 = o64["E"].item()
    eE = abs(E32.item() - E64) / abs(E64)
    eF = relerr(F32, F64)
    say(f"[gpu]   FP32 vs FP64: E {eE:.2e} F {eF:.2e}; force std {F64.std():.3f} eV/A")
    assert eE < 2e-5 and eF < 1e-4
    # central differences of the FP64 GPU energy on 250 random atoms
    rng = np.random.default_rng(8)
    atoms = rng.choice(w.N, size=250, replace=False)
    h = 1e-5
    tpos = torch.tensor(pos_r, dtype=torch.float64, device="cuda")
    tc = torch.tensor(c_r, dtype=torch.float64, device="cuda")
    Eb = torch.empty(1, dtype=torch.float64, device="cuda")
    fd = np.zeros((len(atoms), 3))
    for ii, a in enumerate(atoms):
        for d in range(3):
            vals = []
            for sgn in (1.0, -1.0):
                tpos[a, d] += sgn * h
                pod.pod_energy_forces(m64.h, w.N, nb.P, tpos, w.cell, nb.offsets, nb.nbr_j, nb.shift, tc,
                                      None, Eb, None, None, None)
                vals.append(Eb.item())
                tpos[a, d] -= sgn * h
            fd[ii, d] = -(vals[0] - vals[1]) / (2 * h)
    m64.check()
    efd64 = np.abs(fd - F64[atoms]).max() / np.abs(F64[atoms]).max()
    efd32 = np.abs(fd - F32[atoms]).max() / np.abs(F64[atoms]).max()
    say(f"[gpu]   central differences (250 atoms): FP64 forces {efd64:.2e}, FP32 forces {efd32:.2e}")
    assert efd64 < 1e-6 and efd32 < 1e-4


def test_cfg4_full_box_vs_compiled_oracle(box54k):
    """The 54,000-atom box against the compiled FP64 oracle (oracle.cpp, pinned
    to the NumPy oracle at 1e-12), every atom: the differentiable energy's
    FP64 forces, dE/dc and virial at 1e-10, its FP32 forces at 1e-4 and
    energy at 2e-5 (both sides on the FP32-rounded inputs).  The models take
    the oracle's basis Q, so the comparison does not depend on the sign
    convention of the eigenvectors."""
    from oracle import oracle_c
    w = box54k
    s = w.setup
    op = oracle_params(s)
    Q, _ = po.pod_basis(op)
    K = op.K
    m64 = pod.PodModel(pod.setup_from_workload(s), "f64", Q=Q[:, :K])
    nb = pod.DeviceNeighbors.from_list(w.nl)
    nb.build_reverse(m64)
    D = m64.descriptors(w.pos, w.cell, nb).cpu().numpy()
    c = wl.standardised_coefficients(D, s, seed=9)
    args = (w.nl.offsets.astype(np.int64), w.nl.nbr_j, w.nl.shift3, op, Q)
    say(f"[gpu] cfg4 against the compiled oracle, N={w.N}, {oracle_c.host_threads()} host threads")
    ref = oracle_c.energy_forces(w.pos, w.cell, *args, c, threads=oracle_c.host_threads())
    x = torch.tensor(w.pos, dtype=torch.float64, device="cuda", requires_grad=True)
    cc = torch.tensor(c, dtype=torch.float64, device="cuda", requires_grad=True)
    E, W = pod_energy(x, cc, m64, nb, w.cell)
    E.backward()
    assert abs(E.item() - ref["E"]) < 1e-10 * abs(ref["E"])
    assert relerr(-x.grad.cpu().numpy(), ref["F"]) < 1e-10
    assert relerr(cc.grad.cpu().numpy(), ref["G"]) < 1e-10
    assert relerr(W.cpu().numpy(), ref["W"]) < 1e-10
    # FP32 on the FP32-rounded inputs, against the oracle on the same inputs
    m32 = pod.PodModel(pod.setup_from_workload(s), "f32", Q=Q[:, :K])
    x32 = torch.tensor(w.pos, dtype=torch.float32, device="cuda", requires_grad=True)
    c32 = torch.tensor(c, dtype=torch.float32, device="cuda")
    E32, _ = pod_energy(x32, c32, m32, nb, w.cell)
    E32.backward()
    ref32 = oracle_c.energy_forces(x32.detach().double().cpu().numpy(), w.cell, *args, c32.double().cpu().numpy(),
                                   threads=oracle_c.host_threads())
    eE = abs(E32.item() - ref32["E"]) / abs(ref32["E"])
    eF = relerr(-x32.grad.double().cpu().numpy(), ref32["F"])
    say(f"[gpu]   FP32 against the oracle: E {eE:.2e}, F {eF:.2e}")
    assert eE < 2e-5 and eF < 1e-4


def test_dE_dc_is_G_and_virial_is_strain_derivative():
    s, pos, cell, nl = _setup_small()
    m = pod.PodModel(pod.setup_from_workload(s), "f64")
    nb = pod.DeviceNeighbors.from_list(nl)
    c = wl.coefficients(s.M, 5)
    o = m.energy_forces(pos, cell, nb, c)
    G = o["G"].cpu().numpy()
    d = np.random.default_rng(1).normal(size=s.M)
    E1 = m.energy_forces(pos, cell, nb, c + d)["E"].item()
    assert E1 - o["E"].item() == pytest.approx(d @ G, rel=1e-9)
    W = o["W"].cpu().numpy()
    h = 1e-6
    Wfd = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            eps = np.zeros((3, 3)); eps[a, b] += 0.5 * h; eps[b, a] += 0.5 * h
            Ep = m.energy_forces(pos @ (np.eye(3) + eps).T, cell @ (np.eye(3) + eps).T, nb, c)["E"].item()
            Em = m.energy_forces(pos @ (np.eye(3) - eps).T, cell @ (np.eye(3) - eps).T, nb, c)["E"].item()
            Wfd[a, b] = -(Ep - Em) / (2 * h)
    assert np.abs(W - Wfd).max() < 1e-6 * np.abs(W).max()
