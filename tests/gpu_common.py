"""Helpers shared by the GPU parity tests: oracle parameter objects, relative
error norms and the case runner.  Inputs come from the seeded workload
generator; expected values come only from the oracle."""
import sys

import numpy as np

from oracle import pod_oracle as po
from paper_2212_14446_amd import pod, workloads as wl


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_params(s) -> po.PodParams:
    if isinstance(s, wl.PodSetup):
        a, b, g, k = s.snapshot_family()
    else:
        a, b, g, k = s.alpha, s.beta, s.gamma, s.kappa
    return po.PodParams(s.rin, s.rcut, np.asarray(a, float), np.asarray(b, float), np.asarray(g, float),
                        np.asarray(k, float), s.K2, s.K3, s.K4, s.P3, s.P4)


def lib_setup(s) -> pod.Setup:
    if isinstance(s, wl.PodSetup):
        return pod.setup_from_workload(s)
    return s


def relerr(x, ref):
    """Normwise relative error ||x - ref||_inf / ||ref||_inf."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.max(np.abs(ref)) if ref.size else 0.0
    num = np.max(np.abs(x - ref)) if ref.size else 0.0
    return num / den if den > 0 else num


def colerr(D, ref):
    """Per-descriptor-column normwise relative error (max over columns)."""
    D = np.asarray(D, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    worst = 0.0
    for k in range(ref.shape[1]):
        worst = max(worst, relerr(D[:, k], ref[:, k]))
    return worst


class Case:
    """One system: positions, cell, neighbour list and parameters, with the
    oracle's basis Q (passed to the library so both sides share it)."""

    def __init__(self, pos, cell, nl, setup, c, name="case"):
        self.pos = np.asarray(pos, dtype=np.float64)
        self.cell = None if cell is None else np.asarray(cell, dtype=np.float64)
        self.nl = nl
        self.setup = setup
        self.op = oracle_params(setup)
        self.Q, _ = po.pod_basis(self.op)
        self.K = self.op.K
        self.c = np.asarray(c, dtype=np.float64)
        self.name = name

    @classmethod
    def from_workload(cls, w):
        return cls(w.pos, w.cell, w.nl, w.setup, w.c, w.name)

    def oracle_descriptors(self, atoms=None, pos=None):
        pos = self.pos if pos is None else pos
        return po.descriptors_fast(pos, self.cell, self.nl.offsets.astype(np.int64), self.nl.nbr_j,
                                   self.nl.shift3, self.op, self.Q, atoms)

    def oracle_ef(self, pos=None):
        pos = self.pos if pos is None else pos
        return po.energy_forces(pos, self.cell, self.nl.offsets.astype(np.int64), self.nl.nbr_j,
                                self.nl.shift3, self.op, self.Q, self.c)

    def model(self, dtype):
        return pod.PodModel(lib_setup(self.setup), dtype, Q=self.Q[:, : self.K])

    def run(self, dtype, pos=None):
        """Descriptors and energy/forces from the GPU, as float64 numpy.  Forces
        are taken on both force paths: atomics ("F") and the reverse-index
        gather ("F_gather"); the gather path's E, W, G must agree too."""
        import torch
        pos = self.pos if pos is None else pos
        m = self.model(dtype)
        nb = pod.DeviceNeighbors.from_list(self.nl)
        D = m.descriptors(pos, self.cell, nb)
        o = m.energy_forces(pos, self.cell, nb, self.c)
        torch.cuda.synchronize()
        res = {"D": D.double().cpu().numpy(), "E": float(o["E"].item()),
               "E_atom": o["E_atom"].double().cpu().numpy(), "F": o["F"].double().cpu().numpy(),
               "W": o["W"].cpu().numpy(), "G": o["G"].cpu().numpy()}
        nb.build_reverse(m)
        o2 = m.energy_forces(pos, self.cell, nb, self.c)
        torch.cuda.synchronize()
        res["F_gather"] = o2["F"].double().cpu().numpy()
        res["E_gather"] = float(o2["E"].item())
        res["W_gather"] = o2["W"].cpu().numpy()
        res["rev"] = nb.rev[: nb.P].cpu().numpy()
        return res


def reverse_index(nl):
    """Host reference of the reverse-pair index (dictionary lookup)."""
    N = len(nl.offsets) - 1
    centre = np.repeat(np.arange(N), np.diff(nl.offsets))
    key = {(int(i), int(j), int(a), int(b), int(c)): p
           for p, (i, j, (a, b, c)) in enumerate(zip(centre, nl.nbr_j, nl.shift3))}
    return np.array([key[(int(j), int(i), -int(a), -int(b), -int(c))]
                     for i, j, (a, b, c) in zip(centre, nl.nbr_j, nl.shift3)], dtype=np.int64)


def positions_for(dtype, pos):
    """The exact input positions a dtype path sees (FP32 rounds them)."""
    if dtype == "f32":
        return np.asarray(pos, dtype=np.float32).astype(np.float64)
    return np.asarray(pos, dtype=np.float64)
