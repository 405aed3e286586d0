"""Molecular dynamics driver over the C ABI: velocity Verlet chunks
(pod_md_verlet) with a skin neighbour list built on the device
(pod_build_neighbors) and rebuilt once an atom has moved more than half the
skin (pod_md_max_displacement).  Argument marshalling and the rebuild
decision only; every step runs in the library's kernels."""
from __future__ import annotations

import numpy as np

from paper_2212_14446_amd import pod

MASS_TA = 180.94788   # amu


class MD:
    """NVE dynamics of one periodic (or open) system with a linear POD model."""

    def __init__(self, model: pod.PodModel, pos, vel, cell, c, mass=MASS_TA, skin=0.5):
        import torch
        self.m = model
        self.cell = None if cell is None else np.asarray(cell, dtype=np.float64)
        self.x = model._pos(pos).clone()
        self.v = torch.as_tensor(np.asarray(vel), dtype=model.torch_dtype, device=model.device).contiguous().clone()
        self.c = torch.as_tensor(np.asarray(c), dtype=model.torch_dtype, device=model.device).contiguous()
        self.mass = float(mass)
        self.skin = float(skin)
        self.N = int(self.x.shape[0])
        self.F = torch.empty_like(self.x)
        self.E = torch.empty(1, dtype=torch.float64, device=model.device)
        self.disp = torch.empty(1, dtype=torch.float64, device=model.device)
        self.rebuilds = 0
        self._rebuild()
        pod.pod_energy_forces(model.h, self.N, self.nb.P, self.x, self.cell, self.nb.offsets, self.nb.nbr_j,
                              self.nb.shift, self.c, None, self.E, self.F, None, None, rev=self.nb.rev)
        model.check()

    def _rebuild(self):
        self.nb = pod.DeviceNeighbors.build(self.m, self.x, self.cell, rlist=self.m.setup.rcut + self.skin)
        self.nb.build_reverse(self.m)
        self.x_ref = self.x.clone()
        self.rebuilds += 1

    def _chunk(self, k, dt, ep, ek):
        pod.pod_md_verlet(self.m.h, self.N, self.nb.P, self.x, self.v, self.F, self.cell, self.nb.offsets,
                          self.nb.nbr_j, self.nb.shift, self.nb.rev, self.c, self.mass, dt, k, ep, ek,
                          self.x_ref, self.disp)
        d = float(self.disp.item())
        if not np.isfinite(d):
            raise RuntimeError("non-finite positions in the dynamics")
        return d

    def run(self, nsteps: int, chunk: int = 10, dt: float = 1.0):
        """nsteps steps of dt fs; returns per-step potential and kinetic
        energy (eV).  A chunk of steps whose atoms moved more than half the
        skin from the list's positions (measured on the device after every
        step) is undone and run again on a list rebuilt at its start, with
        fewer steps if needed, so every step runs on a valid list."""
        import torch
        ep = torch.empty(max(nsteps, 1), dtype=torch.float64, device=self.m.device)
        ek = torch.empty(max(nsteps, 1), dtype=torch.float64, device=self.m.device)
        done = 0
        d_prev = 0.0
        while done < nsteps:
            k = min(chunk, nsteps - done)
            saved = (self.x.clone(), self.v.clone(), self.F.clone())
            d = self._chunk(k, dt, ep[done:], ek[done:])
            rebuilt = False
            while d > 0.5 * self.skin:
                self.x.copy_(saved[0])
                self.v.copy_(saved[1])
                self.F.copy_(saved[2])
                if not rebuilt:
                    self._rebuild()
                    rebuilt = True
                elif k > 1:
                    k = max(1, k // 2)
                else:
                    raise RuntimeError("atoms move more than half the skin in one step")
                d = self._chunk(k, dt, ep[done:], ek[done:])
            done += k
            if rebuilt:
                d_prev = 0.0
            # rebuild ahead when the next chunk would likely cross half the skin
            if d + 1.5 * max(d - d_prev, 0.0) > 0.5 * self.skin:
                self._rebuild()
                d = 0.0
            d_prev = d
        self.m.check()
        return ep[:nsteps], ek[:nsteps]
