"""Plain FP64 CPU oracle of molecular dynamics with a POD potential.

Test infrastructure, not product code.  Only the test suite, the smoke check
and the benchmark's CPU leg import this module; the HIP library and its
binding never call it, and it shares no code with them.

The paper measures its potentials by the cost of molecular-dynamics steps
(Sec. V, Fig. 4); this module is the reference integrator for that use: the
velocity Verlet scheme (Swope, Andersen, Berens and Wilson, J. Chem. Phys. 76,
637 (1982)),

    v(t + dt/2) = v(t) + dt/2 F(t) / m
    x(t + dt)   = x(t) + dt v(t + dt/2)
    v(t + dt)   = v(t + dt/2) + dt/2 F(t + dt) / m,

in units of angstrom, femtosecond, atomic mass unit and electronvolt, so that
an acceleration F/m in eV/(A amu) is ACC A/fs^2 and a kinetic energy
m v^2 / 2 in amu A^2/fs^2 is that value divided by ACC in eV.
"""
from __future__ import annotations

import numpy as np

# 1 eV / (1 A * 1 amu) in A / fs^2: 1.602176634e-19 J / 1e-10 m / 1.66053906660e-27 kg
ACC = 1.602176634e-19 / 1e-10 / 1.66053906660e-27 * 1e-20


def kinetic_energy(vel, mass: float) -> float:
    """sum_n m |v_n|^2 / 2 in eV (vel in A/fs, mass in amu)."""
    v = np.asarray(vel, dtype=np.float64)
    return float(0.5 * mass * (v * v).sum() / ACC)


def velocity_verlet(pos, vel, mass: float, dt: float, nsteps: int, force_fn):
    """nsteps of velocity Verlet from (pos, vel); force_fn(pos) -> (E, F).

    Returns the final positions and velocities and, per step (including the
    start), the potential and kinetic energies."""
    x = np.array(pos, dtype=np.float64)
    v = np.array(vel, dtype=np.float64)
    E, F = force_fn(x)
    epot, ekin = [E], [kinetic_energy(v, mass)]
    a = ACC / mass
    for _ in range(nsteps):
        v = v + 0.5 * dt * a * F
        x = x + dt * v
        E, F = force_fn(x)
        v = v + 0.5 * dt * a * F
        epot.append(E)
        ekin.append(kinetic_energy(v, mass))
    return x, v, np.array(epot), np.array(ekin)


def pod_force_fn(cell, p, Q, c, rlist=None):
    """force_fn for the POD oracle: the neighbour list is rebuilt from scratch
    (brute force over images) at every step, so it is always exact."""
    from oracle import pod_oracle as po

    rl = p.rcut if rlist is None else rlist

    def fn(x):
        off, nj, sh = po.neighbors_bruteforce(x, cell, rl)
        out = po.energy_forces(x, cell, off, nj, sh, p, Q, c)
        return out["E"], out["F"]
    return fn
