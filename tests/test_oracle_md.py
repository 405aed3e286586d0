"""Pins of the molecular-dynamics oracle (velocity Verlet with POD forces).

The integrator is checked against the exact discrete solution of velocity
Verlet for a harmonic oscillator; with POD forces, against time reversal,
momentum conservation and the second-order decay of the energy error."""
import numpy as np

from oracle import md_oracle as mo
from oracle import pod_oracle as po
from paper_2212_14446_amd import workloads as wl


def test_unit_constant():
    # 1 eV/(A amu) = 9.6485e-3 A/fs^2 (CODATA constants)
    assert abs(mo.ACC - 9.648533212e-3) < 1e-11


def test_harmonic_oscillator_exact_discrete_solution():
    """For F = -k x, velocity Verlet gives x_{n+1} - 2 x_n + x_{n-1} =
    -(h w)^2 x_n, so x_n = A cos(n t) + B sin(n t), cos t = 1 - (h w)^2 / 2."""
    m, k, h = 2.5, 0.7, 0.9
    w2 = k * mo.ACC / m
    x0, v0 = np.array([[0.3, -0.1, 0.2]]), np.array([[0.01, 0.02, -0.015]])
    n = 40
    x, v, _, _ = mo.velocity_verlet(x0, v0, m, h, n, lambda x: (0.5 * k * float((x * x).sum()), -k * x))
    th = np.arccos(1.0 - 0.5 * h * h * w2)
    x1 = x0 + h * v0 - 0.5 * h * h * w2 * x0
    A = x0
    B = (x1 - x0 * np.cos(th)) / np.sin(th)
    want = A * np.cos(n * th) + B * np.sin(n * th)
    assert np.abs(x - want).max() <= 1e-12 * np.abs(want).max()


def _small(seed=5):
    s = wl.PodSetup(0.5, 5.0, 6, 3, 3, 2, 2, 2)
    pos, cell = wl.bcc(2)
    pos = wl.displace(pos, 0.05, seed)
    p = po.PodParams(s.rin, s.rcut, *s.snapshot_family(), s.K2, s.K3, s.K4, s.P3, s.P4)
    Q, _ = po.pod_basis(p)
    # a gentle potential: small random coefficients
    c = 0.02 * wl.coefficients(s.M, seed + 1)
    vel = np.random.default_rng(seed + 2).normal(0.0, 0.005, size=pos.shape)
    vel -= vel.mean(0)
    return pos, cell, vel, p, Q, c


def test_time_reversal_and_momentum():
    pos, cell, vel, p, Q, c = _small()
    fn = mo.pod_force_fn(cell, p, Q, c)
    m, dt, n = 180.95, 1.0, 8
    x, v, _, _ = mo.velocity_verlet(pos, vel, m, dt, n, fn)
    assert np.abs(v.sum(0) - vel.sum(0)).max() <= 1e-12
    xb, vb, _, _ = mo.velocity_verlet(x, -v, m, dt, n, fn)
    assert np.abs(xb - pos).max() <= 1e-10
    assert np.abs(vb + vel).max() <= 1e-10 * max(1.0, np.abs(vel).max())


def test_energy_error_is_second_order():
    pos, cell, vel, p, Q, c = _small(7)
    fn = mo.pod_force_fn(cell, p, Q, c)
    m, T = 180.95, 8.0
    drift = []
    for dt in (2.0, 1.0):
        _, _, ep, ek = mo.velocity_verlet(pos, vel * 20, m, dt, int(T / dt), fn)
        et = ep + ek
        drift.append(np.abs(et - et[0]).max())
    assert drift[1] < 0.4 * drift[0]      # ~ 1/4 for a second-order scheme
