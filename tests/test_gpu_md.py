"""Molecular dynamics on the device (pod_md_verlet, pod_md_max_displacement,
the md.MD driver with a device-built skin list) against the velocity-Verlet
oracle with POD oracle forces on an exact list at every step.

FP64 tolerance: the two sides differ only by summation order in the forces
(~1e-15 relative per step); over 20 steps of a smooth, gentle potential the
difference stays below 1e-10 relative, checked at 1e-9."""
import numpy as np
import pytest
import torch

from gpu_common import oracle_params, relerr, say
from oracle import md_oracle as mo
from oracle import pod_oracle as po
from paper_2212_14446_amd import md, pod, workloads as wl

pytestmark = pytest.mark.gpu

S = wl.PodSetup(0.5, 5.0, 6, 3, 3, 2, 2, 2)


def _system(n=2, seed=5, vscale=0.005, cscale=0.02):
    pos, cell = wl.bcc(n)
    pos = wl.displace(pos, 0.05, seed)
    c = cscale * wl.coefficients(S.M, seed + 1)
    vel = np.random.default_rng(seed + 2).normal(0.0, vscale, size=pos.shape)
    vel -= vel.mean(0)
    return pos, cell, vel, c


def _model(dtype="f64"):
    p = oracle_params(S)
    Q, _ = po.pod_basis(p)
    return pod.PodModel(pod.setup_from_workload(S), dtype, Q=Q[:, :p.K]), p, Q


def test_verlet_matches_oracle():
    pos, cell, vel, c = _system()
    m, p, Q = _model()
    dyn = md.MD(m, pos, vel, cell, c, skin=0.5)
    ep, ek = dyn.run(20, chunk=7, dt=1.0)
    x, v, oep, oek = mo.velocity_verlet(pos, vel, md.MASS_TA, 1.0, 20, mo.pod_force_fn(cell, p, Q, c))
    say(f"[gpu] md vs oracle: rebuilds {dyn.rebuilds}")
    assert relerr(dyn.x.cpu().numpy() - pos, x - pos) <= 1e-9
    assert relerr(dyn.v.cpu().numpy(), v) <= 1e-9
    assert relerr(ep.cpu().numpy(), oep[1:]) <= 1e-9
    assert relerr(ek.cpu().numpy(), oek[1:]) <= 1e-9


def test_rebuilds_momentum_and_energy():
    """Hot atoms force list rebuilds (and chunk retries); the trajectory
    equals one that rebuilds before every step, momentum is conserved and the
    total energy stays within the integrator's error."""
    pos, cell, vel, c = _system(3, seed=9, vscale=0.008)
    m, p, Q = _model()
    a = md.MD(m, pos, vel, cell, c, skin=0.15)
    ep, ek = a.run(120, chunk=10, dt=0.5)
    b = md.MD(m, pos, vel, cell, c, skin=0.15)
    for _ in range(120):
        b._rebuild()
        b.run(1, chunk=1, dt=0.5)
    say(f"[gpu] md rebuilds: {a.rebuilds} (every-step reference {b.rebuilds})")
    assert a.rebuilds > 2
    assert relerr(a.x.cpu().numpy() - pos, b.x.cpu().numpy() - pos) <= 1e-9
    mom0 = vel.sum(0)
    mom = a.v.cpu().numpy().sum(0)
    assert np.abs(mom - mom0).max() <= 1e-12 * max(1.0, np.abs(vel).sum())
    et = (ep + ek).cpu().numpy()
    e0 = float(ek[0].item())
    assert np.abs(et - et[0]).max() <= 1e-3 * e0


def test_fp32_follows_fp64():
    pos, cell, vel, c = _system(seed=11)
    m64, _, _ = _model("f64")
    m32, _, _ = _model("f32")
    a = md.MD(m64, pos, vel, cell, c)
    b = md.MD(m32, pos, vel, cell, c)
    a.run(20, dt=1.0)
    b.run(20, dt=1.0)
    dx = a.x.cpu().numpy() - pos
    assert relerr(b.x.double().cpu().numpy() - pos, dx) <= 1e-3


def test_max_displacement_and_errors():
    m, _, _ = _model()
    x = torch.zeros((5, 3), dtype=torch.float64, device="cuda")
    xr = torch.zeros_like(x)
    x[3, 1] = 0.25
    x[1, 0] = -0.1
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    pod.pod_md_max_displacement(m.h, 5, x, xr, out)
    assert out.item() == 0.25
    x[2, 2] = float("nan")
    pod.pod_md_max_displacement(m.h, 5, x, xr, out)
    assert np.isnan(out.item())
    pos, cell, vel, c = _system()
    dyn = md.MD(m, pos, vel, cell, c)
    nb = dyn.nb
    args = (m.h, dyn.N, nb.P, dyn.x, dyn.v, dyn.F, cell, nb.offsets, nb.nbr_j, nb.shift, nb.rev, dyn.c)
    for mass, dt, extra in ((0.0, 1.0, {}), (180.0, float("nan"), {}), (180.0, 1.0, {"max_disp": out})):
        with pytest.raises(pod.PodError) as e:
            pod.pod_md_verlet(*args, mass, dt, 1, **extra)
        assert pod.ERRORS[e.value.code] == "POD_EINVAL"
