"""The C-ABI library on the CPU: it loads, exports every declared entry point,
and its host-only pieces (parameter validation, the POD basis of Sec. II.B)
agree with the oracle.  No compute call is made here."""
import ctypes

import numpy as np
import pytest

from oracle import pod_oracle as po
from paper_2212_14446_amd import pod, workloads as wl


def test_library_exports_every_header_symbol():
    L = pod.lib()
    names = pod.header_symbols()
    assert "pod_init" in names and "pod_energy_forces" in names and "pod_descriptors" in names
    for n in names:
        assert hasattr(L, n), n


def test_binding_has_every_header_symbol():
    """The Python binding offers each C entry point under the same name."""
    for n in pod.header_symbols():
        assert callable(getattr(pod, n, None)), n
    for n in ("pod_acsf_create", "pod_five_body_energy_forces", "pod_md_verlet", "pod_fit_solve"):
        assert n in pod.header_symbols()


def _setup(s: wl.PodSetup):
    return pod.setup_from_workload(s)


@pytest.mark.parametrize("s", [wl.SETUP_CFG1, wl.SETUP_CFG2])
def test_host_basis_matches_oracle(s):
    Q, e = pod.pod_compute_basis(_setup(s))
    p = po.PodParams(s.rin, s.rcut, *s.snapshot_family(), s.K2, s.K3, s.K4, s.P3, s.P4)
    Qo, eo = po.pod_basis(p)
    assert np.allclose(e, eo, rtol=1e-10, atol=1e-13 * eo[0])
    # the retained columns are well separated: same vectors, same sign rule
    K = max(s.K2, s.K3, s.K4)
    assert np.max(np.abs(Q[:, :K] - Qo[:, :K])) < 1e-9


def test_host_basis_general_snapshots():
    # non-integer alpha, two betas, mixed kappa and a non-integer gamma
    s = pod.Setup(0.3, 4.5, np.array([1.0, 2.5, 1.0, 3.0, 0.0]), np.array([2.0, 2.0, 5.0, 5.0, 0.0]),
                  np.array([0.0, 0.0, 0.0, 1.5, 1.5]), np.array([1.0, 1.0, 0.7, 1.0, 0.0]), 3, 3, 0, 2, 0)
    Q, e = pod.pod_compute_basis(s)
    p = po.PodParams(s.rin, s.rcut, s.alpha, s.beta, s.gamma, s.kappa, 3, 3, 0, 2, 0)
    Qo, eo = po.pod_basis(p)
    assert np.allclose(e, eo, rtol=1e-9, atol=1e-12 * eo[0])
    assert np.max(np.abs(Q[:, :3] - Qo[:, :3])) < 1e-8


@pytest.mark.parametrize("change,code", [
    (dict(rin=5.0), "POD_EINVAL"),            # rin >= rcut
    (dict(K2=0, K3=0, K4=0), "POD_EINVAL"),   # nothing to compute
    (dict(K2=9), "POD_EINVAL"),               # K > L
    (dict(P3=-1), "POD_EINVAL"),
    (dict(P4=7), "POD_ENOTSUP"),              # beyond compiled angular degree
])
def test_host_validation(change, code):
    s = _setup(wl.SETUP_CFG2)
    for k, v in change.items():
        setattr(s, k, v)
    with pytest.raises(pod.PodError) as ei:
        pod.pod_compute_basis(s)
    assert pod.ERRORS[ei.value.code] == code


def test_strerror_covers_codes():
    L = pod.lib()
    for code in pod.ERRORS:
        assert L.pod_strerror(code)
    assert L.pod_strerror(-99) == b"unknown error"
