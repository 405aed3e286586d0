"""The allocation-free energy entry point (pod_energy_forces_noalloc) against
pod_energy_forces on the same inputs, through the C ABI: two calls in a row
on the static scratch, the second with a smaller system, on both force
paths and both dtypes.  On the reverse-index path the two entry points run
the same kernels in the same order, so every output must agree bit for bit;
on the atomic path the order of the FP64 force additions is not fixed, so
forces and virial are compared at the parity tolerances (FP64 1e-10, FP32
1e-4)."""
import numpy as np
import pytest

from gpu_common import relerr, say
from paper_2212_14446_amd import pod, workloads as wl

pytestmark = pytest.mark.gpu


def _outputs(m, N):
    import torch
    dt = m.torch_dtype
    return {"E": torch.zeros(1, dtype=torch.float64, device="cuda"),
            "E_atom": torch.zeros(N, dtype=dt, device="cuda"),
            "F": torch.zeros((N, 3), dtype=dt, device="cuda"),
            "W": torch.zeros((3, 3), dtype=torch.float64, device="cuda"),
            "G": torch.zeros(m.M, dtype=torch.float64, device="cuda")}


def _call(fn, m, nb, x, cell, c, rev):
    import torch
    o = _outputs(m, nb.N)
    fn(m.h, nb.N, nb.P, x, cell, nb.offsets, nb.nbr_j, nb.shift, c, o["E_atom"], o["E"], o["F"], o["W"], o["G"],
       rev=rev)
    pod.pod_check(m.h)
    torch.cuda.synchronize()
    return {k: v.double().cpu().numpy() for k, v in o.items()}


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_two_calls_match_energy_forces(dtype):
    import torch
    big = wl.config2(5.0)                        # 15,840 atoms, 397,508 pairs
    small = wl.small_bcc(3, sigma=0.1, seed=5)   # a later, smaller call on the same scratch
    m = pod.PodModel(pod.setup_from_workload(big.setup), dtype)
    for w in (big, small):
        nb = pod.DeviceNeighbors.from_list(w.nl)
        nb.build_reverse(m)
        x = m._pos(w.pos)
        c = torch.as_tensor(w.c, dtype=m.torch_dtype, device="cuda")
        for rev in (nb.rev, None):
            ref = _call(pod.pod_energy_forces, m, nb, x, w.cell, c, rev)
            got = _call(pod.pod_energy_forces_noalloc, m, nb, x, w.cell, c, rev)
            path = "gather" if rev is not None else "atomic"
            errs = {k: relerr(got[k], ref[k]) for k in ref}
            say(f"[gpu] noalloc {dtype} N={nb.N} P={nb.P} {path}: " + " ".join(f"{k}={v:.1e}" for k, v in errs.items()))
            if rev is not None:
                for k in ref:
                    assert np.array_equal(got[k], ref[k]), (k, errs[k])
            else:
                for k in ("E", "E_atom", "G"):
                    assert np.array_equal(got[k], ref[k]), (k, errs[k])
                tol = 1e-10 if dtype == "f64" else 1e-4
                assert errs["F"] < tol and errs["W"] < tol, errs


def test_noalloc_rejects_beyond_static_scratch():
    import torch
    w = wl.config1()
    m = pod.PodModel(pod.setup_from_workload(w.setup), "f64")
    nb = pod.DeviceNeighbors.from_list(w.nl)
    x = m._pos(w.pos)
    c = torch.as_tensor(w.c, dtype=torch.float64, device="cuda")
    o = _outputs(m, nb.N)
    # a pair count whose pair arrays alone exceed the static scratch: refused
    # before any kernel is launched (the list arrays are never read)
    P_big = pod.POD_STATIC_SCRATCH_BYTES // 8
    with pytest.raises(pod.PodError) as e:
        pod.pod_energy_forces_noalloc(m.h, nb.N, P_big, x, w.cell, nb.offsets, nb.nbr_j, nb.shift, c,
                                      o["E_atom"], o["E"], o["F"], o["W"], o["G"])
    assert "POD_ETOOBIG" in str(e.value)
    pod.pod_check(m.h)
