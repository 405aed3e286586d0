"""Register and scratch use of the energy path's benchmark kernel instances
(FP64 and FP32, K = 6, angular degree 4, standard snapshot family), of the
surrogate's per-atom kernel with the network inside, and of the wide-degree
kernels, read from the compiler's resource-usage remarks of a
device-only gfx950 compile of csrc/pod_kernels.hip and csrc/pod_wide.hip with
the library's flags.  The test fails when an
instance spills (scratch above the recorded bound) or loses occupancy, so a
change that pushes a hot kernel into scratch memory is caught on the CPU."""
import shutil

import pytest

from paper_2212_14446_amd import build_lib

# instance: (max scratch bytes per lane, min waves per SIMD, VGPRs when recorded)
RECORDED = {
    "void atom_kernel_occ2<double, 4, 1, true>(KArgs<double>)": (0, 2, 222),
    "void atom_kernel<float, 4, 1, true>(KArgs<float>)": (0, 4, 109),
    "void pair_kernel<double, 4, 6, true>(PArgs<double>)": (0, 4, 128),
    "void pair_kernel<float, 4, 6, true>(PArgs<float>)": (0, 7, 72),
    "void finalize_kernel<double>(FinArgs<double>)": (0, 8, 28),
    "void finalize_kernel<float>(FinArgs<float>)": (0, 8, 28),
    # the surrogate's per-atom kernel with the network inside (FP32 benchmark model)
    "void atom_net_kernel<float, 4, true, 3>(KArgs<float>)": (0, 3, 140),
    "void atom_net_kernel<double, 4, true, 2>(KArgs<double>)": (0, 2, 223),
}


# wide-degree path (degree 7 to 10, K up to 12): no spill in any instance
WIDE_RECORDED = {
    "void wide_kernel<double, 0>(pod::WideArgs<double>)": (0, 4),
    "void wide_kernel<double, 1>(pod::WideArgs<double>)": (0, 2),
    "void wide_kernel<float, 1>(pod::WideArgs<float>)": (0, 2),
}


@pytest.fixture(scope="module")
def resources():
    if not shutil.which(build_lib.hipcc()) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    return build_lib.kernel_resources("pod_kernels.hip")


@pytest.fixture(scope="module")
def wide_resources():
    if not shutil.which(build_lib.hipcc()) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    return build_lib.kernel_resources("pod_wide.hip")


@pytest.mark.parametrize("name", sorted(RECORDED))
def test_benchmark_instance_within_recorded_registers(resources, name):
    assert name in resources, f"instance {name} not compiled"
    max_scratch, min_occ, _ = RECORDED[name]
    r = resources[name]
    assert r["scratch"] <= max_scratch, (name, r)
    assert r["occupancy"] >= min_occ, (name, r)


def test_no_energy_path_instance_spills_much(resources):
    # every instance of the energy path: at most the 20 bytes per lane of the
    # degree-6 FP64 descriptor instance (one wavefront per SIMD, 256 + 256 registers)
    worst = max((r["scratch"], n) for n, r in resources.items())
    assert worst[0] <= 20, worst


@pytest.mark.parametrize("name", sorted(WIDE_RECORDED))
def test_wide_instances_within_recorded_registers(wide_resources, name):
    assert name in wide_resources, f"instance {name} not compiled"
    max_scratch, min_occ = WIDE_RECORDED[name]
    r = wide_resources[name]
    assert r["scratch"] <= max_scratch and r["occupancy"] >= min_occ, (name, r)
    assert max(v["scratch"] for v in wide_resources.values()) == 0
