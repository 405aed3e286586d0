"""Host logic of libpod under AddressSanitizer and UndefinedBehaviorSanitizer,
on the CPU: tests/host_driver.cpp and csrc/pod_plan.cpp (parameter
validation, the POD basis, pod_strerror, neighbour-list bin geometry, the
batch-assembly plan) built with g++ -fsanitize=address,undefined and run on
valid and malformed inputs.  Any sanitizer report aborts the driver
(-fno-sanitize-recover), so a clean exit means no report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2212_14446_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
@pytest.mark.parametrize("opt", ["-O0", "-O2"])
def test_host_logic_under_asan_ubsan(tmp_path, opt):
    exe = str(tmp_path / "host_driver")
    cmd = ["g++", "-std=c++17", opt, "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-o", exe, os.path.join(ROOT, "tests", "host_driver.cpp"), os.path.join(CSRC, "pod_plan.cpp")]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:halt_on_error=1:detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out
    assert "all checks passed" in r.stdout
    assert "runtime error" not in out and "AddressSanitizer" not in out and "LeakSanitizer" not in out
