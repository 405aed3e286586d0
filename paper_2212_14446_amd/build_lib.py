"""Build libpod.so (HIP, gfx950) in-tree with hipcc.

Every source is compiled to an object of its own (in parallel, under
``_build/``) and the objects are linked into ``libpod.so``.  Each object
carries the code of its own kernels, so no relocatable device code is needed.

Usage: python -m paper_2212_14446_amd.build_lib [extra hipcc flags]
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libpod.so")
OBJDIR = os.path.join(ROOT, "_build")

SOURCES = ["pod_host.cpp", "pod_plan.cpp", "pod_kernels.hip", "pod_batch.hip", "pod_mlp.hip", "pod_neighbors.hip",
           "pod_fit.hip", "pod_opod.hip", "pod_md.hip", "pod_acsf.hip", "pod_five.hip", "pod_wide.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++20",
    "-fPIC",
    # packed FP32 instructions are kept out of every HIP code object
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # hardware FP atomics for the force scatter (device memory from hipMalloc)
    "-munsafe-fp-atomics",
    "-fconstexpr-steps=50000000",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def _jobs() -> int:
    for var in ("MAX_JOBS", "CMAKE_BUILD_PARALLEL_LEVEL"):
        v = os.environ.get(var)
        if v and v.isdigit() and int(v) > 0:
            return min(int(v), 16)
    return max(1, min(os.cpu_count() or 1, 16))


def kernel_resources(src: str = "pod_kernels.hip") -> dict:
    """Register and scratch use of every kernel instance of one source, from
    the compiler's resource-usage remarks of a device-only gfx950 compile
    with the library's flags: {demangled name: {"vgpr", "agpr", "scratch"
    (bytes per lane), "occupancy" (waves per SIMD)}}."""
    import re
    import tempfile
    with tempfile.TemporaryDirectory() as td:
        cmd = [hipcc(), *HIPCC_FLAGS, "--offload-device-only", "-Rpass-analysis=kernel-resource-usage",
               "-I", INCLUDE, "-I", CSRC, "-c", "-o", os.path.join(td, "k.o"), os.path.join(CSRC, src)]
        r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compilation of {src} failed:\n{r.stderr[-4000:]}")
    rows, cur = [], None
    keys = {"VGPRs:": "vgpr", "AGPRs:": "agpr", "ScratchSize [bytes/lane]:": "scratch",
            "Occupancy [waves/SIMD]:": "occupancy"}
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = {"mangled": m.group(1)}
            rows.append(cur)
            continue
        for k, name in keys.items():
            if cur is not None and k in line:
                cur[name] = int(line.split(k)[1].split()[0])
    names = subprocess.run(["c++filt"], input="\n".join(r_["mangled"] for r_ in rows), capture_output=True,
                           text=True, check=True).stdout.splitlines()
    out = {}
    for row, name in zip(rows, names):
        name = name.replace("pod::(anonymous namespace)::", "")
        out[name] = {k: row.get(k) for k in keys.values()}
    return out


def build(verbose: bool = True, extra=None, out: str = LIB) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    extra = list(extra or [])

    def compile_one(src):
        obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc(), *HIPCC_FLAGS, *extra, "-I", INCLUDE, "-I", CSRC, "-c", "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        return src, obj, r

    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        results = list(ex.map(compile_one, SOURCES))
    failed = [(s, r) for s, _, r in results if r.returncode != 0]
    for s, _, r in results:
        msg = "\n".join(l for l in (r.stderr or "").splitlines() if "packed-fp32-ops" not in l)
        if msg.strip() and (verbose or r.returncode != 0):
            print(f"--- {s}\n{msg}", file=sys.stderr, flush=True)
    if failed:
        raise RuntimeError("compilation failed: " + ", ".join(s for s, _ in failed))
    tmp = out + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *(o for _, o, _ in results)]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(extra=sys.argv[1:])
