"""Loader of the compiled FP64 CPU oracle (oracle/oracle.cpp).

Test infrastructure, not product code: only the tests, the smoke check and
the benchmark's CPU-baseline leg use it.  It computes what
oracle.pod_oracle.energy_forces computes (the fast atom-density form with
analytic forces, arXiv:2212.14446 Sec. II.E-II.G and Sec. IV.A), compiled
with OpenMP over atoms, so that the CPU baseline runs at compiled speed on
every host core.  Built with g++ -O3 for x86-64-v3 (AVX2 and FMA, which both
the container's and the GPU host's CPUs have) and -fopenmp; no fast-math.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")
CXXFLAGS = ["-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared", "-std=c++17"]

_lib = None


def build(verbose: bool = False) -> str:
    """Compile oracle.cpp into liboracle.so next to it."""
    tmp = LIB + ".tmp"
    cmd = ["g++", *CXXFLAGS, "-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    L = ctypes.CDLL(LIB)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    L.pod_oracle_energy_forces.argtypes = [i, vp, vp, vp, vp, vp, d, d, i, vp, vp, vp, vp, i, i, i, i, i, vp, i,
                                           vp, i, vp, vp, vp, vp, vp]
    L.pod_oracle_energy_forces.restype = i
    _lib = L
    return L


def host_threads() -> int:
    """Threads this process may use: the CPU affinity set, capped by
    OMP_NUM_THREADS when it is set."""
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return n


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def energy_forces(pos, cell, offsets, nbr_j, shift3, p, Q, c, threads: int = 1):
    """E_atom [N], E, G [M], F [N, 3], W [3, 3] of the linear POD model.
    p: oracle.pod_oracle.PodParams; Q: [L, >= K] POD basis; shift3: [P, 3]."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    N = pos.shape[0]
    cellv = None if cell is None else np.ascontiguousarray(cell, dtype=np.float64).reshape(9)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    nj = np.ascontiguousarray(nbr_j, dtype=np.int32)
    sh = np.ascontiguousarray(shift3, dtype=np.int32).reshape(-1, 3)
    Qm = np.ascontiguousarray(Q, dtype=np.float64)
    cv = np.ascontiguousarray(c, dtype=np.float64)
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (p.alpha, p.beta, p.gamma, p.kappa)]
    M = cv.shape[0]
    E_atom = np.zeros(N)
    E = np.zeros(1)
    G = np.zeros(M)
    F = np.zeros((N, 3))
    W = np.zeros(9)
    ptr = lambda a: None if a is None else a.ctypes.data
    rc = lib().pod_oracle_energy_forces(
        N, ptr(pos), ptr(cellv), ptr(off), ptr(nj), ptr(sh), float(p.rin), float(p.rcut), int(p.L),
        *(ptr(a) for a in arrs), int(p.K2), int(p.K3), int(p.K4), int(p.P3), int(p.P4), ptr(Qm), int(Qm.shape[1]),
        ptr(cv), int(threads), ptr(E_atom), ptr(E), ptr(G), ptr(F), ptr(W))
    if rc == -1:
        raise ValueError("a pair distance outside (rin, rcut) or non-finite")
    if rc != 0:
        raise ValueError(f"oracle error {rc}")
    return {"E_atom": E_atom, "E": float(E[0]), "G": G, "F": F, "W": W.reshape(3, 3)}
