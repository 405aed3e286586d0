"""Benchmark: atoms/s of POD energies + forces on one MI355X.

One step = one pod_energy_forces call on the 15,840-atom BCC box (20^3 cells,
1% vacancies, sigma 0.15 A, rcut 5 A, L = 8 snapshots -> K = 6, angular
degree 4, 2/3/4-body, M = 103): radial basis, atomic basis, 2/3/4-body
contractions, energies, adjoint, per-pair gradients, force scatter, virial
and global descriptors, with inputs already resident in HBM.

Prints one JSON line (rank 0).  Extra objects: ``roofline`` for the main
per-atom kernel (timed with HIP events inside the library, on its stream),
``cpu_baseline`` (the FP64 oracle on the host, single thread), ``f32``
(the same workload on the FP32 path), ``batch`` (the batched
descriptor-matrix assembly of 2,000 uneven cells with dG/dR, FP64, at the
autotuner's launch shape), ``rcut6`` (the same box at rcut 6 A, ~56 pairs
per atom), ``autograd`` (the differentiable energy on the 54,000-atom box,
FP32, forward + backward), ``neighbors`` (the device neighbour-list build,
outside the step), ``md`` (velocity-Verlet dynamics on the same box with the
device skin list, per step and per atom-step), ``opod_vs_fast`` (the paper's cost comparison: exclusive-sum
2/3-body energy + forces and exclusive 4-body descriptors against the fast
forms at the Table 6 sizes) and ``surrogate`` (the 4-body network surrogate:
trained on the exact 4-body energies of 19 displaced 54,000-atom boxes, then
timed and scored against exact FP32 2/3/4-body energies and forces on a
1,024,000-atom box, beside the 2/3-body model without it).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "atoms/s for POD energy+forces (FP64/FP32) and MLP-surrogate speedup at fixed RMSE"
PEAK_F64 = 78.6e12    # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz, FP64 vector
PEAK_F32 = 157.3e12   # published FP32 vector peak (packed); unpacked issue gives 78.6e12
KERNEL_SOURCES = ["paper_2212_14446_amd/csrc/pod_kernels.hip", "paper_2212_14446_amd/csrc/pod_tables.h",
                  "paper_2212_14446_amd/csrc/pod_device.h", "paper_2212_14446_amd/csrc/pod_internal.h",
                  "paper_2212_14446_amd/csrc/pod_wide.h", "paper_2212_14446_amd/csrc/pod_net.h"]


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_traffic(dtype, kernel="atom_kernel"):
    """HBM bytes per launch of one kernel of the energy path from the
    committed counter summary, if it was taken on the current kernel source;
    else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_bcc20_15840.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith(("|", "#", " ")):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_hash") != kernel_hash():
        return None
    v = vals.get(f"{dtype}_bytes_per_launch")
    return None if v is None else int(v)


def on_stream(fn):
    """Run a leg on a dedicated HIP stream: handles bind to torch's current
    stream at creation, so the library, every allocation and the timing
    events share it (the legacy default stream adds implicit
    synchronisation to every launch)."""
    def wrapped(*a, **k):
        import torch
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            return fn(*a, **k)
    return wrapped


@on_stream
def run_gpu(w, dtype, steps, warmup):
    import torch
    from paper_2212_14446_amd import pod

    m = pod.PodModel(pod.setup_from_workload(w.setup), dtype)
    tdt = m.torch_dtype
    nb = pod.DeviceNeighbors.from_list(w.nl)
    pos = torch.as_tensor(w.pos, dtype=tdt, device="cuda").contiguous()
    c = torch.as_tensor(w.c, dtype=tdt, device="cuda").contiguous()
    N = w.N
    out = {"E": torch.empty(1, dtype=torch.float64, device="cuda"),
           "E_atom": torch.empty(N, dtype=tdt, device="cuda"),
           "F": torch.empty((N, 3), dtype=tdt, device="cuda"),
           "W": torch.empty((3, 3), dtype=torch.float64, device="cuda"),
           "G": torch.empty(m.M, dtype=torch.float64, device="cuda")}
    cell = w.cell

    # the reverse-pair index belongs to the neighbour list (built once per
    # list, outside the timed region, like the list itself)
    nb.build_reverse(m)

    def step():
        pod.pod_energy_forces(m.h, N, nb.P, pos, cell, nb.offsets, nb.nbr_j, nb.shift, c,
                              out["E_atom"], out["E"], out["F"], out["W"], out["G"], rev=nb.rev)

    for _ in range(warmup):
        step()
    m.check()
    stream = torch.cuda.current_stream()

    def timed_pass(kernel_events):
        # kernel_events: the library records HIP events around each of its
        # launches on its stream (per-kernel durations); they add a few us
        # per step, so throughput comes from a pass without them
        if kernel_events:
            pod.pod_set_kernel_timing(m.h, steps)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    total_ms = timed_pass(False)
    ev_ms = timed_pass(True)
    kms, kn = pod.pod_get_kernel_time(m.h, 1)
    gms, gn = pod.pod_get_kernel_time(m.h, 4)
    pms, pn = pod.pod_get_kernel_time(m.h, 0)
    pod.pod_set_kernel_timing(m.h, 0)
    m.check()
    return {"ms_per_step": total_ms / steps, "kernel_ms": kms / max(kn, 1), "kernel_launches": kn,
            "pair_kernel_ms": gms / max(gn, 1), "pair_kernel_launches": gn,
            "finalize_kernel_ms": pms / max(pn, 1), "ms_per_step_with_kernel_events": ev_ms / steps,
            "E": float(out["E"].item())}


def _relerr(x, ref):
    """Normwise relative error max|x - ref| / max|ref| (host float64)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = float(np.max(np.abs(ref))) if ref.size else 0.0
    num = float(np.max(np.abs(x - ref))) if ref.size else 0.0
    return num / den if den > 0 else num


def _colerr(D, ref):
    """Worst per-column normwise relative error of a descriptor matrix."""
    return max(_relerr(D[:, k], ref[:, k]) for k in range(ref.shape[1]))


@on_stream
def precision_errors(pos, cell, nl, setup, c, descriptors=True):
    """FP32 path against the FP64 path on the same inputs (positions and
    coefficients rounded to FP32 first, so only the arithmetic differs):
    normwise relative error of E, E_atom, F, W, G and, per column, D.  The
    FP64 path is the reference: its own parity with the FP64 oracle is
    1e-10 (tests/test_gpu_workloads.py)."""
    import torch

    from paper_2212_14446_amd import pod
    pos32 = np.asarray(pos, dtype=np.float32).astype(np.float64)
    c32 = np.asarray(c, dtype=np.float32).astype(np.float64)
    nb = pod.DeviceNeighbors.from_list(nl)
    res = {}
    for dt in ("f64", "f32"):
        m = pod.PodModel(pod.setup_from_workload(setup), dt)
        nb.build_reverse(m)
        o = m.energy_forces(pos32, cell, nb, c32)
        r = {k: (v.double().cpu().numpy() if k != "E" else float(v.item())) for k, v in o.items()}
        if descriptors:
            r["D"] = m.descriptors(pos32, cell, nb).double().cpu().numpy()
        res[dt] = r
        del m
    a, b = res["f32"], res["f64"]
    out = {"E": abs(a["E"] - b["E"]) / abs(b["E"]), "E_atom": _relerr(a["E_atom"], b["E_atom"]),
           "F": _relerr(a["F"], b["F"]), "W": _relerr(a["W"], b["W"]), "G": _relerr(a["G"], b["G"])}
    if descriptors:
        out["D_worst_column"] = _colerr(a["D"], b["D"])
    out["definition"] = ("normwise max|x32 - x64| / max|x64| per output (D per column, worst column), "
                         "both paths on the same FP32-rounded inputs")
    return out


def roofline(w, r, dtype, traffic=True):
    """Roofline of the energy path's two main kernels from the algorithmic
    flop model in paper_2212_14446_amd.flops: the per-atom kernel (radial
    basis and R, atomic basis, contractions, energy, adjoint rows) and the
    pair kernel (R', monomials, pair gradients, virial).  The headline
    object is the dominant (longer) kernel; both are listed, with the
    finalize kernel's time beside them."""
    from paper_2212_14446_amd import flops as fl
    s = w.setup
    K = max(s.K2, s.K3, s.K4)
    PA = max(s.P3 if s.K3 else 0, s.P4 if s.K4 else 0)
    sp = fl.split_counts(K, s.L, PA, s.P4)
    P, N = w.nl.n_pairs, w.N
    f_atom = sp["atom_per_pair"] * P + sp["per_atom"] * N
    f_pair = sp["pair_per_pair"] * P
    peak = PEAK_F64 if dtype == "f64" else PEAK_F32
    legs = {"atom_kernel": (f_atom, r["kernel_ms"]), "pair_kernel": (f_pair, r["pair_kernel_ms"])}
    dom = max(legs, key=lambda k: legs[k][1])
    f_dom, t_dom = legs[dom]
    achieved = f_dom / (t_dom * 1e-3)
    tr = committed_traffic(dtype, dom) if traffic else None
    both = (f_atom + f_pair) / ((r["kernel_ms"] + r["pair_kernel_ms"]) * 1e-3)
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": tr,
            "hbm_GBps": (tr / (t_dom * 1e-3) / 1e9) if tr else None, "hbm_peak_GBps": 8000.0,
            "kernel": dom, "kernel_ms": t_dom, "flops_per_launch": f_dom,
            "kernels": {k: {"ms": t, "flops_per_launch": f, "achieved_TFLOPs": f / (t * 1e-3) / 1e12 if t else None,
                            "frac": f / (t * 1e-3) / peak if t else None} for k, (f, t) in legs.items()},
            "two_kernels_frac": both / peak,
            "finalize_kernel_ms": r["finalize_kernel_ms"],
            "kernel_timing": f"HIP events around each launch on the library stream, second pass of the same "
                             f"steps ({r['ms_per_step_with_kernel_events']:.4f} ms/step with the events)"}


@on_stream
def run_batch(steps, warmup):
    """Batched assembly of 2,000 cells (2..250 atoms; BCC/FCC/A15/liquid):
    D, G and dG/dR per cell in one launch, FP64, autotuned launch shape."""
    import torch

    from paper_2212_14446_amd import autotune as at, flops as fl, pod, workloads as wl
    b = wl.config3()
    print(f"[bench] batch: {b.n_cfg} cells, N={b.N}, P={b.nl.n_pairs}", file=sys.stderr, flush=True)
    s = b.setup
    m = pod.PodModel(pod.setup_from_workload(s), "f64")
    db = pod.DeviceBatch.from_batch(b)
    tune = at.tune_batch(m, db, reps=2)
    out = None
    for _ in range(warmup):
        out = pod.batch_assemble(m, db, tune=tune, out=out)
    torch.cuda.synchronize()
    pod.pod_set_kernel_timing(m.h, steps)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        pod.batch_assemble(m, db, tune=tune, out=out, check=False)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    kms, kn = pod.pod_get_kernel_time(m.h, 1)
    pod.pod_set_kernel_timing(m.h, 0)
    m.check()
    kms /= max(kn, 1)
    K = max(s.K2, s.K3, s.K4)
    PA = max(s.P3 if s.K3 else 0, s.P4 if s.K4 else 0)
    f = fl.batch_counts(K, s.L, PA, s.P4, s.M, b.nl.n_pairs, b.N)
    ach = f["total"] / (kms * 1e-3)
    rec = {"workload": f"{b.n_cfg} cells, 2..250 atoms, bcc/fcc/a15/liquid, rcut {s.rcut}",
           "cells": b.n_cfg, "atoms": b.N, "pairs": b.nl.n_pairs, "outputs": "D, G, dG/dR (FP64)",
           "ms_per_assembly": ms, "cells_per_s": b.n_cfg / (ms * 1e-3), "atoms_per_s": b.N / (ms * 1e-3),
           "tune": list(tune), "kernel_ms": kms,
           "roofline": {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_F64 / 1e12, "unit": "TFLOP/s",
                        "frac": ach / PEAK_F64, "flops_per_launch": f["total"]}}
    rec["fit"] = run_fit(m, b, out, steps, warmup)
    return rec


def run_fit(m, b, out, steps, warmup):
    """Linear fit (eq. (63a), weights 100 : 1, gamma 1e-12) from the assembled
    matrix: Gram of the 2,000 energy rows and 3N force rows on the FP64 matrix
    cores, then the Cholesky solve.  Labels are seeded synthetic values."""
    import torch

    from paper_2212_14446_amd import pod
    M = m.M
    rng = np.random.default_rng(12)
    E = torch.tensor(rng.normal(size=b.n_cfg), dtype=torch.float64, device="cuda")
    F = torch.tensor(rng.normal(size=3 * b.N), dtype=torch.float64, device="cuda")
    Z = torch.empty((M + 1, M + 1), dtype=torch.float64, device="cuda")
    c = torch.empty(M, dtype=torch.float64, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")

    def step():
        pod.pod_fit_gram(m.h, M, b.n_cfg, out["G"], E, 100.0, 3 * b.N, out["dGdR"], F, 1.0, Z)
        pod.pod_fit_solve(m.h, M, Z, 1e-12, c, loss)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    pod.pod_set_kernel_timing(m.h, steps)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    gms, gn = pod.pod_get_kernel_time(m.h, 3)
    pod.pod_set_kernel_timing(m.h, 0)
    m.check()
    gms /= max(gn, 1)
    rows = b.n_cfg + 3 * b.N
    D = M + 1
    flops = rows * D * (D + 1)          # upper triangle of [A b]^T [A b], FMA = 2
    bytes_ = rows * D * 8               # every row and its label read once
    return {"workload": f"{b.n_cfg} energy rows + {3 * b.N} force rows, M = {M}",
            "ms_per_fit": ms, "gram_kernel_ms": gms,
            "roofline": {"bound": "mfma", "achieved": flops / (gms * 1e-3) / 1e12, "peak": PEAK_F64 / 1e12,
                         "unit": "TFLOP/s", "frac": flops / (gms * 1e-3) / PEAK_F64, "flops_per_launch": flops,
                         "hbm_GBps": bytes_ / (gms * 1e-3) / 1e9, "hbm_peak_GBps": 8000.0,
                         "note": "FP64 matrix-core peak equals the FP64 vector peak on this GPU"}}


PEAK_BF16 = 2.5e15     # dense bfloat16 MFMA peak


@on_stream
def run_autograd(steps, warmup):
    """Differentiable energy on the 54,000-atom box (FP32): one step = forward
    (pod_energy_forces through PodEnergy) + backward (dE/dpos and dE/dc)."""
    import torch

    from paper_2212_14446_amd import autograd, pod, workloads as wl
    w = wl.config4()
    s = w.setup
    m64 = pod.PodModel(pod.setup_from_workload(s), "f64")
    nb = pod.DeviceNeighbors.from_list(w.nl)
    c = wl.standardised_coefficients(m64.descriptors(w.pos, w.cell, nb).cpu().numpy(), s, seed=8)
    m = pod.PodModel(pod.setup_from_workload(s), "f32")
    nb.build_reverse(m)
    x = torch.tensor(w.pos, dtype=torch.float32, device="cuda", requires_grad=True)
    cc = torch.tensor(c, dtype=torch.float32, device="cuda", requires_grad=True)

    def step():
        x.grad = None
        cc.grad = None
        E, W = autograd.pod_energy(x, cc, m, nb, w.cell)
        E.backward()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    m.check()
    ms = e0.elapsed_time(e1) / steps
    return {"workload": f"{w.name}: {w.N} atoms, {w.nl.n_pairs} pairs, FP32",
            "step": "E forward + backward to dE/dpos and dE/dc (torch.autograd.Function)",
            "ms_per_step": ms, "atoms_per_s": w.N / (ms * 1e-3),
            "error_vs_f64": precision_errors(w.pos, w.cell, w.nl, s, c, descriptors=False)}


@on_stream
def run_neighbors(reps, warmup=2):
    """Device neighbour-list build (pod_build_neighbors, a blocking call),
    reported beside the step and not part of it: the 15,840-atom box (FP64)
    and the 1,024,000-atom box (FP32)."""
    from paper_2212_14446_amd import pod, workloads as wl
    out = {}
    w = wl.config2(5.0)
    p, cell = wl.bcc(80)
    big = ("bcc80_1024000_s0.15", wl.displace(p, 0.15, 10), cell, wl.SETUP_CFG5)
    for name, pos, cell, s, dt in ((w.name, w.pos, w.cell, w.setup, "f64"), (*big, "f32")):
        m = pod.PodModel(pod.setup_from_workload(s), dt)
        x = m._pos(pos)
        nb = pod.DeviceNeighbors.build(m, x, cell)
        cap = nb.P
        for _ in range(warmup):
            pod.DeviceNeighbors.build(m, x, cell, capacity=cap)
        t0 = time.perf_counter()
        for _ in range(reps):
            pod.DeviceNeighbors.build(m, x, cell, capacity=cap, check=False)
        ms = (time.perf_counter() - t0) * 1e3 / reps
        m.check()
        out[dt] = {"workload": name, "atoms": int(x.shape[0]), "pairs": nb.P, "ms_per_build": ms,
                   "atoms_per_s": x.shape[0] / (ms * 1e-3)}
    return out


# (L, K2, K3, P3, K4, P4) of the six rows of Table 6 (M3 = 6, 15, 31, 56, 92,
# 141); rows 5 and 6 need K up to 12, so their snapshot family has L = 14
# (12 Bessel + 2 inverse powers)
TABLE6 = [(8, 2, 1, 2, 1, 1), (8, 5, 3, 2, 3, 2), (8, 5, 5, 4, 5, 3), (8, 6, 7, 6, 7, 4),
          (14, 10, 9, 8, 9, 5), (14, 8, 12, 10, 12, 6)]


@on_stream
def run_opod(steps, warmup=3):
    """The paper's cost comparison on the 15,840-atom box (FP64): the
    exclusive-sum 2/3-body model (OPOD, eq. (15b), O(N_i^2) per atom) against
    the fast form (FPOD3, eq. (26a)) for energy + forces, and the exclusive
    4-body descriptors (eq. (20a), O(N_i^3)) against the fast ones (eq. (30a)),
    at the Table 6 sizes."""
    import torch

    from paper_2212_14446_amd import pod, workloads as wl
    w = wl.config2(5.0)
    nb = pod.DeviceNeighbors.from_list(w.nl)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    rows = []
    for (L, K2, K3, P3, K4, P4) in TABLE6:
        s3 = wl.PodSetup(0.5, 5.0, L, K2, K3, 0, P3, 0)
        m3 = pod.PodModel(pod.setup_from_workload(s3), "f64")
        nb.build_reverse(m3)
        c = torch.tensor(wl.coefficients(s3.M, 3), device="cuda")
        x3 = m3._pos(w.pos)
        out = m3.energy_forces(x3, w.cell, nb, c)
        oout = m3.opod_energy_forces(x3, w.cell, nb, c)
        t_fast = timed(lambda: m3.energy_forces(x3, w.cell, nb, c, check=False, out=out))
        t_excl = timed(lambda: m3.opod_energy_forces(x3, w.cell, nb, c, check=False, out=oout))
        m3.check()
        s4 = wl.PodSetup(0.5, 5.0, L, K2, K3, K4, P3, P4)
        m4 = pod.PodModel(pod.setup_from_workload(s4), "f64")
        D = torch.empty((w.N, s4.M), dtype=torch.float64, device="cuda")
        x = m4._pos(w.pos)
        t_d_fast = timed(lambda: pod.pod_descriptors(m4.h, w.N, nb.P, x, w.cell, nb.offsets, nb.nbr_j, nb.shift, D))
        t_d_excl = timed(lambda: pod.pod_opod_descriptors(m4.h, w.N, nb.P, x, w.cell, nb.offsets, nb.nbr_j,
                                                          nb.shift, D))
        m4.check()
        rows.append({"L": L, "K2": K2, "K3": K3, "P3": P3, "M3": s3.M, "fpod3_ef_ms": t_fast, "opod_ef_ms": t_excl,
                     "opod_over_fpod3": t_excl / t_fast, "K4": K4, "P4": P4, "M4": s4.M,
                     "fast_desc4_ms": t_d_fast, "excl_desc4_ms": t_d_excl, "excl_over_fast": t_d_excl / t_d_fast})
        print(f"[bench] opod row {rows[-1]}", file=sys.stderr, flush=True)
    return {"workload": f"{w.name}: {w.N} atoms, {w.nl.n_pairs} pairs, FP64", "rows": rows}


@on_stream
def run_acsf(steps, warmup=3):
    """Atom-centred symmetry functions (eqs. (21c), (22c), (22d)) through the
    atomic basis on the 15,840-atom box: the 34-function set of
    workloads.acsf_standard (8 radial, 18 angular, 8 four-body functions, 11
    radial channels), the functions alone and the forces of E = sum_i W . G_i
    with the functions, FP64 and FP32; per-kernel times from HIP events on
    the leg's stream."""
    import numpy as np
    import torch

    from paper_2212_14446_amd import pod, workloads as wl
    w = wl.config2(5.0)
    spec = wl.acsf_standard()
    setup = wl.PodSetup(w.setup.rin, w.setup.rcut, 6, 2, 2, 0, 2, 0)   # rin, rcut of the box's potential

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    out = {"workload": f"{w.name}: {w.N} atoms, {w.nl.n_pairs} pairs, {spec.n} functions"}
    for dt in ("f64", "f32"):
        m = pod.PodModel(pod.setup_from_workload(setup), dt)
        a = m.acsf(spec)
        nb = pod.DeviceNeighbors.from_list(w.nl)
        nb.build_reverse(m)
        x = m._pos(w.pos)
        G = torch.empty((w.N, a.n), dtype=m.torch_dtype, device="cuda")
        F = torch.empty((w.N, 3), dtype=m.torch_dtype, device="cuda")
        W = torch.tensor(np.random.default_rng(5).normal(size=a.n), dtype=m.torch_dtype, device="cuda")
        args = (w.N, nb.P, x, w.cell, nb.offsets, nb.nbr_j, nb.shift)
        t_d = timed(lambda: pod.pod_acsf_descriptors(m.h, a, *args, G))
        t_f = timed(lambda: pod.pod_acsf_forces(m.h, a, *args, nb.rev, W, 0, F, G))
        pod.pod_set_kernel_timing(m.h, steps)
        for _ in range(steps):
            pod.pod_acsf_forces(m.h, a, *args, nb.rev, W, 0, F, G)
        kb, nkb = pod.pod_get_kernel_time(m.h, 1)
        kp, nkp = pod.pod_get_kernel_time(m.h, 0)
        pod.pod_set_kernel_timing(m.h, 0)
        m.check()
        out[dt] = {"descriptors_ms": t_d, "forces_ms": t_f, "descriptors_atoms_per_s": w.N / (t_d * 1e-3),
                   "forces_atoms_per_s": w.N / (t_f * 1e-3), "basis_kernels_ms": kb / steps,
                   "pair_and_gather_ms": kp / steps}
        print(f"[bench] acsf {dt} {out[dt]}", file=sys.stderr, flush=True)
    return out


@on_stream
def run_five(steps, warmup=3):
    """Five-body descriptors (the extension of Sec. II.F to body order five)
    on the 15,840-atom box with the box's radial basis (K = 6): P5 = 2 (5
    orbits) and P5 = 4 (22 orbits) per radial function, and the energy and
    forces of c5 . D5 at P5 = 4, FP64 and FP32; kernel times from HIP events
    on the leg's stream."""
    import numpy as np
    import torch

    from paper_2212_14446_amd import pod, workloads as wl
    w = wl.config2(5.0)
    out = {"workload": f"{w.name}: {w.N} atoms, {w.nl.n_pairs} pairs, K5 = 6"}
    for dt in ("f64", "f32"):
        m = pod.PodModel(pod.setup_from_workload(w.setup), dt)
        nb = pod.DeviceNeighbors.from_list(w.nl)
        x = m._pos(w.pos)
        for P5 in (2, 4):
            n = pod.pod_five_body_count(P5)
            D5 = torch.empty((w.N, 6 * n), dtype=m.torch_dtype, device="cuda")
            call = lambda: pod.pod_five_body_descriptors(m.h, w.N, nb.P, x, w.cell, nb.offsets, nb.nbr_j, nb.shift,
                                                         6, P5, D5)
            for _ in range(warmup):
                call()
            pod.pod_set_kernel_timing(m.h, steps)
            for _ in range(steps):
                call()
            kms, kn = pod.pod_get_kernel_time(m.h, 1)
            pms, pn = pod.pod_get_kernel_time(m.h, 0)
            pod.pod_set_kernel_timing(m.h, 0)
            m.check()
            t = kms / max(kn, 1) + pms / max(pn, 1)
            out[f"{dt}_P5_{P5}"] = {"descriptors": 6 * n, "kernel_ms": t, "pair_record_ms": pms / max(pn, 1),
                                    "five_body_ms": kms / max(kn, 1), "atoms_per_s": w.N / (t * 1e-3)}
            print(f"[bench] five-body {dt} P5={P5} {out[f'{dt}_P5_{P5}']}", file=sys.stderr, flush=True)
        # energy and forces of c5 . D5 at P5 = 4
        n = pod.pod_five_body_count(4)
        nb.build_reverse(m)
        c5 = torch.tensor(np.random.default_rng(3).normal(size=6 * n) * 1e-3, dtype=m.torch_dtype, device="cuda")
        E_atom = torch.empty(w.N, dtype=m.torch_dtype, device="cuda")
        F = torch.empty((w.N, 3), dtype=m.torch_dtype, device="cuda")
        call = lambda: pod.pod_five_body_energy_forces(m.h, w.N, nb.P, x, w.cell, nb.offsets, nb.nbr_j, nb.shift,
                                                       nb.rev, 6, 4, c5, E_atom, F)
        for _ in range(warmup):
            call()
        pod.pod_set_kernel_timing(m.h, steps)
        for _ in range(steps):
            call()
        kms, kn = pod.pod_get_kernel_time(m.h, 1)
        pms, pn = pod.pod_get_kernel_time(m.h, 0)
        pod.pod_set_kernel_timing(m.h, 0)
        m.check()
        t = (kms + pms) / steps   # all timed intervals of the calls: records, basis, gradients + gather
        out[f"{dt}_P5_4_energy_forces"] = {"kernel_ms": t, "atoms_per_s": w.N / (t * 1e-3)}
        print(f"[bench] five-body {dt} E+F {out[f'{dt}_P5_4_energy_forces']}", file=sys.stderr, flush=True)
    return out


@on_stream
def run_md(steps, dtype="f64", T=300.0, dt=1.0):
    """NVE molecular dynamics on the 15,840-atom box (the use by which the
    paper prices its potentials, Fig. 4): velocity Verlet with the 2/3/4-body
    model of the main leg (synthetic coefficients standardised on the box's
    descriptors and scaled to a gentle potential), Maxwell-Boltzmann
    velocities at T, skin list built and
    rebuilt on the device.  Reported per step and per atom-step."""
    import torch

    from paper_2212_14446_amd import md, pod, workloads as wl
    w = wl.config2(5.0)
    m = pod.PodModel(pod.setup_from_workload(w.setup), dtype)
    kB = 8.617333262e-5   # eV / K
    acc = 1.602176634e-19 / 1e-10 / 1.66053906660e-27 * 1e-20
    rng = np.random.default_rng(21)
    vel = rng.normal(0.0, np.sqrt(kB * T * acc / md.MASS_TA), size=w.pos.shape)
    vel -= vel.mean(0)
    nb0 = pod.DeviceNeighbors.from_list(w.nl)
    D = m.descriptors(w.pos, w.cell, nb0).double().cpu().numpy()
    c = 0.02 * wl.standardised_coefficients(D, w.setup, seed=8)   # forces below ~0.2 eV/A
    dyn = md.MD(m, w.pos, vel, w.cell, c, skin=0.4)   # fastest of 0.2-0.5 A at chunks of 10 and 20
    dyn.run(20, chunk=20, dt=dt)                 # warm-up
    torch.cuda.synchronize()
    r0 = dyn.rebuilds
    t0 = time.perf_counter()
    ep, ek = dyn.run(steps, chunk=20, dt=dt)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    et = (ep + ek).cpu().numpy()
    err = precision_errors(w.pos, w.cell, w.nl, w.setup, c, descriptors=False) if dtype == "f32" else None
    return {"force_error_vs_f64_first_step": err,
            "workload": f"{w.name}: {w.N} atoms, {dtype.upper()}, {T:g} K, dt {dt:g} fs, skin 0.4 A",
            "steps": steps, "ms_per_step": ms, "s_per_atom_step": ms * 1e-3 / w.N,
            "atom_steps_per_s": w.N / (ms * 1e-3), "rebuilds": dyn.rebuilds - r0,
            "energy_drift_eV_per_atom": float(np.abs(et - et[0]).max() / w.N)}


@on_stream
def run_surrogate(steps, epochs=30):
    """Config-5 experiment, all on the device through the library, for two
    exact models: 2/3/4-body at P3 = P4 = 4, and the same 2/3-body part with
    4-body terms up to degree 6 (P4 > P3), where the exact atomic basis grows
    from 35 to 84 monomials while the surrogate keeps the degree-4 one (its
    network trained for four times the epochs, against the larger 4-body
    energies).  The training boxes and the 1,024,000-atom box are built once
    for both."""
    import torch

    from paper_2212_14446_amd import pod, surrogate, workloads as wl
    t0 = time.perf_counter()
    boxes = [(p, cl, nl) for p, cl, nl, _ in wl.config5_train_boxes()]
    w = wl.config5_infer()
    t_lists = time.perf_counter() - t0
    nb = pod.DeviceNeighbors.from_list(w.nl)
    pos = torch.tensor(w.pos, dtype=torch.float32, device="cuda")
    nb.build_reverse(pod.PodModel(pod.setup_from_workload(wl.SETUP_CFG5_23), "f32"))

    def timed(fn, model):
        o = fn()
        torch.cuda.synchronize()
        pod.pod_set_kernel_timing(model.h, steps)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        kt = {k: pod.pod_get_kernel_time(model.h, k) for k in (0, 1, 2, 4)}
        pod.pod_set_kernel_timing(model.h, 0)
        model.check()
        return o, e0.elapsed_time(e1) / steps, {k: (v[0] / v[1] if v[1] else 0.0) for k, v in kt.items()}

    rm = lambda a, b: float(torch.sqrt(((a.double() - b.double()) ** 2).mean()))
    out = {"workload": f"{w.name}: {w.N} atoms, {w.nl.n_pairs} pairs, FP32", "neighbour_lists_s": t_lists}
    for label, S, S23, epochs in (("P3=4,P4=4", wl.SETUP_CFG5, wl.SETUP_CFG5_23, epochs),
                                  ("P3=4,P4=6", wl.SETUP_CFG5_P6, wl.SETUP_CFG5_23, 4 * epochs)):
        n_in = S23.M - 1
        m23 = pod.PodModel(pod.setup_from_workload(S23), "f32")
        m64 = pod.PodModel(pod.setup_from_workload(S), "f64")
        nb0 = pod.DeviceNeighbors.from_list(boxes[0][2])
        c = wl.standardised_coefficients(m64.descriptors(boxes[0][0], boxes[0][1], nb0).cpu().numpy(), S, seed=9)
        t0 = time.perf_counter()
        in64 = None if S23.P3 == S.P3 else pod.PodModel(pod.setup_from_workload(S23), "f64")
        X, T = surrogate.four_body_dataset(m64, boxes, c, n_in, input_model=in64)
        del in64
        t_data = time.perf_counter() - t0
        net = surrogate.Network(n_in, seed=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist = surrogate.fit(m23.h, net, X, T, epochs=epochs, batch=8192, lr=3e-3, seed=2)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        y, _ = net.forward(m23.h, X, grad=False)
        e_train = float(torch.sqrt(((y - T) ** 2).mean()))
        print(f"[bench] surrogate {label}: trained on {X.shape[0]} environments in {t_train:.2f} s "
              f"(labels {t_data:.1f} s), energy rmse {e_train:.4f} eV", file=sys.stderr, flush=True)
        del X, T, y
        m32 = pod.PodModel(pod.setup_from_workload(S), "f32")
        c23 = wl.embed_23_coefficients(c, S, S23)
        ex, t_ex, k_ex = timed(lambda: m32.energy_forces(pos, w.cell, nb, c, virial=False, global_desc=False,
                                                         check=False), m32)
        su, t_su, k_su = timed(lambda: m23.energy_forces_surrogate(pos, w.cell, nb, c23, net, virial=False,
                                                                   check=False), m23)
        n4, t_n4, k_n4 = timed(lambda: m23.energy_forces(pos, w.cell, nb, c23, virial=False, global_desc=False,
                                                          check=False), m23)
        err_exact = precision_errors(w.pos, w.cell, w.nl, S, c, descriptors=False)
        f_net = 2 * (n_in * 64 + 64 * 64 + 64) + 2 * (64 * 64 + 64 * n_in)   # forward + input gradient per atom
        # the network runs inside the surrogate's per-atom kernel: its time is
        # that kernel's minus the same kernel's on the 2/3-body model alone
        net_ms = max(k_su[1] - k_n4[1], 0.0)
        ach = f_net * w.N / (net_ms * 1e-3) if net_ms > 0 else 0.0
        f_rmse = rm(su["F"], ex["F"])
        out[label] = {
            "exact_model": f"K2 = K3 = K4 = 6, P3 = {S.P3}, P4 = {S.P4}, M = {S.M}",
            "surrogate_model": f"2/3-body K2 = K3 = 6, P3 = {S23.P3} ({n_in} inputs) + network {n_in} -> 64 -> 64 -> 1",
            "train": {"environments": sum(len(b[0]) for b in boxes), "boxes": len(boxes), "epochs": epochs,
                      "batch": 8192, "seconds": t_train, "label_seconds": t_data, "energy_rmse_eV": e_train,
                      "final_loss_std_units": hist[-1]},
            "ms_exact": t_ex, "ms_surrogate": t_su, "ms_without_4body": t_n4,
            "speedup_vs_exact": t_ex / t_su, "speedup_ceiling_free_network": t_ex / t_n4,
            "atoms_per_s_exact": w.N / (t_ex * 1e-3), "atoms_per_s_surrogate": w.N / (t_su * 1e-3),
            "force_rmse_eV_per_A": {"surrogate": f_rmse, "without_4body": rm(n4["F"], ex["F"])},
            "force_rmse_target_met": f_rmse <= 0.02,
            "force_std_exact_eV_per_A": float(ex["F"].double().std()),
            "energy_rmse_eV_per_atom": {"surrogate": rm(su["E_atom"], ex["E_atom"]),
                                        "without_4body": rm(n4["E_atom"], ex["E_atom"])},
            "exact_f32_error_vs_f64": err_exact,
            "exact_kernels_ms": {"per_atom_kernel": k_ex[1], "pair_kernel": k_ex[4], "finalize": k_ex[0]},
            "surrogate_kernels_ms": {"per_atom_kernel_with_network": k_su[1],
                                     "per_atom_kernel_2_3_body_alone": k_n4[1], "pair_kernel": k_su[4],
                                     "weight_packing": k_su[2], "finalize": k_su[0]},
            "network_mfma": {"bound": "mfma", "achieved": ach / 1e12, "peak": PEAK_BF16 / 1e12, "unit": "TFLOP/s",
                             "frac": ach / PEAK_BF16, "flops_per_atom": f_net, "network_ms": net_ms}}
        print(f"[bench] surrogate {label}: exact {t_ex:.3f} ms, surrogate {t_su:.3f} ms, without 4-body "
              f"{t_n4:.3f} ms, force rmse {f_rmse:.4f} eV/A", file=sys.stderr, flush=True)
        del m64, m32, m23, net
    return out


def cpu_baseline(w, min_seconds=2.5):
    """The compiled FP64 oracle (oracle/oracle.cpp: fast form, analytic
    forces, OpenMP over atoms) on the host: full energy + forces + virial +
    G passes over the whole box, on every thread this process may use and on
    one thread, each repeated until at least min_seconds of wall time."""
    from oracle import oracle_c, pod_oracle as po
    s = w.setup
    p = po.PodParams(s.rin, s.rcut, *s.snapshot_family(), s.K2, s.K3, s.K4, s.P3, s.P4)
    Q, _ = po.pod_basis(p)
    args = (w.pos, w.cell, w.nl.offsets.astype(np.int64), w.nl.nbr_j, w.nl.shift3, p, Q, w.c)
    oracle_c.lib()

    def timed(threads):
        oracle_c.energy_forces(*args, threads=threads)       # warm-up pass
        n, t0 = 0, time.perf_counter()
        while True:
            oracle_c.energy_forces(*args, threads=threads)
            n += 1
            dt = time.perf_counter() - t0
            if dt >= min_seconds:
                return n, dt

    nth = oracle_c.host_threads()
    n_all, t_all = timed(nth)
    n_one, t_one = timed(1)
    return {"value": n_all * w.N / t_all, "unit": "atoms/s", "cores": nth, "kind": "oracle",
            "sample": f"{n_all} full energy + forces + virial passes over the {w.N}-atom box on {nth} threads "
                      f"(compiled FP64 oracle, g++ -O3 -march=x86-64-v3 -fopenmp); {n_one} passes on 1 thread",
            "seconds": t_all, "single_thread": {"value": n_one * w.N / t_one, "cores": 1, "seconds": t_one},
            "cpu_model": oracle_c.cpu_model()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--rcut", type=float, default=5.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f32", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-rc6", action="store_true")
    ap.add_argument("--no-autograd", action="store_true")
    ap.add_argument("--no-neighbors", action="store_true")
    ap.add_argument("--no-opod", action="store_true")
    ap.add_argument("--no-md", action="store_true")
    ap.add_argument("--no-acsf", action="store_true")
    ap.add_argument("--no-five", action="store_true")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (a known-size "
                         "kernel for scaling hardware traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the spatial decomposition is described in the design notes).", file=sys.stderr)
        sys.exit(2)

    from paper_2212_14446_amd import workloads as wl
    if args.copy_calibration_mb > 0:
        import torch
        n = args.copy_calibration_mb * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: {n * 8} bytes read, {n * 8} bytes written", file=sys.stderr, flush=True)
        del src, dst
    w = wl.config2(args.rcut)
    print(f"[bench] workload {w.name}: N={w.N} P={w.nl.n_pairs} M={w.setup.M}", file=sys.stderr, flush=True)
    r64 = run_gpu(w, "f64", args.steps, args.warmup)
    print(f"[bench] f64 {r64}", file=sys.stderr, flush=True)
    rec = {
        "metric": METRIC,
        "value": w.N / (r64["ms_per_step"] * 1e-3),
        "unit": "atoms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "atoms": w.N, "pairs": w.nl.n_pairs,
                   "pairs_per_atom": w.nl.n_pairs / w.N, "rcut": w.setup.rcut, "L": w.setup.L,
                   "K": max(w.setup.K2, w.setup.K3, w.setup.K4), "P3": w.setup.P3, "P4": w.setup.P4,
                   "M": w.setup.M, "body_orders": "2/3/4"},
        "roofline": roofline(w, r64, "f64"),
    }
    if not args.no_f32:
        r32 = run_gpu(w, "f32", args.steps, args.warmup)
        print(f"[bench] f32 {r32}", file=sys.stderr, flush=True)
        rec["f32"] = {"value": w.N / (r32["ms_per_step"] * 1e-3), "ms_per_step": r32["ms_per_step"],
                      "roofline": roofline(w, r32, "f32"),
                      "error_vs_f64": precision_errors(w.pos, w.cell, w.nl, w.setup, w.c)}
        print(f"[bench] f32 error vs f64 {rec['f32']['error_vs_f64']}", file=sys.stderr, flush=True)
    if not args.no_rc6 and args.rcut != 6.0:
        # the same box at rcut 6 A (the first five BCC shells, ~56 pairs per atom)
        w6 = wl.config2(6.0)
        print(f"[bench] workload {w6.name}: N={w6.N} P={w6.nl.n_pairs}", file=sys.stderr, flush=True)
        rc6 = {"workload": w6.name, "pairs": w6.nl.n_pairs, "pairs_per_atom": w6.nl.n_pairs / w6.N}
        for dt in ("f64", "f32"):
            r6 = run_gpu(w6, dt, args.steps, args.warmup)
            rc6[dt] = {"value": w6.N / (r6["ms_per_step"] * 1e-3), "unit": "atoms/s",
                       "ms_per_step": r6["ms_per_step"], "roofline": roofline(w6, r6, dt, traffic=False)}
        rc6["f32"]["error_vs_f64"] = precision_errors(w6.pos, w6.cell, w6.nl, w6.setup, w6.c)
        rec["rcut6"] = rc6
        print(f"[bench] rcut6 {rc6}", file=sys.stderr, flush=True)
    if not args.no_autograd:
        rec["autograd"] = run_autograd(50, 5)
        print(f"[bench] autograd {rec['autograd']}", file=sys.stderr, flush=True)
    if not args.no_neighbors:
        rec["neighbors"] = run_neighbors(10)
        print(f"[bench] neighbors {rec['neighbors']}", file=sys.stderr, flush=True)
    if not args.no_md:
        rec["md"] = {dt: run_md(200, dt) for dt in ("f64", "f32")}
        print(f"[bench] md {rec['md']}", file=sys.stderr, flush=True)
    if not args.no_opod:
        rec["opod_vs_fast"] = run_opod(20)
    if not args.no_acsf:
        rec["acsf"] = run_acsf(20)
    if not args.no_five:
        rec["five_body"] = run_five(20)
    if not args.no_batch:
        rec["batch"] = run_batch(10, 2)
        print(f"[bench] batch {rec['batch']}", file=sys.stderr, flush=True)
    if not args.no_surrogate:
        rec["surrogate"] = run_surrogate(20)
        print(f"[bench] surrogate {rec['surrogate']}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
