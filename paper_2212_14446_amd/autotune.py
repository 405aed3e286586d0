"""Autotuner of the batched assembly's launch shape.

pod_batch_assemble takes a pod_tune triple (cw, nblocks, threads):
descriptor columns per dG/dR chunk, persistent workgroups and threads per
workgroup.
The best triple depends on the batch (cell sizes, pair counts) and on the
descriptor set (M, K, angular degree).  This module times a fixed candidate
list through the library (HIP events on the handle's stream), picks the
fastest and keeps the pick in a JSON cache keyed by a signature of the
workload, so that a later run with the same cache makes the same choice
without measuring.

Ties and near-ties are broken deterministically: a candidate must beat the
best one so far by more than `margin` (relative) to replace it, scanning the
candidates in their fixed order.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Callable, Iterable, Sequence

import numpy as np

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "pod_batch_tune.json")

CW = (6, 9, 12, 17)
NBLOCKS = (256, 512, 1024)
THREADS = (256, 512)


def candidates(cw: Iterable[int] = CW, nblocks: Iterable[int] = NBLOCKS, threads: Iterable[int] = THREADS):
    """Fixed, ordered candidate list."""
    return [(c, b, t) for c in cw for b in nblocks for t in threads]


def signature(n_cfg: int, cell_atoms: Sequence[int], cell_pairs: Sequence[int], M: int, K: int, PA: int,
              device: str = "") -> str:
    """Cache key: the descriptor set and a coarse summary of the batch (cell
    count, totals, largest cell, a histogram of cell sizes)."""
    a = np.asarray(cell_atoms, dtype=np.int64)
    p = np.asarray(cell_pairs, dtype=np.int64)
    hist = np.histogram(a, bins=8, range=(0, max(int(a.max(initial=0)), 1) + 1))[0] if a.size else []
    desc = {"n_cfg": int(n_cfg), "N": int(a.sum()), "P": int(p.sum()), "max_atoms": int(a.max(initial=0)),
            "max_pairs": int(p.max(initial=0)), "hist": [int(x) for x in hist], "M": int(M), "K": int(K),
            "PA": int(PA), "device": device}
    return hashlib.sha1(json.dumps(desc, sort_keys=True).encode()).hexdigest()[:16]


def load_cache(path: str) -> dict:
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(path: str, data: dict) -> None:
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def pick(times: Sequence[float], cands: Sequence[tuple], margin: float = 0.02) -> tuple:
    """Fastest candidate; a later one must be faster by more than `margin`."""
    best, best_t = None, None
    for c, t in zip(cands, times):
        if t is None or not np.isfinite(t):
            continue
        if best is None or t < best_t * (1.0 - margin):
            best, best_t = tuple(int(x) for x in c), float(t)
    if best is None:
        raise RuntimeError("no candidate could be timed")
    return best


def tune(key: str, measure: Callable[[tuple], float], cache_path: str | None = DEFAULT_CACHE,
         cands: Sequence[tuple] | None = None, margin: float = 0.02) -> tuple:
    """The cached pick for `key`, else measure every candidate (measure(c)
    returns seconds, or None when the launch shape is refused), pick and
    store."""
    cands = candidates() if cands is None else list(cands)
    data = load_cache(cache_path) if cache_path else {}
    hit = data.get(key)
    if hit is not None and isinstance(hit.get("tune"), list) and len(hit["tune"]) == 3:
        return tuple(int(x) for x in hit["tune"])
    times = [measure(c) for c in cands]
    best = pick(times, cands, margin)
    if cache_path:
        data = load_cache(cache_path)
        data[key] = {"tune": list(best), "times_us": {",".join(map(str, c)): (None if t is None else 1e6 * t)
                                                      for c, t in zip(cands, times)}}
        save_cache(cache_path, data)
    return best


# --------------------------------------------------------------------------
# Library-facing part (needs the GPU)
# --------------------------------------------------------------------------
def batch_signature(model, batch) -> str:
    """Signature of a pod.DeviceBatch for a pod.PodModel."""
    import torch
    off = batch.cfg_atom_off.cpu().numpy().astype(np.int64)
    aoff = batch.nbrs.offsets.cpu().numpy().astype(np.int64)
    atoms = np.diff(off)
    pairs = aoff[off[1:]] - aoff[off[:-1]]
    s = model.setup
    PA = max(s.P3 if s.K3 > 0 else 0, s.P4 if s.K4 > 0 else 0)
    dev = torch.cuda.get_device_name(model.device) if torch.cuda.is_available() else ""
    return signature(batch.n_cfg, atoms, pairs, model.M, max(s.K2, s.K3, s.K4), PA, dev)


def measure_batch(model, batch, reps: int = 3, outputs=None):
    """A measure(c) for tune(): mean kernel time of pod_batch_assemble with
    launch shape c (one untimed warm-up call, then `reps` timed calls)."""
    from . import pod
    o = outputs

    def run(c):
        nonlocal o
        try:
            o = pod.batch_assemble(model, batch, tune=c, check=False, out=o)
            pod.pod_check(model.h)
            pod.pod_set_kernel_timing(model.h, reps)
            for _ in range(reps):
                pod.batch_assemble(model, batch, tune=c, check=False, out=o)
            ms, n = pod.pod_get_kernel_time(model.h, 1)
            pod.pod_set_kernel_timing(model.h, 0)
        except pod.PodError:
            pod.pod_set_kernel_timing(model.h, 0)
            return None
        return ms * 1e-3 / max(n, 1)

    return run


def tune_batch(model, batch, cache_path: str | None = DEFAULT_CACHE, cands=None, reps: int = 3) -> tuple:
    """Launch shape for pod_batch_assemble on this batch (cached)."""
    key = batch_signature(model, batch)
    return tune(key, measure_batch(model, batch, reps), cache_path, cands)
