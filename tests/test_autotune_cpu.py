"""Host logic of the batched-assembly autotuner: the pick is the fastest
candidate with deterministic tie-breaking, it is cached under the workload
signature, and a cached pick is returned without measuring."""
import json

import numpy as np
import pytest

from paper_2212_14446_amd import autotune as at


def test_candidates_fixed_order():
    c = at.candidates()
    assert len(c) == len(at.CW) * len(at.NBLOCKS) * len(at.THREADS)
    assert c == at.candidates()
    assert c[0] == (at.CW[0], at.NBLOCKS[0], at.THREADS[0])


def test_pick_fastest_and_ties():
    cands = [(1, 1, 1), (2, 2, 2), (3, 3, 3)]
    assert at.pick([3.0, 1.0, 2.0], cands) == (2, 2, 2)
    # within the margin the earlier candidate stays
    assert at.pick([1.0, 0.99, 1.5], cands, margin=0.02) == (1, 1, 1)
    assert at.pick([1.0, 0.97, 1.5], cands, margin=0.02) == (2, 2, 2)
    # refused launch shapes (None) are skipped
    assert at.pick([None, 2.0, float("nan")], cands) == (2, 2, 2)
    with pytest.raises(RuntimeError):
        at.pick([None, None, None], cands)


def test_signature_depends_on_workload():
    a = at.signature(3, [2, 10, 250], [20, 200, 6000], 103, 6, 4)
    assert a == at.signature(3, [2, 10, 250], [20, 200, 6000], 103, 6, 4)
    assert a != at.signature(3, [2, 10, 249], [20, 200, 6000], 103, 6, 4)
    assert a != at.signature(3, [2, 10, 250], [20, 200, 6000], 21, 4, 3)
    assert a != at.signature(3, [2, 10, 250], [20, 200, 6000], 103, 6, 4, device="other")


def test_tune_caches_and_is_deterministic(tmp_path):
    path = str(tmp_path / "tune.json")
    cands = at.candidates(cw=(3, 6), nblocks=(4,), threads=(256, 512))
    calls = []

    def measure(c):
        calls.append(c)
        return {(3, 4, 256): 5.0, (3, 4, 512): 4.0, (6, 4, 256): 3.0, (6, 4, 512): 3.01}[c]

    best = at.tune("k1", measure, path, cands)
    assert best == (6, 4, 256) and len(calls) == len(cands)
    data = json.load(open(path))
    assert data["k1"]["tune"] == [6, 4, 256]

    def never(c):
        raise AssertionError("cached pick must not measure")

    for _ in range(3):
        assert at.tune("k1", never, path, cands) == (6, 4, 256)
    # another key measures again and leaves the first entry alone
    best2 = at.tune("k2", lambda c: float(np.prod(c)), path, cands)
    assert best2 == (3, 4, 256)
    data = json.load(open(path))
    assert data["k1"]["tune"] == [6, 4, 256] and data["k2"]["tune"] == [3, 4, 256]


def test_corrupt_cache_is_ignored(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    best = at.tune("k", lambda c: 1.0 / c[0], str(path), [(1, 1, 1), (2, 1, 1)])
    assert best == (2, 1, 1)
    assert json.load(open(path))["k"]["tune"] == [2, 1, 1]


def test_no_cache_path_measures_each_time():
    n = []
    for _ in range(2):
        at.tune("k", lambda c: n.append(c) or 1.0, None, [(1, 1, 1)])
    assert len(n) == 2
