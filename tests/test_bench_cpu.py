"""Host-side contract of bench.py: more than one GPU is refused with a
message before anything touches a device, and the flop models the roofline
uses are the documented per-pair / per-atom counts."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_flop_model_counts():
    sys.path.insert(0, ROOT)
    from paper_2212_14446_amd import flops as fl
    c = fl.counts(6, 8, 4, 4)
    assert (c["Na"], c["Ga"], c["NT"]) == (35, 60, 121)
    assert c["radial_per_pair"] == 302 and c["forward_per_pair"] == 454 and c["backward_per_pair"] == 1420
    assert c["per_atom"] == 10902
    b = fl.batch_counts(6, 8, 4, 4, 103, 1000, 40)
    assert b["per_pair_column"] == 212
    assert b["derivatives"] == 1000 * (102 * 212 + 6 * 34)


def test_flop_split_between_kernels():
    # the two kernels of the energy path share the per-pair work without
    # double counting: snapshots and R in the atom kernel, R' and the
    # backward sweep in the pair kernel
    sys.path.insert(0, ROOT)
    from paper_2212_14446_amd import flops as fl
    c = fl.counts(6, 8, 4, 4)
    sp = fl.split_counts(6, 8, 4, 4)
    assert sp["atom_per_pair"] + sp["pair_per_pair"] == (c["radial_per_pair"] + c["forward_per_pair"]
                                                         + c["backward_per_pair"])
    assert sp["per_atom"] == c["per_atom"]
    assert sp["pair_per_pair"] == 2 * 8 * 6 + c["backward_per_pair"]

