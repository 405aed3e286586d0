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



def test_embedded_two_three_body_coefficients_reproduce_the_model_energy():
    """The surrogate's exact part: a model's constant, 2- and 3-body
    coefficients placed in the layout of a 2/3-body setup with a higher
    3-body degree give, through the oracle, the model's energy with its
    4-body coefficients set to zero."""
    import numpy as np

    from oracle import pod_oracle as po
    from paper_2212_14446_amd import workloads as wl
    S = wl.PodSetup(rin=0.5, rcut=5.0, L=6, K2=3, K3=2, K4=2, P3=2, P4=3)
    S23 = wl.PodSetup(rin=0.5, rcut=5.0, L=6, K2=3, K3=2, K4=0, P3=4, P4=0)
    mk = lambda s: po.PodParams(s.rin, s.rcut, *s.snapshot_family(), s.K2, s.K3, s.K4, s.P3, s.P4)
    p, p23 = mk(S), mk(S23)
    Q, _ = po.pod_basis(p, n_quad=400)
    pos, cell = wl.bcc(1)
    pos = wl.displace(pos, 0.2, 7)
    off, nj, sh = po.neighbors_bruteforce(pos, cell, p.rcut)
    c = np.random.default_rng(3).normal(size=S.M)
    c23 = wl.embed_23_coefficients(c, S, S23)
    assert c23.shape == (S23.M,)
    c_no4 = c.copy()
    c_no4[1 + S.K2 + S.K3 * (S.P3 + 1):] = 0.0
    e_ref = po.total_energy(pos, cell, off, nj, sh, p, Q, c_no4)
    e_23 = po.total_energy(pos, cell, off, nj, sh, p23, Q, c23)
    assert abs(e_23 - e_ref) <= 1e-12 * max(1.0, abs(e_ref))
    with __import__("pytest").raises(ValueError):
        wl.embed_23_coefficients(c, S, wl.PodSetup(rin=0.5, rcut=5.0, L=6, K2=3, K3=2, K4=0, P3=1, P4=0))
