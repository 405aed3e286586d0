"""Batched descriptor-matrix assembly (Sec. IV.A, eqs. (58a), (63a)) through
pod_batch_assemble: per-atom descriptors D, per-cell global descriptors G and
per-cell derivatives dG/dR of many uneven cells in one persistent launch,
FP64, against the oracle (descriptors_fast and global_descriptor_derivatives,
cell by cell) and against the single-system library call."""
import numpy as np
import pytest

from gpu_common import colerr, oracle_params, relerr, say
from oracle import pod_oracle as po
from paper_2212_14446_amd import pod, workloads as wl

pytestmark = pytest.mark.gpu

TOL = 1e-10


class Ref:
    """Oracle parameters and basis of one setup."""

    def __init__(self, setup):
        self.setup = setup
        self.op = oracle_params(setup)
        self.Q, _ = po.pod_basis(self.op)
        self.K = self.op.K

    def model(self):
        return pod.PodModel(pod.setup_from_workload(self.setup), "f64", Q=self.Q[:, : self.K])

    def cell_refs(self, batch, c):
        pos, cell, nl = batch.config(c)
        args = (pos, cell, nl.offsets.astype(np.int64), nl.nbr_j, nl.shift3, self.op, self.Q)
        D = po.descriptors_fast(*args)
        dG = po.global_descriptor_derivatives(*args)          # [N_c, 3, M]
        return D, D.sum(axis=0), dG.reshape(-1, dG.shape[2])


def host(o):
    import torch
    torch.cuda.synchronize()
    return {k: (None if v is None else v.cpu().numpy()) for k, v in o.items()}


def check_cell(batch, got, ref, c):
    a0, a1 = int(batch.cfg_atom_off[c]), int(batch.cfg_atom_off[c + 1])
    D, G, dG = ref.cell_refs(batch, c)
    e = {"D": colerr(got["D"][a0:a1], D), "G": relerr(got["G"][c], G),
         "dGdR": colerr(got["dGdR"][3 * a0:3 * a1], dG)}
    assert np.all(got["dGdR"][3 * a0:3 * a1, 0] == 0.0)
    return e


@pytest.fixture(scope="module")
def ref2():
    return Ref(wl.SETUP_CFG2)


@pytest.fixture(scope="module")
def small_batch():
    return wl.make_batch(24, 11, wl.SETUP_CFG2, n_min=2, n_max=250)


@pytest.fixture(scope="module")
def small_got(ref2, small_batch):
    m = ref2.model()
    db = pod.DeviceBatch.from_batch(small_batch)
    return host(pod.batch_assemble(m, db)), m, db


def test_batch_small_every_cell(ref2, small_batch, small_got):
    got = small_got[0]
    say(f"[gpu] batch small n_cfg={small_batch.n_cfg} N={small_batch.N} P={small_batch.nl.n_pairs}")
    worst = {"D": 0.0, "G": 0.0, "dGdR": 0.0}
    for c in range(small_batch.n_cfg):
        e = check_cell(small_batch, got, ref2, c)
        for k in worst:
            worst[k] = max(worst[k], e[k])
    say("[gpu]   " + " ".join(f"{k}={v:.3e}" for k, v in worst.items()))
    for k, v in worst.items():
        assert v < TOL, (k, v)


def test_batch_matches_single_system_call(ref2, small_batch, small_got):
    got, m, _ = small_got
    for c in range(small_batch.n_cfg):
        pos, cell, nl = small_batch.config(c)
        nb = pod.DeviceNeighbors.from_list(nl)
        D1 = m.descriptors(pos, cell, nb).cpu().numpy()
        a0, a1 = int(small_batch.cfg_atom_off[c]), int(small_batch.cfg_atom_off[c + 1])
        assert colerr(got["D"][a0:a1], D1) < 1e-12
        assert relerr(got["G"][c], D1.sum(axis=0)) < 1e-12


@pytest.mark.parametrize("tune", [(1, 7, 64), (3, 64, 128), (6, 512, 256), (12, 4096, 512), (17, 1, 192)])
def test_batch_tunes_agree(ref2, small_batch, small_got, tune):
    got, m, db = small_got
    say(f"[gpu] batch tune {tune}")
    t = host(pod.batch_assemble(m, db, tune=tune))
    for k in ("D", "G", "dGdR"):
        assert relerr(t[k], got[k]) < 1e-12, k


def test_batch_partial_outputs(ref2, small_batch, small_got):
    got, m, db = small_got
    only_d = host(pod.batch_assemble(m, db, D=True, G=False, dGdR=False))
    assert relerr(only_d["D"], got["D"]) < 1e-12
    only_dg = host(pod.batch_assemble(m, db, D=False, G=False, dGdR=True))
    assert relerr(only_dg["dGdR"], got["dGdR"]) < 1e-12


def test_batch_empty_and_tiny_cells(ref2):
    """Cells of 0 atoms between others, and cells of 2 atoms whose lists are
    all periodic images."""
    import torch
    b = wl.make_batch(5, 12, wl.SETUP_CFG2, n_min=2, n_max=4)
    off = np.asarray(b.cfg_atom_off, dtype=np.int64)
    off2 = np.concatenate([[0, 0], off[1:3], [off[2]], off[3:]]).astype(np.int32)   # empty cells 0 and 3
    cells = np.concatenate([b.cells[:1], b.cells[:2], b.cells[1:2], b.cells[2:]], axis=0)
    m = ref2.model()
    db = pod.DeviceBatch(off2, b.pos, cells, b.nl.offsets, b.nl.nbr_j, b.nl.shift)
    got = host(pod.batch_assemble(m, db))
    assert np.all(got["G"][0] == 0.0) and np.all(got["G"][3] == 0.0)
    mapping = [1, 2, 4, 5, 6]
    for c in range(b.n_cfg):
        D, G, dG = ref2.cell_refs(b, c)
        a0, a1 = int(off[c]), int(off[c + 1])
        assert colerr(got["D"][a0:a1], D) < TOL
        assert relerr(got["G"][mapping[c]], G) < TOL
        assert colerr(got["dGdR"][3 * a0:3 * a1], dG) < TOL
    # n_cfg = 0 and N = 0 are no-ops
    z = torch.zeros(1, dtype=torch.int32, device="cuda")
    pod.pod_batch_assemble(m.h, 0, 0, 0, z, db.pos, db.cells, z, z, z)


def test_batch_errors(ref2, small_batch):
    import torch
    m = ref2.model()
    b = small_batch
    # a neighbour outside its own cell is skipped and latched
    nbr = b.nl.nbr_j.copy()
    a1 = int(b.cfg_atom_off[1])
    nbr[int(b.nl.offsets[a1])] = 0                   # first pair of cell 1 -> atom of cell 0
    db = pod.DeviceBatch(b.cfg_atom_off, b.pos, b.cells, b.nl.offsets, nbr, b.nl.shift)
    o = pod.batch_assemble(m, db, check=False)
    with pytest.raises(pod.PodError) as e:
        m.check()
    assert e.value.code == -7
    del o
    # inconsistent offsets are refused on the host
    bad = np.asarray(b.cfg_atom_off).copy()
    bad[-1] -= 1
    db2 = pod.DeviceBatch(bad, b.pos, b.cells, b.nl.offsets, b.nl.nbr_j, b.nl.shift)
    with pytest.raises(pod.PodError) as e:
        pod.batch_assemble(m, db2)
    assert e.value.code == -1
    # launch shapes the kernel is not built for
    for bad_tune in ((6, 64, 100), (6, 64, 1024)):
        with pytest.raises(pod.PodError) as e:
            pod.batch_assemble(m, pod.DeviceBatch.from_batch(b), tune=bad_tune)
        assert e.value.code == -1
    # a non-finite coordinate
    pos = np.asarray(b.pos).copy()
    pos[0, 1] = np.nan
    db3 = pod.DeviceBatch(b.cfg_atom_off, pos, b.cells, b.nl.offsets, b.nl.nbr_j, b.nl.shift)
    pod.batch_assemble(m, db3, check=False)
    with pytest.raises(pod.PodError) as e:
        m.check()
    assert e.value.code == -3
    # FP32 handles are not supported by the FP64 assembly
    m32 = pod.PodModel(pod.setup_from_workload(wl.SETUP_CFG2), "f32", Q=ref2.Q[:, : ref2.K])
    db = pod.DeviceBatch.from_batch(b)
    with pytest.raises(pod.PodError) as e:
        pod.batch_assemble(m32, db)
    assert e.value.code == -6
    torch.cuda.synchronize()


def test_batch_config3_full(ref2):
    """2,000 cells (2..250 atoms; BCC/FCC/A15 and liquid) in one launch:
    sampled cells against the oracle, and at every cell the identities
    G_c = sum_{i in c} D_i and sum_{n in c} dG_c/dr_n = 0 (translation)."""
    import torch
    b = wl.config3()
    say(f"[gpu] config3 n_cfg={b.n_cfg} N={b.N} P={b.nl.n_pairs}")
    m = ref2.model()
    db = pod.DeviceBatch.from_batch(b)
    o = pod.batch_assemble(m, db)
    torch.cuda.synchronize()
    cid = torch.repeat_interleave(torch.arange(b.n_cfg, device="cuda"),
                                  torch.as_tensor(np.diff(b.cfg_atom_off).astype(np.int64), device="cuda"))
    Gs = torch.zeros_like(o["G"]).index_add_(0, cid, o["D"])
    assert float((Gs - o["G"]).abs().max()) <= 1e-12 * float(o["G"].abs().max())
    dG = o["dGdR"].view(b.N, 3, m.M)
    tr = torch.zeros((b.n_cfg, 3, m.M), dtype=torch.float64, device="cuda").index_add_(0, cid, dG)
    tr_rel = float(tr.abs().max()) / float(dG.abs().max())
    say(f"[gpu]   translation sum rel={tr_rel:.3e}")
    assert tr_rel < 1e-12
    got = {"D": o["D"].cpu().numpy(), "G": o["G"].cpu().numpy(), "dGdR": o["dGdR"].cpu().numpy()}
    sizes = np.diff(b.cfg_atom_off)
    rng = np.random.default_rng(99)
    sample = sorted(set([int(np.argmax(sizes)), int(np.argmin(sizes))]
                        + [int(x) for x in rng.choice(b.n_cfg, 6, replace=False)]))
    for c in sample:
        e = check_cell(b, got, ref2, c)
        say(f"[gpu]   cell {c} ({b.kinds[c]}, {sizes[c]} atoms) " + " ".join(f"{k}={v:.2e}" for k, v in e.items()))
        for k, v in e.items():
            assert v < TOL, (c, k, v)


def test_batch_autotuner_deterministic(ref2, small_batch, small_got, tmp_path):
    """The autotuner times candidates through the library, caches its pick
    and returns the same pick from the cache; the pick's results agree."""
    from paper_2212_14446_amd import autotune as at
    got, m, db = small_got
    path = str(tmp_path / "tune.json")
    cands = at.candidates(cw=(3, 6), nblocks=(64, 256), threads=(128, 256))
    best = at.tune_batch(m, db, path, cands, reps=2)
    say(f"[gpu] autotune pick {best}")
    assert best in cands
    for _ in range(2):
        assert at.tune_batch(m, db, path, cands) == best
    t = host(pod.batch_assemble(m, db, tune=best))
    for k in ("D", "G", "dGdR"):
        assert relerr(t[k], got[k]) < 1e-12, k


@pytest.mark.parametrize("setup", [
    wl.SETUP_CFG1,                                                   # L 6 -> K 4, 2/3-body, P3 = 3
    wl.PodSetup(rin=0.5, rcut=4.5, L=8, K2=3, K3=5, K4=2, P3=2, P4=6),  # P_a = 6 (largest instance)
    wl.PodSetup(rin=0.5, rcut=5.0, L=9, K2=7, K3=0, K4=7, P3=0, P4=3),  # no 3-body block
], ids=["cfg1", "p6", "no3body"])
def test_batch_other_descriptor_sets(setup):
    """Every cell of a small batch against the oracle for descriptor sets
    other than the benchmark's (other K, angular degrees and blocks)."""
    ref = Ref(setup)
    b = wl.make_batch(8, 13, setup, n_min=2, n_max=120)
    say(f"[gpu] batch other set M={setup.M} n_cfg={b.n_cfg} N={b.N}")
    got = host(pod.batch_assemble(ref.model(), pod.DeviceBatch.from_batch(b)))
    for c in range(b.n_cfg):
        e = check_cell(b, got, ref, c)
        for k, v in e.items():
            assert v < TOL, (c, k, v)
