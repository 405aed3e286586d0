"""Seeded synthetic inputs: Ta-like lattices, liquids and neighbour lists.

This module holds no descriptor, energy or force arithmetic.  It builds the
inputs of the POD path -- positions, periodic cells, full neighbour lists in
CSR form and coefficient vectors -- from fixed numpy seeds, with the shapes of
the paper's workloads: BCC tantalum boxes like the 20x20x20 (16,000-atom)
molecular-dynamics cell of its timing study (Sec. V.A), and mixed BCC / FCC /
A15 / liquid cells like its training set (Sec. V.A).  The training set itself
is not reproduced; these synthetic structures only share its shapes.

Neighbour-list contract (what the library expects):
  * a full list, both directions, sorted by centre atom;
  * every (i, j, n) with 0 < |r_j + n.cell - r_i| < rcut, n in Z^3;
  * periodic images are distinct entries, i == j allowed for n != 0;
  * ``shift`` packs n as three signed bytes (x | y << 8 | z << 16).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

A_TA = 3.31  # BCC lattice constant used for the tantalum-like boxes (angstrom)


# --------------------------------------------------------------------------
# Lattices
# --------------------------------------------------------------------------
_BASIS = {
    "bcc": np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]]),
    "fcc": np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]]),
    # A15 (Cr3Si type, all sites the same species): 2a + 6c Wyckoff positions
    "a15": np.array([
        [0.0, 0.0, 0.0], [0.5, 0.5, 0.5],
        [0.25, 0.5, 0.0], [0.75, 0.5, 0.0],
        [0.0, 0.25, 0.5], [0.0, 0.75, 0.5],
        [0.5, 0.0, 0.25], [0.5, 0.0, 0.75],
    ]),
}


def lattice(kind: str, n1: int, n2: int, n3: int, a: float):
    """Sites of an n1 x n2 x n3 supercell of a cubic lattice; returns (pos, cell)."""
    basis = _BASIS[kind]
    g = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij"), -1)
    g = g.reshape(-1, 1, 3) + basis[None, :, :]
    pos = g.reshape(-1, 3) * a
    cell = np.diag([n1 * a, n2 * a, n3 * a]).astype(np.float64)
    return pos.astype(np.float64), cell


def bcc(n: int, a: float = A_TA):
    return lattice("bcc", n, n, n, a)


def displace(pos, sigma: float, seed: int):
    rng = np.random.default_rng(seed)
    return pos + rng.normal(0.0, sigma, size=pos.shape)


def remove_sites(pos, n_remove: int, seed: int):
    rng = np.random.default_rng(seed)
    keep = np.sort(rng.choice(pos.shape[0], size=pos.shape[0] - n_remove, replace=False))
    return pos[keep]


def random_liquid(n: int, box: float, dmin: float, seed: int, max_tries: int = 200000):
    """Random sequential insertion of n points in a periodic cube, keeping every
    periodic distance >= dmin."""
    rng = np.random.default_rng(seed)
    pts = np.zeros((0, 3))
    tries = 0
    while pts.shape[0] < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("random_liquid: packing too dense")
        x = rng.uniform(0.0, box, size=3)
        if pts.shape[0]:
            d = pts - x
            d -= box * np.round(d / box)
            if np.min((d * d).sum(1)) < dmin * dmin:
                continue
        pts = np.vstack([pts, x])
    return pts, np.eye(3) * box


# --------------------------------------------------------------------------
# Neighbour lists
# --------------------------------------------------------------------------
@dataclass
class NeighborList:
    offsets: np.ndarray   # int32 [N+1]
    nbr_j: np.ndarray     # int32 [P]
    shift3: np.ndarray    # int32 [P, 3]
    shift: np.ndarray     # int32 [P], packed signed bytes

    @property
    def n_pairs(self) -> int:
        return int(self.offsets[-1])


def pack_shift(shift3):
    s = np.asarray(shift3, dtype=np.int64)
    if s.size and (s.min() < -128 or s.max() > 127):
        raise ValueError("image shift outside the signed-byte range")
    s = s & 0xFF
    return (s[:, 0] | (s[:, 1] << 8) | (s[:, 2] << 16)).astype(np.int32)


def _finish(N, i, j, sh):
    order = np.lexsort((sh[:, 2], sh[:, 1], sh[:, 0], j, i))
    i, j, sh = i[order], j[order], sh[order]
    counts = np.bincount(i, minlength=N)
    offsets = np.zeros(N + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    if offsets[-1] > np.iinfo(np.int32).max:
        raise ValueError("too many pairs for 32-bit offsets")
    sh = sh.astype(np.int32)
    return NeighborList(offsets.astype(np.int32), j.astype(np.int32), sh, pack_shift(sh))


def neighbor_list(pos, cell, rcut: float) -> NeighborList:
    """Full neighbour list within rcut (strict) for a periodic cell (rows are
    lattice vectors) or an open system (cell None)."""
    from scipy.spatial import cKDTree

    pos = np.asarray(pos, dtype=np.float64)
    N = pos.shape[0]
    if N == 0:
        return _finish(0, np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros((0, 3), np.int64))
    if cell is None:
        tree = cKDTree(pos)
        sm = tree.sparse_distance_matrix(tree, rcut, output_type="ndarray")
        i, j = sm["i"].astype(np.int64), sm["j"].astype(np.int64)
        d = pos[j] - pos[i]
        r = np.sqrt((d * d).sum(1))
        keep = (r > 0) & (r < rcut)
        return _finish(N, i[keep], j[keep], np.zeros((int(keep.sum()), 3), np.int64))
    cell = np.asarray(cell, dtype=np.float64)
    diag = np.diag(cell)
    ortho = np.allclose(cell, np.diag(diag))
    if ortho and np.all(diag > 2.0 * rcut + 1e-9):
        # minimum image is unique: periodic KD-tree
        wrapped = np.mod(pos, diag)
        wrapped[wrapped >= diag] = 0.0
        tree = cKDTree(wrapped, boxsize=diag)
        sm = tree.sparse_distance_matrix(tree, rcut, output_type="ndarray")
        i, j = sm["i"].astype(np.int64), sm["j"].astype(np.int64)
        raw = pos[j] - pos[i]
        n = -np.round(raw / diag).astype(np.int64)
        d = raw + n * diag
        r = np.sqrt((d * d).sum(1))
        keep = (r > 0) & (r < rcut)
        return _finish(N, i[keep], j[keep], n[keep])
    # general / small cell: replicate images
    inv = np.linalg.inv(cell)
    spacing = 1.0 / np.linalg.norm(inv, axis=0)
    nimg = np.ceil(rcut / spacing).astype(int) + 1
    rng = [np.arange(-k, k + 1) for k in nimg]
    imgs = np.array([[a, b, c] for a in rng[0] for b in rng[1] for c in rng[2]], dtype=np.int64)
    big = (pos[None, :, :] + (imgs @ cell)[:, None, :]).reshape(-1, 3)
    tree = cKDTree(big)
    hits = tree.query_ball_point(pos, rcut)
    ii, jj, nn = [], [], []
    for a, lst in enumerate(hits):
        if not lst:
            continue
        lst = np.asarray(lst, dtype=np.int64)
        im, j = lst // N, lst % N
        d = big[lst] - pos[a]
        r = np.sqrt((d * d).sum(1))
        keep = (r > 0) & (r < rcut)
        ii.append(np.full(int(keep.sum()), a, np.int64))
        jj.append(j[keep])
        nn.append(imgs[im[keep]])
    if not ii:
        return _finish(N, np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros((0, 3), np.int64))
    return _finish(N, np.concatenate(ii), np.concatenate(jj), np.concatenate(nn))


def min_pair_distance(pos, cell, nl: NeighborList) -> float:
    if nl.n_pairs == 0:
        return np.inf
    i = np.repeat(np.arange(pos.shape[0]), np.diff(nl.offsets))
    cellm = np.zeros((3, 3)) if cell is None else np.asarray(cell)
    d = pos[nl.nbr_j] + nl.shift3 @ cellm - pos[i]
    return float(np.sqrt((d * d).sum(1)).min())


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------
@dataclass
class PodSetup:
    """Radial / angular / body-order parameters of one workload."""
    rin: float
    rcut: float
    L: int
    K2: int
    K3: int
    K4: int
    P3: int
    P4: int
    beta: float = 3.0

    def snapshot_family(self):
        """Bessel snapshots alpha = 1..L-2 at one beta (kappa = 1) plus
        inverse-power snapshots gamma = 1, 2 (kappa = 0)."""
        nb = self.L - 2
        alpha = np.concatenate([np.arange(1, nb + 1, dtype=float), np.zeros(2)])
        beta = np.concatenate([np.full(nb, self.beta), np.zeros(2)])
        gamma = np.concatenate([np.zeros(nb), np.array([1.0, 2.0])])
        kappa = np.concatenate([np.ones(nb), np.zeros(2)])
        return alpha, beta, gamma, kappa

    @property
    def M(self) -> int:
        ka = _n_partitions3(self.P4) if self.K4 > 0 else 0
        return 1 + self.K2 + (self.K3 * (self.P3 + 1) if self.K3 else 0) + self.K4 * ka


def _n_partitions3(P):
    return sum(1 for n in range(P + 1) for a in range(n + 1) for b in range(a + 1)
               if 0 <= n - a - b <= b)


@dataclass
class Workload:
    name: str
    pos: np.ndarray
    cell: np.ndarray | None
    nl: NeighborList
    setup: PodSetup
    c: np.ndarray

    @property
    def N(self) -> int:
        return self.pos.shape[0]


SETUP_CFG1 = PodSetup(rin=0.5, rcut=5.0, L=6, K2=4, K3=4, K4=0, P3=3, P4=0)
SETUP_CFG2 = PodSetup(rin=0.5, rcut=5.0, L=8, K2=6, K3=6, K4=6, P3=4, P4=4)


def coefficients(M: int, seed: int):
    return np.random.default_rng(seed).normal(0.0, 1.0, size=M)


def config1() -> Workload:
    """128-atom BCC cell (4x4x4 conventional cells), sigma 0.1, 2+3-body."""
    pos, cell = bcc(4)
    pos = displace(pos, 0.1, seed=1)
    s = SETUP_CFG1
    nl = neighbor_list(pos, cell, s.rcut)
    return Workload("bcc4_128_f64_23body", pos, cell, nl, s, coefficients(s.M, seed=2))


def config2(rcut: float = 5.0) -> Workload:
    """20x20x20 BCC box, 1% vacancies (160 sites), sigma 0.15, 2/3/4-body."""
    pos, cell = bcc(20)
    pos = remove_sites(pos, 160, seed=3)
    pos = displace(pos, 0.15, seed=4)
    s = PodSetup(rin=0.5, rcut=rcut, L=8, K2=6, K3=6, K4=6, P3=4, P4=4)
    nl = neighbor_list(pos, cell, s.rcut)
    return Workload(f"bcc20_vac1pct_15840_rc{rcut:g}", pos, cell, nl, s, coefficients(s.M, seed=5))


def config4_positions():
    """30x30x30 BCC box (54,000 atoms), sigma 0.2."""
    pos, cell = bcc(30)
    return displace(pos, 0.2, seed=7), cell


def small_bcc(n: int = 2, sigma: float = 0.1, seed: int = 11, setup: PodSetup = SETUP_CFG2):
    pos, cell = bcc(n)
    pos = displace(pos, sigma, seed)
    nl = neighbor_list(pos, cell, setup.rcut)
    return Workload(f"bcc{n}_s{sigma}", pos, cell, nl, setup, coefficients(setup.M, seed + 1))


def config4() -> Workload:
    """54,000-atom BCC box (30^3 cells), sigma 0.2, 2/3/4-body (FP32 path),
    coefficients set per body order from descriptor statistics by
    ``standardised_coefficients``."""
    pos, cell = config4_positions()
    s = PodSetup(rin=0.5, rcut=5.0, L=8, K2=6, K3=6, K4=6, P3=4, P4=4)
    nl = neighbor_list(pos, cell, s.rcut)
    return Workload("bcc30_54000_s0.2", pos, cell, nl, s, np.zeros(s.M))


SETUP_CFG5 = PodSetup(rin=0.5, rcut=5.0, L=8, K2=6, K3=6, K4=6, P3=4, P4=4)
SETUP_CFG5_23 = PodSetup(rin=0.5, rcut=5.0, L=8, K2=6, K3=6, K4=0, P3=4, P4=0)
# the same 2/3-body part with 4-body terms up to angular degree 6 (P4 > P3):
# the exact model's atomic basis grows from 35 to 84 monomials, while the
# surrogate keeps the degree-4 basis of SETUP_CFG5_23
SETUP_CFG5_P6 = PodSetup(rin=0.5, rcut=5.0, L=8, K2=6, K3=6, K4=6, P3=4, P4=6)


def embed_23_coefficients(c, setup: PodSetup, setup23: PodSetup):
    """The constant, 2-body and 3-body coefficients of a model (setup) in the
    descriptor layout of a 2/3-body setup with the same K2, K3 and a 3-body
    degree P3 at least as high: columns of degrees above setup.P3 get zero,
    so that c23 . D23 is the model's 2/3-body energy."""
    if setup23.K2 != setup.K2 or setup23.K3 != setup.K3 or setup23.P3 < setup.P3:
        raise ValueError("2/3-body layout does not contain the model's")
    c = np.asarray(c, dtype=np.float64)
    out = np.zeros(setup23.M)
    out[: 1 + setup.K2] = c[: 1 + setup.K2]
    o, o23 = 1 + setup.K2, 1 + setup23.K2
    for m in range(setup.K3):
        out[o23 + m * (setup23.P3 + 1): o23 + m * (setup23.P3 + 1) + setup.P3 + 1] = \
            c[o + m * (setup.P3 + 1): o + (m + 1) * (setup.P3 + 1)]
    return out


def config5_train_boxes(n_boxes: int = 19, seed: int = 9):
    """Training environments for the 4-body surrogate: n_boxes BCC 30^3
    boxes (54,000 atoms each), each displaced with its own sigma drawn
    uniformly from [0.05, 0.3] A.  Yields (pos, cell, nl, sigma)."""
    rng = np.random.default_rng(seed)
    sigmas = rng.uniform(0.05, 0.3, size=n_boxes)
    seeds = rng.integers(1, 1 << 31, size=n_boxes)
    base, cell = bcc(30)
    for k in range(n_boxes):
        pos = displace(base, float(sigmas[k]), int(seeds[k]))
        yield pos, cell, neighbor_list(pos, cell, SETUP_CFG5.rcut), float(sigmas[k])


def config5_infer() -> Workload:
    """1,024,000-atom BCC box (80^3 cells), sigma 0.15 A, for surrogate
    inference."""
    pos, cell = bcc(80)
    pos = displace(pos, 0.15, 10)
    nl = neighbor_list(pos, cell, SETUP_CFG5.rcut)
    return Workload("bcc80_1024000_s0.15", pos, cell, nl, SETUP_CFG5, np.zeros(SETUP_CFG5.M))


def standardised_coefficients(D, setup: PodSetup, seed: int, targets=(1.0, 0.3, 0.1)):
    """Coefficients c_m = z_m s_b / (sigma_m sqrt(n_b)) with z ~ N(0, 1),
    sigma_m the standard deviation of descriptor m over the rows of D and
    n_b the size of its body-order block, so that the per-atom energy of the
    2-, 3- and 4-body blocks has a spread of about s_b = targets (eV)."""
    rng = np.random.default_rng(seed)
    M = D.shape[1]
    c = np.zeros(M)
    sig = D.std(axis=0)
    sig[sig == 0] = 1.0
    m2 = setup.K2
    m3 = setup.K3 * (setup.P3 + 1) if setup.K3 else 0
    blocks = [(1, 1 + m2), (1 + m2, 1 + m2 + m3), (1 + m2 + m3, M)]
    for (lo, hi), s in zip(blocks, targets):
        if hi > lo:
            z = rng.normal(size=hi - lo)
            c[lo:hi] = z * s / (sig[lo:hi] * np.sqrt(hi - lo))
    return c


# --------------------------------------------------------------------------
# Batches of small cells (descriptor-matrix assembly)
# --------------------------------------------------------------------------
V_ATOM = A_TA ** 3 / 2.0          # volume per atom of the BCC reference (A^3)
_SITES_PER_CELL = {"bcc": 2, "fcc": 4, "a15": 8}


@dataclass
class Batch:
    """Many periodic cells, concatenated: atoms of cell c are
    cfg_atom_off[c]:cfg_atom_off[c+1]; neighbour indices are global."""
    kinds: list
    cfg_atom_off: np.ndarray   # int32 [n_cfg + 1]
    pos: np.ndarray            # [N_tot, 3]
    cells: np.ndarray          # [n_cfg, 3, 3]
    nl: NeighborList           # global CSR
    setup: PodSetup

    @property
    def n_cfg(self) -> int:
        return len(self.cfg_atom_off) - 1

    @property
    def N(self) -> int:
        return self.pos.shape[0]

    def config(self, c):
        """(pos, cell, local neighbour list) of cell c."""
        a0, a1 = int(self.cfg_atom_off[c]), int(self.cfg_atom_off[c + 1])
        o = self.nl.offsets[a0:a1 + 1].astype(np.int64)
        p0, p1 = int(o[0]), int(o[-1])
        nl = NeighborList((o - p0).astype(np.int32), (self.nl.nbr_j[p0:p1] - a0).astype(np.int32),
                          self.nl.shift3[p0:p1], self.nl.shift[p0:p1])
        return self.pos[a0:a1], self.cells[c], nl


def small_cell(kind: str, n_atoms: int, vol_scale: float, sigma: float, rng):
    """One cell of n_atoms: a lattice supercell (the smallest n1 x n2 x n3 with
    at least n_atoms sites, random sites deleted down to n_atoms) or a random
    liquid (sequential insertion, minimum distance 2 A), at volume per atom
    V_ATOM * vol_scale."""
    if kind == "liquid":
        box = (n_atoms * V_ATOM * vol_scale) ** (1.0 / 3.0)
        seed = int(rng.integers(1 << 31))
        pos, cell = random_liquid(n_atoms, box, 2.0, seed)
        return pos, cell
    spc = _SITES_PER_CELL[kind]
    best = None
    for n1 in range(1, 8):
        for n2 in range(1, n1 + 1):
            for n3 in range(1, n2 + 1):
                if n1 * n2 * n3 * spc >= n_atoms:
                    key = (n1 * n2 * n3, n1 - n3)
                    if best is None or key < best[0]:
                        best = (key, (n1, n2, n3))
    n1, n2, n3 = best[1]
    a = (spc * V_ATOM * vol_scale) ** (1.0 / 3.0)
    pos, cell = lattice(kind, n1, n2, n3, a)
    if pos.shape[0] > n_atoms:
        keep = np.sort(rng.choice(pos.shape[0], size=n_atoms, replace=False))
        pos = pos[keep]
    pos = pos + rng.normal(0.0, sigma, size=pos.shape)
    return pos, cell


def make_batch(n_cfg: int, seed: int, setup: PodSetup, n_min: int = 2, n_max: int = 250, sigma: float = 0.1):
    """n_cfg cells, atom counts uniform in [n_min, n_max], kinds uniform over
    BCC / FCC / A15 / liquid, volume per atom scaled by U[0.9, 1.1]."""
    rng = np.random.default_rng(seed)
    kinds, poss, cells, lists = [], [], [], []
    for _ in range(n_cfg):
        kind = ["bcc", "fcc", "a15", "liquid"][int(rng.integers(4))]
        n = int(rng.integers(n_min, n_max + 1))
        scale = float(rng.uniform(0.9, 1.1))
        pos, cell = small_cell(kind, n, scale, sigma, rng)
        kinds.append(kind)
        poss.append(pos)
        cells.append(cell)
        lists.append(neighbor_list(pos, cell, setup.rcut))
    counts = np.array([p.shape[0] for p in poss])
    cfg_off = np.zeros(n_cfg + 1, dtype=np.int64)
    cfg_off[1:] = np.cumsum(counts)
    pair_counts = np.array([nl.n_pairs for nl in lists])
    pair_off = np.zeros(n_cfg + 1, dtype=np.int64)
    pair_off[1:] = np.cumsum(pair_counts)
    offsets = np.concatenate([[0]] + [nl.offsets[1:].astype(np.int64) + pair_off[c] for c, nl in enumerate(lists)])
    nbr_j = np.concatenate([nl.nbr_j.astype(np.int64) + cfg_off[c] for c, nl in enumerate(lists)])
    shift3 = np.concatenate([nl.shift3 for nl in lists]).astype(np.int32)
    nl = NeighborList(offsets.astype(np.int32), nbr_j.astype(np.int32), shift3, pack_shift(shift3))
    return Batch(kinds, cfg_off.astype(np.int32), np.concatenate(poss), np.stack(cells), nl, setup)


def config3(n_cfg: int = 2000) -> Batch:
    """2,000 cells of 2-250 atoms (seed 6), 2/3/4-body parameters of the
    15,840-atom box."""
    return make_batch(n_cfg, seed=6, setup=SETUP_CFG2)


@dataclass
class AcsfSpec:
    """Parameters of a set of atom-centred symmetry functions (Sec. III.B):
    radial functions G2 (eta, r_s), angular functions G3 (eta, zeta, lambda)
    and four-body functions G4 (eta, a, b, c, alpha, beta, gamma), with
    non-negative integer exponents zeta, a, b, c.  Descriptor order: all G2,
    then all G3, then all G4, each in the order given."""
    g2: tuple = ()
    g3: tuple = ()
    g4: tuple = ()

    @property
    def n(self) -> int:
        return len(self.g2) + len(self.g3) + len(self.g4)


def acsf_standard() -> AcsfSpec:
    """34 functions in the usual Behler-Parrinello pattern for a 5 A cut-off:
    8 radial shells (eta = 2 / A^2, r_s = 1.5 .. 5.0 A), 18 angular functions
    (eta in {0.005, 0.05, 0.2} / A^2, zeta in {1, 2, 4}, lambda = +-1) and 8
    four-body functions (eta in {0.005, 0.05}, (a, b, c) in {(1,1,1),
    (2,1,1)}, alpha = beta = gamma = +-1)."""
    g2 = tuple((2.0, 1.5 + 0.5 * k) for k in range(8))
    g3 = tuple((eta, z, lam) for eta in (0.005, 0.05, 0.2) for z in (1, 2, 4) for lam in (1.0, -1.0))
    g4 = tuple((eta, a, b, c, s, s, s) for eta in (0.005, 0.05) for (a, b, c) in ((1, 1, 1), (2, 1, 1))
               for s in (1.0, -1.0))
    return AcsfSpec(g2, g3, g4)
