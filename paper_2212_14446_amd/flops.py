"""Algorithmic operation counts of the fast POD energy + force path.

Counts are floating-point operations of the algorithm (an FMA counts 2, a
transcendental counts 1), not instructions issued.  They are the numerators
of the roofline fractions the benchmark reports.

Per directed pair (N_a monomials of degree <= P_a, K radial functions, L
snapshots, G_a nonzero partial derivatives of the monomials):
  radial     2 * (2 L K)           projections R = Phi Q and R' = Phi' Q
             + 10 L + 30           snapshots, cut-off, geometry
  forward    (N_a - 1) + 2 K N_a   monomials + atomic-basis FMAs (eq. (24b))
  backward   (N_a - 1) + K (2 N_a + 2 G_a + 4 (P_a + 1) + 12) + 6 K + 18
             monomials; per radial index: adjoint contraction, its gradient,
             degree sums and the chain rule of eq. (24c); share reduction,
             virial
Per atom (NT merged eq. (30a) terms, K_a four-body functions):
  K (3 N_a + 4 NT + 3 N_a + 9 NT + 2 (2 + P_a + K_a))
             D3 (eq. (26a)), D4 (eq. (30a)), their adjoints, energy

Batched assembly with descriptor derivatives (batch_counts): radial with
derivatives and forward as above, the per-atom forward contraction
K (3 N_a + 4 NT), and for dG/dR, per pair and radial index m the monomials
(N_a - 1), and per pair and descriptor column
  2 N_a + 6 N_a(P_a - 1) + 2 (P_a + 1) + 12
  (h = J . A, its u-gradient from the monomials of degree < P_a, the degree
  sums, and v of eq. (24c) with its two scatters).
"""
from __future__ import annotations


def monomials(P):
    return [(a, b, n - a - b) for n in range(P + 1) for a in range(n, -1, -1) for b in range(n - a, -1, -1)]


def four_body(P):
    out = []
    for n in range(P + 1):
        for a in range(n, -1, -1):
            for b in range(min(a, n - a), -1, -1):
                c = n - a - b
                if 0 <= c <= b:
                    out.append((a, b, c))
    return out


def merged_terms(P):
    """Number of distinct sorted monomial triples of eq. (30a) over all p with
    (b, c) != (0, 0)."""
    look = {e: i for i, e in enumerate(monomials(P))}
    total = 0
    for (a, b, c) in four_body(P):
        if b == 0 and c == 0:
            continue
        seen = set()
        for ea in [e for e in monomials(a) if sum(e) == a]:
            for eb in [e for e in monomials(b) if sum(e) == b]:
                for ec in [e for e in monomials(c) if sum(e) == c]:
                    x = look[tuple(u + v for u, v in zip(ea, eb))]
                    y = look[tuple(u + v for u, v in zip(ea, ec))]
                    z = look[tuple(u + v for u, v in zip(eb, ec))]
                    seen.add(tuple(sorted((x, y, z))))
        total += len(seen)
    return total


def counts(K, L, PA, P4=None):
    """Dict of per-pair and per-atom algorithmic flops."""
    P4 = PA if P4 is None else P4
    mons = monomials(PA)
    Na = len(mons)
    Ga = sum((a > 0) + (b > 0) + (c > 0) for a, b, c in mons)
    NT = merged_terms(PA)
    Ka = len(four_body(P4))
    radial = 2 * (2 * L * K) + 10 * L + 30
    fwd = (Na - 1) + 2 * K * Na
    bwd = (Na - 1) + K * (2 * Na + 2 * Ga + 4 * (PA + 1) + 12) + 6 * K + 18
    atom = K * (3 * Na + 4 * NT + 3 * Na + 9 * NT + 2 * (2 + PA + Ka))
    return {"radial_per_pair": radial, "forward_per_pair": fwd, "backward_per_pair": bwd,
            "per_atom": atom, "Na": Na, "Ga": Ga, "NT": NT}


def batch_counts(K, L, PA, P4, M, n_pairs, n_atoms):
    """Algorithmic flops of one batched assembly (D, G and dG/dR)."""
    c = counts(K, L, PA, P4)
    Na, NT = c["Na"], c["NT"]
    Na_low = len(monomials(PA - 1)) if PA > 0 else 0
    per_col = 2 * Na + 6 * Na_low + 2 * (PA + 1) + 12
    fwd = (c["radial_per_pair"] + c["forward_per_pair"]) * n_pairs + K * (3 * Na + 4 * NT) * n_atoms
    deriv = n_pairs * ((M - 1) * per_col + K * (Na - 1))
    return {"forward": fwd, "derivatives": deriv, "total": fwd + deriv, "per_pair_column": per_col}


def split_counts(K, L, PA, P4=None):
    """The same work divided between the two kernels of the energy path:
    the per-atom kernel evaluates the snapshots and R = Phi Q, the atomic
    basis, the contractions, energy and adjoint rows; the pair kernel
    evaluates R' = Phi' Q and the backward sweep of each pair."""
    c = counts(K, L, PA, P4)
    proj = 2 * L * K
    snap = c["radial_per_pair"] - 2 * proj
    return {"atom_per_pair": snap + proj + c["forward_per_pair"], "per_atom": c["per_atom"],
            "pair_per_pair": proj + c["backward_per_pair"]}

