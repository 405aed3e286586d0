"""Oracle index tables against the integer tables printed in the paper
(Tables 1, 3, 4, 5, 6 of Sec. II and Sec. V)."""
import os

import numpy as np

from oracle import pod_oracle as po

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    out = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                out.append([int(x) for x in line.split()])
    return out


def test_monomials_match_table3_per_degree():
    printed = _rows("table3_monomials.txt")
    mine = po.monomial_exponents(4)
    assert len(mine) == len(printed) == 35
    for n in range(5):
        want = sorted(tuple(r[1:]) for r in printed if r[0] == n)
        got = sorted(e for e in mine if sum(e) == n)
        assert got == want
        assert len(got) == (n + 1) * (n + 2) // 2        # count stated with eq. (23b)


def test_multinomials_match_table4_in_table3_order():
    printed3 = _rows("table3_monomials.txt")
    printed4 = {r[0]: r[1:] for r in _rows("table4_multinomials.txt")}
    for n in range(5):
        mons = [tuple(r[1:]) for r in printed3 if r[0] == n]
        assert [po.multinomial(e) for e in mons] == printed4[n]
        # multinomial theorem: the coefficients sum to 3^n
        assert sum(printed4[n]) == 3 ** n


def test_four_body_triples_match_table1():
    printed = [tuple(r[1:]) for r in _rows("table1_four_body.txt")]
    assert po.four_body_triples(4) == printed


def test_table5_counts():
    for P, Ka, Na, Ca, ratio in _rows("table5_angular_counts.txt"):
        assert po.n_four_body(P) == Ka
        assert len(po.monomial_exponents(P)) == Na == (P + 1) * (P + 2) * (P + 3) // 6
        # C_a: number of (q, s, t) terms of eq. (30a) summed over the p of Table 1
        nd = lambda n: (n + 1) * (n + 2) // 2
        ca = sum(nd(a) * nd(b) * nd(c) for (a, b, c) in po.four_body_triples(P))
        assert ca == Ca
        r = int(np.floor(Ca / Na + 0.5))
        if P == 10:
            assert (r, ratio) == (74, 75)       # printed ratio is a misprint
        else:
            assert r == ratio


def test_table6_descriptor_counts():
    for K2, K3, P3, M3, K4, P4, _ka_printed, M4 in _rows("table6_descriptor_counts.txt"):
        p3 = po.PodParams(0.5, 5.0, *po.default_snapshot_family(8), K2, K3, 0, P3, 0)
        assert po.num_descriptors(p3)[0] == M3
        p4 = po.PodParams(0.5, 5.0, *po.default_snapshot_family(8), K2, K3, K4, P3, P4)
        assert po.num_descriptors(p4)[0] == M4


def test_four_body_term_count_after_merging_duplicates():
    # distinct sorted (x, y, z) monomial triples of eq. (30a) per p; the paper
    # does not print this, it is a derived count used by the GPU tables
    look = {e: i for i, e in enumerate(po.monomial_exponents(4))}
    total = 0
    for (a, b, c) in po.four_body_triples(4):
        if b == 0 and c == 0:
            continue
        seen = set()
        for ea in po.monomial_exponents(a)[po._deg_start(a):]:
            for eb in po.monomial_exponents(b)[po._deg_start(b):]:
                for ec in po.monomial_exponents(c)[po._deg_start(c):]:
                    t = tuple(sorted((look[po._add(ea, eb)], look[po._add(ea, ec)],
                                      look[po._add(eb, ec)])))
                    seen.add(t)
        total += len(seen)
    assert total > 0
