// Compile-time index tables of the device path.
//
// * angular monomials x^a y^b z^c, a + b + c = n <= PA (Sec. II.E, eq. (23b));
// * multinomial coefficients n!/(a! b! c!) of (x + y + z)^n (Table 4);
// * 4-body angular index p = (a, b, c), a >= b >= c >= 0, in Table 1 order;
// * the terms of eq. (30a): for each p with (b, c) != (0, 0), every product
//   c_aq c_bs c_ct B_{alpha+beta} B_{alpha+gamma} B_{beta+gamma}, with equal
//   monomial triples (after sorting) merged into one term with the summed
//   coefficient.  (a, 0, 0) uses eq. (27a) instead.
//
// Everything here is constexpr so that kernels can unroll over the tables and
// keep the per-atom basis in registers with constant indices.
#pragma once

namespace pod {

constexpr int n_mono(int P) { return P < 0 ? 0 : (P + 1) * (P + 2) * (P + 3) / 6; }
constexpr int n_of_degree(int n) { return (n + 1) * (n + 2) / 2; }
constexpr int factorial(int n) { return n <= 1 ? 1 : n * factorial(n - 1); }

// Device monomial order: degree-major; within degree n, c ascending, then b
// ascending (a = n - b - c).
constexpr int mono_index(int a, int b, int c) {
    const int n = a + b + c;
    return n_mono(n - 1) + c * (n + 1) - c * (c - 1) / 2 + b;
}

constexpr int n_partitions(int P) {
    int k = 0;
    for (int n = 0; n <= P; ++n)
        for (int a = n; a >= 0; --a)
            for (int b = (a < n - a ? a : n - a); b >= 0; --b) {
                const int c = n - a - b;
                if (c >= 0 && c <= b) ++k;
            }
    return k;
}

template <int PA>
struct MonoTable {
    static constexpr int NA = n_mono(PA);
    int ex[NA][3];
    int deg[NA];
    int mult[NA];
    int par[NA];    // lower-degree monomial this one is built from (-1 for index 0)
    int axis[NA];   // coordinate multiplied in to build it
    int down[NA][3];// index of mu - e_d, or -1 when that exponent is 0
    constexpr MonoTable() : ex{}, deg{}, mult{}, par{}, axis{}, down{} {
        for (int n = 0; n <= PA; ++n)
            for (int c = 0; c <= n; ++c)
                for (int b = 0; b <= n - c; ++b) {
                    const int a = n - b - c;
                    const int i = mono_index(a, b, c);
                    ex[i][0] = a; ex[i][1] = b; ex[i][2] = c;
                    deg[i] = n;
                    mult[i] = factorial(n) / (factorial(a) * factorial(b) * factorial(c));
                }
        for (int i = 0; i < NA; ++i) {
            par[i] = -1; axis[i] = -1;
            for (int d = 0; d < 3; ++d) {
                down[i][d] = -1;
                if (ex[i][d] > 0) {
                    int t[3] = {ex[i][0], ex[i][1], ex[i][2]};
                    t[d] -= 1;
                    down[i][d] = mono_index(t[0], t[1], t[2]);
                }
            }
            for (int d = 0; d < 3 && i > 0; ++d)
                if (ex[i][d] > 0) { par[i] = down[i][d]; axis[i] = d; break; }
        }
    }
};

// Worst-case number of merged eq. (30a) terms for PA <= 6 (raw count 1345).
constexpr int D4_CAP = 1400;

template <int PA>
struct D4Build {
    int KA;
    int pa[64], pb[64], pc[64];   // (a, b, c) of each p, Table 1 order
    int tbeg[64], tend[64];       // merged terms of p: [tbeg[p], tend[p])
    int nt;
    int tp[D4_CAP], tx[D4_CAP], ty[D4_CAP], tz[D4_CAP], tc[D4_CAP];
    constexpr D4Build() : KA(0), pa{}, pb{}, pc{}, tbeg{}, tend{}, nt(0), tp{}, tx{}, ty{}, tz{}, tc{} {
        for (int n = 0; n <= PA; ++n)
            for (int a = n; a >= 0; --a)
                for (int b = (a < n - a ? a : n - a); b >= 0; --b) {
                    const int c = n - a - b;
                    if (c < 0 || c > b) continue;
                    const int p = KA++;
                    pa[p] = a; pb[p] = b; pc[p] = c;
                    tbeg[p] = nt; tend[p] = nt;
                    if (b == 0 && c == 0) continue;      // eq. (27a)
                    const int first = nt;
                    // monomials of degree a, b, c: (x1, y1, z1) etc.
                    for (int c1 = 0; c1 <= a; ++c1)
                        for (int b1 = 0; b1 <= a - c1; ++b1) {
                            const int a1 = a - b1 - c1;
                            const int m1 = factorial(a) / (factorial(a1) * factorial(b1) * factorial(c1));
                            for (int c2 = 0; c2 <= b; ++c2)
                                for (int b2 = 0; b2 <= b - c2; ++b2) {
                                    const int a2 = b - b2 - c2;
                                    const int m2 = factorial(b) / (factorial(a2) * factorial(b2) * factorial(c2));
                                    for (int c3 = 0; c3 <= c; ++c3)
                                        for (int b3 = 0; b3 <= c - c3; ++b3) {
                                            const int a3 = c - b3 - c3;
                                            const int m3 = factorial(c) / (factorial(a3) * factorial(b3) * factorial(c3));
                                            // alpha+beta on rhat_ij, alpha+gamma on rhat_ik, beta+gamma on rhat_il
                                            int x = mono_index(a1 + a2, b1 + b2, c1 + c2);
                                            int y = mono_index(a1 + a3, b1 + b3, c1 + c3);
                                            int z = mono_index(a2 + a3, b2 + b3, c2 + c3);
                                            if (x > y) { int s = x; x = y; y = s; }
                                            if (y > z) { int s = y; y = z; z = s; }
                                            if (x > y) { int s = x; x = y; y = s; }
                                            int hit = -1;
                                            for (int k = first; k < nt; ++k)
                                                if (tx[k] == x && ty[k] == y && tz[k] == z) { hit = k; break; }
                                            if (hit >= 0) {
                                                tc[hit] += m1 * m2 * m3;
                                            } else {
                                                tp[nt] = p; tx[nt] = x; ty[nt] = y; tz[nt] = z;
                                                tc[nt] = m1 * m2 * m3;
                                                ++nt;
                                            }
                                        }
                                }
                        }
                    tend[p] = nt;
                }
    }
};

template <int PA>
struct D4Table {
    static constexpr D4Build<PA> build{};
    static constexpr int KA = build.KA;
    static constexpr int NT = build.nt;
};

}  // namespace pod
