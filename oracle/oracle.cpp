// Compiled FP64 CPU oracle of the linear POD energy, its global descriptors,
// forces and virial, by the atom-density (fast) form of arXiv:2212.14446.
//
// Test infrastructure and the benchmark's CPU baseline, not product code:
// only the tests and the benchmark's CPU leg load it (through
// oracle/oracle_c.py); it shares no code, header or table with the HIP
// library.  It computes exactly what oracle/pod_oracle.py's energy_forces
// computes, step by step, in plain double precision with OpenMP over atoms:
//
//   r_ij = r_j + n.cell - r_i                       Sec. II.A
//   snapshots Phi_l = f_c psi(r; mu_l) and Phi'_l   Sec. II.B, eqs. (3)-(8), (11)
//   R_k = sum_l Q_lk Phi_l, R'_k                    eq. (12)
//   A_mu(u) = x^a y^b z^c, u = r_ij / |r_ij|        eq. (23b), Table 3
//   B_i,k,mu = sum_j R_k A_mu                       eq. (24b)
//   D2 = B_k0; D3_kn = sum_{deg mu = n} c_mu B^2    eqs. (25), (26a), Table 4
//   D4 by eq. (27a) for (a, 0, 0), eq. (30a) else   Tables 1, 5
//   E_i = sum_col c_col D_i,col; G = sum_i D_i      eqs. (57a), (58a)
//   dE_i/dB_i by the product rule (eq. (26c) for the 3-body term)
//   g_ij = dE_i/dr_ij = sum dE_i/dB dB/dr_ij        eq. (24c), chain rule through u
//   F_i += g_ij, F_j -= g_ij; W_ab -= r_ij,a g_ij,b
//
// No blocking or reordering beyond these definitions: each atom's pairs are
// walked in list order, and threads own disjoint atoms (their force and
// virial contributions are summed per thread, then over threads in order).
#include <omp.h>

#include <cmath>
#include <cstdlib>
#include <vector>

namespace {

constexpr double kEpsFc = 1e-6;   // epsilon of the cut-off function, eq. (8)
constexpr double kPi = 3.14159265358979323846;

struct Mono {
    int e[3];
    int deg;
    double mult;   // n! / (a! b! c!)
};

double factorial(int n) {
    double f = 1.0;
    for (int k = 2; k <= n; ++k) f *= k;
    return f;
}

// Monomials of degree <= P: degree ascending, then (a, b) descending.
std::vector<Mono> monomials(int P) {
    std::vector<Mono> out;
    for (int n = 0; n <= P; ++n)
        for (int a = n; a >= 0; --a)
            for (int b = n - a; b >= 0; --b) {
                Mono m;
                m.e[0] = a; m.e[1] = b; m.e[2] = n - a - b;
                m.deg = n;
                m.mult = factorial(n) / (factorial(a) * factorial(b) * factorial(n - a - b));
                out.push_back(m);
            }
    return out;
}

int mono_index(const std::vector<Mono>& ms, int a, int b, int c) {
    for (size_t i = 0; i < ms.size(); ++i)
        if (ms[i].e[0] == a && ms[i].e[1] == b && ms[i].e[2] == c) return static_cast<int>(i);
    return -1;
}

// One product of eq. (30a): coefficient and the three monomial indices.
struct Term {
    double coef;
    int x, y, z;
};

// 4-body functions (a, b, c), a >= b >= c >= 0, a + b + c <= P4, Table 1 order.
struct Four {
    int a, b, c;
    std::vector<Term> terms;   // eq. (30a) products when (b, c) != (0, 0)
};

double ipow(double x, int n) {
    double v = 1.0;
    for (int k = 0; k < n; ++k) v *= x;
    return v;
}

}  // namespace

extern "C" {

// Returns 0, or -1 for a pair distance outside (rin, rcut) or a non-finite
// one, -2 for invalid arguments.  Q is L x qcols row-major (qcols >= K).
// Outputs: E_atom[N], E[1], G[M], F[N*3], W[9].
int pod_oracle_energy_forces(int N, const double* pos, const double* cell, const long long* offsets,
                             const int* nbr_j, const int* shift3, double rin, double rcut, int L,
                             const double* alpha, const double* beta, const double* gamma, const double* kappa,
                             int K2, int K3, int K4, int P3, int P4, const double* Q, int qcols, const double* c,
                             int threads, double* E_atom, double* E, double* G, double* F, double* W) {
    const int K = K2 > K3 ? (K2 > K4 ? K2 : K4) : (K3 > K4 ? K3 : K4);
    int PA = 0;
    if (K3 > 0 && P3 > PA) PA = P3;
    if (K4 > 0 && P4 > PA) PA = P4;
    if (N < 0 || L < 1 || K < 1 || qcols < K || threads < 1) return -2;
    const std::vector<Mono> ms = monomials(PA);
    const int NA = static_cast<int>(ms.size());

    std::vector<Four> fours;
    if (K4 > 0) {
        for (int n = 0; n <= P4; ++n)
            for (int a = n; a >= 0; --a)
                for (int b = (a < n - a ? a : n - a); b >= 0; --b) {
                    const int cc = n - a - b;
                    if (cc < 0 || cc > b) continue;
                    Four f;
                    f.a = a; f.b = b; f.c = cc;
                    if (!(b == 0 && cc == 0)) {
                        const std::vector<Mono> ma = monomials(a), mb = monomials(b), mc = monomials(cc);
                        for (const Mono& ea : ma) {
                            if (ea.deg != a) continue;
                            for (const Mono& eb : mb) {
                                if (eb.deg != b) continue;
                                for (const Mono& ec : mc) {
                                    if (ec.deg != cc) continue;
                                    Term t;
                                    t.coef = ea.mult * eb.mult * ec.mult;
                                    t.x = mono_index(ms, ea.e[0] + eb.e[0], ea.e[1] + eb.e[1], ea.e[2] + eb.e[2]);
                                    t.y = mono_index(ms, ea.e[0] + ec.e[0], ea.e[1] + ec.e[1], ea.e[2] + ec.e[2]);
                                    t.z = mono_index(ms, eb.e[0] + ec.e[0], eb.e[1] + ec.e[1], eb.e[2] + ec.e[2]);
                                    f.terms.push_back(t);
                                }
                            }
                        }
                    }
                    fours.push_back(f);
                }
    }
    const int KA = static_cast<int>(fours.size());
    const int M = 1 + K2 + (K3 > 0 ? K3 * (P3 + 1) : 0) + (K4 > 0 ? K4 * KA : 0);
    const int off3 = 1 + K2;
    const int off4 = off3 + (K3 > 0 ? K3 * (P3 + 1) : 0);

    int status = 0;
    std::vector<std::vector<double>> Ft(threads, std::vector<double>(static_cast<size_t>(N) * 3, 0.0));
    std::vector<std::vector<double>> Wt(threads, std::vector<double>(9, 0.0));
    std::vector<std::vector<double>> Gt(threads, std::vector<double>(M, 0.0));

#pragma omp parallel num_threads(threads)
    {
        const int t = omp_get_thread_num();
        std::vector<double>& Fl = Ft[t];
        std::vector<double>& Wl = Wt[t];
        std::vector<double>& Gl = Gt[t];
        std::vector<double> B(static_cast<size_t>(K) * NA), Ab(static_cast<size_t>(K) * NA);
        std::vector<double> D(M), D3(static_cast<size_t>(K) * (PA + 1));
        std::vector<double> pr, pdr, pu, pd, pA;   // per pair of the atom: R, R', u, r_ij, A
        std::vector<double> Phi(L), dPhi(L);

#pragma omp for schedule(static)
        for (int i = 0; i < N; ++i) {
            const long long b0 = offsets[i], b1 = offsets[i + 1];
            const int np = static_cast<int>(b1 - b0);
            pr.assign(static_cast<size_t>(np) * K, 0.0);
            pdr.assign(static_cast<size_t>(np) * K, 0.0);
            pu.assign(static_cast<size_t>(np) * 3, 0.0);
            pd.assign(static_cast<size_t>(np) * 3, 0.0);
            pA.assign(static_cast<size_t>(np) * NA, 0.0);
            std::fill(B.begin(), B.end(), 0.0);
            bool bad = false;
            for (int q = 0; q < np; ++q) {
                const long long p = b0 + q;
                const int j = nbr_j[p];
                double d[3];
                for (int x = 0; x < 3; ++x) {
                    double s = 0.0;
                    if (cell)
                        for (int k = 0; k < 3; ++k) s += shift3[3 * p + k] * cell[3 * k + x];
                    d[x] = pos[3 * j + x] + s - pos[3 * i + x];
                }
                const double r = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                if (!std::isfinite(r) || r <= rin || r >= rcut) { bad = true; break; }
                // cut-off, eq. (8), and its derivative
                const double h = rcut - rin;
                const double tt = (r - rin) / h;
                const double y = 1.0 - tt * tt * tt;
                const double s = y * y + kEpsFc;
                const double fc = std::exp(1.0 - 1.0 / std::sqrt(s));
                const double dfc = fc * (y * std::pow(s, -1.5)) * (-3.0 * tt * tt / h);
                // snapshots, eqs. (3)-(6), (11)
                const double dist = r - rin;
                for (int l = 0; l < L; ++l) {
                    double psi = 0.0, dpsi = 0.0;
                    if (kappa[l] != 0.0) {
                        double xx, dx;
                        if (beta[l] == 0.0) {
                            xx = tt; dx = 1.0 / h;
                        } else {
                            const double den = std::expm1(-beta[l]);
                            xx = std::expm1(-beta[l] * tt) / den;
                            dx = -beta[l] * std::exp(-beta[l] * tt) / den / h;
                        }
                        const double w = alpha[l] * kPi;
                        const double sn = std::sin(w * xx), cs = std::cos(w * xx);
                        psi += kappa[l] * sn / dist;
                        dpsi += kappa[l] * (w * cs * dx * dist - sn) / (dist * dist);
                    }
                    if (kappa[l] != 1.0) {
                        const double g = gamma[l];
                        psi += (1.0 - kappa[l]) * std::pow(r, -g);
                        dpsi += (1.0 - kappa[l]) * (-g) * std::pow(r, -g - 1.0);
                    }
                    Phi[l] = fc * psi;
                    dPhi[l] = dfc * psi + fc * dpsi;
                }
                double* R = &pr[static_cast<size_t>(q) * K];
                double* dR = &pdr[static_cast<size_t>(q) * K];
                for (int k = 0; k < K; ++k) {
                    double a = 0.0, da = 0.0;
                    for (int l = 0; l < L; ++l) {
                        a += Q[l * qcols + k] * Phi[l];
                        da += Q[l * qcols + k] * dPhi[l];
                    }
                    R[k] = a; dR[k] = da;
                }
                double* u = &pu[static_cast<size_t>(q) * 3];
                for (int x = 0; x < 3; ++x) { u[x] = d[x] / r; pd[3 * q + x] = d[x]; }
                double* A = &pA[static_cast<size_t>(q) * NA];
                for (int mu = 0; mu < NA; ++mu)
                    A[mu] = ipow(u[0], ms[mu].e[0]) * ipow(u[1], ms[mu].e[1]) * ipow(u[2], ms[mu].e[2]);
                for (int k = 0; k < K; ++k)
                    for (int mu = 0; mu < NA; ++mu) B[static_cast<size_t>(k) * NA + mu] += R[k] * A[mu];
            }
            if (bad) {
#pragma omp atomic write
                status = -1;
                continue;
            }
            // descriptors
            auto Bv = [&](int k, int mu) { return B[static_cast<size_t>(k) * NA + mu]; };
            std::fill(D.begin(), D.end(), 0.0);
            std::fill(D3.begin(), D3.end(), 0.0);
            for (int k = 0; k < K; ++k)
                for (int mu = 0; mu < NA; ++mu) D3[static_cast<size_t>(k) * (PA + 1) + ms[mu].deg] += ms[mu].mult * Bv(k, mu) * Bv(k, mu);
            D[0] = 1.0;
            for (int k = 0; k < K2; ++k) D[1 + k] = Bv(k, 0);
            for (int k = 0; k < K3; ++k)
                for (int n = 0; n <= P3; ++n) D[off3 + k * (P3 + 1) + n] = D3[static_cast<size_t>(k) * (PA + 1) + n];
            for (int k = 0; k < K4; ++k)
                for (int f = 0; f < KA; ++f) {
                    const Four& fo = fours[f];
                    double v = 0.0;
                    if (fo.b == 0 && fo.c == 0) {
                        v = Bv(k, 0) * D3[static_cast<size_t>(k) * (PA + 1) + fo.a];   // eq. (27a)
                    } else {
                        for (const Term& tm : fo.terms) v += tm.coef * Bv(k, tm.x) * Bv(k, tm.y) * Bv(k, tm.z);
                    }
                    D[off4 + k * KA + f] = v;
                }
            double ei = 0.0;
            for (int col = 0; col < M; ++col) {
                ei += c[col] * D[col];
                Gl[col] += D[col];
            }
            E_atom[i] = ei;
            // adjoint dE_i/dB_i by the product rule
            std::fill(Ab.begin(), Ab.end(), 0.0);
            auto Aa = [&](int k, int mu) -> double& { return Ab[static_cast<size_t>(k) * NA + mu]; };
            for (int k = 0; k < K2; ++k) Aa(k, 0) += c[1 + k];
            for (int k = 0; k < K3; ++k)
                for (int mu = 0; mu < NA; ++mu)
                    if (ms[mu].deg <= P3) Aa(k, mu) += c[off3 + k * (P3 + 1) + ms[mu].deg] * 2.0 * ms[mu].mult * Bv(k, mu);
            for (int k = 0; k < K4; ++k)
                for (int f = 0; f < KA; ++f) {
                    const Four& fo = fours[f];
                    const double w = c[off4 + k * KA + f];
                    if (fo.b == 0 && fo.c == 0) {
                        Aa(k, 0) += w * D3[static_cast<size_t>(k) * (PA + 1) + fo.a];
                        for (int mu = 0; mu < NA; ++mu)
                            if (ms[mu].deg == fo.a) Aa(k, mu) += w * Bv(k, 0) * 2.0 * ms[mu].mult * Bv(k, mu);
                    } else {
                        for (const Term& tm : fo.terms) {
                            Aa(k, tm.x) += w * tm.coef * Bv(k, tm.y) * Bv(k, tm.z);
                            Aa(k, tm.y) += w * tm.coef * Bv(k, tm.x) * Bv(k, tm.z);
                            Aa(k, tm.z) += w * tm.coef * Bv(k, tm.x) * Bv(k, tm.y);
                        }
                    }
                }
            // pair gradients, eq. (24c): dB_k,mu/dr_ij = R'_k A_mu u + R_k (I - u u^T) grad_u A_mu / r
            for (int q = 0; q < np; ++q) {
                const double* R = &pr[static_cast<size_t>(q) * K];
                const double* dR = &pdr[static_cast<size_t>(q) * K];
                const double* u = &pu[static_cast<size_t>(q) * 3];
                const double* d = &pd[static_cast<size_t>(q) * 3];
                const double* A = &pA[static_cast<size_t>(q) * NA];
                const double r = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                double g[3] = {0.0, 0.0, 0.0};
                for (int mu = 0; mu < NA; ++mu) {
                    const int ea = ms[mu].e[0], eb = ms[mu].e[1], ec = ms[mu].e[2];
                    double gr[3] = {0.0, 0.0, 0.0};
                    if (ea > 0) gr[0] = ea * ipow(u[0], ea - 1) * ipow(u[1], eb) * ipow(u[2], ec);
                    if (eb > 0) gr[1] = eb * ipow(u[0], ea) * ipow(u[1], eb - 1) * ipow(u[2], ec);
                    if (ec > 0) gr[2] = ec * ipow(u[0], ea) * ipow(u[1], eb) * ipow(u[2], ec - 1);
                    const double ug = u[0] * gr[0] + u[1] * gr[1] + u[2] * gr[2];
                    double dA[3];
                    for (int x = 0; x < 3; ++x) dA[x] = (gr[x] - ug * u[x]) / r;
                    for (int k = 0; k < K; ++k) {
                        const double ab = Aa(k, mu);
                        for (int x = 0; x < 3; ++x) g[x] += ab * (dR[k] * A[mu] * u[x] + R[k] * dA[x]);
                    }
                }
                const int j = nbr_j[b0 + q];
                for (int x = 0; x < 3; ++x) {
                    Fl[3 * static_cast<size_t>(i) + x] += g[x];
                    Fl[3 * static_cast<size_t>(j) + x] -= g[x];
                }
                for (int x = 0; x < 3; ++x)
                    for (int yy = 0; yy < 3; ++yy) Wl[3 * x + yy] -= d[x] * g[yy];
            }
        }
    }
    if (status != 0) return status;
    double Et = 0.0;
    for (int i = 0; i < N; ++i) Et += E_atom[i];
    *E = Et;
    for (size_t k = 0; k < static_cast<size_t>(N) * 3; ++k) {
        double s = 0.0;
        for (int t = 0; t < threads; ++t) s += Ft[t][k];
        F[k] = s;
    }
    for (int k = 0; k < 9; ++k) {
        double s = 0.0;
        for (int t = 0; t < threads; ++t) s += Wt[t][k];
        W[k] = s;
    }
    for (int k = 0; k < M; ++k) {
        double s = 0.0;
        for (int t = 0; t < threads; ++t) s += Gt[t][k];
        G[k] = s;
    }
    return 0;
}

}  // extern "C"
