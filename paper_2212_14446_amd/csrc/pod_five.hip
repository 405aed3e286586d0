// Five-body descriptors through the atomic basis (the extension of Sec. II.F
// to higher body order): with the four neighbours j, k, l, n of atom i and
// the six angles between them,
//   D5_{i m e} = sum_{j,k,l,n} R_m(r_ij) R_m(r_ik) R_m(r_il) R_m(r_in)
//                w_jk^e1 w_jl^e2 w_jn^e3 w_kl^e4 w_kn^e5 w_ln^e6,
// one descriptor per orbit of exponent tuples under the 24 relabellings of
// (j, k, l, n), |e| <= P5.  Expanding every power as
// (u . v)^a = sum_{|alpha| = a} mult(alpha) u^alpha v^alpha and collecting
// the monomials of each neighbour,
//   D5 = sum mult(alpha_1) ... mult(alpha_6)
//        B_{alpha_1 + alpha_2 + alpha_3} B_{alpha_1 + alpha_4 + alpha_5}
//        B_{alpha_2 + alpha_4 + alpha_6} B_{alpha_3 + alpha_5 + alpha_6},
// the five-body counterpart of eq. (30a) with the atomic basis
// B_{i m mu} = sum_j R_m(r_ij) u_ij^mu of eq. (24b).  Products with equal
// sorted index quadruples are merged into one term at compile time.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <utility>

#include "pod.h"
#include "pod_device.h"
#include "pod_internal.h"
#include "pod_tables.h"

namespace pod {
namespace {

constexpr int FIVE_MAX_ORBITS = 22;   // orbits with |e| <= 4
constexpr int FIVE_CAP = 700;         // merged terms (at most the 680 raw products for |e| <= 4)
constexpr int FIVE_THREADS = 256;
// Lanes per (atom, radial function) sharing its neighbours: two for the
// descriptors; one with the adjoint, whose per-atom work both lanes would
// otherwise repeat.
constexpr int five_split(bool adj) { return adj ? 1 : 2; }
constexpr int FIVE_PAIR_LANES = 16;   // lanes per atom in the pair-record kernel

// angle positions (j,k), (j,l), (j,n), (k,l), (k,n), (l,n) with j,k,l,n = 0..3
constexpr int FIVE_EDGE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

constexpr int edge_of(int a, int b) {
    if (a > b) { const int t = a; a = b; b = t; }
    for (int t = 0; t < 6; ++t)
        if (FIVE_EDGE[t][0] == a && FIVE_EDGE[t][1] == b) return t;
    return -1;
}

constexpr bool lex_less(const int (&a)[6], const int (&b)[6]) {
    for (int t = 0; t < 6; ++t)
        if (a[t] != b[t]) return a[t] < b[t];
    return false;
}

// k-th monomial of degree n in the device order (c ascending, then b)
constexpr void mono_of_degree(int n, int k, int& a, int& b, int& c) {
    int q = 0;
    for (int cc = 0; cc <= n; ++cc)
        for (int bb = 0; bb <= n - cc; ++bb) {
            if (q == k) { a = n - bb - cc; b = bb; c = cc; return; }
            ++q;
        }
    a = b = c = 0;
}

template <int PD>
struct FiveBuild {
    int nd;                          // orbits with |e| <= PD, in descriptor order
    int ex[FIVE_MAX_ORBITS][6];      // largest tuple of each orbit
    int nt;
    int td[FIVE_CAP], tx[FIVE_CAP], ty[FIVE_CAP], tz[FIVE_CAP], tw[FIVE_CAP], tc[FIVE_CAP];

    constexpr FiveBuild() : nd(0), ex{}, nt(0), td{}, tx{}, ty{}, tz{}, tw{}, tc{} {
        int perm[24][4] = {};
        int np = 0;
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
                for (int c = 0; c < 4; ++c)
                    for (int d = 0; d < 4; ++d)
                        if (a != b && a != c && a != d && b != c && b != d && c != d) {
                            perm[np][0] = a; perm[np][1] = b; perm[np][2] = c; perm[np][3] = d;
                            ++np;
                        }
        // orbits, degree by degree, each by its largest tuple, descending
        for (int n = 0; n <= PD; ++n) {
            const int first = nd;
            int e[6] = {};
            for (e[0] = 0; e[0] <= n; ++e[0])
                for (e[1] = 0; e[1] <= n - e[0]; ++e[1])
                    for (e[2] = 0; e[2] <= n - e[0] - e[1]; ++e[2])
                        for (e[3] = 0; e[3] <= n - e[0] - e[1] - e[2]; ++e[3])
                            for (e[4] = 0; e[4] <= n - e[0] - e[1] - e[2] - e[3]; ++e[4]) {
                                e[5] = n - e[0] - e[1] - e[2] - e[3] - e[4];
                                int best[6] = {};
                                for (int q = 0; q < np; ++q) {
                                    int img[6] = {};
                                    for (int t = 0; t < 6; ++t)
                                        img[edge_of(perm[q][FIVE_EDGE[t][0]], perm[q][FIVE_EDGE[t][1]])] = e[t];
                                    if (q == 0 || lex_less(best, img))
                                        for (int t = 0; t < 6; ++t) best[t] = img[t];
                                }
                                bool seen = false;
                                for (int d = first; d < nd; ++d) {
                                    bool same = true;
                                    for (int t = 0; t < 6; ++t) same = same && ex[d][t] == best[t];
                                    seen = seen || same;
                                }
                                if (!seen) {
                                    for (int t = 0; t < 6; ++t) ex[nd][t] = best[t];
                                    ++nd;
                                }
                            }
            for (int x = first + 1; x < nd; ++x)          // insertion sort, descending
                for (int y = x; y > first && lex_less(ex[y - 1], ex[y]); --y)
                    for (int t = 0; t < 6; ++t) {
                        const int s = ex[y][t];
                        ex[y][t] = ex[y - 1][t];
                        ex[y - 1][t] = s;
                    }
        }
        // merged products of each orbit
        for (int d = 0; d < nd; ++d) {
            const int first = nt;
            int cnt[6] = {}, idx[6] = {};
            for (int t = 0; t < 6; ++t) cnt[t] = n_of_degree(ex[d][t]);
            bool more = true;
            while (more) {
                int m[6][3] = {};
                int coef = 1;
                for (int t = 0; t < 6; ++t) {
                    mono_of_degree(ex[d][t], idx[t], m[t][0], m[t][1], m[t][2]);
                    coef *= factorial(ex[d][t]) / (factorial(m[t][0]) * factorial(m[t][1]) * factorial(m[t][2]));
                }
                int q[4] = {};
                for (int v = 0; v < 4; ++v) {   // monomial of neighbour v: sum over its three angles
                    int s[3] = {0, 0, 0};
                    for (int t = 0; t < 6; ++t)
                        if (FIVE_EDGE[t][0] == v || FIVE_EDGE[t][1] == v)
                            for (int c = 0; c < 3; ++c) s[c] += m[t][c];
                    q[v] = mono_index(s[0], s[1], s[2]);
                }
                for (int x = 1; x < 4; ++x)
                    for (int y = x; y > 0 && q[y - 1] > q[y]; --y) {
                        const int s = q[y];
                        q[y] = q[y - 1];
                        q[y - 1] = s;
                    }
                int hit = -1;
                for (int k = first; k < nt; ++k)
                    if (tx[k] == q[0] && ty[k] == q[1] && tz[k] == q[2] && tw[k] == q[3]) hit = k;
                if (hit >= 0) {
                    tc[hit] += coef;
                } else {
                    td[nt] = d; tx[nt] = q[0]; ty[nt] = q[1]; tz[nt] = q[2]; tw[nt] = q[3]; tc[nt] = coef;
                    ++nt;
                }
                int t = 0;                    // next multi-index (odometer)
                while (t < 6 && ++idx[t] == cnt[t]) idx[t++] = 0;
                more = t < 6;
            }
        }
    }
};

template <int PD>
struct FiveTable {
    static constexpr FiveBuild<PD> build{};
    static constexpr int ND = build.nd;
    static constexpr int NT = build.nt;
};

template <typename T>
struct FArgs {
    ParamsT<T> prm;   // by value: scalar loads
    CellT<T> cell;
    int N, P, K5, nd;
    const T* pos;
    const int* offsets;
    const int* nbr_j;
    const int* shift;
    T* rec;           // per pair: rhat (3), r, R_m (K5) [, R'_m (K5)]; R = R' = 0 for a pair that is not a neighbour
    int rs;           // record stride: 4 + K5, or 4 + 2 K5 with derivatives
    T* D5;            // N x K5 nd, or null
    const T* c5;      // energy: K5 x nd coefficients (m-major), or null
    T* bbar;          // energy: dE_i/dB_{i m .}, [m][i][n_mono] (scratch)
    T* Em;            // energy: per (atom, m) energies, [i][m] (scratch)
    T* V;             // forces: dE_i/dr_ij per pair (3P, scratch)
    const int* rev;
    T* E_atom;
    T* F;
    int* err;
};

// FIVE_PAIR_LANES lanes per atom walk its pairs: geometry, validation and
// the radial basis once per pair for all K5 radial functions.
template <typename T, bool FAST, bool DERIV>
__global__ __launch_bounds__(FIVE_THREADS) void five_pair_kernel(FArgs<T> g) {
    __shared__ T sQ[POD_MAX_L * POD_MAX_K];
    if (FAST) {
        for (int k = threadIdx.x; k < POD_MAX_L * POD_MAX_K; k += FIVE_THREADS) sQ[k] = (&g.prm.Q[0][0])[k];
        __syncthreads();
    }
    const int i = blockIdx.x * (FIVE_THREADS / FIVE_PAIR_LANES) + static_cast<int>(threadIdx.x) / FIVE_PAIR_LANES;
    const int l = static_cast<int>(threadIdx.x) % FIVE_PAIR_LANES;
    if (i >= g.N) return;
    const int p0 = max(g.offsets[i], 0);
    int p1 = g.offsets[i + 1];
    if (p1 > g.P) {
        if (l == 0) atomicOr(g.err, ERR_NEIGH);
        p1 = g.P;
    }
    for (int p = p0 + l; p < p1; p += FIVE_PAIR_LANES) {
        T* row = g.rec + static_cast<size_t>(p) * g.rs;
        T u[3] = {T(0), T(0), T(0)};
        T r = T(0.5) * (g.prm.rin + g.prm.rcut);
        bool ok = false;
        const int j = g.nbr_j[p];
        const int sh = g.shift[p];
        if (j < 0 || j >= g.N || (!g.cell.periodic && (sh & 0xFFFFFF) != 0)) {
            atomicOr(g.err, ERR_NEIGH);
        } else {
            const T sx = static_cast<T>(dev::unpack_shift(sh, 0));
            const T sy = static_cast<T>(dev::unpack_shift(sh, 1));
            const T sz = static_cast<T>(dev::unpack_shift(sh, 2));
            const T* c = g.cell.a;
            const T d0 = g.pos[3 * j] - g.pos[3 * i] + sx * c[0] + sy * c[3] + sz * c[6];
            const T d1 = g.pos[3 * j + 1] - g.pos[3 * i + 1] + sx * c[1] + sy * c[4] + sz * c[7];
            const T d2 = g.pos[3 * j + 2] - g.pos[3 * i + 2] + sx * c[2] + sy * c[5] + sz * c[8];
            const T r2 = d0 * d0 + d1 * d1 + d2 * d2;
            if (!dev::d_finite(r2)) {
                atomicOr(g.err, ERR_NONFINITE);
            } else {
                const T rr = dev::d_sqrt(r2);
                if (rr <= g.prm.rin) {
                    atomicOr(g.err, ERR_RANGE);
                } else if (rr < g.prm.rcut) {   // beyond rcut: a skin-list entry, not a neighbour
                    ok = true;
                    r = rr;
                    u[0] = d0 / rr;
                    u[1] = d1 / rr;
                    u[2] = d2 / rr;
                }
            }
        }
        T R[FAST_MAX_K], dR[FAST_MAX_K];
        if constexpr (FAST) dev::radial_std<T, DERIV>(&g.prm, sQ, r, T(1) / r, R, dR);
        else dev::radial<T, DERIV>(&g.prm, r, T(1) / r, R, dR);
        row[0] = u[0];
        row[1] = u[1];
        row[2] = u[2];
        row[3] = r;
#pragma unroll
        for (int k = 0; k < FAST_MAX_K; ++k)
            if (k < g.K5) {
                row[4 + k] = ok ? R[k] : T(0);
                if (DERIV) row[4 + g.K5 + k] = ok ? dR[k] : T(0);
            }
    }
}

template <typename T, int PD, bool ADJ>
__global__ __launch_bounds__(FIVE_THREADS) void five_kernel(FArgs<T> g) {
    constexpr int NA = n_mono(PD);
    using Tab = FiveTable<PD>;
    const int m = blockIdx.y;
    constexpr int SPLIT = five_split(ADJ);
    const int i = blockIdx.x * (FIVE_THREADS / SPLIT) + static_cast<int>(threadIdx.x) / SPLIT;
    const int sub = static_cast<int>(threadIdx.x) % SPLIT;
    if (i >= g.N) return;   // the whole group of the atom
    T B[NA];
#pragma unroll
    for (int mu = 0; mu < NA; ++mu) B[mu] = T(0);
    const int p0 = max(g.offsets[i], 0);
    int p1 = g.offsets[i + 1];
    if (p1 > g.P) {
        if (sub == 0) atomicOr(g.err, ERR_NEIGH);
        p1 = g.P;
    }
    for (int p = p0 + sub; p < p1; p += SPLIT) {
        const T* row = g.rec + static_cast<size_t>(p) * g.rs;
        dev::accumulate_basis<T, PD>(B, row[4 + m], row[0], row[1], row[2]);
    }
#pragma unroll
    for (int mu = 0; mu < NA; ++mu) {
        T v = B[mu];
#pragma unroll
        for (int o = 1; o < SPLIT; o <<= 1) v += __shfl_xor(v, o);
        B[mu] = v;
    }
    T acc[Tab::ND];
#pragma unroll
    for (int d = 0; d < Tab::ND; ++d) acc[d] = T(0);
#pragma unroll
    for (int t = 0; t < Tab::NT; ++t)
        acc[Tab::build.td[t]] += T(Tab::build.tc[t]) * B[Tab::build.tx[t]] * B[Tab::build.ty[t]] *
                                 B[Tab::build.tz[t]] * B[Tab::build.tw[t]];
    if constexpr (!ADJ) {
        if (sub == 0) {
            T* out = g.D5 + static_cast<size_t>(i) * g.K5 * g.nd + static_cast<size_t>(m) * g.nd;
#pragma unroll
            for (int d = 0; d < Tab::ND; ++d)
                if (d < g.nd) out[d] = acc[d];
        }
    } else {
        // E_im = sum_d c5_{m d} D5_{i m d} and dE_im/dB by the product rule on
        // every merged product (orbits beyond P5 weigh 0)
        const T* cm = g.c5 + static_cast<size_t>(m) * g.nd;
        T cw[Tab::ND];
        T e = T(0);
#pragma unroll
        for (int d = 0; d < Tab::ND; ++d) {
            cw[d] = d < g.nd ? cm[d] : T(0);
            e += cw[d] * acc[d];
        }
        T bb[NA];
#pragma unroll
        for (int mu = 0; mu < NA; ++mu) bb[mu] = T(0);
        // one instance per merged product, so every index is a constant
        auto term = [&]<int t>() {
            constexpr int x = Tab::build.tx[t], y = Tab::build.ty[t], z = Tab::build.tz[t], w = Tab::build.tw[t];
            const T c = cw[Tab::build.td[t]] * T(Tab::build.tc[t]);
            const T pxy = B[x] * B[y], pzw = B[z] * B[w];
            bb[x] += c * B[y] * pzw;
            bb[y] += c * B[x] * pzw;
            bb[z] += c * pxy * B[w];
            bb[w] += c * pxy * B[z];
        };
        [&]<int... ts>(std::integer_sequence<int, ts...>) {
            (term.template operator()<ts>(), ...);
        }(std::make_integer_sequence<int, Tab::NT>{});
        if (sub == 0) {
            g.Em[static_cast<size_t>(i) * g.K5 + m] = e;
            T* out = g.bbar + (static_cast<size_t>(m) * g.N + i) * NA;
#pragma unroll
            for (int mu = 0; mu < NA; ++mu) out[mu] = bb[mu];
        }
    }
}

// FIVE_PAIR_LANES lanes per atom: for each pair, d E_i / d r_ij =
// sum_m [R'_m h_m rhat + R_m (grad_u h_m - (u . grad_u h_m) u) / r] with
// h_m(u) = sum_mu dE_i/dB_{i m mu} u^mu (eq. (24c) with the five-body adjoint).
template <typename T, int PD>
__global__ __launch_bounds__(FIVE_THREADS) void five_grad_kernel(FArgs<T> g) {
    constexpr MonoTable<PD> mt{};
    constexpr int NA = n_mono(PD);
    const int i = blockIdx.x * (FIVE_THREADS / FIVE_PAIR_LANES) + static_cast<int>(threadIdx.x) / FIVE_PAIR_LANES;
    const int l = static_cast<int>(threadIdx.x) % FIVE_PAIR_LANES;
    if (i >= g.N) return;
    const int p0 = max(g.offsets[i], 0);
    const int p1 = min(g.offsets[i + 1], g.P);
    for (int p = p0 + l; p < p1; p += FIVE_PAIR_LANES) {
        const T* row = g.rec + static_cast<size_t>(p) * g.rs;
        const T ux = row[0], uy = row[1], uz = row[2], ir = T(1) / row[3];
        T A[NA];
        A[0] = T(1);
#pragma unroll
        for (int mu = 1; mu < NA; ++mu) {
            const T u = mt.axis[mu] == 0 ? ux : (mt.axis[mu] == 1 ? uy : uz);
            A[mu] = A[mt.par[mu]] * u;
        }
        T v0 = T(0), v1 = T(0), v2 = T(0);
        for (int m = 0; m < g.K5; ++m) {
            const T Rm = row[4 + m], dRm = row[4 + g.K5 + m];
            const T* bb = g.bbar + (static_cast<size_t>(m) * g.N + i) * NA;
            T h = T(0), eul = T(0), q0 = T(0), q1 = T(0), q2 = T(0);
#pragma unroll
            for (int mu = 0; mu < NA; ++mu) {
                const T b = bb[mu];
                const T ba = b * A[mu];
                h += ba;
                if (mt.deg[mu] > 0) eul += T(mt.deg[mu]) * ba;
                if (mt.down[mu][0] >= 0) q0 += T(mt.ex[mu][0]) * b * A[mt.down[mu][0]];
                if (mt.down[mu][1] >= 0) q1 += T(mt.ex[mu][1]) * b * A[mt.down[mu][1]];
                if (mt.down[mu][2] >= 0) q2 += T(mt.ex[mu][2]) * b * A[mt.down[mu][2]];
            }
            const T c1 = dRm * h - Rm * eul * ir;
            const T c2 = Rm * ir;
            v0 += c1 * ux + c2 * q0;
            v1 += c1 * uy + c2 * q1;
            v2 += c1 * uz + c2 * q2;
        }
        g.V[3 * static_cast<size_t>(p)] = v0;
        g.V[3 * static_cast<size_t>(p) + 1] = v1;
        g.V[3 * static_cast<size_t>(p) + 2] = v2;
    }
}

// F_i = sum over the pairs p of i of (V_p - V_rev(p)); E_i = sum_m E_im.
template <typename T>
__global__ __launch_bounds__(FIVE_THREADS) void five_gather_kernel(FArgs<T> g) {
    const int i = blockIdx.x * (FIVE_THREADS / FIVE_PAIR_LANES) + static_cast<int>(threadIdx.x) / FIVE_PAIR_LANES;
    const int l = static_cast<int>(threadIdx.x) % FIVE_PAIR_LANES;
    if (i >= g.N) return;
    if (g.E_atom && l == 0) {
        T e = T(0);
        for (int m = 0; m < g.K5; ++m) e += g.Em[static_cast<size_t>(i) * g.K5 + m];
        g.E_atom[i] = e;
    }
    if (!g.F) return;
    const int p0 = max(g.offsets[i], 0);
    const int p1 = min(g.offsets[i + 1], g.P);
    T f0 = T(0), f1 = T(0), f2 = T(0);
    for (int p = p0 + l; p < p1; p += FIVE_PAIR_LANES) {
        const int q = g.rev[p];
        f0 += g.V[3 * static_cast<size_t>(p)];
        f1 += g.V[3 * static_cast<size_t>(p) + 1];
        f2 += g.V[3 * static_cast<size_t>(p) + 2];
        if (q < 0 || q >= g.P) {
            atomicOr(g.err, ERR_NEIGH);
            continue;
        }
        f0 -= g.V[3 * static_cast<size_t>(q)];
        f1 -= g.V[3 * static_cast<size_t>(q) + 1];
        f2 -= g.V[3 * static_cast<size_t>(q) + 2];
    }
#pragma unroll
    for (int o = 1; o < FIVE_PAIR_LANES; o <<= 1) {
        f0 += __shfl_xor(f0, o);
        f1 += __shfl_xor(f1, o);
        f2 += __shfl_xor(f2, o);
    }
    if (l == 0) {
        g.F[3 * static_cast<size_t>(i)] = f0;
        g.F[3 * static_cast<size_t>(i) + 1] = f1;
        g.F[3 * static_cast<size_t>(i) + 2] = f2;
    }
}

int n_orbits(int P5) {
    constexpr FiveBuild<4> b{};
    int n = 0;
    for (int d = 0; d < b.nd; ++d) {
        int s = 0;
        for (int t = 0; t < 6; ++t) s += b.ex[d][t];
        if (s <= P5) ++n;
    }
    return n;
}

size_t align256(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

// Descriptors (D5), or with coefficients the energy and forces.
template <typename T>
int five_impl(pod_handle* h, const ParamsT<T>& prm, int N, int P, const void* pos, const double* cell,
              const int* offsets, const int* nbr_j, const int* shift, const int* rev, int K5, int P5, void* D5,
              const void* c5, void* E_atom, void* F) {
    FArgs<T> g;
    g.prm = prm;
    g.cell.periodic = cell != nullptr;
    for (int k = 0; k < 9; ++k) {
        const double v = cell ? cell[k] : 0.0;
        if (!std::isfinite(v)) return POD_EINVAL;
        g.cell.a[k] = static_cast<T>(v);
    }
    const bool energy = c5 != nullptr;
    const bool deriv = energy && F != nullptr;
    g.N = N;
    g.P = P;
    g.K5 = K5;
    g.nd = n_orbits(P5);
    g.pos = static_cast<const T*>(pos);
    g.offsets = offsets;
    g.nbr_j = nbr_j;
    g.shift = shift;
    g.rs = 4 + (deriv ? 2 : 1) * K5;
    g.D5 = static_cast<T*>(D5);
    g.c5 = static_cast<const T*>(c5);
    g.rev = rev;
    g.E_atom = static_cast<T*>(E_atom);
    g.F = static_cast<T*>(F);
    g.err = h->d_err;
    const int NA = P5 <= 2 ? n_mono(2) : n_mono(4);
    const size_t b_rec = align256(sizeof(T) * static_cast<size_t>(P) * g.rs);
    const size_t b_bar = energy ? align256(sizeof(T) * static_cast<size_t>(N) * K5 * NA) : 0;
    const size_t b_em = energy ? align256(sizeof(T) * static_cast<size_t>(N) * K5) : 0;
    const size_t b_v = deriv ? align256(sizeof(T) * 3 * static_cast<size_t>(P)) : 0;
    const int rc = ensure_scratch(h, b_rec + b_bar + b_em + b_v + 256);
    if (rc != POD_OK) return rc;
    char* base = static_cast<char*>(h->d_scratch);
    g.rec = reinterpret_cast<T*>(base);
    g.bbar = energy ? reinterpret_cast<T*>(base + b_rec) : nullptr;
    g.Em = energy ? reinterpret_cast<T*>(base + b_rec + b_bar) : nullptr;
    g.V = deriv ? reinterpret_cast<T*>(base + b_rec + b_bar + b_em) : nullptr;
    const int apb = FIVE_THREADS / FIVE_PAIR_LANES;
    const dim3 agrid((N + apb - 1) / apb);
    if (P > 0) {
        timing_begin(h, 0);
        if (prm.std_ok) {
            if (deriv) hipLaunchKernelGGL((five_pair_kernel<T, true, true>), agrid, dim3(FIVE_THREADS), 0, h->stream, g);
            else hipLaunchKernelGGL((five_pair_kernel<T, true, false>), agrid, dim3(FIVE_THREADS), 0, h->stream, g);
        } else {
            if (deriv) hipLaunchKernelGGL((five_pair_kernel<T, false, true>), agrid, dim3(FIVE_THREADS), 0, h->stream, g);
            else hipLaunchKernelGGL((five_pair_kernel<T, false, false>), agrid, dim3(FIVE_THREADS), 0, h->stream, g);
        }
        timing_end(h, 0);
    }
    const int fpb = FIVE_THREADS / five_split(energy);
    const dim3 grid((N + fpb - 1) / fpb, K5);
    timing_begin(h, 1);
    if (P5 <= 2) {
        if (energy) hipLaunchKernelGGL((five_kernel<T, 2, true>), grid, dim3(FIVE_THREADS), 0, h->stream, g);
        else hipLaunchKernelGGL((five_kernel<T, 2, false>), grid, dim3(FIVE_THREADS), 0, h->stream, g);
    } else {
        if (energy) hipLaunchKernelGGL((five_kernel<T, 4, true>), grid, dim3(FIVE_THREADS), 0, h->stream, g);
        else hipLaunchKernelGGL((five_kernel<T, 4, false>), grid, dim3(FIVE_THREADS), 0, h->stream, g);
    }
    timing_end(h, 1);
    if (energy) {
        timing_begin(h, 0);
        if (deriv && P > 0) {
            if (P5 <= 2) hipLaunchKernelGGL((five_grad_kernel<T, 2>), agrid, dim3(FIVE_THREADS), 0, h->stream, g);
            else hipLaunchKernelGGL((five_grad_kernel<T, 4>), agrid, dim3(FIVE_THREADS), 0, h->stream, g);
        }
        hipLaunchKernelGGL((five_gather_kernel<T>), agrid, dim3(FIVE_THREADS), 0, h->stream, g);
        timing_end(h, 0);
    }
    return hipGetLastError() == hipSuccess ? POD_OK : POD_EHIP;
}

static_assert(FiveTable<4>::ND == FIVE_MAX_ORBITS, "orbit count for |e| <= 4");
static_assert(FiveTable<4>::NT <= FIVE_CAP, "merged five-body terms");

}  // namespace
}  // namespace pod

extern "C" {

int pod_five_body_count(int P5, int* n) {
    if (!n || P5 < 0) return POD_EINVAL;
    if (P5 > POD_FIVE_MAX_P) return POD_ENOTSUP;
    *n = pod::n_orbits(P5);
    return POD_OK;
}

int pod_five_body_descriptors(pod_handle* h, int N, int P, const void* pos, const double* cell, const int* offsets,
                              const int* nbr_j, const int* shift, int K5, int P5, void* D5) {
    using namespace pod;
    if (!h || N < 0 || P < 0 || K5 < 1 || K5 > h->K || P5 < 0) return POD_EINVAL;
    if (P5 > POD_FIVE_MAX_P || K5 > FAST_MAX_K) return POD_ENOTSUP;
    if (N > 0 && (!pos || !offsets || !D5 || (P > 0 && (!nbr_j || !shift)))) return POD_EINVAL;
    if (N == 0) return POD_OK;
    if (h->dtype == POD_F64)
        return five_impl<double>(h, h->hp_d, N, P, pos, cell, offsets, nbr_j, shift, nullptr, K5, P5, D5, nullptr,
                                 nullptr, nullptr);
    return five_impl<float>(h, h->hp_f, N, P, pos, cell, offsets, nbr_j, shift, nullptr, K5, P5, D5, nullptr,
                            nullptr, nullptr);
}

int pod_five_body_energy_forces(pod_handle* h, int N, int P, const void* pos, const double* cell, const int* offsets,
                                const int* nbr_j, const int* shift, const int* rev, int K5, int P5, const void* c5,
                                void* E_atom, void* F) {
    using namespace pod;
    if (!h || N < 0 || P < 0 || K5 < 1 || K5 > h->K || P5 < 0) return POD_EINVAL;
    if (P5 > POD_FIVE_MAX_P || K5 > FAST_MAX_K) return POD_ENOTSUP;
    if (N > 0 && (!pos || !offsets || !c5 || (!E_atom && !F) || (P > 0 && (!nbr_j || !shift))))
        return POD_EINVAL;
    if (N > 0 && F && P > 0 && !rev) return POD_EINVAL;
    if (N == 0) return POD_OK;
    if (h->dtype == POD_F64)
        return five_impl<double>(h, h->hp_d, N, P, pos, cell, offsets, nbr_j, shift, rev, K5, P5, nullptr, c5,
                                 E_atom, F);
    return five_impl<float>(h, h->hp_f, N, P, pos, cell, offsets, nbr_j, shift, rev, K5, P5, nullptr, c5, E_atom,
                            F);
}

}  // extern "C"
