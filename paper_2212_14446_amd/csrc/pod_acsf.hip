// Atom-centred symmetry functions (Sec. III.B) evaluated through the atomic
// basis of Sec. II.E: the radial functions G2 of eq. (21c), the angular
// functions G3 of eq. (22c) and the four-body functions G4 of eq. (22d), in
// work linear in the number of neighbours.
//
// A radial channel (eta, r_s) has g(r) = exp(-eta (r - r_s)^2) f_c(r) and the
// atomic basis B_mu = sum_j g(r_ij) u_ij^mu (eq. (24b) with g in place of
// R_m).  Expanding the integer powers binomially and using
// (u . v)^n = sum_{|mu| = n} mult(mu) u^mu v^mu,
//   G2 = B_0,
//   G3 = 2^(1-zeta) sum_n C(zeta, n) lambda^n S_n,
//        S_n = sum_{|mu| = n} mult(mu) B_mu^2                   (eq. (26a)),
//   G4 = sum_{n1 <= a, n2 <= b, n3 <= c} C(a, n1) C(b, n2) C(c, n3)
//        alpha^n1 beta^n2 gamma^n3 T(n1, n2, n3),
// where T(n1, n2, n3) = sum_{j,k,l} g_j g_k g_l w_jk^n1 w_jl^n2 w_kl^n3 is
// symmetric in its arguments and is the four-body sum of eq. (30a) (eq. (27a)
// for (n, 0, 0)) at the sorted triple.  Every function is thus a fixed linear
// combination of the invariants of its channel,
//   I = [B_0 | S_0 .. S_6 | T_p for the 23 sorted triples of degree <= 6],
// with coefficients built once on the host.
//
// Kernels (handle dtype T):
//   basis_kernel<PD>  2-4 lanes per atom, a few channels of angular degree
//                     class PD (0, 2, 4, 6) per grid row: B in registers,
//                     invariants, functions; with weights W, the adjoint
//                     dL/dB of each channel (written to scratch).
//   pair_kernel<PDM>  16 lanes per atom, one pair per lane: the derivative of
//                     sum_c dL/dB_c . B_c with respect to r_ij (eq. (24c) with
//                     g, g' in place of R_m, R'_m), summed over channels.
//   gather_kernel     F_i = sum over the pairs p of i of (V_p - V_rev(p)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "pod.h"
#include "pod_device.h"
#include "pod_internal.h"
#include "pod_tables.h"

namespace pod {
namespace {

constexpr int ACSF_NI = 31;          // [B_0 | S_0..S_6 | T_p, p < 23]
constexpr int ACSF_S0 = 1;
constexpr int ACSF_T0 = 8;
constexpr int ACSF_THREADS = 256;
// Lanes per atom in the basis kernels: four, or two for the FP64 adjoint of
// degree 4 and above, whose per-atom work (repeated by every lane of the
// atom) then outweighs the shorter neighbour loop (measured: 45.6 -> 35.1 us
// for the angular channels of the 15,840-atom box; slower in the other cases).
template <typename T, int PD, bool ADJ>
constexpr int acsf_split() { return (ADJ && PD >= 4 && sizeof(T) == 8) ? 2 : 4; }
constexpr int GATHER_LANES = 16;                       // lanes per atom in the force gather
constexpr int PAIR_LANES = 16;                         // lanes per atom in the pair-gradient kernel

// Channels of one degree class a basis thread carries at once.
constexpr int channels_per_thread(int pd) { return pd == 0 ? 8 : (pd == 2 ? 2 : 1); }

// Degree class of a channel: the smallest instantiated PD >= need.
int degree_class(int need) { return need <= 0 ? 0 : (need <= 2 ? 2 : (need <= 4 ? 4 : 6)); }

template <typename T>
struct AChan {
    T eta, rs;
    int pd;       // degree class
    int d0, d1;   // functions of this channel in the sorted order
    int bpre;     // adjoint scratch: sum of n_mono(pd) over the earlier channels
};

}  // namespace
}  // namespace pod

struct pod_acsf {
    int dtype;
    int nd, nch, pd_max, bsum;
    std::vector<int> cls_ch[4];   // channels of each degree class (0, 2, 4, 6)
    void* d_ch;                   // nch AChan<T>
    void* d_coef;                 // nd x ACSF_NI, sorted order
    int* d_col;                   // nd: output column of each sorted function
    int* d_cls;                   // channels of each class, concatenated
    int cls_off[5];
};

namespace pod {
namespace {

template <typename T>
struct AArgs {
    int N, nd;
    T rin, rcut, inv_h;
    int periodic;
    T cell[9];
    const T* pos;
    const int* offsets;
    const int* nbr_j;
    const int* shift;
    const AChan<T>* ch;
    const T* coef;
    const int* col;
    T* G;            // N x nd or null
    const T* W;      // weights: row i at W + i * ldw (ldw 0: one shared row)
    long ldw;
    T* bbar;         // adjoint scratch, channel-major [c][i][mu]
    T* V;            // P x 3 pair gradients
    const int* rev;
    T* F;
    int P;
    int* err;
};

// Pair p of atom i: unit vector and distance when 0 < r < rcut; errors of the
// list and of the coordinates are latched as in the POD kernels.
template <typename T>
__device__ __forceinline__ bool pair_geometry(const AArgs<T>& g, int i, int p, T& r, T& ux, T& uy, T& uz) {
    const int j = g.nbr_j[p];
    const int sh = g.shift[p];
    if (j < 0 || j >= g.N || (!g.periodic && (sh & 0xFFFFFF) != 0)) {
        atomicOr(g.err, ERR_NEIGH);
        return false;
    }
    const T sx = static_cast<T>(dev::unpack_shift(sh, 0));
    const T sy = static_cast<T>(dev::unpack_shift(sh, 1));
    const T sz = static_cast<T>(dev::unpack_shift(sh, 2));
    const T* c = g.cell;
    const T d0 = g.pos[3 * j] - g.pos[3 * i] + sx * c[0] + sy * c[3] + sz * c[6];
    const T d1 = g.pos[3 * j + 1] - g.pos[3 * i + 1] + sx * c[1] + sy * c[4] + sz * c[7];
    const T d2 = g.pos[3 * j + 2] - g.pos[3 * i + 2] + sx * c[2] + sy * c[5] + sz * c[8];
    const T r2 = d0 * d0 + d1 * d1 + d2 * d2;
    if (!dev::d_finite(r2)) {
        atomicOr(g.err, ERR_NONFINITE);
        return false;
    }
    r = dev::d_sqrt(r2);
    if (r <= g.rin) {
        atomicOr(g.err, ERR_RANGE);
        return false;
    }
    if (r >= g.rcut) return false;   // a skin-list entry: not a neighbour
    const T ir = T(1) / r;
    ux = d0 * ir;
    uy = d1 * ir;
    uz = d2 * ir;
    return true;
}

// Pair range of atom i clamped to [0, P); a range beyond P is a list error.
template <typename T>
__device__ __forceinline__ void pair_range(const AArgs<T>& g, int i, int& p0, int& p1) {
    p0 = max(g.offsets[i], 0);
    p1 = g.offsets[i + 1];
    if (p1 > g.P) {
        atomicOr(g.err, ERR_NEIGH);
        p1 = g.P;
    }
}

// Cut-off function of eq. (8) and its derivative.
template <typename T>
__device__ __forceinline__ void cutoff(T r, T rin, T inv_h, T& fc, T& dfc) {
    const T t = (r - rin) * inv_h;
    const T t2 = t * t;
    const T y = T(1) - t2 * t;
    const T s = y * y + T(1e-6);
    const T rs = dev::d_rsqrt(s);
    fc = dev::d_exp(T(1) - rs);
    dfc = fc * y * (rs * rs * rs) * (T(-3) * t2 * inv_h);
}

// Invariants of one channel from its basis B, the functions of the channel
// and (ADJ) the adjoint dL/dB for L = sum_d W_d G_d; written when `write`.
template <typename T, int PD, bool ADJ>
__device__ __forceinline__ void finish_channel(const AArgs<T>& g, const AChan<T>& ch, int i,
                                               const T (&B)[n_mono(PD)], bool write) {
    constexpr MonoTable<PD> mt{};
    constexpr int NA = n_mono(PD);
    using Tab = D4Table<PD>;
    constexpr int KA = Tab::KA;
    constexpr int NT = Tab::NT;
    T S[PD + 1];
#pragma unroll
    for (int n = 0; n <= PD; ++n) S[n] = T(0);
#pragma unroll
    for (int mu = 0; mu < NA; ++mu) S[mt.deg[mu]] += T(mt.mult[mu]) * B[mu] * B[mu];
    T Tq[KA];
#pragma unroll
    for (int p = 0; p < KA; ++p) Tq[p] = (Tab::build.pb[p] == 0) ? B[0] * S[Tab::build.pa[p]] : T(0);
#pragma unroll
    for (int t = 0; t < NT; ++t)
        Tq[Tab::build.tp[t]] += T(Tab::build.tc[t]) * B[Tab::build.tx[t]] * B[Tab::build.ty[t]] * B[Tab::build.tz[t]];

    if (g.G && write) {
        for (int d = ch.d0; d < ch.d1; ++d) {
            const T* cf = g.coef + static_cast<size_t>(d) * ACSF_NI;
            T v = cf[0] * B[0];
#pragma unroll
            for (int n = 0; n <= PD; ++n) v += cf[ACSF_S0 + n] * S[n];
#pragma unroll
            for (int p = 0; p < KA; ++p) v += cf[ACSF_T0 + p] * Tq[p];
            g.G[static_cast<size_t>(i) * g.nd + g.col[d]] = v;
        }
    }
    if constexpr (ADJ) {
        // adjoint of the invariants: Ibar_k = sum_d W_d coef_dk
        T b0 = T(0);
        T Sb[PD + 1];
        T Tb[KA];
#pragma unroll
        for (int n = 0; n <= PD; ++n) Sb[n] = T(0);
#pragma unroll
        for (int p = 0; p < KA; ++p) Tb[p] = T(0);
        const T* wrow = g.W + static_cast<size_t>(i) * g.ldw;
        for (int d = ch.d0; d < ch.d1; ++d) {
            const T* cf = g.coef + static_cast<size_t>(d) * ACSF_NI;
            const T w = wrow[g.col[d]];
            b0 += w * cf[0];
#pragma unroll
            for (int n = 0; n <= PD; ++n) Sb[n] += w * cf[ACSF_S0 + n];
#pragma unroll
            for (int p = 0; p < KA; ++p) Tb[p] += w * cf[ACSF_T0 + p];
        }
        // T_(n,0,0) = B_0 S_n (eq. (27a)); the other T_p are sums of triple products
        T bb[NA];
#pragma unroll
        for (int mu = 0; mu < NA; ++mu) bb[mu] = T(0);
#pragma unroll
        for (int p = 0; p < KA; ++p)
            if (Tab::build.pb[p] == 0) {
                b0 += Tb[p] * S[Tab::build.pa[p]];
                Sb[Tab::build.pa[p]] += Tb[p] * B[0];
            }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const T w = Tb[Tab::build.tp[t]] * T(Tab::build.tc[t]);
            const int x = Tab::build.tx[t], y = Tab::build.ty[t], z = Tab::build.tz[t];
            bb[x] += w * B[y] * B[z];
            bb[y] += w * B[x] * B[z];
            bb[z] += w * B[x] * B[y];
        }
        bb[0] += b0;
#pragma unroll
        for (int mu = 0; mu < NA; ++mu) bb[mu] += T(2 * mt.mult[mu]) * B[mu] * Sb[mt.deg[mu]];
        if (write) {
            T* out = g.bbar + static_cast<size_t>(g.N) * ch.bpre + static_cast<size_t>(i) * NA;
#pragma unroll
            for (int mu = 0; mu < NA; ++mu) out[mu] = bb[mu];
        }
    }
}

// One atom per SPLIT consecutive lanes, which share its neighbours (lane s
// takes pairs s, s + SPLIT, ...) and sum their partial bases with
// butterfly shuffles (a fixed order, identical on the lanes); each thread
// carries the bases of up to channels_per_thread(PD) channels of the class,
// so the pair geometry and f_c are computed once for all of them.
template <typename T, int PD, bool ADJ>
__global__ __launch_bounds__(ACSF_THREADS) void basis_kernel(AArgs<T> g, const int* __restrict__ chans, int nclass) {
    constexpr int NA = n_mono(PD);
    constexpr int NC = channels_per_thread(PD);
    const int c0 = blockIdx.y * NC;
    const int nc = min(NC, nclass - c0);
    AChan<T> ch[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) ch[k] = g.ch[chans[c0 + (k < nc ? k : 0)]];
    constexpr int SPLIT = acsf_split<T, PD, ADJ>();
    const int i = blockIdx.x * (ACSF_THREADS / SPLIT) + static_cast<int>(threadIdx.x) / SPLIT;
    const int sub = static_cast<int>(threadIdx.x) % SPLIT;
    if (i >= g.N) return;   // the whole group of the atom

    T B[NC][NA];
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
        for (int mu = 0; mu < NA; ++mu) B[k][mu] = T(0);
    int p0, p1;
    pair_range(g, i, p0, p1);
    for (int p = p0 + sub; p < p1; p += SPLIT) {
        T r, ux, uy, uz;
        if (!pair_geometry(g, i, p, r, ux, uy, uz)) continue;
        T fc, dfc;
        cutoff(r, g.rin, g.inv_h, fc, dfc);
#pragma unroll
        for (int k = 0; k < NC; ++k)
            if (k < nc) {
                const T x = r - ch[k].rs;
                dev::accumulate_basis<T, PD>(B[k], dev::d_exp(-ch[k].eta * x * x) * fc, ux, uy, uz);
            }
    }
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
        for (int mu = 0; mu < NA; ++mu) {
            T v = B[k][mu];
#pragma unroll
            for (int o = 1; o < SPLIT; o <<= 1) v += __shfl_xor(v, o);
            B[k][mu] = v;
        }
#pragma unroll
    for (int k = 0; k < NC; ++k)
        if (k < nc) finish_channel<T, PD, ADJ>(g, ch[k], i, B[k], sub == 0);
}

// sum_mu bb_mu A_mu (h), its u-gradient (q) and the Euler sum u . grad h =
// sum_mu deg(mu) bb_mu A_mu for the first n_mono(PD) monomials.
template <typename T, int PD, int PDM>
__device__ __forceinline__ void contract(const T* __restrict__ bb, const T (&A)[n_mono(PDM)], T& h, T& eul, T& q0,
                                         T& q1, T& q2) {
    constexpr MonoTable<PDM> mt{};
    constexpr int NA = n_mono(PD);
    h = eul = q0 = q1 = q2 = T(0);
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
}

// PAIR_LANES lanes per atom walk its pairs (pairs outside every atom's
// range keep whatever the caller's buffer held and are never read).
template <typename T, int PDM>
__global__ __launch_bounds__(ACSF_THREADS) void pair_kernel(AArgs<T> g, int nch) {
    constexpr MonoTable<PDM> mt{};
    constexpr int NAM = n_mono(PDM);
    const int i = blockIdx.x * (ACSF_THREADS / PAIR_LANES) + static_cast<int>(threadIdx.x) / PAIR_LANES;
    const int l = static_cast<int>(threadIdx.x) % PAIR_LANES;
    if (i >= g.N) return;
    int p0, p1;
    pair_range(g, i, p0, p1);
    for (int p = p0 + l; p < p1; p += PAIR_LANES) {
    T v0 = T(0), v1 = T(0), v2 = T(0);
    T r, ux, uy, uz;
    if (pair_geometry(g, i, p, r, ux, uy, uz)) {
        T fc, dfc;
        cutoff(r, g.rin, g.inv_h, fc, dfc);
        const T ir = T(1) / r;
        T A[NAM];
        A[0] = T(1);
#pragma unroll
        for (int mu = 1; mu < NAM; ++mu) {
            const T u = mt.axis[mu] == 0 ? ux : (mt.axis[mu] == 1 ? uy : uz);
            A[mu] = A[mt.par[mu]] * u;
        }
        for (int c = 0; c < nch; ++c) {
            const AChan<T> ch = g.ch[c];
            const T x = r - ch.rs;
            const T e = dev::d_exp(-ch.eta * x * x);
            const T gv = e * fc;
            const T gd = e * (dfc - T(2) * ch.eta * x * fc);
            T h, eul, q0, q1, q2;
            const T* bb = g.bbar + static_cast<size_t>(g.N) * ch.bpre + static_cast<size_t>(i) * n_mono(ch.pd);
            switch (ch.pd) {
                case 0: contract<T, 0, PDM>(bb, A, h, eul, q0, q1, q2); break;
                case 2: if constexpr (PDM >= 2) contract<T, 2, PDM>(bb, A, h, eul, q0, q1, q2); break;
                case 4: if constexpr (PDM >= 4) contract<T, 4, PDM>(bb, A, h, eul, q0, q1, q2); break;
                default: if constexpr (PDM >= 6) contract<T, 6, PDM>(bb, A, h, eul, q0, q1, q2); break;
            }
            // d/dr_ij of g(r) h(u): g' h rhat + g (grad_u h - (u . grad_u h) u) / r
            const T c1 = gd * h - gv * eul * ir;
            const T c2 = gv * ir;
            v0 += c1 * ux + c2 * q0;
            v1 += c1 * uy + c2 * q1;
            v2 += c1 * uz + c2 * q2;
        }
    }
    g.V[3 * static_cast<size_t>(p)] = v0;
    g.V[3 * static_cast<size_t>(p) + 1] = v1;
    g.V[3 * static_cast<size_t>(p) + 2] = v2;
    }
}

// F_i = -dE/dx_i: E_i depends on x_j - x_i through the pairs of i, and x_i
// enters the pairs (j -> i) of its neighbours, which rev finds.
// GATHER_LANES lanes per atom share its pairs and sum with butterfly shuffles.
template <typename T>
__global__ __launch_bounds__(ACSF_THREADS) void gather_kernel(AArgs<T> g) {
    const int i = blockIdx.x * (ACSF_THREADS / GATHER_LANES) + static_cast<int>(threadIdx.x) / GATHER_LANES;
    const int l = static_cast<int>(threadIdx.x) % GATHER_LANES;
    if (i >= g.N) return;   // the whole group of the atom
    T f0 = T(0), f1 = T(0), f2 = T(0);
    int p0, p1;
    pair_range(g, i, p0, p1);
    for (int p = p0 + l; p < p1; p += GATHER_LANES) {
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
    for (int o = 1; o < GATHER_LANES; o <<= 1) {
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

bool integral(double x, int lo, int hi, int* out) {
    if (!std::isfinite(x) || x != std::floor(x) || x < lo || x > hi) return false;
    *out = static_cast<int>(x);
    return true;
}

double binom(int n, int k) {
    double b = 1.0;
    for (int t = 1; t <= k; ++t) b = b * (n - k + t) / t;
    return b;
}

double ipow(double x, int n) {
    double v = 1.0;
    for (int t = 0; t < n; ++t) v *= x;
    return v;
}

template <typename T>
int upload(pod_acsf* a, const std::vector<AChan<double>>& ch, const std::vector<double>& coef) {
    std::vector<AChan<T>> cht(ch.size());
    for (size_t c = 0; c < ch.size(); ++c)
        cht[c] = AChan<T>{static_cast<T>(ch[c].eta), static_cast<T>(ch[c].rs), ch[c].pd, ch[c].d0, ch[c].d1,
                          ch[c].bpre};
    std::vector<T> cf(coef.begin(), coef.end());
    if (hipMalloc(&a->d_ch, sizeof(AChan<T>) * cht.size()) != hipSuccess) return POD_ENOMEM;
    if (hipMalloc(&a->d_coef, sizeof(T) * cf.size()) != hipSuccess) return POD_ENOMEM;
    if (hipMemcpy(a->d_ch, cht.data(), sizeof(AChan<T>) * cht.size(), hipMemcpyHostToDevice) != hipSuccess)
        return POD_EHIP;
    if (hipMemcpy(a->d_coef, cf.data(), sizeof(T) * cf.size(), hipMemcpyHostToDevice) != hipSuccess)
        return POD_EHIP;
    return POD_OK;
}

template <typename T>
int fill_args(pod_handle* h, const pod_acsf* a, AArgs<T>& g, int N, int P, const void* pos, const double* cell,
              const int* offsets, const int* nbr_j, const int* shift) {
    g.N = N;
    g.P = P;
    g.nd = a->nd;
    g.rin = static_cast<T>(h->rin);
    g.rcut = static_cast<T>(h->rcut);
    g.inv_h = static_cast<T>(1.0 / (h->rcut - h->rin));
    g.periodic = cell != nullptr;
    for (int k = 0; k < 9; ++k) {
        const double v = cell ? cell[k] : 0.0;
        if (!std::isfinite(v)) return POD_EINVAL;
        g.cell[k] = static_cast<T>(v);
    }
    g.pos = static_cast<const T*>(pos);
    g.offsets = offsets;
    g.nbr_j = nbr_j;
    g.shift = shift;
    g.ch = static_cast<const AChan<T>*>(a->d_ch);
    g.coef = static_cast<const T*>(a->d_coef);
    g.col = a->d_col;
    g.G = nullptr;
    g.W = nullptr;
    g.ldw = 0;
    g.bbar = nullptr;
    g.V = nullptr;
    g.rev = nullptr;
    g.F = nullptr;
    g.err = h->d_err;
    return POD_OK;
}

template <typename T, bool ADJ>
void launch_basis(pod_handle* h, const pod_acsf* a, const AArgs<T>& g) {
    for (int k = 0; k < 4; ++k) {
        const int n = a->cls_off[k + 1] - a->cls_off[k];
        if (n == 0) continue;
        const int per = channels_per_thread(2 * k);
        constexpr int splits[4] = {acsf_split<T, 0, ADJ>(), acsf_split<T, 2, ADJ>(), acsf_split<T, 4, ADJ>(),
                                   acsf_split<T, 6, ADJ>()};
        const int apb = ACSF_THREADS / splits[k];
        const dim3 grid((g.N + apb - 1) / apb, (n + per - 1) / per);
        const int* chans = a->d_cls + a->cls_off[k];
        timing_begin(h, 1);
        switch (k) {
            case 0: hipLaunchKernelGGL((basis_kernel<T, 0, ADJ>), grid, dim3(ACSF_THREADS), 0, h->stream, g, chans, n); break;
            case 1: hipLaunchKernelGGL((basis_kernel<T, 2, ADJ>), grid, dim3(ACSF_THREADS), 0, h->stream, g, chans, n); break;
            case 2: hipLaunchKernelGGL((basis_kernel<T, 4, ADJ>), grid, dim3(ACSF_THREADS), 0, h->stream, g, chans, n); break;
            default: hipLaunchKernelGGL((basis_kernel<T, 6, ADJ>), grid, dim3(ACSF_THREADS), 0, h->stream, g, chans, n); break;
        }
        timing_end(h, 1);
    }
}

template <typename T>
int descriptors_impl(pod_handle* h, const pod_acsf* a, int N, int P, const void* pos, const double* cell,
                     const int* offsets, const int* nbr_j, const int* shift, void* G) {
    AArgs<T> g;
    const int rc = fill_args<T>(h, a, g, N, P, pos, cell, offsets, nbr_j, shift);
    if (rc != POD_OK) return rc;
    g.G = static_cast<T*>(G);
    launch_basis<T, false>(h, a, g);
    return hipGetLastError() == hipSuccess ? POD_OK : POD_EHIP;
}

template <typename T>
int forces_impl(pod_handle* h, const pod_acsf* a, int N, int P, const void* pos, const double* cell,
                const int* offsets, const int* nbr_j, const int* shift, const int* rev, const void* W, long ldw,
                void* G, void* F) {
    AArgs<T> g;
    int rc = fill_args<T>(h, a, g, N, P, pos, cell, offsets, nbr_j, shift);
    if (rc != POD_OK) return rc;
    const size_t nb = static_cast<size_t>(N) * a->bsum;
    const size_t nv = 3 * static_cast<size_t>(P);
    rc = ensure_scratch(h, sizeof(T) * (nb + nv) + 256);
    if (rc != POD_OK) return rc;
    g.bbar = static_cast<T*>(h->d_scratch);
    g.V = g.bbar + nb;
    g.G = static_cast<T*>(G);
    g.W = static_cast<const T*>(W);
    g.ldw = ldw;
    g.rev = rev;
    g.F = static_cast<T*>(F);
    launch_basis<T, true>(h, a, g);
    const int ppb = ACSF_THREADS / PAIR_LANES;
    const dim3 pgrid((N + ppb - 1) / ppb);
    timing_begin(h, 0);
    switch (a->pd_max) {
        case 0: hipLaunchKernelGGL((pair_kernel<T, 0>), pgrid, dim3(ACSF_THREADS), 0, h->stream, g, a->nch); break;
        case 2: hipLaunchKernelGGL((pair_kernel<T, 2>), pgrid, dim3(ACSF_THREADS), 0, h->stream, g, a->nch); break;
        case 4: hipLaunchKernelGGL((pair_kernel<T, 4>), pgrid, dim3(ACSF_THREADS), 0, h->stream, g, a->nch); break;
        default: hipLaunchKernelGGL((pair_kernel<T, 6>), pgrid, dim3(ACSF_THREADS), 0, h->stream, g, a->nch); break;
    }
    const int apg = ACSF_THREADS / GATHER_LANES;
    hipLaunchKernelGGL((gather_kernel<T>), dim3((N + apg - 1) / apg), dim3(ACSF_THREADS), 0, h->stream, g);
    timing_end(h, 0);
    return hipGetLastError() == hipSuccess ? POD_OK : POD_EHIP;
}

void release(pod_acsf* a) {
    if (!a) return;
    if (a->d_ch) (void)hipFree(a->d_ch);
    if (a->d_coef) (void)hipFree(a->d_coef);
    if (a->d_col) (void)hipFree(a->d_col);
    if (a->d_cls) (void)hipFree(a->d_cls);
    delete a;
}

}  // namespace
}  // namespace pod

extern "C" {

int pod_acsf_create(pod_handle* h, int n2, const double* g2, int n3, const double* g3, int n4, const double* g4,
                    pod_acsf** out) {
    using namespace pod;
    if (!h || !out || n2 < 0 || n3 < 0 || n4 < 0) return POD_EINVAL;
    *out = nullptr;
    const int nd = n2 + n3 + n4;
    if (nd == 0 || nd > POD_ACSF_MAX_FUNCTIONS) return POD_EINVAL;
    if ((n2 && !g2) || (n3 && !g3) || (n4 && !g4)) return POD_EINVAL;

    // per function: channel key, degree need and coefficient row
    struct Fn { double eta, rs; int need; double coef[ACSF_NI]; };
    std::vector<Fn> fn(nd);
    constexpr D4Build<6> tab{};
    for (int o = 0; o < nd; ++o) {
        Fn& f = fn[o];
        for (double& v : f.coef) v = 0.0;
        if (o < n2) {
            f.eta = g2[2 * o];
            f.rs = g2[2 * o + 1];
            f.need = 0;
            f.coef[0] = 1.0;
        } else if (o < n2 + n3) {
            const double* q = g3 + 3 * (o - n2);
            int zeta;
            if (!integral(q[1], 0, POD_ACSF_MAX_DEGREE, &zeta)) {
                if (std::isfinite(q[1]) && q[1] == std::floor(q[1]) && q[1] > POD_ACSF_MAX_DEGREE) return POD_ENOTSUP;
                return POD_EINVAL;
            }
            if (!std::isfinite(q[2])) return POD_EINVAL;
            f.eta = q[0];
            f.rs = 0.0;
            f.need = zeta;
            const double norm = std::ldexp(1.0, 1 - zeta);
            for (int n = 0; n <= zeta; ++n) f.coef[ACSF_S0 + n] = norm * binom(zeta, n) * ipow(q[2], n);
        } else {
            const double* q = g4 + 7 * (o - n2 - n3);
            int e[3];
            for (int k = 0; k < 3; ++k) {
                if (!integral(q[1 + k], 0, 1 << 20, &e[k])) return POD_EINVAL;
                if (!std::isfinite(q[4 + k])) return POD_EINVAL;
            }
            if (e[0] + e[1] + e[2] > POD_ACSF_MAX_DEGREE) return POD_ENOTSUP;
            f.eta = q[0];
            f.rs = 0.0;
            f.need = e[0] + e[1] + e[2];
            for (int n1 = 0; n1 <= e[0]; ++n1)
                for (int n2_ = 0; n2_ <= e[1]; ++n2_)
                    for (int n3_ = 0; n3_ <= e[2]; ++n3_) {
                        const double w = binom(e[0], n1) * ipow(q[4], n1) * binom(e[1], n2_) * ipow(q[5], n2_) *
                                         binom(e[2], n3_) * ipow(q[6], n3_);
                        int s[3] = {n1, n2_, n3_};
                        std::sort(s, s + 3);
                        int p = -1;
                        for (int t = 0; t < tab.KA; ++t)
                            if (tab.pa[t] == s[2] && tab.pb[t] == s[1] && tab.pc[t] == s[0]) p = t;
                        if (p < 0) return POD_EINVAL;   // unreachable: every sorted triple of degree <= 6 is listed
                        f.coef[ACSF_T0 + p] += w;
                    }
        }
        if (!std::isfinite(f.eta) || !std::isfinite(f.rs)) return POD_EINVAL;
    }

    // channels: distinct (eta, r_s), in order of first appearance
    std::vector<AChan<double>> ch;
    std::vector<int> fch(nd);
    std::vector<int> need;
    for (int o = 0; o < nd; ++o) {
        int c = -1;
        for (size_t k = 0; k < ch.size(); ++k)
            if (ch[k].eta == fn[o].eta && ch[k].rs == fn[o].rs) c = static_cast<int>(k);
        if (c < 0) {
            c = static_cast<int>(ch.size());
            if (c >= POD_ACSF_MAX_CHANNELS) return POD_ENOTSUP;
            ch.push_back(AChan<double>{fn[o].eta, fn[o].rs, 0, 0, 0, 0});
            need.push_back(0);
        }
        fch[o] = c;
        need[c] = std::max(need[c], fn[o].need);
    }
    const int nch = static_cast<int>(ch.size());
    std::vector<int> col;
    std::vector<double> coef;
    int bpre = 0, pd_max = 0;
    auto* a = new pod_acsf{};
    a->dtype = h->dtype;
    a->nd = nd;
    a->nch = nch;
    for (int c = 0; c < nch; ++c) {
        ch[c].pd = degree_class(need[c]);
        ch[c].d0 = static_cast<int>(col.size());
        for (int o = 0; o < nd; ++o)
            if (fch[o] == c) {
                col.push_back(o);
                coef.insert(coef.end(), fn[o].coef, fn[o].coef + ACSF_NI);
            }
        ch[c].d1 = static_cast<int>(col.size());
        ch[c].bpre = bpre;
        bpre += n_mono(ch[c].pd);
        pd_max = std::max(pd_max, ch[c].pd);
        a->cls_ch[ch[c].pd / 2].push_back(c);
    }
    a->pd_max = pd_max;
    a->bsum = bpre;
    std::vector<int> cls;
    a->cls_off[0] = 0;
    for (int k = 0; k < 4; ++k) {
        cls.insert(cls.end(), a->cls_ch[k].begin(), a->cls_ch[k].end());
        a->cls_off[k + 1] = static_cast<int>(cls.size());
    }
    int rc = h->dtype == POD_F64 ? upload<double>(a, ch, coef) : upload<float>(a, ch, coef);
    if (rc == POD_OK && (hipMalloc(&a->d_col, sizeof(int) * nd) != hipSuccess ||
                         hipMalloc(&a->d_cls, sizeof(int) * nch) != hipSuccess))
        rc = POD_ENOMEM;
    if (rc == POD_OK && (hipMemcpy(a->d_col, col.data(), sizeof(int) * nd, hipMemcpyHostToDevice) != hipSuccess ||
                         hipMemcpy(a->d_cls, cls.data(), sizeof(int) * nch, hipMemcpyHostToDevice) != hipSuccess))
        rc = POD_EHIP;
    if (rc != POD_OK) {
        release(a);
        return rc;
    }
    *out = a;
    return POD_OK;
}

int pod_acsf_num_functions(const pod_acsf* a, int* n_functions, int* n_channels) {
    if (!a) return POD_EINVAL;
    if (n_functions) *n_functions = a->nd;
    if (n_channels) *n_channels = a->nch;
    return POD_OK;
}

int pod_acsf_descriptors(pod_handle* h, const pod_acsf* a, int N, int P, const void* pos, const double* cell,
                         const int* offsets, const int* nbr_j, const int* shift, void* G) {
    using namespace pod;
    if (!h || !a || N < 0 || P < 0) return POD_EINVAL;
    if (a->dtype != h->dtype) return POD_EINVAL;
    if (N > 0 && (!pos || !offsets || !G || (P > 0 && (!nbr_j || !shift)))) return POD_EINVAL;
    if (N == 0) return POD_OK;
    return h->dtype == POD_F64 ? descriptors_impl<double>(h, a, N, P, pos, cell, offsets, nbr_j, shift, G)
                               : descriptors_impl<float>(h, a, N, P, pos, cell, offsets, nbr_j, shift, G);
}

int pod_acsf_forces(pod_handle* h, const pod_acsf* a, int N, int P, const void* pos, const double* cell,
                    const int* offsets, const int* nbr_j, const int* shift, const int* rev, const void* W, long ldw,
                    void* G, void* F) {
    using namespace pod;
    if (!h || !a || N < 0 || P < 0) return POD_EINVAL;
    if (a->dtype != h->dtype) return POD_EINVAL;
    if (ldw != 0 && ldw < a->nd) return POD_EINVAL;
    if (N > 0 && (!pos || !offsets || !W || !F || (P > 0 && (!nbr_j || !shift || !rev)))) return POD_EINVAL;
    if (N == 0) return POD_OK;
    return h->dtype == POD_F64
               ? forces_impl<double>(h, a, N, P, pos, cell, offsets, nbr_j, shift, rev, W, ldw, G, F)
               : forces_impl<float>(h, a, N, P, pos, cell, offsets, nbr_j, shift, rev, W, ldw, G, F);
}

void pod_acsf_free(pod_acsf* a) { pod::release(a); }

}  // extern "C"
