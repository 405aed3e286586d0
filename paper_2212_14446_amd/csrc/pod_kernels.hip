// Fused per-atom kernels of the fast POD path for gfx950 (CDNA4).
//
// Work mapping.  One workgroup is one 64-lane wavefront and owns APW = 64 / K
// consecutive atoms (K = max(K2, K3, K4)).  Lane l serves atom a = l / K and
// index q = l % K, which is used two ways:
//   * pair stage   : q is a neighbour slot; each lane evaluates one pair
//                    r_ij -> (rhat, 1/r, R_k(r), R'_k(r)) and stages it in LDS;
//                    neighbour slots are consumed K at a time per atom.
//   * basis stage  : q is the radial index m; the lane accumulates the row
//                    B_{i m .} = sum_j R_m(r_ij) A_.(rhat_ij) of the atomic
//                    basis (Sec. II.E, eq. (24b)) in registers.
// Every contraction of Sec. II.E is diagonal in m (the same radial function in
// all factors, eqs. (14), (17a)), so D3, D4, the energy and the adjoint
// dE_i/dB_{i m .} are computed by each lane from its own row without any
// exchange.  The backward sweep recomputes the pair stage (nothing per pair is
// stored) and reduces the per-m gradient contributions of each pair through
// LDS; forces are scattered with device-scope atomics, block totals of E, W
// and G go to a partial-sum buffer reduced by a second kernel.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "pod.h"
#include "pod_internal.h"
#include "pod_tables.h"

namespace pod {
namespace {

template <typename T> __device__ __forceinline__ T d_exp(T x);
template <> __device__ __forceinline__ double d_exp(double x) { return exp(x); }
template <> __device__ __forceinline__ float d_exp(float x) { return expf(x); }
template <typename T> __device__ __forceinline__ T d_expm1(T x);
template <> __device__ __forceinline__ double d_expm1(double x) { return expm1(x); }
template <> __device__ __forceinline__ float d_expm1(float x) { return expm1f(x); }
template <typename T> __device__ __forceinline__ T d_log(T x);
template <> __device__ __forceinline__ double d_log(double x) { return log(x); }
template <> __device__ __forceinline__ float d_log(float x) { return logf(x); }
template <typename T> __device__ __forceinline__ T d_sqrt(T x);
template <> __device__ __forceinline__ double d_sqrt(double x) { return sqrt(x); }
template <> __device__ __forceinline__ float d_sqrt(float x) { return sqrtf(x); }
template <typename T> __device__ __forceinline__ T d_rsqrt(T x);
template <> __device__ __forceinline__ double d_rsqrt(double x) { return rsqrt(x); }
template <> __device__ __forceinline__ float d_rsqrt(float x) { return rsqrtf(x); }
template <typename T> __device__ __forceinline__ void d_sincos(T x, T* s, T* c);
template <> __device__ __forceinline__ void d_sincos(double x, double* s, double* c) { sincos(x, s, c); }
template <> __device__ __forceinline__ void d_sincos(float x, float* s, float* c) { sincosf(x, s, c); }
template <typename T> __device__ __forceinline__ bool d_finite(T x) { return isfinite(x); }

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ int unpack_shift(int sh, int d) {
    return static_cast<int>(static_cast<int8_t>((sh >> (8 * d)) & 0xFF));
}

// Radial functions R_k(r) = sum_l Q_lk Phi_l(r) and (DERIV) R'_k(r) for k <
// POD_MAX_K (Sec. II.B, eqs. (3)-(8), (11), (12)).  Q is zero beyond K.
template <typename T, bool DERIV>
__device__ __forceinline__ void radial(const ParamsT<T>* __restrict__ P, T r, T rinv,
                                       T (&R)[POD_MAX_K], T (&dR)[POD_MAX_K]) {
    const T inv_h = P->inv_h;
    const T dist = r - P->rin;
    const T t = dist * inv_h;
    const T t2 = t * t;
    const T y = T(1) - t2 * t;
    const T s = y * y + T(1e-6);
    const T rs = d_rsqrt(s);
    const T fc = d_exp(T(1) - rs);
    const T dfc = DERIV ? fc * y * (rs * rs * rs) * (T(-3) * t2 * inv_h) : T(0);
    const T idist = T(1) / dist;
    constexpr T kPi = T(3.14159265358979323846);
    T x = 0, dx = 0, s1 = 0, c1 = 1, sk = 0, ck = 1;
#pragma unroll
    for (int k = 0; k < POD_MAX_K; ++k) { R[k] = 0; dR[k] = 0; }
    const int L = P->L;
    for (int l = 0; l < L; ++l) {
        const SnapT<T>& sn = P->s[l];
        T psi = 0, dpsi = 0;
        if (sn.bessel) {
            if (sn.newbeta) {
                if (sn.bh == T(0)) {
                    x = t; dx = inv_h;
                } else {
                    const T em = d_expm1(-sn.bh * dist);
                    x = em * sn.inv_em1;
                    dx = -sn.bh * (em + T(1)) * sn.inv_em1;
                }
                d_sincos(kPi * x, &s1, &c1);
                sk = 0; ck = 1;
            }
            T sa, ca;
            if (sn.steps >= 0) {
                for (int q = 0; q < sn.steps; ++q) {
                    const T ns = sk * c1 + ck * s1;
                    const T nc = ck * c1 - sk * s1;
                    sk = ns; ck = nc;
                }
                sa = sk; ca = ck;
            } else {
                d_sincos(sn.apix * x, &sa, &ca);
            }
            const T phi = sa * idist;
            psi = sn.kappa * phi;
            if (DERIV) dpsi = sn.kappa * (sn.apix * ca * dx - phi) * idist;
        }
        if (sn.power) {
            T v;
            if (sn.power == 1) {
                v = rinv;
                for (int q = 1; q < sn.igamma; ++q) v *= rinv;
            } else {
                v = d_exp(-sn.gamma * d_log(r));
            }
            const T w = T(1) - sn.kappa;
            psi += w * v;
            if (DERIV) dpsi -= w * sn.gamma * v * rinv;
        }
        const T ph = fc * psi;
        const T dph = DERIV ? dfc * psi + fc * dpsi : T(0);
#pragma unroll
        for (int k = 0; k < POD_MAX_K; ++k) {
            const T qlk = P->Q[l][k];
            R[k] += qlk * ph;
            if (DERIV) dR[k] += qlk * dph;
        }
    }
}

template <typename T>
struct KArgs {
    const ParamsT<T>* prm;
    int N, P;
    const T* pos;
    CellT<T> cell;
    const int* offsets;
    const int* nbr_j;
    const int* shift;
    const T* coef;     // energy coefficients (mode 1)
    T* D;              // descriptors (mode 0)
    T* E_atom;         // per-atom energy or null (mode 1)
    T* F;              // forces or null (mode 1)
    double* part;      // per-block partials: E, W[9], G[M] (mode 1)
    int want_G;
    int want_back;     // run the backward sweep (forces or virial requested)
    int* err;
};

// Pair stage: lane evaluates neighbour slot `slot` of its atom (valid) and
// writes rhat, 1/r, R_k, (R'_k) to LDS column `col`.  Returns the pair vector.
template <typename T, bool DERIV>
__device__ __forceinline__ void pair_stage(const KArgs<T>& g, int i, int p, bool valid, int col, int K,
                                           T* sU, T* sRinv, T* sR, T* sdR, T (&dvec)[3]) {
    T d0 = 0, d1 = 0, d2 = 0;
    bool ok = false;
    if (valid) {
        const int j = g.nbr_j[p];
        const int sh = g.shift[p];
        if (j < 0 || j >= g.N || (!g.cell.periodic && (sh & 0xFFFFFF) != 0)) {
            atomicOr(g.err, ERR_NEIGH);
        } else {
            const T sx = T(unpack_shift(sh, 0)), sy = T(unpack_shift(sh, 1)), sz = T(unpack_shift(sh, 2));
            const T* a = g.cell.a;
            d0 = g.pos[3 * j + 0] - g.pos[3 * i + 0] + sx * a[0] + sy * a[3] + sz * a[6];
            d1 = g.pos[3 * j + 1] - g.pos[3 * i + 1] + sx * a[1] + sy * a[4] + sz * a[7];
            d2 = g.pos[3 * j + 2] - g.pos[3 * i + 2] + sx * a[2] + sy * a[5] + sz * a[8];
            const T r2 = d0 * d0 + d1 * d1 + d2 * d2;
            if (!d_finite(r2)) {
                atomicOr(g.err, ERR_NONFINITE);
            } else {
                const T r = d_sqrt(r2);
                if (r <= g.prm->rin || r >= g.prm->rcut) atomicOr(g.err, ERR_RANGE);
                else ok = true;
            }
        }
    }
    // invalid lanes evaluate a harmless mid-range distance and store zeros
    const T rmid = T(0.5) * (g.prm->rin + g.prm->rcut);
    const T r = ok ? d_sqrt(d0 * d0 + d1 * d1 + d2 * d2) : rmid;
    const T rinv = T(1) / r;
    T R[POD_MAX_K], dR[POD_MAX_K];
    radial<T, DERIV>(g.prm, r, rinv, R, dR);
    const T z = ok ? T(1) : T(0);
    sU[col] = d0 * rinv * z;
    sU[WAVE + col] = d1 * rinv * z;
    sU[2 * WAVE + col] = d2 * rinv * z;
    sRinv[col] = rinv;
#pragma unroll
    for (int k = 0; k < POD_MAX_K; ++k) {
        if (k < K) {
            sR[k * WAVE + col] = R[k] * z;
            if (DERIV) sdR[k * WAVE + col] = dR[k] * z;
        }
    }
    dvec[0] = d0 * z; dvec[1] = d1 * z; dvec[2] = d2 * z;
}

template <typename T, int PA>
__device__ __forceinline__ void accumulate_basis(T (&acc)[n_mono(PA)], T Rm, T ux, T uy, T uz) {
    constexpr MonoTable<PA> mt{};
    constexpr int NA = n_mono(PA);
    T A[NA];
    A[0] = Rm;
    acc[0] += Rm;
#pragma unroll
    for (int mu = 1; mu < NA; ++mu) {
        const T u = mt.axis[mu] == 0 ? ux : (mt.axis[mu] == 1 ? uy : uz);
        A[mu] = A[mt.par[mu]] * u;
        acc[mu] += A[mu];
    }
}

template <typename T, int PA, int MODE>
__global__ __launch_bounds__(64) void atom_kernel(KArgs<T> g) {
    constexpr MonoTable<PA> mt{};
    constexpr int NA = n_mono(PA);
    using Tab = D4Table<PA>;
    constexpr int KA = Tab::KA;
    constexpr int NT = Tab::NT;

    const ParamsT<T>* __restrict__ P = g.prm;
    const int K = P->K;
    const int lane = threadIdx.x;
    const int apw = WAVE / K;
    const int al = lane / K;
    const int q = lane - al * K;
    const int atom = blockIdx.x * apw + al;
    const bool act = (al < apw) && (atom < g.N);

    int beg = 0, cnt = 0;
    if (act) {
        const int b = g.offsets[atom], e = g.offsets[atom + 1];
        if (b < 0 || e < b || e > g.P) {
            if (q == 0) atomicOr(g.err, ERR_NEIGH);
        } else {
            beg = b; cnt = e - b;
        }
    }
    const int nround = (wave_max(cnt) + K - 1) / K;

    extern __shared__ unsigned char smem_raw[];
    T* sU = reinterpret_cast<T*>(smem_raw);
    T* sRinv = sU + 3 * WAVE;
    T* sR = sRinv + WAVE;
    T* sdR = sR + K * WAVE;
    T* sRed = sdR + (MODE == 1 ? K * WAVE : 0);

    // ---------------- forward: atomic basis row B_{i, m=q, .} ----------------
    T acc[NA];
#pragma unroll
    for (int mu = 0; mu < NA; ++mu) acc[mu] = 0;
    for (int rd = 0; rd < nround; ++rd) {
        {
            const int sl = rd * K + q;
            T dv[3];
            pair_stage<T, false>(g, atom, beg + sl, act && sl < cnt, lane, K, sU, sRinv, sR, sdR, dv);
        }
        __syncthreads();
        for (int s = 0; s < K; ++s) {
            if (act && rd * K + s < cnt) {
                const int col = al * K + s;
                accumulate_basis<T, PA>(acc, sR[q * WAVE + col], sU[col], sU[WAVE + col], sU[2 * WAVE + col]);
            }
        }
        __syncthreads();
    }

    // ---------------- contractions (Sec. II.E) ----------------
    T d3[PA + 1];
#pragma unroll
    for (int n = 0; n <= PA; ++n) d3[n] = 0;
#pragma unroll
    for (int mu = 0; mu < NA; ++mu) d3[mt.deg[mu]] += T(mt.mult[mu]) * acc[mu] * acc[mu];  // eq. (26a)
    T d4[KA];
#pragma unroll
    for (int p = 0; p < KA; ++p) d4[p] = 0;
#pragma unroll
    for (int p = 0; p < KA; ++p)
        if (Tab::build.pb[p] == 0) d4[p] = acc[0] * d3[Tab::build.pa[p]];                   // eq. (27a)
#pragma unroll
    for (int t = 0; t < NT; ++t)                                                             // eq. (30a)
        d4[Tab::build.tp[t]] += T(Tab::build.tc[t]) * acc[Tab::build.tx[t]] * acc[Tab::build.ty[t]] *
                                acc[Tab::build.tz[t]];

    const int m = q;
    const bool has2 = act && m < P->K2;
    const bool has3 = act && m < P->K3;
    const bool has4 = act && m < P->K4;
    const int P3 = P->P3, Ka4 = P->Ka4;

    if (MODE == 0) {
        if (act) {
            T* Drow = g.D + static_cast<size_t>(atom) * P->M;
            if (q == 0) Drow[0] = T(1);
            if (has2) Drow[1 + m] = acc[0];
            if (has3) {
#pragma unroll
                for (int n = 0; n <= PA; ++n)
                    if (n <= P3) Drow[P->off3 + m * (P3 + 1) + n] = d3[n];
            }
            if (has4) {
#pragma unroll
                for (int p = 0; p < KA; ++p)
                    if (p < Ka4) Drow[P->off4 + m * Ka4 + p] = d4[p];
            }
        }
        return;
    }

    // ---------------- energy (eq. (57a)) and adjoint dE_i/dB ----------------
    const T* c = g.coef;
    T w2 = has2 ? c[1 + m] : T(0);
    T w3[PA + 1], w4[KA];
#pragma unroll
    for (int n = 0; n <= PA; ++n) w3[n] = (has3 && n <= P3) ? c[P->off3 + m * (P3 + 1) + n] : T(0);
#pragma unroll
    for (int p = 0; p < KA; ++p) w4[p] = (has4 && p < Ka4) ? c[P->off4 + m * Ka4 + p] : T(0);

    double e = 0.0;
    if (act) {
        T ev = w2 * acc[0];
#pragma unroll
        for (int n = 0; n <= PA; ++n) ev += w3[n] * d3[n];
#pragma unroll
        for (int p = 0; p < KA; ++p) ev += w4[p] * d4[p];
        e = static_cast<double>(ev);
        if (q == 0) e += static_cast<double>(c[0]);
    }
    // effective weights of D2 and D3 including the (a, 0, 0) 4-body terms
    T eff2 = w2;
    T eff3[PA + 1];
#pragma unroll
    for (int n = 0; n <= PA; ++n) eff3[n] = w3[n];
#pragma unroll
    for (int p = 0; p < KA; ++p)
        if (Tab::build.pb[p] == 0) {
            eff2 += w4[p] * d3[Tab::build.pa[p]];
            eff3[Tab::build.pa[p]] += w4[p] * acc[0];
        }
    T ab[NA];
#pragma unroll
    for (int mu = 0; mu < NA; ++mu) ab[mu] = T(2 * mt.mult[mu]) * eff3[mt.deg[mu]] * acc[mu];  // eq. (26c)
    ab[0] += eff2;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int x = Tab::build.tx[t], y = Tab::build.ty[t], z = Tab::build.tz[t];
        const T wc = w4[Tab::build.tp[t]] * T(Tab::build.tc[t]);
        ab[x] += wc * acc[y] * acc[z];
        ab[y] += wc * acc[x] * acc[z];
        ab[z] += wc * acc[x] * acc[y];
    }

    // per-atom energy: sum the K lanes of the atom through LDS
    {
        double* sE = reinterpret_cast<double*>(smem_raw);
        sE[lane] = e;
        __syncthreads();
        double ei = 0.0;
        if (act && q == 0) {
            for (int k = 0; k < K; ++k) ei += sE[al * K + k];
            if (g.E_atom) g.E_atom[atom] = static_cast<T>(ei);
        }
        __syncthreads();
        const double eb = wave_sum(ei);
        if (lane == 0) g.part[static_cast<size_t>(blockIdx.x) * (10 + P->M)] = eb;
    }
    // block partial of the global descriptors G = sum_i D_i (eq. (58a))
    if (g.want_G) {
        double* sG = reinterpret_cast<double*>(smem_raw);
        const int M = P->M;
        for (int k = lane; k < M; k += WAVE) sG[k] = 0.0;
        __syncthreads();
        for (int a2 = 0; a2 < apw; ++a2) {
            if (al == a2 && act) {
                if (q == 0) sG[0] += 1.0;
                if (has2) sG[1 + m] += static_cast<double>(acc[0]);
                if (has3)
#pragma unroll
                    for (int n = 0; n <= PA; ++n)
                        if (n <= P3) sG[P->off3 + m * (P3 + 1) + n] += static_cast<double>(d3[n]);
                if (has4)
#pragma unroll
                    for (int p = 0; p < KA; ++p)
                        if (p < Ka4) sG[P->off4 + m * Ka4 + p] += static_cast<double>(d4[p]);
            }
            __syncthreads();
        }
        double* pg = g.part + static_cast<size_t>(blockIdx.x) * (10 + M) + 10;
        for (int k = lane; k < M; k += WAVE) pg[k] = sG[k];
        __syncthreads();
    }

    if (!g.want_back) return;

    // ---------------- backward sweep: g_ij = dE_i/dr_ij (eq. (24c)) ----------------
    double vir[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) vir[k] = 0.0;
    T fown0 = 0, fown1 = 0, fown2 = 0;
    for (int rd = 0; rd < nround; ++rd) {
        const int myslot = rd * K + q;
        const bool mine = act && myslot < cnt;
        T dv[3];
        pair_stage<T, true>(g, atom, beg + myslot, mine, lane, K, sU, sRinv, sR, sdR, dv);
        __syncthreads();
        for (int s = 0; s < K; ++s) {
            T gx = 0, gy = 0, gz = 0;
            const int col = al * K + s;
            if (act && rd * K + s < cnt) {
                const T Rm = sR[m * WAVE + col], dRm = sdR[m * WAVE + col];
                const T ux = sU[col], uy = sU[WAVE + col], uz = sU[2 * WAVE + col];
                const T ri = sRinv[col];
                T A[NA];
                A[0] = T(1);
#pragma unroll
                for (int mu = 1; mu < NA; ++mu) {
                    const T u = mt.axis[mu] == 0 ? ux : (mt.axis[mu] == 1 ? uy : uz);
                    A[mu] = A[mt.par[mu]] * u;
                }
                T hd[PA + 1];
#pragma unroll
                for (int n = 0; n <= PA; ++n) hd[n] = 0;
                T g0 = 0, g1 = 0, g2 = 0;
#pragma unroll
                for (int mu = 0; mu < NA; ++mu) {
                    hd[mt.deg[mu]] += ab[mu] * A[mu];
                    if (mt.down[mu][0] >= 0) g0 += (ab[mu] * T(mt.ex[mu][0])) * A[mt.down[mu][0]];
                    if (mt.down[mu][1] >= 0) g1 += (ab[mu] * T(mt.ex[mu][1])) * A[mt.down[mu][1]];
                    if (mt.down[mu][2] >= 0) g2 += (ab[mu] * T(mt.ex[mu][2])) * A[mt.down[mu][2]];
                }
                T hsum = 0, eul = 0;
#pragma unroll
                for (int n = 0; n <= PA; ++n) { hsum += hd[n]; eul += T(n) * hd[n]; }
                // d/dr_ij [R_m(r) h(rhat)] = R'_m h rhat + R_m (grad_u h - (rhat . grad_u h) rhat)/r,
                // with rhat . grad_u h = sum_n n h_n for the degree-n parts h_n (Euler)
                const T a1 = dRm * hsum - Rm * eul * ri;
                const T a2 = Rm * ri;
                gx = a1 * ux + a2 * g0;
                gy = a1 * uy + a2 * g1;
                gz = a1 * uz + a2 * g2;
            }
            T* red = sRed + (static_cast<size_t>(col) * K + m) * 3;
            if (act) { red[0] = gx; red[1] = gy; red[2] = gz; }
        }
        __syncthreads();
        if (mine) {
            T gx = 0, gy = 0, gz = 0;
            const T* red = sRed + static_cast<size_t>(lane) * K * 3;
            for (int k = 0; k < K; ++k) { gx += red[3 * k]; gy += red[3 * k + 1]; gz += red[3 * k + 2]; }
            fown0 += gx; fown1 += gy; fown2 += gz;
            if (g.F) {
                const int j = g.nbr_j[beg + myslot];
                atomicAdd(&g.F[3 * j + 0], -gx);
                atomicAdd(&g.F[3 * j + 1], -gy);
                atomicAdd(&g.F[3 * j + 2], -gz);
            }
            const double dd[3] = {double(dv[0]), double(dv[1]), double(dv[2])};
            const double gg[3] = {double(gx), double(gy), double(gz)};
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) vir[3 * a + b] -= dd[a] * gg[b];
        }
        __syncthreads();
    }
    // own-atom force: F_i += sum_j g_ij, summed over the atom's K lanes
    {
        T* sF = sRed;
        sF[3 * lane + 0] = fown0; sF[3 * lane + 1] = fown1; sF[3 * lane + 2] = fown2;
        __syncthreads();
        if (act && q == 0 && g.F) {
            T f0 = 0, f1 = 0, f2 = 0;
            for (int k = 0; k < K; ++k) {
                const int l2 = al * K + k;
                f0 += sF[3 * l2]; f1 += sF[3 * l2 + 1]; f2 += sF[3 * l2 + 2];
            }
            atomicAdd(&g.F[3 * atom + 0], f0);
            atomicAdd(&g.F[3 * atom + 1], f1);
            atomicAdd(&g.F[3 * atom + 2], f2);
        }
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double v = wave_sum(vir[k]);
        if (lane == 0) g.part[static_cast<size_t>(blockIdx.x) * (10 + P->M) + 1 + k] = v;
    }
}

// Column sums of the block partials: column 0 -> E, 1..9 -> W, 10.. -> G.
__global__ __launch_bounds__(256) void finalize_kernel(const double* __restrict__ part, int nblk, int stride,
                                                       double* E, double* W, double* G) {
    const int col = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) s += part[static_cast<size_t>(b) * stride + col];
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if (static_cast<int>(threadIdx.x) < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double v = red[0];
        if (col == 0) { if (E) *E = v; }
        else if (col < 10) { if (W) W[col - 1] = v; }
        else if (G) G[col - 10] = v;
    }
}

template <typename T>
__global__ void zero_kernel(T* __restrict__ x, long n) {
    for (long i = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<long>(gridDim.x) * blockDim.x)
        x[i] = T(0);
}

template <typename T, int PA, int MODE>
hipError_t launch_atom(const KArgs<T>& a, int nblk, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL((atom_kernel<T, PA, MODE>), dim3(nblk), dim3(WAVE), lds, st, a);
    return hipGetLastError();
}

template <typename T, int MODE>
hipError_t dispatch_pa(int PA, const KArgs<T>& a, int nblk, size_t lds, hipStream_t st) {
    switch (PA) {
        case 0: return launch_atom<T, 0, MODE>(a, nblk, lds, st);
        case 1: return launch_atom<T, 1, MODE>(a, nblk, lds, st);
        case 2: return launch_atom<T, 2, MODE>(a, nblk, lds, st);
        case 3: return launch_atom<T, 3, MODE>(a, nblk, lds, st);
        case 4: return launch_atom<T, 4, MODE>(a, nblk, lds, st);
        case 5: return launch_atom<T, 5, MODE>(a, nblk, lds, st);
        case 6: return launch_atom<T, 6, MODE>(a, nblk, lds, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
int fill_common(pod_handle* h, KArgs<T>& a, int N, int P, const void* pos, const double* cell,
                const int* offsets, const int* nbr_j, const int* shift) {
    a.prm = static_cast<const ParamsT<T>*>(h->d_params);
    a.N = N; a.P = P;
    a.pos = static_cast<const T*>(pos);
    a.cell.periodic = cell != nullptr;
    for (int k = 0; k < 9; ++k) {
        const double v = cell ? cell[k] : 0.0;
        if (!std::isfinite(v)) return POD_EINVAL;
        a.cell.a[k] = static_cast<T>(v);
    }
    a.offsets = offsets; a.nbr_j = nbr_j; a.shift = shift;
    a.coef = nullptr; a.D = nullptr; a.E_atom = nullptr; a.F = nullptr; a.part = nullptr;
    a.want_G = 0;
    a.want_back = 0;
    a.err = h->d_err;
    return POD_OK;
}

size_t lds_bytes(int K, int mode, size_t tsize, int M) {
    size_t n = static_cast<size_t>(4 + K) * WAVE;
    if (mode == 1) n += static_cast<size_t>(K) * WAVE + static_cast<size_t>(WAVE) * K * 3;
    size_t bytes = n * tsize;
    const size_t need_d = static_cast<size_t>(WAVE > M ? WAVE : M) * sizeof(double);
    return bytes > need_d ? bytes : need_d;
}

template <typename T>
int descriptors_impl(pod_handle* h, int N, int P, const void* pos, const double* cell, const int* offsets,
                     const int* nbr_j, const int* shift, void* D) {
    KArgs<T> a;
    int rc = fill_common<T>(h, a, N, P, pos, cell, offsets, nbr_j, shift);
    if (rc != POD_OK) return rc;
    a.D = static_cast<T*>(D);
    const int apw = WAVE / h->K;
    const int nblk = (N + apw - 1) / apw;
    if (nblk == 0) return POD_OK;
    const size_t lds = lds_bytes(h->K, 0, sizeof(T), h->M);
    timing_begin(h);
    const hipError_t e = dispatch_pa<T, 0>(h->PA, a, nblk, lds, h->stream);
    timing_end(h);
    return e == hipSuccess ? POD_OK : POD_EHIP;
}

template <typename T>
int energy_forces_impl(pod_handle* h, int N, int P, const void* pos, const double* cell, const int* offsets,
                       const int* nbr_j, const int* shift, const void* c, void* E_atom, double* E, void* F,
                       double* W, double* G) {
    KArgs<T> a;
    int rc = fill_common<T>(h, a, N, P, pos, cell, offsets, nbr_j, shift);
    if (rc != POD_OK) return rc;
    a.coef = static_cast<const T*>(c);
    a.E_atom = static_cast<T*>(E_atom);
    a.F = static_cast<T*>(F);
    a.want_G = G != nullptr;
    a.want_back = (F != nullptr) || (W != nullptr);
    const int apw = WAVE / h->K;
    const int nblk = (N + apw - 1) / apw;
    const int stride = 10 + h->M;
    hipStream_t st = h->stream;
    if (F && N > 0) {
        const long n = 3L * N;
        const int zb = static_cast<int>((n + 255) / 256 < 2048 ? (n + 255) / 256 : 2048);
        hipLaunchKernelGGL((zero_kernel<T>), dim3(zb), dim3(256), 0, st, static_cast<T*>(F), n);
        if (hipGetLastError() != hipSuccess) return POD_EHIP;
    }
    if (nblk > 0) {
        rc = ensure_scratch(h, static_cast<size_t>(nblk) * stride * sizeof(double));
        if (rc != POD_OK) return rc;
        a.part = static_cast<double*>(h->d_scratch);
        const size_t lds = lds_bytes(h->K, 1, sizeof(T), h->M);
        timing_begin(h);
        const hipError_t e = dispatch_pa<T, 1>(h->PA, a, nblk, lds, st);
        timing_end(h);
        if (e != hipSuccess) return POD_EHIP;
    }
    const int ncol = G ? stride : 10;
    if (E || W || G) {
        hipLaunchKernelGGL(finalize_kernel, dim3(ncol), dim3(256), 0, st,
                           static_cast<const double*>(h->d_scratch), nblk, stride, E, W, G);
        if (hipGetLastError() != hipSuccess) return POD_EHIP;
    }
    return POD_OK;
}

bool bad_common(pod_handle* h, int N, int P, const void* pos, const int* offsets, const int* nbr_j,
                const int* shift) {
    if (!h || N < 0 || P < 0) return true;
    if (N > 0 && (!pos || !offsets)) return true;
    if (P > 0 && (!nbr_j || !shift)) return true;
    return false;
}

}  // namespace
}  // namespace pod

extern "C" {

int pod_descriptors(pod_handle* h, int N, int P, const void* pos, const double* cell, const int* offsets,
                    const int* nbr_j, const int* shift, void* D) {
    if (pod::bad_common(h, N, P, pos, offsets, nbr_j, shift)) return POD_EINVAL;
    if (N > 0 && !D) return POD_EINVAL;
    if (h->dtype == POD_F64)
        return pod::descriptors_impl<double>(h, N, P, pos, cell, offsets, nbr_j, shift, D);
    return pod::descriptors_impl<float>(h, N, P, pos, cell, offsets, nbr_j, shift, D);
}

int pod_energy_forces(pod_handle* h, int N, int P, const void* pos, const double* cell, const int* offsets,
                      const int* nbr_j, const int* shift, const void* c, void* E_atom, double* E, void* F,
                      double* W, double* G) {
    if (pod::bad_common(h, N, P, pos, offsets, nbr_j, shift)) return POD_EINVAL;
    if (!c) return POD_EINVAL;
    if (h->dtype == POD_F64)
        return pod::energy_forces_impl<double>(h, N, P, pos, cell, offsets, nbr_j, shift, c, E_atom, E, F, W, G);
    return pod::energy_forces_impl<float>(h, N, P, pos, cell, offsets, nbr_j, shift, c, E_atom, E, F, W, G);
}

}  // extern "C"
