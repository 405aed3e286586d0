// Device helpers shared by the kernels of libpod: math wrappers, wavefront
// reductions, the radial basis (Sec. II.B) and the atomic-basis update
// (Sec. II.E, eq. (24b)).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "pod.h"
#include "pod_internal.h"
#include "pod_tables.h"

namespace pod {
namespace dev {

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

// Ordering point for a workgroup of one wavefront.  A wavefront performs its
// LDS accesses in program order, so lanes see each other's LDS writes once
// the compiler keeps the accesses on their side of this point; unlike a
// workgroup barrier it does not wait for outstanding global-memory loads.
__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_wave_barrier(); }

__device__ __forceinline__ int wave_or(int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v |= __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Sums of nine values over the 64 lanes of a wavefront, in a fixed order:
// halving exchanges in which each lane keeps half of the values it still
// carries (a transposed reduction: 17 exchanges instead of 54).  Returns
// the sum of value c in lane 4 c (c = 0..8); other lanes get c >= 9.
__device__ __forceinline__ double wave_sum9(const double (&v)[9], int lane, int& c) {
    double a[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i] = i < 9 ? v[i] : 0.0;
    // xor 32: lanes < 32 keep values 0..7, lanes >= 32 keep 8..15
    const bool hi32 = (lane & 32) != 0;
    double b[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const double send = hi32 ? a[i] : a[i + 8];
        const double recv = __shfl_xor(send, 32);
        b[i] = (hi32 ? a[i + 8] : a[i]) + recv;
    }
    // xor 16: keep 4
    const bool hi16 = (lane & 16) != 0;
    double e[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double send = hi16 ? b[i] : b[i + 4];
        const double recv = __shfl_xor(send, 16);
        e[i] = (hi16 ? b[i + 4] : b[i]) + recv;
    }
    // xor 8: keep 2
    const bool hi8 = (lane & 8) != 0;
    double f[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double send = hi8 ? e[i] : e[i + 2];
        const double recv = __shfl_xor(send, 8);
        f[i] = (hi8 ? e[i + 2] : e[i]) + recv;
    }
    // xor 4: keep 1
    const bool hi4 = (lane & 4) != 0;
    double t;
    {
        const double send = hi4 ? f[0] : f[1];
        const double recv = __shfl_xor(send, 4);
        t = (hi4 ? f[1] : f[0]) + recv;
    }
    t += __shfl_xor(t, 2);
    t += __shfl_xor(t, 1);
    // lane bits 5, 4, 3, 2 chose halves 8, 4, 2, 1 of the 16 values
    const int idx = (hi32 ? 8 : 0) + (hi16 ? 4 : 0) + (hi8 ? 2 : 0) + (hi4 ? 1 : 0);
    c = (lane & 3) == 0 ? idx : 16;
    return t;
}

__device__ __forceinline__ int unpack_shift(int sh, int d) {
    return static_cast<int>(static_cast<int8_t>((sh >> (8 * d)) & 0xFF));
}

// One neighbour slot of an atom: index and packed image shift.
struct SlotIdx {
    int j;    // neighbour index, -1 for an empty slot
    int sh;   // packed image shift
};

// The loads of a slot are issued on every lane (an empty slot reads entry 0,
// which exists whenever the list is not empty): with a fixed number of
// loads per round the compiler can wait for exactly the ones a round needs
// and leave the prefetched ones in flight.
template <typename A>
__device__ __forceinline__ SlotIdx slot_index(const A& g, bool valid, int p) {
    const int pc = valid ? p : 0;
    SlotIdx s;
    s.j = g.nbr_j[pc];
    s.sh = g.shift[pc];
    if (!valid) { s.j = -1; s.sh = 0; }
    return s;
}

template <typename T, typename A>
__device__ __forceinline__ void slot_pos(const A& g, const SlotIdx& s, T (&pj)[3]) {
    const int jc = (s.j >= 0 && s.j < g.N) ? s.j : 0;
    pj[0] = g.pos[3 * jc + 0];
    pj[1] = g.pos[3 * jc + 1];
    pj[2] = g.pos[3 * jc + 2];
}

// r_ij = r_j + n.cell - r_i, |r_ij| and validity of one fetched slot.  Data
// errors are collected in `eb` (error-word bits).
template <typename T, typename A>
__device__ __forceinline__ bool slot_geometry(const A& g, bool valid, const SlotIdx& s, const T (&pj)[3],
                                              const T (&pi)[3], int& eb, T (&d)[3], T& r) {
    d[0] = d[1] = d[2] = T(0);
    r = T(0.5) * (g.prm.rin + g.prm.rcut);
    if (!valid) return false;
    if (s.j < 0 || s.j >= g.N || (!g.cell.periodic && (s.sh & 0xFFFFFF) != 0)) {
        eb |= ERR_NEIGH;
        return false;
    }
    const T sx = T(unpack_shift(s.sh, 0)), sy = T(unpack_shift(s.sh, 1)), sz = T(unpack_shift(s.sh, 2));
    const T* a = g.cell.a;
    const T d0 = pj[0] - pi[0] + sx * a[0] + sy * a[3] + sz * a[6];
    const T d1 = pj[1] - pi[1] + sx * a[1] + sy * a[4] + sz * a[7];
    const T d2 = pj[2] - pi[2] + sx * a[2] + sy * a[5] + sz * a[8];
    const T r2 = d0 * d0 + d1 * d1 + d2 * d2;
    if (!d_finite(r2)) {
        eb |= ERR_NONFINITE;
        return false;
    }
    const T rr = d_sqrt(r2);
    if (rr <= g.prm.rin) {
        eb |= ERR_RANGE;
        return false;
    }
    if (rr >= g.prm.rcut) return false;   // not a neighbour (Sec. II.A): no contribution
    d[0] = d0; d[1] = d1; d[2] = d2;
    r = rr;
    return true;
}

// Radial functions R_k(r) = sum_l Q_lk Phi_l(r) and (DERIV) R'_k(r) for k <
// NR (Sec. II.B, eqs. (3)-(8), (11), (12)).  Q is zero beyond K.
template <typename T, bool DERIV, int NR>
__device__ __forceinline__ void radial(const ParamsT<T>* __restrict__ P, T r, T rinv, T (&R)[NR], T (&dR)[NR]) {
    static_assert(NR <= POD_MAX_K, "radial functions beyond the parameter block");
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
    for (int k = 0; k < NR; ++k) { R[k] = 0; dR[k] = 0; }
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
        for (int k = 0; k < NR; ++k) {
            const T qlk = P->Q[l][k];
            R[k] += qlk * ph;
            if (DERIV) dR[k] += qlk * dph;
        }
    }
}


// sin(pi x) and cos(pi x) for -0.25 <= x <= 1.25 (here x is the scaled
// distance, in [0, 1]).  Quadrant reduction t = x - k/2 with k = rint(2x) is
// exact (Sterbenz); sin and cos of theta = pi t, |theta| <= pi/4, come from
// their Taylor series (terms to theta^17 / theta^18 in double, theta^9 /
// theta^10 in float: truncation below half an ulp).
template <typename T>
__device__ __forceinline__ void sincospi_unit(T x, T* sp, T* cp) {
    const T k = rint(T(2) * x);
    const T t = x - T(0.5) * k;
    const T th = T(3.14159265358979323846) * t;
    const T z = th * th;
    T sn, cs;
    if constexpr (sizeof(T) == 8) {
        T ps = T(1.0 / 355687428096000.0);                      //  1/17!
        ps = ps * z - T(1.0 / 1307674368000.0);                 // -1/15!
        ps = ps * z + T(1.0 / 6227020800.0);                    //  1/13!
        ps = ps * z - T(1.0 / 39916800.0);                      // -1/11!
        ps = ps * z + T(1.0 / 362880.0);                        //  1/9!
        ps = ps * z - T(1.0 / 5040.0);                          // -1/7!
        ps = ps * z + T(1.0 / 120.0);                           //  1/5!
        ps = ps * z - T(1.0 / 6.0);                             // -1/3!
        T pc = -T(1.0 / 6402373705728000.0);                    // -1/18!
        pc = pc * z + T(1.0 / 20922789888000.0);                //  1/16!
        pc = pc * z - T(1.0 / 87178291200.0);                   // -1/14!
        pc = pc * z + T(1.0 / 479001600.0);                     //  1/12!
        pc = pc * z - T(1.0 / 3628800.0);                       // -1/10!
        pc = pc * z + T(1.0 / 40320.0);                         //  1/8!
        pc = pc * z - T(1.0 / 720.0);                           // -1/6!
        pc = pc * z + T(1.0 / 24.0);                            //  1/4!
        pc = pc * z - T(0.5);                                   // -1/2!
        sn = th + th * z * ps;
        cs = T(1) + z * pc;
    } else {
        T ps = T(1.0 / 362880.0);                               //  1/9!
        ps = ps * z - T(1.0 / 5040.0);                          // -1/7!
        ps = ps * z + T(1.0 / 120.0);                           //  1/5!
        ps = ps * z - T(1.0 / 6.0);                             // -1/3!
        T pc = -T(1.0 / 3628800.0);                             // -1/10!
        pc = pc * z + T(1.0 / 40320.0);                         //  1/8!
        pc = pc * z - T(1.0 / 720.0);                           // -1/6!
        pc = pc * z + T(1.0 / 24.0);                            //  1/4!
        pc = pc * z - T(0.5);                                   // -1/2!
        sn = th + th * z * ps;
        cs = T(1) + z * pc;
    }
    // rotate by k quarter turns
    const int q = static_cast<int>(k) & 3;
    T so = sn, co = cs;
    if (q == 1) { so = cs; co = -sn; }
    else if (q == 2) { so = -sn; co = -cs; }
    else if (q == 3) { so = -cs; co = sn; }
    *sp = so;
    *cp = co;
}

// Radial functions for the standard snapshot family (Bessel alpha = 1..nb at
// one beta, inverse powers gamma = 1..ni): one expm1, one sincos and one exp
// per pair; sin/cos(alpha pi x) by angle addition; Q read from LDS.
// KR: number of radial functions to form (the others are left zero; -1 =
// all NR).  sQ holds Q with row stride POD_MAX_K.
template <typename T, bool DERIV, int KR = -1, int NR>
__device__ __forceinline__ void radial_std(const ParamsT<T>* __restrict__ P, const T* __restrict__ sQ, T r,
                                           T rinv, T (&R)[NR], T (&dR)[NR]) {
    constexpr int KF = KR < 0 ? NR : KR;
    static_assert(KF <= NR && NR <= POD_MAX_K, "radial functions beyond the array or the parameter block");
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
#pragma unroll
    for (int k = 0; k < NR; ++k) { R[k] = 0; dR[k] = 0; }
    const int nb = P->std_nb, ni = P->std_ni;
    if (nb > 0) {
        T x, dx;
        const T bh = P->std_bh;
        if (bh == T(0)) {
            x = t; dx = inv_h;
        } else {
            const T em = d_expm1(-bh * dist);
            x = em * P->std_inv_em1;
            dx = -bh * (em + T(1)) * P->std_inv_em1;
        }
        T s1, c1;
        sincospi_unit(x, &s1, &c1);
        const T fci = fc * idist;
        const T dfci = DERIV ? dfc * idist : T(0);
        const T pdx = kPi * dx;
        T sk = 0, ck = 1;
        for (int l = 0; l < nb; ++l) {
            const T ns = sk * c1 + ck * s1;
            const T nc = ck * c1 - sk * s1;
            sk = ns; ck = nc;
            // Phi = f_c sin/(r - rin); Phi' = f_c' sin/(r-rin) + f_c (alpha pi cos dx - sin/(r-rin))/(r-rin)
            const T ph = fci * sk;
            const T dph = DERIV ? dfci * sk + fci * (T(l + 1) * pdx * ck - sk * idist) : T(0);
            const T* q = sQ + l * POD_MAX_K;
#pragma unroll
            for (int k = 0; k < KF; ++k) {
                R[k] += q[k] * ph;
                if (DERIV) dR[k] += q[k] * dph;
            }
        }
    }
    T pw = T(1);
    for (int g = 1; g <= ni; ++g) {
        pw *= rinv;                                  // r^-g
        const T ph = fc * pw;
        const T dph = DERIV ? (dfc - T(g) * fc * rinv) * pw : T(0);
        const T* q = sQ + (nb + g - 1) * POD_MAX_K;
#pragma unroll
        for (int k = 0; k < KF; ++k) {
            R[k] += q[k] * ph;
            if (DERIV) dR[k] += q[k] * dph;
        }
    }
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

}  // namespace dev
}  // namespace pod
