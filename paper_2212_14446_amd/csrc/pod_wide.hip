// Energy path for angular degree 7 to 10 (and K up to 12): the largest POD
// models of Table 6, whose atomic-basis rows (up to 286 monomials per radial
// function, eq. (23b)) do not fit a lane's registers.  Two kernels:
//
// wide_pair_kernel (16 lanes per atom): one record per listed pair --
//   [rhat (3), r, R_k (K) (, R'_k (K))] (Sec. II.A, II.B) -- with R = R' = 0
//   and rhat = 0 for a listed pair beyond the cut-off.
// wide_kernel: one 256-thread workgroup serves one atom at a time
//   (persistent over the atoms i = blk, blk + nblk, ...):
//   1. basis (eq. (24b)): the records of WIDE_CHUNK pairs and the powers of
//      their unit vectors' components are staged in LDS, and thread t
//      accumulates B_{k n} for its monomials n = t, t + 256 and every k in
//      registers; the rows then go to LDS;
//   2. contraction: degree sums S_{k a} = sum_{|n| = a} c_n B_{k n}^2,
//      thread d forms descriptor d: D2 = B_{k 0} (eq. (25)), D3 = S
//      (eq. (26a)), D4 by eq. (27a) for (a, 0, 0) and by the merged terms of
//      eq. (30a) otherwise; the energy (eq. (57a)) and the G partials;
//   3. adjoint dE_i/dB_{k n} by the product rule on the same formulas, the
//      4-body part gathered per monomial from a table of its occurrences in
//      the eq. (30a) terms (fixed order, no atomics); row k overwrites basis
//      row k in LDS;
//   4. pair gradients (eq. (24c)): eight lanes per pair split the monomials,
//      g_ij = sum_{k n} Abar_{k n} [R'_k A_n rhat + R_k (grad A_n - |n| A_n
//      rhat) / r] (Euler identity for the homogeneous A_n), summed over the
//      eight lanes by shuffles in a fixed order, then stored at the pair's
//      own and reverse slots (or added to the force accumulator).
// E, G and the virial leave as per-workgroup partials that the energy path's
// finalize kernel sums in a fixed order.  Evaluating the radial functions in
// a kernel of their own keeps their constants and temporaries out of the
// per-atom kernel's registers and leaves it one dependent load (the record)
// per pair instead of three (index, position, then the arithmetic).
#include <hip/hip_runtime.h>

#include <cmath>

#include "pod.h"
#include "pod_device.h"
#include "pod_internal.h"
#include "pod_tables.h"
#include "pod_wide.h"

namespace pod {
namespace {

using namespace dev;

constexpr int WT = WIDE_THREADS;
constexpr int CH = WIDE_CHUNK;
constexpr int GSUB = WT / CH;                               // lanes per pair in the gradient pass
constexpr int NA_MAX = n_mono(POD_MAX_P);                   // 286
constexpr int MPT = (NA_MAX + WT - 1) / WT;                 // monomials per thread in the basis pass
constexpr int DPT = 2;                                      // descriptor columns per thread
constexpr int NA4 = n_mono(POD_MAX_P4);                     // monomials that enter eq. (30a)
constexpr int KA4 = n_partitions(POD_MAX_P4);               // 23
constexpr int NT4 = D4Table<POD_MAX_P4>::NT;                // merged eq. (30a) terms

static_assert(1 + POD_MAX_K + POD_MAX_K * (POD_MAX_P + 1) + POD_MAX_K * KA4 <= DPT * WT,
              "descriptor columns per thread");
static_assert(GSUB == 8, "the gradient reduction assumes eight lanes per pair");

// Monomial codes: a | b << 4 | c << 8 | degree << 12 | multinomial << 16
// (device order of pod_tables.h).  Packed eq. (30a) tables for 4-body indices
// p up to degree POD_MAX_P4 (Table 1 order, so a lower P4 uses a prefix):
// per p its triple a | b << 4 | c << 8 and term range; every merged term
// x | y << 7 | z << 14 | coefficient << 21 (sorted monomial indices); and for
// every monomial n < NA4 its occurrences in the terms, p | u << 5 | v << 12 |
// coefficient << 19 (u, v the other two monomials).  The packed layout is
// the one copied to LDS: [ptri KA4][tbeg KA4][tend KA4][term NT4][obeg NA4+1]
// [occ 3 NT4][index of (a, 0, 0) for a <= POD_MAX_P4].  The occurrences of a
// monomial are in term order, hence sorted by p.
struct WideTables {
    int code[NA_MAX];
    int tab[wide_tab_ints()];
};
constexpr int T_PTRI = 0, T_TBEG = KA4, T_TEND = 2 * KA4, T_TERM = 3 * KA4, T_OBEG = 3 * KA4 + NT4,
              T_OCC = 3 * KA4 + NT4 + NA4 + 1, T_PA00 = 3 * KA4 + 4 * NT4 + NA4 + 1;

constexpr WideTables make_wide_tables() {
    WideTables w{};
    constexpr MonoTable<POD_MAX_P> mt{};
    for (int n = 0; n < NA_MAX; ++n)
        w.code[n] = mt.ex[n][0] | (mt.ex[n][1] << 4) | (mt.ex[n][2] << 8) | (mt.deg[n] << 12) | (mt.mult[n] << 16);
    constexpr D4Build<POD_MAX_P4> d4{};
    for (int p = 0; p < KA4; ++p) {
        w.tab[T_PTRI + p] = d4.pa[p] | (d4.pb[p] << 4) | (d4.pc[p] << 8);
        w.tab[T_TBEG + p] = d4.tbeg[p];
        w.tab[T_TEND + p] = d4.tend[p];
    }
    for (int k = 0; k < NT4; ++k)
        w.tab[T_TERM + k] = d4.tx[k] | (d4.ty[k] << 7) | (d4.tz[k] << 14) | (d4.tc[k] << 21);
    for (int a = 0; a <= POD_MAX_P4; ++a) w.tab[T_PA00 + a] = n_partitions(a - 1);
    int cnt[NA4] = {};
    for (int k = 0; k < NT4; ++k) { ++cnt[d4.tx[k]]; ++cnt[d4.ty[k]]; ++cnt[d4.tz[k]]; }
    w.tab[T_OBEG] = 0;
    for (int n = 0; n < NA4; ++n) w.tab[T_OBEG + n + 1] = w.tab[T_OBEG + n] + cnt[n];
    int at[NA4] = {};
    for (int n = 0; n < NA4; ++n) at[n] = w.tab[T_OBEG + n];
    for (int k = 0; k < NT4; ++k) {
        const int x = d4.tx[k], y = d4.ty[k], z = d4.tz[k];
        const int own[3] = {x, y, z}, u[3] = {y, x, x}, v[3] = {z, z, y};
        for (int r = 0; r < 3; ++r)
            w.tab[T_OCC + at[own[r]]++] = d4.tp[k] | (u[r] << 5) | (v[r] << 12) | (d4.tc[k] << 19);
    }
    return w;
}

// field limits of the packing
constexpr int wide_max_term_coef() {
    constexpr D4Build<POD_MAX_P4> d4{};
    int mx = 0;
    for (int k = 0; k < NT4; ++k) mx = d4.tc[k] > mx ? d4.tc[k] : mx;
    return mx;
}
static_assert(NA4 <= 128 && KA4 <= 32 && POD_MAX_P <= 15 && wide_max_term_coef() < 2048, "packed table fields");

__device__ const WideTables kWide = make_wide_tables();

// 4-body index of the triple (a, 0, 0): the first triple of degree a.
__device__ __forceinline__ int p_a00(const int* tab, int a) { return tab[T_PA00 + a]; }

// Sum over the workgroup in a fixed order (shuffles within each wavefront,
// then the four wavefront sums in order); every thread gets the result.
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int tid = threadIdx.x;
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    const double s = (red[0] + red[1]) + (red[2] + red[3]);
    return s;
}

// Pair records: 16 lanes per atom walk its list range.
template <typename T, bool DERIV, bool FAST>
__global__ __launch_bounds__(WT) void wide_pair_kernel(WideArgs<T> g) {
    __shared__ T sQ[POD_MAX_L * POD_MAX_K];
    const ParamsT<T>& prm = g.prm;
    const int tid = threadIdx.x;
    if (FAST)
        for (int k = tid; k < POD_MAX_L * POD_MAX_K; k += WT) sQ[k] = (&prm.Q[0][0])[k];
    __syncthreads();
    const int K = prm.K, RS = g.rs;
    const int i = blockIdx.x * (WT / 16) + tid / 16, l = tid % 16;
    int eb = 0;
    if (i < g.N) {
        const int b = g.offsets[i], e = g.offsets[i + 1];
        if (b < 0 || e < b || e > g.P) {
            eb |= ERR_NEIGH;
        } else {
            const T pi[3] = {g.pos[3 * i], g.pos[3 * i + 1], g.pos[3 * i + 2]};
            for (int p = b + l; p < e; p += 16) {
                const SlotIdx si = slot_index(g, true, p);
                T pj[3], d[3], r;
                slot_pos<T>(g, si, pj);
                const bool ok = slot_geometry<T>(g, true, si, pj, pi, eb, d, r);
                const T ri = T(1) / r;
                T R[POD_MAX_K], dR[POD_MAX_K];
                if constexpr (FAST) radial_std<T, DERIV>(&prm, sQ, r, ri, R, dR);
                else radial<T, DERIV>(&prm, r, ri, R, dR);
                T* rec = g.rec + static_cast<size_t>(p) * RS;
                rec[0] = ok ? d[0] * ri : T(0);
                rec[1] = ok ? d[1] * ri : T(0);
                rec[2] = ok ? d[2] * ri : T(0);
                rec[3] = r;
#pragma unroll
                for (int k = 0; k < POD_MAX_K; ++k)
                    if (k < K) {
                        rec[4 + k] = ok ? R[k] : T(0);
                        if (DERIV) rec[4 + K + k] = ok ? dR[k] : T(0);
                    }
            }
        }
    }
    eb = wave_or(eb);
    if ((tid & 63) == 0 && eb) atomicOr(g.err, eb);
}

template <typename T, int MODE>
__global__ __launch_bounds__(WT) void wide_kernel(WideArgs<T> g) {
    extern __shared__ __align__(16) unsigned char smem[];
    const ParamsT<T>& prm = g.prm;
    const int K = prm.K, PA = prm.PA, M = prm.M;
    const int NA = n_mono(PA);
    const int PA1 = PA + 1;
    const bool four = prm.K4 > 0;
    const WideLds L = wide_lds(K, PA, M, four, static_cast<int>(sizeof(T)));
    T* sC = reinterpret_cast<T*>(smem + L.coef);
    int* sCode = reinterpret_cast<int*>(smem + L.code);
    int* sTab = reinterpret_cast<int*>(smem + L.tab);
    T* sB = reinterpret_cast<T*>(smem + L.b);
    T* sS = reinterpret_cast<T*>(smem + L.s);
    T* sR = reinterpret_cast<T*>(smem + L.r);      // [q][POD_MAX_K] R, then [q][POD_MAX_K] R'
    T* sdR = sR + CH * POD_MAX_K;
    T* sU = reinterpret_cast<T*>(smem + L.u);      // [q][4]: rhat, r
    T* sP = reinterpret_cast<T*>(smem + L.pw);
    double* sRed = reinterpret_cast<double*>(smem + L.red);
    const int tid = threadIdx.x;

    for (int n = tid; n < NA; n += WT) sCode[n] = kWide.code[n];
    if (MODE == 1)
        for (int k = tid; k < M; k += WT) sC[k] = g.coef[k];
    if (four)
        for (int k = tid; k < wide_tab_ints(); k += WT) sTab[k] = kWide.tab[k];
    __syncthreads();

    const int K2 = prm.K2, K3 = prm.K3, K4 = prm.K4, P3 = prm.P3, P4 = prm.P4, KA = prm.Ka4;
    const int off3 = prm.off3, off4 = prm.off4;
    // this thread's monomials in the basis pass
    int mcode[MPT];
#pragma unroll
    for (int j = 0; j < MPT; ++j) mcode[j] = (tid + j * WT < NA) ? sCode[tid + j * WT] : 0;

    double gacc[DPT] = {0.0, 0.0};
    double eacc = 0.0;
    double vir[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) vir[c] = 0.0;
    int eb = 0;

    for (int i = blockIdx.x; i < g.N; i += gridDim.x) {
        int b = g.offsets[i], e = g.offsets[i + 1];
        if (b < 0 || e < b || e > g.P) {
            eb |= ERR_NEIGH;
            b = e = 0;
        }
        const int n = e - b;
        const int RS = g.rs;

        // ---- 1. atomic basis
        T acc[MPT][POD_MAX_K];
#pragma unroll
        for (int j = 0; j < MPT; ++j)
#pragma unroll
            for (int k = 0; k < POD_MAX_K; ++k) acc[j][k] = T(0);
        for (int c0 = 0; c0 < n; c0 += CH) {
            const int nc = n - c0 < CH ? n - c0 : CH;
            // stage the chunk: R_k of every pair, and the powers u_x^a, u_y^b,
            // u_z^c of its unit vector
            const T* rc = g.rec + static_cast<size_t>(b + c0) * RS;
            for (int t = tid; t < nc * K; t += WT) {
                const int q = t / K, k = t - q * K;
                sR[q * POD_MAX_K + k] = rc[static_cast<size_t>(q) * RS + 4 + k];
            }
            for (int t = tid; t < nc * 3; t += WT) {
                const int q = t / 3, ax = t - 3 * q;
                const T u = rc[static_cast<size_t>(q) * RS + ax];
                T* pw = sP + (q * 3 + ax) * PA1;
                T v = T(1);
                for (int a = 0; a <= PA; ++a) {
                    pw[a] = v;
                    v *= u;
                }
            }
            __syncthreads();
#pragma unroll 1
            for (int q = 0; q < nc; ++q) {
                const T* pw = sP + q * 3 * PA1;
                const T* Rq = sR + q * POD_MAX_K;
                T Rv[POD_MAX_K];
#pragma unroll
                for (int k = 0; k < POD_MAX_K; ++k) Rv[k] = k < K ? Rq[k] : T(0);
#pragma unroll
                for (int j = 0; j < MPT; ++j) {
                    if (tid + j * WT < NA) {
                        const int cd = mcode[j];
                        const T A = pw[cd & 15] * pw[PA1 + ((cd >> 4) & 15)] * pw[2 * PA1 + ((cd >> 8) & 15)];
#pragma unroll
                        for (int k = 0; k < POD_MAX_K; ++k) acc[j][k] += Rv[k] * A;
                    }
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int j = 0; j < MPT; ++j) {
            const int nn = tid + j * WT;
            if (nn < NA)
#pragma unroll
                for (int k = 0; k < POD_MAX_K; ++k)
                    if (k < K) sB[k * NA + nn] = acc[j][k];
        }
        __syncthreads();

        // ---- 2. degree sums and descriptors
        for (int w = tid; w < K * PA1; w += WT) {
            const int k = w / PA1, a = w - k * PA1;
            const int n0 = n_mono(a - 1), n1 = n_mono(a);
            const T* Bk = sB + k * NA;
            T s = T(0);
            for (int nn = n0; nn < n1; ++nn) {
                const T v = Bk[nn];
                s += T(sCode[nn] >> 16) * v * v;
            }
            sS[w] = s;
        }
        __syncthreads();
        double ep = 0.0;
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int dc = tid + j * WT;
            if (dc >= M) continue;
            T v;
            if (dc == 0) {
                v = T(1);
            } else if (dc < off3) {
                v = sB[(dc - 1) * NA];
            } else if (dc < off4) {
                const int k = (dc - off3) / (P3 + 1), a = (dc - off3) - k * (P3 + 1);
                v = sS[k * PA1 + a];
            } else {
                const int k = (dc - off4) / KA, p = (dc - off4) - k * KA;
                const T* Bk = sB + k * NA;
                const int tri = sTab[T_PTRI + p];
                if ((tri >> 4) == 0) {
                    v = Bk[0] * sS[k * PA1 + (tri & 15)];                           // eq. (27a)
                } else {
                    T v0 = T(0), v1 = T(0);
                    const int t1 = sTab[T_TEND + p];
                    int t = sTab[T_TBEG + p];
                    for (; t + 1 < t1; t += 2) {                                    // eq. (30a)
                        const int ta = sTab[T_TERM + t], tb = sTab[T_TERM + t + 1];
                        v0 += T(ta >> 21) * Bk[ta & 127] * Bk[(ta >> 7) & 127] * Bk[(ta >> 14) & 127];
                        v1 += T(tb >> 21) * Bk[tb & 127] * Bk[(tb >> 7) & 127] * Bk[(tb >> 14) & 127];
                    }
                    if (t < t1) {
                        const int ta = sTab[T_TERM + t];
                        v0 += T(ta >> 21) * Bk[ta & 127] * Bk[(ta >> 7) & 127] * Bk[(ta >> 14) & 127];
                    }
                    v = v0 + v1;
                }
            }
            if constexpr (MODE == 0) {
                g.D[static_cast<size_t>(i) * M + dc] = v;
            } else {
                ep += static_cast<double>(sC[dc]) * static_cast<double>(v);
                gacc[j] += static_cast<double>(v);
            }
        }
        if constexpr (MODE == 0) {
            __syncthreads();   // sB and sS are rewritten by the next atom
            continue;
        } else {
            const double Ei = block_sum(ep, sRed);
            if (tid == 0) {
                if (g.E_atom) g.E_atom[i] = static_cast<T>(Ei);
                eacc += Ei;
            }
            if (!g.want_back) {
                __syncthreads();
                continue;
            }

            // ---- 3. adjoint dE_i/dB_{k n}, one radial index at a time: the
            // contractions are diagonal in k, so row k of the adjoint needs
            // only row k of the basis and overwrites it in place
            const T* cf = sC;
#pragma unroll 1
            for (int k = 0; k < K; ++k) {
                T* Bk = sB + k * NA;
                const T B0 = Bk[0];
                T ab[MPT];
#pragma unroll
                for (int j = 0; j < MPT; ++j) {
                    ab[j] = T(0);
                    const int nn = tid + j * WT;
                    if (nn >= NA) continue;
                    const int cd = sCode[nn];
                    const int dg = (cd >> 12) & 15;
                    const T mult = T(cd >> 16);
                    const T Bn = Bk[nn];
                    T v = T(0);
                    if (nn == 0 && k < K2) v += cf[1 + k];
                    if (k < K3 && dg <= P3) v += T(2) * cf[off3 + k * (P3 + 1) + dg] * mult * Bn;
                    if (k < K4) {
                        const T* c4 = cf + off4 + k * KA;
                        if (nn == 0)
                            for (int a = 0; a <= P4; ++a) v += c4[p_a00(sTab, a)] * sS[k * PA1 + a];   // eq. (27a)
                        if (dg <= P4) v += c4[p_a00(sTab, dg)] * B0 * T(2) * mult * Bn;
                        if (nn < NA4) {
                            // occurrences are sorted by p: stop at the first p of a
                            // higher degree than the model's; four at a time
                            const int o0 = sTab[T_OBEG + nn], o1 = sTab[T_OBEG + nn + 1];
                            T v4 = T(0);
                            int o = o0;
                            for (; o + 3 < o1; o += 4) {                                      // eq. (30a)
                                const int oa = sTab[T_OCC + o], ob = sTab[T_OCC + o + 1];
                                const int oc = sTab[T_OCC + o + 2], od = sTab[T_OCC + o + 3];
                                if ((od & 31) >= KA) break;
                                v4 += c4[oa & 31] * T(oa >> 19) * Bk[(oa >> 5) & 127] * Bk[(oa >> 12) & 127];
                                v4 += c4[ob & 31] * T(ob >> 19) * Bk[(ob >> 5) & 127] * Bk[(ob >> 12) & 127];
                                v4 += c4[oc & 31] * T(oc >> 19) * Bk[(oc >> 5) & 127] * Bk[(oc >> 12) & 127];
                                v4 += c4[od & 31] * T(od >> 19) * Bk[(od >> 5) & 127] * Bk[(od >> 12) & 127];
                            }
                            for (; o < o1; ++o) {
                                const int oa = sTab[T_OCC + o];
                                if ((oa & 31) >= KA) break;
                                v4 += c4[oa & 31] * T(oa >> 19) * Bk[(oa >> 5) & 127] * Bk[(oa >> 12) & 127];
                            }
                            v += v4;
                        }
                    }
                    ab[j] = v;
                }
                __syncthreads();   // every read of row k is done
#pragma unroll
                for (int j = 0; j < MPT; ++j)
                    if (tid + j * WT < NA) Bk[tid + j * WT] = ab[j];
            }
            __syncthreads();
            const T* sA = sB;   // adjoint rows [K][NA]

            // ---- 4. pair gradients, eq. (24c)
            const int q = tid / GSUB, s = tid - q * GSUB;
            for (int c0 = 0; c0 < n; c0 += CH) {
                const int nc = n - c0 < CH ? n - c0 : CH;
                const T* rc = g.rec + static_cast<size_t>(b + c0) * RS;
                for (int t = tid; t < nc * K; t += WT) {
                    const int qq = t / K, k = t - qq * K;
                    sR[qq * POD_MAX_K + k] = rc[static_cast<size_t>(qq) * RS + 4 + k];
                    sdR[qq * POD_MAX_K + k] = rc[static_cast<size_t>(qq) * RS + 4 + K + k];
                }
                for (int t = tid; t < nc * 4; t += WT) {
                    const int qq = t / 4, c = t - 4 * qq;
                    const T v = rc[static_cast<size_t>(qq) * RS + c];
                    sU[qq * 4 + c] = v;
                    if (c < 3) {
                        T* pw = sP + (qq * 3 + c) * PA1;
                        T x = T(1);
                        for (int a = 0; a <= PA; ++a) {
                            pw[a] = x;
                            x *= v;
                        }
                    }
                }
                __syncthreads();
                const bool in = q < nc;
                const int p = b + c0 + q;
                const int qc = in ? q : 0;
                const T u[3] = {sU[qc * 4 + 0], sU[qc * 4 + 1], sU[qc * 4 + 2]};
                const T r = sU[qc * 4 + 3];
                const T ri = T(1) / r;
                const bool ok = in && (u[0] * u[0] + u[1] * u[1] + u[2] * u[2] > T(0.5));
                T R[POD_MAX_K], dR[POD_MAX_K];
#pragma unroll
                for (int k = 0; k < POD_MAX_K; ++k) {
                    R[k] = k < K ? sR[qc * POD_MAX_K + k] : T(0);
                    dR[k] = k < K ? sdR[qc * POD_MAX_K + k] : T(0);
                }
                const T* pw = sP + qc * 3 * PA1;
                T sa = T(0), gv0 = T(0), gv1 = T(0), gv2 = T(0);
#pragma unroll 1
                for (int nn = s; nn < NA; nn += GSUB) {
                    const int cd = sCode[nn];
                    const int ea = cd & 15, ebx = (cd >> 4) & 15, ec = (cd >> 8) & 15, dg = (cd >> 12) & 15;
                    const T xa = pw[ea], yb = pw[PA1 + ebx], zc = pw[2 * PA1 + ec];
                    T w1 = T(0), w2 = T(0);
#pragma unroll
                    for (int k = 0; k < POD_MAX_K; ++k) {
                        if (k < K) {
                            const T av = sA[k * NA + nn];
                            w1 += av * dR[k];
                            w2 += av * R[k];
                        }
                    }
                    const T A = xa * yb * zc;
                    sa += (w1 - T(dg) * ri * w2) * A;
                    if (ea > 0) gv0 += w2 * T(ea) * pw[ea - 1] * yb * zc;
                    if (ebx > 0) gv1 += w2 * T(ebx) * xa * pw[PA1 + ebx - 1] * zc;
                    if (ec > 0) gv2 += w2 * T(ec) * xa * yb * pw[2 * PA1 + ec - 1];
                }
                // sum over the eight lanes of the pair (fixed order)
#pragma unroll
                for (int o = 1; o < GSUB; o <<= 1) {
                    sa += __shfl_xor(sa, o);
                    gv0 += __shfl_xor(gv0, o);
                    gv1 += __shfl_xor(gv1, o);
                    gv2 += __shfl_xor(gv2, o);
                }
                const T gx = ok ? sa * u[0] + ri * gv0 : T(0);
                const T gy = ok ? sa * u[1] + ri * gv1 : T(0);
                const T gz = ok ? sa * u[2] + ri * gv2 : T(0);
                if (s == 0 && in) {
                    if (g.gbuf) {
                        T* go = g.gown + 3 * static_cast<size_t>(p);
                        go[0] = gx; go[1] = gy; go[2] = gz;
                        const int rv = g.rev[p];
                        if (rv >= 0 && rv < g.P) {
                            T* gp3 = g.gbuf + 3 * static_cast<size_t>(rv);
                            gp3[0] = gx; gp3[1] = gy; gp3[2] = gz;
                        } else {
                            eb |= ERR_NEIGH;
                        }
                    } else if (ok && g.Facc) {
                        const int j = g.nbr_j[p];
                        atomicAdd(&g.Facc[3 * j + 0], -static_cast<double>(gx));
                        atomicAdd(&g.Facc[3 * j + 1], -static_cast<double>(gy));
                        atomicAdd(&g.Facc[3 * j + 2], -static_cast<double>(gz));
                        atomicAdd(&g.Facc[3 * i + 0], static_cast<double>(gx));
                        atomicAdd(&g.Facc[3 * i + 1], static_cast<double>(gy));
                        atomicAdd(&g.Facc[3 * i + 2], static_cast<double>(gz));
                    }
                    if (ok) {
                        const double dd[3] = {static_cast<double>(u[0] * r), static_cast<double>(u[1] * r),
                                              static_cast<double>(u[2] * r)};
                        const double gg[3] = {static_cast<double>(gx), static_cast<double>(gy),
                                              static_cast<double>(gz)};
#pragma unroll
                        for (int x = 0; x < 3; ++x)
#pragma unroll
                            for (int y = 0; y < 3; ++y) vir[3 * x + y] -= dd[x] * gg[y];
                    }
                }
                __syncthreads();   // the chunk's staging is rewritten next
            }
            __syncthreads();   // LDS is rewritten by the next atom
        }
    }

    // block partials (every thread takes part in the reductions)
    const int blk = blockIdx.x, nblk = gridDim.x;
    if constexpr (MODE == 1) {
        if (tid == 0) g.part[blk] = eacc;
        if (g.want_G) {
#pragma unroll
            for (int j = 0; j < DPT; ++j) {
                const int dc = tid + j * WT;
                if (dc < M) g.part[static_cast<size_t>(10 + dc) * nblk + blk] = gacc[j];
            }
        }
        if (g.want_W) {
#pragma unroll
            for (int c = 0; c < 9; ++c) {
                const double v = block_sum(vir[c], sRed);
                if (tid == 0) g.wpart[static_cast<size_t>(c) * nblk + blk] = v;
                __syncthreads();
            }
        }
    }
    eb = wave_or(eb);
    if ((tid & 63) == 0 && eb) atomicOr(g.err, eb);
}

template <typename T, int MODE>
hipError_t launch_mode(const WideArgs<T>& a, bool fast, int nblk, hipStream_t st) {
    const int nrec = (a.N + WT / 16 - 1) / (WT / 16);
    constexpr bool DERIV = MODE == 1;
    if (a.N > 0) {
        if (fast) hipLaunchKernelGGL((wide_pair_kernel<T, DERIV, true>), dim3(nrec), dim3(WT), 0, st, a);
        else hipLaunchKernelGGL((wide_pair_kernel<T, DERIV, false>), dim3(nrec), dim3(WT), 0, st, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const size_t lds = wide_lds(a.prm.K, a.prm.PA, a.prm.M, a.prm.K4 > 0, static_cast<int>(sizeof(T))).total;
    hipLaunchKernelGGL((wide_kernel<T, MODE>), dim3(nblk), dim3(WT), lds, st, a);
    return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_wide(const WideArgs<T>& a, int mode, bool fast, int nblk, hipStream_t st) {
    if (nblk <= 0) return hipSuccess;
    return mode == 0 ? launch_mode<T, 0>(a, fast, nblk, st) : launch_mode<T, 1>(a, fast, nblk, st);
}

template hipError_t launch_wide<double>(const WideArgs<double>&, int, bool, int, hipStream_t);
template hipError_t launch_wide<float>(const WideArgs<float>&, int, bool, int, hipStream_t);

}  // namespace pod
