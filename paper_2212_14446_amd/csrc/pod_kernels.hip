// Kernels of the fast POD path for gfx950 (CDNA4).
//
// atom_kernel  (one 64-lane wavefront per workgroup, APW = 64 / K atoms):
//   lane l serves atom a = l / K and radial index m = l % K and keeps the row
//   B_{i m .} = sum_j R_m(r_ij) A_.(rhat_ij) of the atomic basis (Sec. II.E,
//   eq. (24b)) in registers.  Neighbours are taken K at a time per atom
//   ("rounds"): in a round, lane (a, s) evaluates slot s of atom a -- pair
//   geometry and the radial basis (Sec. II.B, eqs. (3)-(8), (11), (12)) --
//   and stages {rhat, R_k} in LDS for the atom's K lanes, with the next
//   slot's indices and positions prefetched.  Every contraction of Sec. II.E
//   is diagonal in m (the same radial function in all factors, eqs. (14),
//   (17a)), so D3, D4, the energy and the adjoint dE_i/dB_{i m .} come from
//   the lane's own row with compile-time tables.  The backward sweep walks
//   the slots again, forms dE_i/dr_ij (eq. (24c)) from the K adjoint rows of
//   the atom, and either stores it at the reverse slot of the pair (gather
//   path, with a reverse-pair index) or adds it to an FP64 accumulator with
//   device atomics.  E, the virial and G leave as per-workgroup partials.
// finalize_kernel  sums the partials in a fixed order (E, W, G) and forms the
//   forces: on the gather path each atom adds its own sum_j g_ij to the
//   values stored in its list range (32 lanes per atom); otherwise it copies
//   and clears the accumulator.
// reverse_kernel  builds the reverse-pair index of a list once.
// The per-atom basis B and its adjoint never leave the chip; only the
// pair gradients of the gather path go through memory.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "pod.h"
#include "pod_device.h"
#include "pod_internal.h"
#include "pod_tables.h"

namespace pod {
namespace {

using namespace dev;

template <typename T>
struct KArgs {
    ParamsT<T> prm;    // by value: read with scalar loads
    int N, P;
    const T* pos;
    CellT<T> cell;
    const int* offsets;
    const int* nbr_j;
    const int* shift;
    const T* coef;     // energy coefficients (mode 1)
    T* D;              // descriptors (mode 0)
    T* E_atom;         // per-atom energy or null (mode 1)
    double* Facc;      // force accumulator (3N, zero on entry) (mode 1, backward, no gbuf)
    T* gbuf;           // gather path: g_ij stored at the reverse slot rev[p] (3P)
    double* fown;      // gather path: own-atom force sum_j g_ij (3N)
    const int* rev;    // reverse-pair index (gather path)
    double* part;      // block partials, column-major [10 + M][nblk] (mode 1)
    int want_G;        // block partials of G requested
    int want_back;     // run the backward sweep (forces or virial requested)
    const float* y_net;  // mode 2: per-atom network energy (N)
    const float* g_net;  // mode 2: per-atom dy/dD for descriptor columns 1.. (N x n_net)
    int n_net;
    int* err;
};

// Neighbour slots are fetched two rounds ahead: the index and image shift of
// round r + 2 and the neighbour position of round r + 1 are requested before
// the arithmetic of round r.
struct SlotIdx {
    int j;    // neighbour index, -1 for an empty slot
    int sh;   // packed image shift
    int rv;   // reverse pair (gather path), -1 otherwise
};

template <typename T>
__device__ __forceinline__ SlotIdx slot_index(const KArgs<T>& g, bool valid, int p) {
    SlotIdx s;
    s.j = -1; s.sh = 0; s.rv = -1;
    if (valid) {
        s.j = g.nbr_j[p]; s.sh = g.shift[p];
        if (g.rev) s.rv = g.rev[p];
    }
    return s;
}

template <typename T>
__device__ __forceinline__ void slot_pos(const KArgs<T>& g, const SlotIdx& s, T (&pj)[3]) {
    pj[0] = pj[1] = pj[2] = T(0);
    if (s.j >= 0 && s.j < g.N) {
        pj[0] = g.pos[3 * s.j + 0];
        pj[1] = g.pos[3 * s.j + 1];
        pj[2] = g.pos[3 * s.j + 2];
    }
}

// r_ij = r_j + n.cell - r_i, |r_ij| and validity of one fetched slot.  Data
// errors are latched in the error word when `report` is set.
template <typename T>
__device__ __forceinline__ bool slot_geometry(const KArgs<T>& g, bool valid, const SlotIdx& s, const T (&pj)[3],
                                              const T (&pi)[3], bool report, T (&d)[3], T& r) {
    d[0] = d[1] = d[2] = T(0);
    r = T(0.5) * (g.prm.rin + g.prm.rcut);
    if (!valid) return false;
    if (s.j < 0 || s.j >= g.N || (!g.cell.periodic && (s.sh & 0xFFFFFF) != 0)) {
        if (report) atomicOr(g.err, ERR_NEIGH);
        return false;
    }
    const T sx = T(unpack_shift(s.sh, 0)), sy = T(unpack_shift(s.sh, 1)), sz = T(unpack_shift(s.sh, 2));
    const T* a = g.cell.a;
    const T d0 = pj[0] - pi[0] + sx * a[0] + sy * a[3] + sz * a[6];
    const T d1 = pj[1] - pi[1] + sx * a[1] + sy * a[4] + sz * a[7];
    const T d2 = pj[2] - pi[2] + sx * a[2] + sy * a[5] + sz * a[8];
    const T r2 = d0 * d0 + d1 * d1 + d2 * d2;
    if (!d_finite(r2)) {
        if (report) atomicOr(g.err, ERR_NONFINITE);
        return false;
    }
    const T rr = d_sqrt(r2);
    if (rr <= g.prm.rin) {
        if (report) atomicOr(g.err, ERR_RANGE);
        return false;
    }
    if (rr >= g.prm.rcut) return false;   // not a neighbour (Sec. II.A): no contribution
    d[0] = d0; d[1] = d1; d[2] = d2;
    r = rr;
    return true;
}

template <typename T, bool DERIV, bool FAST>
__device__ __forceinline__ void radial_any(const ParamsT<T>* __restrict__ P, const T* sQ, T r, T rinv,
                                           T (&R)[POD_MAX_K], T (&dR)[POD_MAX_K]) {
    if constexpr (FAST) radial_std<T, DERIV>(P, sQ, r, rinv, R, dR);
    else radial<T, DERIV>(P, r, rinv, R, dR);
}

// LDS layout of atom_kernel (per 64-lane workgroup), in bytes:
//   [Q (L x POD_MAX_K)] [per-lane double scratch (max(64, M), 3 x 64)]
//   [T area: union { round staging [64][stage_stride(K)], adjoint rows [APW][K][NA | 1] }]
__host__ __device__ constexpr int stage_stride(int K) { return (3 + K) | 1; }
__host__ __device__ constexpr int odd_len(int n) { return n | 1; }

struct AtomLds {
    size_t off_q, off_e, off_f, off_t, total;
};

__host__ __device__ inline AtomLds atom_lds_layout(int K, int NA, int M, size_t tsize) {
    const int apw = WAVE / K;
    AtomLds L;
    L.off_q = 0;
    L.off_e = ((static_cast<size_t>(POD_MAX_L) * POD_MAX_K * tsize + 15) / 16) * 16;
    const size_t ne = static_cast<size_t>(M > WAVE ? M : WAVE);
    L.off_f = L.off_e + ((ne * sizeof(double) + 15) / 16) * 16;
    L.off_t = L.off_f + static_cast<size_t>(3) * WAVE * sizeof(double);
    const size_t stage = static_cast<size_t>(WAVE) * stage_stride(K) * tsize;
    const size_t adj = static_cast<size_t>(apw) * K * odd_len(NA) * tsize;
    L.total = L.off_t + (stage > adj ? stage : adj);
    return L;
}

// dE_i/dr_ij of one pair from the atom's K adjoint rows abr[k * NAP + mu]
// (eq. (24c)): d/dr [R_k(r) h_k(rhat)] = R'_k h_k rhat + R_k (grad_u h_k -
// (rhat . grad_u h_k) rhat) / r with h_k = sum_mu Abar_{k mu} A_mu, and
// rhat . grad_u h = sum_n n h_n over the degree-n parts (Euler).
//
// pair_gradient_k contracts over the radial index first, for a K fixed at
// compile time: W1_mu = sum_k Abar_{k mu} R'_k, W2_mu = sum_k Abar_{k mu} R_k,
// then g = (sum_mu W1_mu A_mu - sum_n n H_n / r) rhat + (1/r) sum_mu W2_mu
// grad A_mu with H_n = sum_{deg mu = n} W2_mu A_mu: 2 K + ~3 FMAs per
// monomial instead of ~3 K.
//
// Each monomial is its own basic block, entered under a condition the
// compiler cannot fold (an SGPR set to 1 by an s_mov_b32): within one block
// the code generator would otherwise issue all K * NA reads of the adjoint
// rows before the first FMA and spill them.  The K values of monomial mu + 1
// are read at the top of the block that contracts monomial mu.
template <typename T, int PA, int KK>
__device__ __forceinline__ void pair_gradient_k(const T* __restrict__ abr, const T (&A)[n_mono(PA)],
                                                const T (&R)[POD_MAX_K], const T (&dR)[POD_MAX_K], T ri, T ux,
                                                T uy, T uz, T& gx, T& gy, T& gz) {
    constexpr MonoTable<PA> mt{};
    constexpr int NA = n_mono(PA);
    constexpr int NAP = odd_len(NA);
    T s1 = 0;
    T hd[PA + 1];
    T gp[3][PA + 1];   // gradient sums grouped by the exponent being lowered
#pragma unroll
    for (int n = 0; n <= PA; ++n) { hd[n] = 0; gp[0][n] = 0; gp[1][n] = 0; gp[2][n] = 0; }
    T buf[2][KK];      // double buffer: values of monomial mu in buf[mu & 1]
#pragma unroll
    for (int k = 0; k < KK; ++k) buf[0][k] = abr[k * NAP];
#pragma unroll
    for (int mu = 0; mu < NA; ++mu) {
        int on;
        asm volatile("s_mov_b32 %0, 1" : "=s"(on));
        if (on) {
            const int cb = mu & 1;
            if (mu + 1 < NA) {
#pragma unroll
                for (int k = 0; k < KK; ++k) buf[cb ^ 1][k] = abr[k * NAP + mu + 1];
            }
            T w1 = 0, w2 = 0;
#pragma unroll
            for (int k = 0; k < KK; ++k) {
                w1 += buf[cb][k] * dR[k];
                w2 += buf[cb][k] * R[k];
            }
            s1 += w1 * A[mu];
            hd[mt.deg[mu]] += w2 * A[mu];
#pragma unroll
            for (int dd = 0; dd < 3; ++dd)
                if (mt.down[mu][dd] >= 0) gp[dd][mt.ex[mu][dd]] += w2 * A[mt.down[mu][dd]];
        }
    }
    T eul = 0, g0 = 0, g1 = 0, g2 = 0;
#pragma unroll
    for (int n = 1; n <= PA; ++n) {
        eul += T(n) * hd[n];
        g0 += T(n) * gp[0][n]; g1 += T(n) * gp[1][n]; g2 += T(n) * gp[2][n];
    }
    const T a1 = s1 - eul * ri;
    gx = a1 * ux + ri * g0;
    gy = a1 * uy + ri * g1;
    gz = a1 * uz + ri * g2;
}

// The same for any K: one pass over the monomials per radial function.
template <typename T, int PA>
__device__ __forceinline__ void pair_gradient_any(const T* __restrict__ abr, int K, const T (&A)[n_mono(PA)],
                                                  const T (&R)[POD_MAX_K], const T (&dR)[POD_MAX_K], T ri, T ux,
                                                  T uy, T uz, T& gx, T& gy, T& gz) {
    constexpr MonoTable<PA> mt{};
    constexpr int NA = n_mono(PA);
    constexpr int NAP = odd_len(NA);
    gx = 0; gy = 0; gz = 0;
#pragma unroll
    for (int k = 0; k < POD_MAX_K; ++k) {
        if (k < K) {
            const T* abk = abr + k * NAP;
            T hd[PA + 1];
            T gp[3][PA + 1];
#pragma unroll
            for (int n = 0; n <= PA; ++n) { hd[n] = 0; gp[0][n] = 0; gp[1][n] = 0; gp[2][n] = 0; }
#pragma unroll
            for (int mu = 0; mu < NA; ++mu) {
                const T w = abk[mu];
                hd[mt.deg[mu]] += w * A[mu];
#pragma unroll
                for (int dd = 0; dd < 3; ++dd)
                    if (mt.down[mu][dd] >= 0) gp[dd][mt.ex[mu][dd]] += w * A[mt.down[mu][dd]];
            }
            T hsum = 0, eul = 0, g0 = 0, g1 = 0, g2 = 0;
#pragma unroll
            for (int n = 0; n <= PA; ++n) {
                hsum += hd[n]; eul += T(n) * hd[n];
                g0 += T(n) * gp[0][n]; g1 += T(n) * gp[1][n]; g2 += T(n) * gp[2][n];
            }
            const T a1 = dR[k] * hsum - R[k] * eul * ri;
            const T a2 = R[k] * ri;
            gx += a1 * ux + a2 * g0;
            gy += a1 * uy + a2 * g1;
            gz += a1 * uz + a2 * g2;
        }
    }
}

// One workgroup = one wavefront = APW = 64 / K atoms.  Neighbour slots are
// processed K at a time per atom ("rounds"); in a round, lane (a, s)
// evaluates slot s of atom a.
template <typename T, int PA, int MODE, bool FAST>
__device__ __forceinline__ void atom_body(const KArgs<T>& g) {
    constexpr MonoTable<PA> mt{};
    constexpr int NA = n_mono(PA);
    constexpr int NAP = odd_len(NA);
    using Tab = D4Table<PA>;
    constexpr int KA = Tab::KA;

    const ParamsT<T>* __restrict__ P = &g.prm;
    const int K = P->K;
    const int M = P->M;
    const int SS = stage_stride(K);
    const int lane = threadIdx.x;
    const int apw = WAVE / K;
    const int al = lane / K;
    const int q = lane - al * K;       // radial index m, or neighbour slot within a round
    const int m = q;
    const int atom = blockIdx.x * apw + al;
    const bool act = (al < apw) && (atom < g.N);

    extern __shared__ __align__(16) unsigned char smem_raw[];
    const AtomLds LY = atom_lds_layout(K, NA, M, sizeof(T));
    T* sQ = reinterpret_cast<T*>(smem_raw + LY.off_q);
    double* sE = reinterpret_cast<double*>(smem_raw + LY.off_e);
    double* sF = reinterpret_cast<double*>(smem_raw + LY.off_f);
    T* sT = reinterpret_cast<T*>(smem_raw + LY.off_t);

    if (FAST)
        for (int i = lane; i < POD_MAX_L * POD_MAX_K; i += WAVE) sQ[i] = (&P->Q[0][0])[i];

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
    T pi[3] = {T(0), T(0), T(0)};
    if (act) { pi[0] = g.pos[3 * atom + 0]; pi[1] = g.pos[3 * atom + 1]; pi[2] = g.pos[3 * atom + 2]; }
    __syncthreads();

    // ---------------- forward: atomic basis row B_{i, m, .} (eq. (24b)) ----------------
    T acc[NA];
#pragma unroll
    for (int mu = 0; mu < NA; ++mu) acc[mu] = 0;
    SlotIdx i0 = slot_index(g, act && q < cnt, beg + q);
    T p0[3];
    slot_pos(g, i0, p0);
    SlotIdx i1 = slot_index(g, act && K + q < cnt, beg + K + q);
    for (int rd = 0; rd < nround; ++rd) {
        {
            // pair stage: rhat and R_k of slot rd*K + q, staged for the atom's K lanes
            const int slot = rd * K + q;
            const SlotIdx ic = i0;
            T pc[3] = {p0[0], p0[1], p0[2]};
            slot_pos(g, i1, p0);
            i0 = i1;
            i1 = slot_index(g, act && slot + 2 * K < cnt, beg + slot + 2 * K);
            T d[3], r;
            const bool ok = slot_geometry<T>(g, act && slot < cnt, ic, pc, pi, true, d, r);
            const T rinv = T(1) / r;
            T R[POD_MAX_K], dR[POD_MAX_K];
            radial_any<T, false, FAST>(P, sQ, r, rinv, R, dR);
            const T z = ok ? T(1) : T(0);
            T* row = sT + lane * SS;
            row[0] = d[0] * rinv; row[1] = d[1] * rinv; row[2] = d[2] * rinv;
#pragma unroll
            for (int k = 0; k < POD_MAX_K; ++k)
                if (k < K) row[3 + k] = R[k] * z;
        }
        __syncthreads();
        if (act) {
            for (int s = 0; s < K; ++s) {
                const T* row = sT + (al * K + s) * SS;
                accumulate_basis<T, PA>(acc, row[3 + m], row[0], row[1], row[2]);
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
    // eq. (30a) for the triples the model uses (none without 4-body terms):
    // the others only ever meet zero weights
    const int ka_used = P->K4 > 0 ? P->Ka4 : 0;
#pragma unroll
    for (int p = 0; p < KA; ++p)
        if (p < ka_used) {
#pragma unroll
            for (int t = Tab::build.tbeg[p]; t < Tab::build.tend[p]; ++t)
                d4[p] += T(Tab::build.tc[t]) * acc[Tab::build.tx[t]] * acc[Tab::build.ty[t]] * acc[Tab::build.tz[t]];
        }

    const bool has2 = act && m < P->K2;
    const bool has3 = act && m < P->K3;
    const bool has4 = act && m < P->K4;
    const int P3 = P->P3, Ka4 = P->Ka4;

    if (MODE == 0) {
        if (act) {
            T* Drow = g.D + static_cast<size_t>(atom) * M;
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
    const T w2 = has2 ? c[1 + m] : T(0);
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
    if constexpr (MODE == 2) {
        // network surrogate (eq. (673a)): energy y_i, adjoint weights c + dy/dD_i
        if (act) {
            const float* gn = g.g_net + static_cast<size_t>(atom) * g.n_net;
            if (has2) eff2 += static_cast<T>(gn[m]);
            if (has3) {
#pragma unroll
                for (int n = 0; n <= PA; ++n)
                    if (n <= P3) eff3[n] += static_cast<T>(gn[P->off3 - 1 + m * (P3 + 1) + n]);
            }
            if (q == 0) e += static_cast<double>(g.y_net[atom]);
        }
    }
#pragma unroll
    for (int p = 0; p < KA; ++p)
        if (Tab::build.pb[p] == 0) {
            eff2 += w4[p] * d3[Tab::build.pa[p]];
            eff3[Tab::build.pa[p]] += w4[p] * acc[0];
        }
    // the adjoint row dE_i/dB_{i m .}: in registers up to P_a = 5; beyond,
    // the row and the basis row do not both fit, so the adjoint row is
    // accumulated in its LDS slot (the staging area is free after the rounds)
    constexpr bool AB_LDS = NA > 60;
    T ab[AB_LDS ? 1 : NA];
    if constexpr (AB_LDS) {
        if (act) {
            T* abrow = sT + (al * K + m) * odd_len(NA);
#pragma unroll
            for (int mu = 0; mu < NA; ++mu)
                abrow[mu] = T(2 * mt.mult[mu]) * eff3[mt.deg[mu]] * acc[mu] + (mu == 0 ? eff2 : T(0));  // eq. (26c)
#pragma unroll
            for (int p = 0; p < KA; ++p)
                if (p < ka_used) {
#pragma unroll
                    for (int t = Tab::build.tbeg[p]; t < Tab::build.tend[p]; ++t) {
                        const int x = Tab::build.tx[t], y = Tab::build.ty[t], z = Tab::build.tz[t];
                        const T wc = w4[p] * T(Tab::build.tc[t]);
                        abrow[x] += wc * acc[y] * acc[z];
                        abrow[y] += wc * acc[x] * acc[z];
                        abrow[z] += wc * acc[x] * acc[y];
                    }
                }
        }
    } else {
#pragma unroll
        for (int mu = 0; mu < NA; ++mu) ab[mu] = T(2 * mt.mult[mu]) * eff3[mt.deg[mu]] * acc[mu];  // eq. (26c)
        ab[0] += eff2;
#pragma unroll
        for (int p = 0; p < KA; ++p)
            if (p < ka_used) {
#pragma unroll
                for (int t = Tab::build.tbeg[p]; t < Tab::build.tend[p]; ++t) {
                    const int x = Tab::build.tx[t], y = Tab::build.ty[t], z = Tab::build.tz[t];
                    const T wc = w4[p] * T(Tab::build.tc[t]);
                    ab[x] += wc * acc[y] * acc[z];
                    ab[y] += wc * acc[x] * acc[z];
                    ab[z] += wc * acc[x] * acc[y];
                }
            }
    }

    // per-atom energy: sum the K lanes of the atom through LDS
    {
        sE[lane] = e;
        __syncthreads();
        double ei = 0.0;
        if (act && q == 0) {
            for (int k = 0; k < K; ++k) ei += sE[al * K + k];
            if (g.E_atom) g.E_atom[atom] = static_cast<T>(ei);
        }
        __syncthreads();
        const double eb = wave_sum(ei);
        if (lane == 0) g.part[blockIdx.x] = eb;
    }
    // global descriptors G = sum_i D_i (eq. (58a)): block partial in LDS
    if (g.want_G) {
        for (int k = lane; k < M; k += WAVE) sE[k] = 0.0;
        __syncthreads();
        for (int a2 = 0; a2 < apw; ++a2) {
            if (al == a2 && act) {
                if (q == 0) sE[0] += 1.0;
                if (has2) sE[1 + m] += static_cast<double>(acc[0]);
                if (has3)
#pragma unroll
                    for (int n = 0; n <= PA; ++n)
                        if (n <= P3) sE[P->off3 + m * (P3 + 1) + n] += static_cast<double>(d3[n]);
                if (has4)
#pragma unroll
                    for (int p = 0; p < KA; ++p)
                        if (p < Ka4) sE[P->off4 + m * Ka4 + p] += static_cast<double>(d4[p]);
            }
            __syncthreads();
        }
        for (int k = lane; k < M; k += WAVE) g.part[static_cast<size_t>(10 + k) * gridDim.x + blockIdx.x] = sE[k];
    }

    if (!g.want_back) return;

    // ---------------- backward: g_ij = dE_i/dr_ij (eq. (24c)) ----------------
    // adjoint rows to LDS; then lane (a, s) takes neighbour slot s of atom a in
    // every round, re-evaluates its radial functions with derivatives and
    // contracts them with the K adjoint rows of atom a
    T* sAb = sT;
    if constexpr (!AB_LDS) {
        if (act) {
#pragma unroll
            for (int mu = 0; mu < NA; ++mu) sAb[(al * K + m) * NAP + mu] = ab[mu];
        }
    }
    __syncthreads();

    double vir[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) vir[k] = 0.0;
    double fo0 = 0.0, fo1 = 0.0, fo2 = 0.0;
    SlotIdx b0 = slot_index(g, act && q < cnt, beg + q);
    T bp0[3];
    slot_pos(g, b0, bp0);
    SlotIdx b1 = slot_index(g, act && K + q < cnt, beg + K + q);
    for (int rd = 0; rd < nround; ++rd) {
        const int slot = rd * K + q;
        const SlotIdx ic = b0;
        T pc[3] = {bp0[0], bp0[1], bp0[2]};
        slot_pos(g, b1, bp0);
        b0 = b1;
        b1 = slot_index(g, act && slot + 2 * K < cnt, beg + slot + 2 * K);
        if (act && slot < cnt) {
            T d[3], r;
            const bool ok = slot_geometry<T>(g, true, ic, pc, pi, false, d, r);
            if (ok) {
                const T ri = T(1) / r;
                T R[POD_MAX_K], dR[POD_MAX_K];
                radial_any<T, true, FAST>(P, sQ, r, ri, R, dR);
                const T ux = d[0] * ri, uy = d[1] * ri, uz = d[2] * ri;
                T A[NA];
                A[0] = T(1);
#pragma unroll
                for (int mu = 1; mu < NA; ++mu) {
                    const T u = mt.axis[mu] == 0 ? ux : (mt.axis[mu] == 1 ? uy : uz);
                    A[mu] = A[mt.par[mu]] * u;
                }
                T gx, gy, gz;
                const T* abr = sAb + (al * K) * NAP;
                // radial index first for the K of the benchmark models (FP64
                // per-atom kernel on the 15,840-atom box 90.5 -> 79.6 us, FP32
                // unchanged at 55.6 us); one pass per radial function otherwise
                if (K == 6) pair_gradient_k<T, PA, 6>(abr, A, R, dR, ri, ux, uy, uz, gx, gy, gz);
                else if (K == 4) pair_gradient_k<T, PA, 4>(abr, A, R, dR, ri, ux, uy, uz, gx, gy, gz);
                else pair_gradient_any<T, PA>(abr, K, A, R, dR, ri, ux, uy, uz, gx, gy, gz);
                if (g.gbuf) {
                    // stored at the reverse slot: the neighbour's gather reads its own list range
                    if (ic.rv >= 0 && ic.rv < g.P) {
                        T* gp3 = g.gbuf + 3 * static_cast<size_t>(ic.rv);
                        gp3[0] = gx; gp3[1] = gy; gp3[2] = gz;
                    } else {
                        atomicOr(g.err, ERR_NEIGH);
                    }
                } else {
                    const int j = ic.j;
                    atomicAdd(&g.Facc[3 * j + 0], -static_cast<double>(gx));
                    atomicAdd(&g.Facc[3 * j + 1], -static_cast<double>(gy));
                    atomicAdd(&g.Facc[3 * j + 2], -static_cast<double>(gz));
                }
                fo0 += gx; fo1 += gy; fo2 += gz;
                const double dd3[3] = {double(d[0]), double(d[1]), double(d[2])};
                const double gg[3] = {double(gx), double(gy), double(gz)};
#pragma unroll
                for (int x = 0; x < 3; ++x)
#pragma unroll
                    for (int y = 0; y < 3; ++y) vir[3 * x + y] -= dd3[x] * gg[y];
            } else if (g.gbuf && ic.rv >= 0 && ic.rv < g.P) {
                T* gp3 = g.gbuf + 3 * static_cast<size_t>(ic.rv);
                gp3[0] = T(0); gp3[1] = T(0); gp3[2] = T(0);
            }
        }
    }
    // own-atom force F_i += sum_j g_ij: sum the K lanes of the atom
    sF[3 * lane + 0] = fo0; sF[3 * lane + 1] = fo1; sF[3 * lane + 2] = fo2;
    __syncthreads();
    if (act && q == 0) {
        double f0 = 0.0, f1 = 0.0, f2 = 0.0;
        for (int k = 0; k < K; ++k) {
            const int l2 = al * K + k;
            f0 += sF[3 * l2]; f1 += sF[3 * l2 + 1]; f2 += sF[3 * l2 + 2];
        }
        if (g.gbuf) {
            g.fown[3 * atom + 0] = f0;
            g.fown[3 * atom + 1] = f1;
            g.fown[3 * atom + 2] = f2;
        } else {
            atomicAdd(&g.Facc[3 * atom + 0], f0);
            atomicAdd(&g.Facc[3 * atom + 1], f1);
            atomicAdd(&g.Facc[3 * atom + 2], f2);
        }
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double v = wave_sum(vir[k]);
        if (lane == 0) g.part[static_cast<size_t>(1 + k) * gridDim.x + blockIdx.x] = v;
    }
}

// Kernel entry points.  The FP64 instances up to angular degree 4 are asked
// to fit two wavefronts per SIMD (at most 256 registers); the others keep the
// compiler's default allocation.
template <typename T, int PA, int MODE, bool FAST>
__global__ __launch_bounds__(64) void atom_kernel(KArgs<T> g) {
    atom_body<T, PA, MODE, FAST>(g);
}

template <typename T, int PA, int MODE, bool FAST>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void atom_kernel_occ2(KArgs<T> g) {
    atom_body<T, PA, MODE, FAST>(g);
}

// Totals and forces.  Blocks 0 .. 9 + M: column sums of the block partials
// (column 0 -> E, 1..9 -> W, 10.. -> G).  Remaining blocks, with a reverse
// index: F_n = sum over the pairs p of n of g_p - g_rev(p) (8 atoms x 32
// lanes per block, deterministic); without one: F = Facc (accumulated with
// atomics) and Facc cleared for the next call.
template <typename T>
struct FinArgs {
    const double* part;
    int nblk, ncol;
    double* E;
    double* W;
    double* G;
    double* Facc;
    T* F;
    long n3;
    const T* gbuf;     // gather path: g stored at reverse slots
    const double* fown;  // gather path: own-atom sums
    const int* rev;
    const int* offsets;
    int N, P;
    int* err;
};

template <typename T>
__global__ __launch_bounds__(256) void finalize_kernel(FinArgs<T> f) {
    const int col = blockIdx.x;
    if (col >= f.ncol) {
        const int fb = col - f.ncol;
        if (f.rev) {
            const int a = fb * 8 + static_cast<int>(threadIdx.x) / 32;
            const int s0 = threadIdx.x % 32;
            double f0 = 0.0, f1 = 0.0, f2 = 0.0;
            if (a < f.N) {
                const int b = f.offsets[a], e = f.offsets[a + 1];
                if (b >= 0 && e >= b && e <= f.P) {
                    // slot p of atom a holds g of the pair (j -> a) whose reverse is p
                    for (int p = b + s0; p < e; p += 32) {
                        f0 -= static_cast<double>(f.gbuf[3 * static_cast<size_t>(p) + 0]);
                        f1 -= static_cast<double>(f.gbuf[3 * static_cast<size_t>(p) + 1]);
                        f2 -= static_cast<double>(f.gbuf[3 * static_cast<size_t>(p) + 2]);
                    }
                }
            }
#pragma unroll
            for (int o = 16; o >= 1; o >>= 1) {
                f0 += __shfl_xor(f0, o, 32);
                f1 += __shfl_xor(f1, o, 32);
                f2 += __shfl_xor(f2, o, 32);
            }
            if (a < f.N && s0 == 0 && f.F) {
                f.F[3 * a + 0] = static_cast<T>(f.fown[3 * a + 0] + f0);
                f.F[3 * a + 1] = static_cast<T>(f.fown[3 * a + 1] + f1);
                f.F[3 * a + 2] = static_cast<T>(f.fown[3 * a + 2] + f2);
            }
        } else {
            const long i = static_cast<long>(fb) * 256 + threadIdx.x;
            if (i < f.n3) {
                if (f.F) f.F[i] = static_cast<T>(f.Facc[i]);
                f.Facc[i] = 0.0;
            }
        }
        return;
    }
    const double* part = f.part;
    const int nblk = f.nblk;
    double* E = f.E;
    double* W = f.W;
    double* G = f.G;
    if ((col == 0 && !E) || (col >= 1 && col < 10 && !W) || (col >= 10 && !G)) return;
    const double* src = part + static_cast<size_t>(col) * nblk;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) s += src[b];
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if (static_cast<int>(threadIdx.x) < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double v = red[0];
        if (col == 0) *E = v;
        else if (col < 10) W[col - 1] = v;
        else G[col - 10] = v;
    }
}

// Reverse-pair index: for pair p = (i -> j, n) find q = (j -> i, -n) in the
// list of j (8 atoms x 32 lanes per 256-thread block).
__global__ __launch_bounds__(256) void reverse_kernel(const int* __restrict__ offsets, const int* __restrict__ nbr_j,
                                                      const int* __restrict__ shift, int N, int P, int* rev,
                                                      int* err) {
    const int a = blockIdx.x * 8 + static_cast<int>(threadIdx.x) / 32;
    const int s0 = threadIdx.x % 32;
    if (a >= N) return;
    const int b = offsets[a], e = offsets[a + 1];
    if (b < 0 || e < b || e > P) {
        if (s0 == 0) atomicOr(err, ERR_NEIGH);
        return;
    }
    for (int p = b + s0; p < e; p += 32) {
        const int j = nbr_j[p];
        const int sh = shift[p];
        int found = -1;
        if (j >= 0 && j < N) {
            const int neg = ((-unpack_shift(sh, 0)) & 0xFF) | (((-unpack_shift(sh, 1)) & 0xFF) << 8) |
                            (((-unpack_shift(sh, 2)) & 0xFF) << 16);
            const int jb = offsets[j], je = offsets[j + 1];
            if (jb >= 0 && je >= jb && je <= P)
                for (int qq = jb; qq < je; ++qq)
                    if (nbr_j[qq] == a && (shift[qq] & 0xFFFFFF) == neg) { found = qq; break; }
        }
        rev[p] = found;
        if (found < 0) atomicOr(err, ERR_NEIGH);
    }
}

template <typename T, int PA, int MODE>
hipError_t launch_atom(const KArgs<T>& a, bool fast, int nblk, size_t lds, hipStream_t st) {
    constexpr bool occ2 = sizeof(T) == 8 && PA <= 4;
    if constexpr (occ2) {
        if (fast) hipLaunchKernelGGL((atom_kernel_occ2<T, PA, MODE, true>), dim3(nblk), dim3(WAVE), lds, st, a);
        else hipLaunchKernelGGL((atom_kernel_occ2<T, PA, MODE, false>), dim3(nblk), dim3(WAVE), lds, st, a);
    } else {
        if (fast) hipLaunchKernelGGL((atom_kernel<T, PA, MODE, true>), dim3(nblk), dim3(WAVE), lds, st, a);
        else hipLaunchKernelGGL((atom_kernel<T, PA, MODE, false>), dim3(nblk), dim3(WAVE), lds, st, a);
    }
    return hipGetLastError();
}

template <typename T, int MODE>
hipError_t dispatch_pa(int PA, const KArgs<T>& a, bool fast, int nblk, size_t lds, hipStream_t st) {
    switch (PA) {
        case 0: return launch_atom<T, 0, MODE>(a, fast, nblk, lds, st);
        case 1: return launch_atom<T, 1, MODE>(a, fast, nblk, lds, st);
        case 2: return launch_atom<T, 2, MODE>(a, fast, nblk, lds, st);
        case 3: return launch_atom<T, 3, MODE>(a, fast, nblk, lds, st);
        case 4: return launch_atom<T, 4, MODE>(a, fast, nblk, lds, st);
        case 5: return launch_atom<T, 5, MODE>(a, fast, nblk, lds, st);
        case 6: return launch_atom<T, 6, MODE>(a, fast, nblk, lds, st);
        default: return hipErrorInvalidValue;
    }
}

size_t lds_bytes(int K, int PA, size_t tsize, int M) { return atom_lds_layout(K, n_mono(PA), M, tsize).total; }

template <typename T>
const ParamsT<T>& host_params(const pod_handle* h);
template <>
const ParamsT<double>& host_params<double>(const pod_handle* h) { return h->hp_d; }
template <>
const ParamsT<float>& host_params<float>(const pod_handle* h) { return h->hp_f; }

template <typename T>
int fill_args(pod_handle* h, KArgs<T>& a, int N, int P, const void* pos, const double* cell, const int* offsets,
              const int* nbr_j, const int* shift) {
    a.prm = host_params<T>(h);
    a.N = N; a.P = P;
    a.pos = static_cast<const T*>(pos);
    a.cell.periodic = cell != nullptr;
    for (int k = 0; k < 9; ++k) {
        const double v = cell ? cell[k] : 0.0;
        if (!std::isfinite(v)) return POD_EINVAL;
        a.cell.a[k] = static_cast<T>(v);
    }
    a.offsets = offsets; a.nbr_j = nbr_j; a.shift = shift;
    a.coef = nullptr; a.D = nullptr; a.E_atom = nullptr; a.Facc = nullptr; a.gbuf = nullptr; a.part = nullptr;
    a.fown = nullptr; a.rev = nullptr;
    a.want_G = 0; a.want_back = 0;
    a.y_net = nullptr; a.g_net = nullptr; a.n_net = 0;
    a.err = h->d_err;
    return POD_OK;
}

template <typename T>
int descriptors_impl(pod_handle* h, int N, int P, const void* pos, const double* cell, const int* offsets,
                     const int* nbr_j, const int* shift, void* D) {
    if (N == 0) return POD_OK;
    KArgs<T> a;
    const int rc = fill_args<T>(h, a, N, P, pos, cell, offsets, nbr_j, shift);
    if (rc != POD_OK) return rc;
    a.D = static_cast<T*>(D);
    const int apw = WAVE / h->K;
    const int nblk = (N + apw - 1) / apw;
    timing_begin(h, 1);
    const hipError_t e = dispatch_pa<T, 0>(h->PA, a, h->std_ok != 0, nblk, lds_bytes(h->K, h->PA, sizeof(T), h->M),
                                           h->stream);
    timing_end(h, 1);
    return e == hipSuccess ? POD_OK : POD_EHIP;
}

template <typename T, int MODE = 1>
int energy_forces_impl(pod_handle* h, int N, int P, const void* pos, const double* cell, const int* offsets,
                       const int* nbr_j, const int* shift, const int* rev, const void* c, void* E_atom, double* E,
                       void* F, double* W, double* G, const float* y_net = nullptr, const float* g_net = nullptr,
                       int n_net = 0) {
    KArgs<T> a;
    int rc = fill_args<T>(h, a, N, P, pos, cell, offsets, nbr_j, shift);
    if (rc != POD_OK) return rc;
    const int apw = WAVE / h->K;
    const int nblk = (N + apw - 1) / apw;
    const int ncol = 10 + h->M;
    const bool gather = rev != nullptr && F != nullptr;
    const size_t part_bytes = (static_cast<size_t>(ncol) * (nblk > 0 ? nblk : 1) * sizeof(double) + 255) & ~size_t(255);
    const size_t g_bytes = gather ? (static_cast<size_t>(P > 0 ? P : 1) * 3 * sizeof(T) + 255) & ~size_t(255) : 0;
    const size_t o_bytes = gather ? static_cast<size_t>(N > 0 ? N : 1) * 3 * sizeof(double) : 0;
    rc = ensure_scratch(h, part_bytes + g_bytes + o_bytes);
    if (rc != POD_OK) return rc;
    rc = ensure_force_acc(h, N);
    if (rc != POD_OK) return rc;
    a.coef = static_cast<const T*>(c);
    a.E_atom = static_cast<T*>(E_atom);
    a.Facc = h->d_facc;
    a.part = static_cast<double*>(h->d_scratch);
    a.gbuf = gather ? reinterpret_cast<T*>(static_cast<char*>(h->d_scratch) + part_bytes) : nullptr;
    a.fown = gather ? reinterpret_cast<double*>(static_cast<char*>(h->d_scratch) + part_bytes + g_bytes) : nullptr;
    a.rev = gather ? rev : nullptr;
    a.want_G = G != nullptr;
    a.want_back = (F != nullptr) || (W != nullptr);
    a.y_net = y_net; a.g_net = g_net; a.n_net = n_net;
    if (nblk > 0) {
        timing_begin(h, 1);
        const hipError_t e = dispatch_pa<T, MODE>(h->PA, a, h->std_ok != 0, nblk,
                                               lds_bytes(h->K, h->PA, sizeof(T), h->M), h->stream);
        timing_end(h, 1);
        if (e != hipSuccess) return POD_EHIP;
    }
    // totals, and the forces: gathered from the per-pair gradients, or copied
    // out of the atomic accumulator (which is re-zeroed)
    FinArgs<T> fa;
    fa.part = static_cast<const double*>(h->d_scratch);
    fa.nblk = nblk; fa.ncol = ncol;
    fa.E = E; fa.W = a.want_back ? W : nullptr; fa.G = G;
    fa.Facc = h->d_facc; fa.F = static_cast<T*>(F);
    fa.n3 = (a.want_back && !gather) ? 3L * N : 0L;
    fa.gbuf = a.gbuf; fa.fown = a.fown; fa.rev = gather ? rev : nullptr; fa.offsets = offsets;
    fa.N = N; fa.P = P; fa.err = h->d_err;
    const int nfb = gather ? (N + 7) / 8 : static_cast<int>((fa.n3 + 255) / 256);
    if (E || W || G || nfb > 0) {
        timing_begin(h, 0);
        hipLaunchKernelGGL((finalize_kernel<T>), dim3(ncol + nfb), dim3(256), 0, h->stream, fa);
        timing_end(h, 0);
        if (hipGetLastError() != hipSuccess) {
            h->facc_dirty = 1;
            return POD_EHIP;
        }
    }
    return POD_OK;
}

// Network surrogate of the 4-body term: descriptors, network forward and
// input gradient, then energy and adjoint with per-atom weights (mode 2).
template <typename T>
int surrogate_impl(pod_handle* h, int N, int P, const void* pos, const double* cell, const int* offsets,
                   const int* nbr_j, const int* shift, const int* rev, const void* c, const float* theta,
                   const float* mu, const float* isg, void* E_atom, double* E, void* F, double* W) {
    const int n_in = h->M - 1;
    const size_t align = 256;
    const size_t d_bytes = (static_cast<size_t>(N) * h->M * sizeof(T) + align - 1) / align * align;
    const size_t y_bytes = (static_cast<size_t>(N) * sizeof(float) + align - 1) / align * align;
    const size_t g_bytes = static_cast<size_t>(N) * n_in * sizeof(float);
    float* y = nullptr;
    float* gr = nullptr;
    if (N > 0) {
        int rc = ensure_mscratch(h, d_bytes + y_bytes + g_bytes);
        if (rc != POD_OK) return rc;
        char* base = static_cast<char*>(h->d_mscratch);
        T* D = reinterpret_cast<T*>(base);
        y = reinterpret_cast<float*>(base + d_bytes);
        gr = reinterpret_cast<float*>(base + d_bytes + y_bytes);
        rc = descriptors_impl<T>(h, N, P, pos, cell, offsets, nbr_j, shift, D);
        if (rc != POD_OK) return rc;
        rc = mlp_forward_launch(h, N, n_in, D + 1, h->M, h->dtype, theta, mu, isg, y, gr);
        if (rc != POD_OK) return rc;
    }
    return energy_forces_impl<T, 2>(h, N, P, pos, cell, offsets, nbr_j, shift, rev, c, E_atom, E, F, W, nullptr,
                                    y, gr, n_in);
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
                      const int* nbr_j, const int* shift, const int* rev, const void* c, void* E_atom, double* E,
                      void* F, double* W, double* G) {
    if (pod::bad_common(h, N, P, pos, offsets, nbr_j, shift)) return POD_EINVAL;
    if (!c) return POD_EINVAL;
    if (h->dtype == POD_F64)
        return pod::energy_forces_impl<double>(h, N, P, pos, cell, offsets, nbr_j, shift, rev, c, E_atom, E, F, W,
                                               G);
    return pod::energy_forces_impl<float>(h, N, P, pos, cell, offsets, nbr_j, shift, rev, c, E_atom, E, F, W, G);
}

int pod_energy_forces_surrogate(pod_handle* h, int N, int P, const void* pos, const double* cell,
                                const int* offsets, const int* nbr_j, const int* shift, const int* rev, const void* c,
                                const float* theta, const float* mu, const float* inv_sigma, void* E_atom, double* E,
                                void* F, double* W) {
    if (pod::bad_common(h, N, P, pos, offsets, nbr_j, shift)) return POD_EINVAL;
    if (!c || !theta || !mu || !inv_sigma) return POD_EINVAL;
    if (h->K4 != 0) return POD_EINVAL;
    if (h->M - 1 < 1 || h->M - 1 > POD_MLP_MAX_IN) return POD_ENOTSUP;
    if (h->dtype == POD_F64)
        return pod::surrogate_impl<double>(h, N, P, pos, cell, offsets, nbr_j, shift, rev, c, theta, mu, inv_sigma,
                                           E_atom, E, F, W);
    return pod::surrogate_impl<float>(h, N, P, pos, cell, offsets, nbr_j, shift, rev, c, theta, mu, inv_sigma,
                                      E_atom, E, F, W);
}

int pod_neighbor_reverse(pod_handle* h, int N, int P, const int* offsets, const int* nbr_j, const int* shift,
                         int* rev) {
    if (!h || N < 0 || P < 0) return POD_EINVAL;
    if (N > 0 && !offsets) return POD_EINVAL;
    if (P > 0 && (!nbr_j || !shift || !rev)) return POD_EINVAL;
    if (N == 0) return POD_OK;
    hipLaunchKernelGGL(pod::reverse_kernel, dim3((N + 7) / 8), dim3(256), 0, h->stream, offsets, nbr_j, shift, N, P,
                       rev, h->d_err);
    return hipGetLastError() == hipSuccess ? POD_OK : POD_EHIP;
}

}  // extern "C"
