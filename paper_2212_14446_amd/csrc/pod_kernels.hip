// Kernels of the fast POD path for gfx950 (CDNA4).
//
// atom_kernel  (one 64-lane wavefront per workgroup, APW = 64 / K atoms):
//   lane l serves atom a = l / K and radial index m = l % K and keeps the row
//   B_{i m .} = sum_j R_m(r_ij) A_.(rhat_ij) of the atomic basis (Sec. II.E,
//   eq. (24b)) in registers.  Neighbours are taken K at a time per atom
//   ("rounds"): in a round, lane (a, s) evaluates slot s of atom a -- pair
//   geometry and the radial basis (Sec. II.B, eqs. (3)-(8), (11), (12)) --
//   and stages {rhat, R_k} in LDS for the atom's K lanes, with the next
//   slots' indices and positions prefetched; it also records the pair's
//   centre atom and vector for the pair kernel.  Every contraction of
//   Sec. II.E is diagonal in m (the same radial function in all factors,
//   eqs. (14), (17a)), so D3, D4, the energy and the adjoint row
//   dE_i/dB_{i m .} come from the lane's own row with compile-time tables.
//   The adjoint rows go to memory, [atom][k][mu]; E and G leave as
//   per-workgroup partials.
// pair_kernel  (one pair per lane, 64 consecutive list slots per block):
//   loads the adjoint rows of the block's centre atoms into LDS, re-evaluates
//   R_k and R'_k and forms dE_i/dr_ij (eq. (24c)); stores it at the pair's
//   own and reverse slots (gather path, with a reverse-pair index) or adds it
//   to an FP64 accumulator with device atomics; the virial leaves as
//   per-block partials.
// finalize_kernel  sums the partials in a fixed order (E, W, G) and forms the
//   forces: on the gather path each atom adds what its own list range holds
//   (32 lanes per atom); otherwise it copies and clears the accumulator.
// reverse_kernel  builds the reverse-pair index of a list once.
// Models beyond these kernels' register budget (angular degree above
// FAST_MAX_PA or more than FAST_MAX_K radial functions) run the whole
// energy path in the wide-degree kernel of pod_wide.hip, whose partials and
// pair gradients have the same layout, so finalize_kernel serves both.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "pod.h"
#include "pod_device.h"
#include "pod_net.h"
#include "pod_internal.h"
#include "pod_tables.h"
#include "pod_wide.h"

namespace pod {

// Scratch of pod_energy_forces_noalloc: one array per GPU, placed with the
// code object.  Host code reaches it only through the device address
// looked up by resolve_static_scratch (the array's name is not a device
// address in host code).
__device__ __align__(256) unsigned char scratch[POD_STATIC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

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
    T* abar;           // adjoint rows dE_i/dB_i, [N][K][NA] (forces or virial requested)
    int* centre;       // centre atom of every pair, for the pair kernel
    T* pdv;            // pair vectors r_ij of every pair (zero when not a neighbour), for the pair kernel
    double* part;      // block partials, column-major [10 + M][nblk] (mode 1)
    int want_G;        // block partials of G requested
    int want_back;     // adjoint rows requested (forces or virial)
    const net::Packed* netw;  // mode 2: network weights (pod_net.h)
    int n_net;                // mode 2: network inputs, descriptor columns 1 .. n_net
    int* err;
};

// Neighbour slots are fetched two rounds ahead: the index and image shift of
// round r + 2 and the neighbour position of round r + 1 are requested before
// the arithmetic of round r (slot helpers in pod_device.h).

// KR: radial functions formed on the standard-family path (K when it is
// fixed at compile time, else all FAST_MAX_K, zero beyond K).
template <typename T, bool DERIV, bool FAST, int KR = FAST_MAX_K>
__device__ __forceinline__ void radial_any(const ParamsT<T>* __restrict__ P, const T* sQ, T r, T rinv,
                                           T (&R)[FAST_MAX_K], T (&dR)[FAST_MAX_K]) {
    if constexpr (FAST) radial_std<T, DERIV, KR>(P, sQ, r, rinv, R, dR);
    else radial<T, DERIV>(P, r, rinv, R, dR);
}

// LDS layout of atom_kernel (per 64-lane workgroup), in bytes:
//   [per-lane double scratch (max(64, M))]
//   [T area: union { round staging [64][stage_stride(K)], G staging
//    [2 + PA + KA][64] doubles, adjoint rows [APW][K][NA] }]
// Per-atom stride of the adjoint rows in memory and LDS, in elements: K * NA
// rounded up to a multiple of 16 bytes (the direct loads into LDS move 16
// bytes per lane).
__host__ __device__ constexpr int abar_stride(int K, int NA, int tsize) {
    return ((K * NA * tsize + 15) / 16 * 16) / tsize;
}

__host__ __device__ constexpr int stage_stride(int K) { return (3 + K) | 1; }
__host__ __device__ constexpr int odd_len(int n) { return n | 1; }

struct AtomLds {
    size_t off_e, off_t, total;
};

// With the network (mode 2) a workgroup is nw wavefronts, each with the
// layout above (its T area holds the basis rows in the adjoint-row slots
// while the network runs), followed by the network tiles of the workgroup's
// nw * APW atoms, 16 atoms per tile.  A tile slot holds the standardised
// inputs [16][MAX_IN] (bfloat16), later overwritten by the input gradients
// [16][MAX_IN] (FP32), and the outputs [16] (FP32).
constexpr size_t NET_LDS = 16 * net::MAX_IN * 4 + 16 * 4;
__host__ __device__ constexpr int net_tiles(int nw, int apw) { return (nw * apw + 15) / 16; }

__host__ __device__ inline AtomLds atom_lds_layout(int K, int NA, int M, size_t tsize, int KA, int PA) {
    const int apw = WAVE / K;
    AtomLds L;
    L.off_e = 0;
    const size_t ne = static_cast<size_t>(M > WAVE ? M : WAVE);
    L.off_t = L.off_e + ((ne * sizeof(double) + 15) / 16) * 16;
    const size_t stage = static_cast<size_t>(WAVE) * stage_stride(K) * tsize;
    const size_t adj = static_cast<size_t>(apw) * abar_stride(K, NA, static_cast<int>(tsize)) * tsize;
    // G staging: [1 + (PA + 1) + KA][64] doubles
    const size_t gst = static_cast<size_t>(2 + PA + KA) * WAVE * sizeof(double);
    size_t t = stage > adj ? stage : adj;
    t = t > gst ? t : gst;
    L.total = L.off_t + t;
    return L;
}

// dE_i/dr_ij of one pair from the atom's K adjoint rows abr[k * NAP + mu]
// (eq. (24c)): d/dr [R_k(r) h_k(rhat)] = R'_k h_k rhat + R_k (grad_u h_k -
// (rhat . grad_u h_k) rhat) / r with h_k = sum_mu Abar_{k mu} A_mu, and
// rhat . grad_u h = sum_n n h_n over the degree-n parts (Euler).

// The same for any K: one pass over the monomials per radial function.
template <typename T, int PA>
__device__ __forceinline__ void pair_gradient_any(const T* __restrict__ abr, int K, const T (&A)[n_mono(PA)],
                                                  const T (&R)[FAST_MAX_K], const T (&dR)[FAST_MAX_K], T ri, T ux,
                                                  T uy, T uz, T& gx, T& gy, T& gz) {
    constexpr MonoTable<PA> mt{};
    constexpr int NA = n_mono(PA);
    constexpr int NAP = NA;    // rows of one atom are contiguous
    gx = 0; gy = 0; gz = 0;
#pragma unroll
    for (int k = 0; k < FAST_MAX_K; ++k) {
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
    const int AST = abar_stride(K, NA, sizeof(T));   // per-atom stride of the adjoint rows
    const int apw = WAVE / K;
    // Mode 2: nw wavefronts per workgroup, wavefront wid taking atom group
    // grp = blockIdx.x * nw + wid of the ngrp groups of APW atoms (the last
    // workgroup may hold groups past the end, which only take part in the
    // workgroup's barriers).  Otherwise one wavefront per workgroup.
    const int nw = MODE == 2 ? static_cast<int>(blockDim.x) / WAVE : 1;
    const int wid = MODE == 2 ? __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / WAVE) : 0;
    const int lane = MODE == 2 ? static_cast<int>(threadIdx.x) % WAVE : static_cast<int>(threadIdx.x);
    const int grp = MODE == 2 ? static_cast<int>(blockIdx.x) * nw + wid : static_cast<int>(blockIdx.x);
    const int ngrp = MODE == 2 ? (g.N + apw - 1) / apw : static_cast<int>(gridDim.x);
    const bool grp_live = MODE != 2 || grp < ngrp;
    const int al = lane / K;
    const int q = lane - al * K;       // radial index m, or neighbour slot within a round
    const int m = q;
    const int atom = grp * apw + al;
    const bool act = (al < apw) && (atom < g.N);

    extern __shared__ __align__(16) unsigned char smem_raw[];
    const AtomLds LY = atom_lds_layout(K, NA, M, sizeof(T), KA, PA);
    unsigned char* wbase = smem_raw + (MODE == 2 ? static_cast<size_t>(wid) * LY.total : 0);
    double* sE = reinterpret_cast<double*>(wbase + LY.off_e);
    T* sT = reinterpret_cast<T*>(wbase + LY.off_t);

    int beg = 0, cnt = 0;
    int eb = 0;                         // error-word bits found by this lane
    if (act) {
        const int b = g.offsets[atom], e = g.offsets[atom + 1];
        if (b < 0 || e < b || e > g.P) eb |= ERR_NEIGH;
        else { beg = b; cnt = e - b; }
    }
    const int wmax = __builtin_amdgcn_readfirstlane(wave_max(cnt));   // the wavefront's longest neighbour list
    const int nround = (wmax + K - 1) / K;
    T pi[3] = {T(0), T(0), T(0)};
    if (act) { pi[0] = g.pos[3 * atom + 0]; pi[1] = g.pos[3 * atom + 1]; pi[2] = g.pos[3 * atom + 2]; }

    // ---------------- forward: atomic basis row B_{i, m, .} (eq. (24b)) ----------------
    T acc[NA];
#pragma unroll
    for (int mu = 0; mu < NA; ++mu) acc[mu] = 0;
    if (nround > 0) {   // some atom has pairs: the list is not empty
        SlotIdx i0 = slot_index(g, act && q < cnt, beg + q);
        T p0[3];
        slot_pos(g, i0, p0);
        SlotIdx i1 = slot_index(g, act && K + q < cnt, beg + K + q);
        for (int rd = 0; rd < nround; ++rd) {
            {
                // pair stage: rhat and R_k of slot rd*K + q, staged for the atom's K lanes
                const int slot = rd * K + q;
                const bool live = act && slot < cnt;
                const SlotIdx ic = i0;
                T pc[3] = {p0[0], p0[1], p0[2]};
                slot_pos(g, i1, p0);
                i0 = i1;
                i1 = slot_index(g, act && slot + 2 * K < cnt, beg + slot + 2 * K);
                T d[3], r;
                const bool ok = slot_geometry<T>(g, live, ic, pc, pi, eb, d, r);
                if constexpr (MODE != 0) {
                    // centre atom and pair vector for the pair kernel (an empty
                    // slot writes the spare entry P)
                    const int pw = live ? beg + slot : g.P;
                    g.centre[pw] = atom;
                    T* pv = g.pdv + 3 * static_cast<size_t>(pw);
                    pv[0] = d[0]; pv[1] = d[1]; pv[2] = d[2];
                }
                const T rinv = T(1) / r;
                T R[FAST_MAX_K], dR[FAST_MAX_K];
                radial_any<T, false, FAST>(P, &P->Q[0][0], r, rinv, R, dR);
                const T z = ok ? T(1) : T(0);
                T* row = sT + lane * SS;
                row[0] = d[0] * rinv; row[1] = d[1] * rinv; row[2] = d[2] * rinv;
#pragma unroll
                for (int k = 0; k < FAST_MAX_K; ++k)
                    if (k < K) row[3 + k] = R[k] * z;
            }
            wave_sync();
            if (act) {
                // slots past the wavefront's longest list (in its last round)
                // hold R = 0 for every atom: not visited
                const int ns = wmax - rd * K < K ? wmax - rd * K : K;
                for (int s = 0; s < ns; ++s) {
                    const T* row = sT + (al * K + s) * SS;
                    accumulate_basis<T, PA>(acc, row[3 + m], row[0], row[1], row[2]);
                }
            }
            wave_sync();
        }
    }
    {
        const int ew = wave_or(eb);
        if (lane == 0 && ew != 0) atomicOr(g.err, ew);
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

    // global descriptors G = sum_i D_i (eq. (58a)): block partial.  Lane
    // (atom, m) holds the values of columns that belong to radial index m
    // only -- D2 (j = 0), D3 (j = 1 .. P3 + 1), D4 (j = P3 + 2 ..) -- so the
    // block sum of column (m, j) adds lanes m, K + m, 2K + m, ...: the values
    // go to LDS as [j][lane] (the round staging area, free here) and thread
    // (m, j) sums its atoms in order.
    if (g.want_G) {
        constexpr int NJ = 1 + (PA + 1) + KA;
        const int P3e = P->K3 > 0 ? P3 : -1;     // D3 rows j = 1 .. P3e + 1, D4 rows after them
        double* sG = reinterpret_cast<double*>(sT);
#pragma unroll
        for (int j = 0; j < NJ; ++j) sG[j * WAVE + lane] = 0.0;
        if (has2) sG[lane] = static_cast<double>(acc[0]);
        if (has3) {
#pragma unroll
            for (int n = 0; n <= PA; ++n)
                if (n <= P3) sG[(1 + n) * WAVE + lane] = static_cast<double>(d3[n]);
        }
        if (has4) {
#pragma unroll
            for (int p = 0; p < KA; ++p)
                if (p < Ka4) sG[(2 + P3e + p) * WAVE + lane] = static_cast<double>(d4[p]);
        }
        wave_sync();
        const int na = (g.N - grp * apw < apw) ? g.N - grp * apw : apw;
        const int nj3 = 2 + P3e + Ka4;     // columns per radial index
        for (int t = lane; t < K * nj3; t += WAVE) {
            const int mm = t / nj3, j = t - mm * nj3;
            int col = -1;
            if (j == 0) col = mm < P->K2 ? 1 + mm : -1;
            else if (j <= P3e + 1) col = mm < P->K3 ? P->off3 + mm * (P3 + 1) + (j - 1) : -1;
            else col = mm < P->K4 ? P->off4 + mm * Ka4 + (j - P3e - 2) : -1;
            if (col < 0) continue;
            double sum = 0.0;
            for (int a2 = 0; a2 < na; ++a2) sum += sG[j * WAVE + a2 * K + mm];
            if (grp_live) g.part[static_cast<size_t>(10 + col) * ngrp + grp] = sum;
        }
        if (lane == 0 && grp_live) g.part[static_cast<size_t>(10) * ngrp + grp] = static_cast<double>(na);
        wave_sync();
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
        // network surrogate (eq. (673a)) on the workgroup's atoms, 16 at a
        // time (pod_net.h): the 2/3-body descriptors standardised and rounded
        // as the network kernels do, then the energy y_i and the adjoint
        // weights c + dy/dD_i.  The basis row waits in its adjoint-row slot
        // in LDS meanwhile (the adjoint is formed there in place below), so
        // the network's registers do not add to the row's.  Every wavefront
        // writes the input rows of its atoms (row wid * APW + a of the
        // workgroup's tiles); the tiles are then shared out over the
        // wavefronts, so a workgroup of nw wavefronts evaluates
        // ceil(nw * APW / 16) tiles rather than nw partly empty ones.
        using namespace net;
        if (act) {
            T* brow = sT + al * AST + m * NA;
#pragma unroll
            for (int mu = 0; mu < NA; ++mu) brow[mu] = acc[mu];
        }
        const int ntile = net_tiles(nw, apw);
        unsigned char* nreg = smem_raw + static_cast<size_t>(nw) * LY.total;
        const int row = wid * apw + al;   // the atom's row in the workgroup's tiles
        unsigned char* rslot = nreg + static_cast<size_t>(row >> 4) * NET_LDS;
        unsigned short* xrow = reinterpret_cast<unsigned short*>(rslot) + (row & 15) * MAX_IN;
        const float* drow = reinterpret_cast<const float*>(rslot) + (row & 15) * MAX_IN;
        const float* yrow = reinterpret_cast<const float*>(rslot) + 16 * MAX_IN + (row & 15);
        const int off3 = P->off3;
        {
            // zero the wavefront's rows (128 bytes each), and with the last
            // wavefront the rows of the last tile past the workgroup's atoms
            const Packed* pk = g.netw;
            const int r0 = wid * apw;
            const int r1 = wid == nw - 1 ? 16 * ntile : r0 + apw;
            for (int idx = lane; idx < (r1 - r0) * 8; idx += WAVE) {
                const int rr = r0 + (idx >> 3);
                uint4* z4 = reinterpret_cast<uint4*>(nreg + static_cast<size_t>(rr >> 4) * NET_LDS) + (rr & 15) * 8;
                z4[idx & 7] = uint4{0u, 0u, 0u, 0u};
            }
            wave_sync();
            if (act) {
                // the lane's standardisation values, requested together (an
                // absent term reads entry 0 and is not written)
                const int k2 = has2 ? m : 0;
                const float mu2 = pk->mu[k2], is2 = pk->isg[k2];
                float mu3[PA + 1], is3[PA + 1];
#pragma unroll
                for (int n = 0; n <= PA; ++n) {
                    const int k = (has3 && n <= P3) ? off3 - 1 + m * (P3 + 1) + n : 0;
                    mu3[n] = pk->mu[k];
                    is3[n] = pk->isg[k];
                }
                if (has2) xrow[m] = to_bf16(static_cast<float>((acc[0] - static_cast<T>(mu2)) * static_cast<T>(is2)));
                if (has3) {
#pragma unroll
                    for (int n = 0; n <= PA; ++n)
                        if (n <= P3)
                            xrow[off3 - 1 + m * (P3 + 1) + n] =
                                to_bf16(static_cast<float>((d3[n] - static_cast<T>(mu3[n])) * static_cast<T>(is3[n])));
                }
            }
        }
        __syncthreads();
        const int r = lane & 15, gq = lane >> 4;
#pragma unroll 1
        for (int t = wid; t < ntile; t += nw) {
            // the weights' address depends on t by a term that is zero at run
            // time but not provably so (t is bounded by the launch, K is not),
            // so their loads stay inside the loop instead of being hoisted in
            // front of it and held in registers across it
            const int zero = (t * K) >> 30;
            const PackedW wts{reinterpret_cast<const Packed*>(reinterpret_cast<const char*>(g.netw) + zero)};
            unsigned char* tslot = nreg + static_cast<size_t>(t) * NET_LDS;
            const unsigned short* sX = reinterpret_cast<const unsigned short*>(tslot);
            float* sD = reinterpret_cast<float*>(tslot);
            float* sY = sD + 16 * MAX_IN;
            bf4 xb[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) xb[s] = *reinterpret_cast<const bf4*>(&sX[r * MAX_IN + 16 * s + 4 * gq]);
            wave_sync();   // the input tile is read before the gradients overwrite it
            f4 z1[4], z2[4], dx[4];
            bf4 h1b[4];
            layers(wts, xb, r, gq, z1, h1b, z2);
            const float y = output(wts, z2, gq);
            input_grad(wts, z1, z2, r, gq, dx);
            if (gq == 0) sY[r] = y;
            // all 64 gradient columns, without branches: the packed isg is
            // zero beyond n_in, and those columns are not read
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const f4 sg = *reinterpret_cast<const f4*>(&wts.p->isg[16 * s + 4 * gq]);
                f4 v;
#pragma unroll
                for (int i = 0; i < 4; ++i) v[i] = dx[s][i] * sg[i];
                *reinterpret_cast<f4*>(&sD[r * MAX_IN + 16 * s + 4 * gq]) = v;
            }
            wave_sync();
        }
        __syncthreads();
        if (act) {
            if (has2) eff2 += static_cast<T>(drow[m]);
            if (has3) {
#pragma unroll
                for (int n = 0; n <= PA; ++n)
                    if (n <= P3) eff3[n] += static_cast<T>(drow[off3 - 1 + m * (P3 + 1) + n]);
            }
            if (q == 0) e += static_cast<double>(*yrow);
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
    constexpr bool AB_LDS = NA > 60 || MODE == 2;
    T ab[AB_LDS ? 1 : NA];
    if constexpr (MODE == 2) {
        // the row waits in its LDS slot; the surrogate's model has no 4-body
        // descriptors (the entry point requires K4 = 0), so eq. (26c) is all
        if (act && g.want_back) {
            T* abrow = sT + al * AST + m * NA;
#pragma unroll
            for (int mu = 0; mu < NA; ++mu)
                abrow[mu] = T(2 * mt.mult[mu]) * eff3[mt.deg[mu]] * abrow[mu] + (mu == 0 ? eff2 : T(0));
        }
    } else if constexpr (AB_LDS) {
        if (act) {
            T* abrow = sT + al * AST + m * NA;
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
        wave_sync();
        double ei = 0.0;
        if (act && q == 0) {
            for (int k = 0; k < K; ++k) ei += sE[al * K + k];
            if (g.E_atom) g.E_atom[atom] = static_cast<T>(ei);
        }
        wave_sync();
        const double eb = wave_sum(ei);
        if (lane == 0 && grp_live) g.part[grp] = eb;
    }
    if (!g.want_back) return;

    // ---------------- adjoint rows to memory ----------------
    // rows dE_i/dB_{i k .} of the workgroup's atoms, [atom][k][mu] (K * NA
    // values per atom, contiguous over the workgroup's atoms): staged in LDS
    // (the round staging area is free) and copied out coalesced
    T* sAb = sT;
    if constexpr (!AB_LDS) {
        if (act) {
#pragma unroll
            for (int mu = 0; mu < NA; ++mu) sAb[al * AST + m * NA + mu] = ab[mu];
        }
    }
    wave_sync();
    {
        const int a0 = grp * apw;
        const int na = (g.N - a0 < apw) ? g.N - a0 : apw;
        const int nv = na * AST;
        T* dst = g.abar + static_cast<size_t>(a0) * AST;
        for (int idx = lane; idx < nv; idx += WAVE) dst[idx] = sAb[idx];
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

// The surrogate instances (mode 2) run up to four wavefronts per workgroup,
// held to WPE wavefronts per SIMD: three in FP32 (which their LDS allows
// anyway), two in FP64 up to angular degree 4, as the mode-1 instances.
template <typename T, int PA, bool FAST, int WPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void atom_net_kernel(KArgs<T> g) {
    atom_body<T, PA, 2, FAST>(g);
}

// ---------------------------------------------------------------------------
// Pair kernel: g_ij = dE_i/dr_ij for one pair per lane (eq. (24c)).
//
// Block w (one 64-lane wavefront) takes pairs 64 w .. 64 w + 63 of the list.
// The centre atom of every pair was written by the atom kernel.  The adjoint
// rows of the block's atoms, K * NA values per atom, are copied from memory
// into LDS (the loads for the first pair_acap atoms are issued before the
// radial functions are evaluated; a block whose pairs span more atoms takes
// the rest in further chunks).  Each lane re-evaluates the radial functions
// with their derivatives and contracts the monomials of its pair with the K
// rows of its centre atom.
//
// Outputs: on the gather path g is stored at the pair's own slot p and at
// its reverse slot rev(p), and the finalize kernel forms each atom's force
// from its own list range in a fixed order; without a reverse index, g is
// added to an FP64 accumulator with atomics.  The virial leaves as one
// partial per block.
template <typename T>
struct PArgs {
    ParamsT<T> prm;    // by value: read with scalar loads
    int N, P;
    const T* pos;
    CellT<T> cell;
    const int* offsets;
    const int* nbr_j;
    const int* shift;
    const int* rev;          // reverse-pair index (gather path) or null
    const T* abar;           // adjoint rows [N][K][NA]
    const int* centre;       // centre atom of every pair (written by the atom kernel)
    const T* pdv;            // pair vectors r_ij, zero for a listed pair that is not a neighbour (same)
    T* gbuf;                 // gather: g_ij stored at slot rev(p) (3P)
    T* gown;                 // gather: g_ij stored at slot p (3P)
    double* Facc;            // scatter: FP64 accumulator (3N, zero on entry)
    double* wpart;           // virial partials, column-major [9][nblk]
    int want_W;
    int gate;                // always 1 (see pair_gradient_blocks)
    int* err;
};

// Pairs per pair-kernel block: one per lane.
constexpr int PAIR_BLOCK = WAVE;

// Atoms whose adjoint rows one pair block holds in LDS at a time (at most
// 8 KB; 64 pairs of atoms with 21 or more pairs each span at most 5 atoms).
__host__ __device__ constexpr int pair_acap(int K, int NA, int tsize) {
    const int per = abar_stride(K, NA, tsize) * tsize;
    const int a = 8192 / per;
    return a < 1 ? 1 : (a > 8 ? 8 : a);
}

__host__ __device__ inline size_t pair_lds_bytes(int K, int NA, size_t tsize) {
    const int t = static_cast<int>(tsize);
    return static_cast<size_t>(pair_acap(K, NA, t)) * abar_stride(K, NA, t) * tsize;
}

// dE_i/dr_ij of one pair for a radial count KK fixed at compile time
// (eq. (24c)): W1_mu = sum_k Abar_{k mu} R'_k, W2_mu = sum_k Abar_{k mu} R_k,
// then g = (sum_mu W1_mu A_mu - sum_n n H_n / r) rhat + (1/r) sum_mu W2_mu
// grad A_mu with H_n = sum_{deg mu = n} W2_mu A_mu and the gradient sums
// grouped by the exponent being lowered.
//
// Each monomial is contracted in a basic block of its own, entered under
// `gate`, a kernel argument that is always 1 but unknown to the compiler:
// with all monomials in one block the code generator issues the K * NA LDS
// reads of the adjoint rows ahead of the arithmetic and runs out of
// registers (FP64: 256 VGPRs + 256 AGPRs and scratch, against 180 VGPRs).
template <typename T, int PA, int KK>
__device__ __forceinline__ void pair_gradient_blocks(const T* __restrict__ abr, const T (&R)[FAST_MAX_K],
                                                     const T (&dR)[FAST_MAX_K], T ri, T ux, T uy, T uz, int gate,
                                                     T& gx, T& gy, T& gz) {
    constexpr MonoTable<PA> mt{};
    constexpr int NA = n_mono(PA);
    constexpr int NAP = NA;    // rows of one atom are contiguous
    T A[NA];           // monomials, formed in the block that contracts them
    T s1 = 0, eul = 0, g0 = 0, g1 = 0, g2 = 0;
    T buf[2][KK];      // the K values of monomial mu in buf[mu & 1]; mu + 1 read ahead
#pragma unroll
    for (int k = 0; k < KK; ++k) buf[0][k] = abr[k * NAP];
#pragma unroll
    for (int mu = 0; mu < NA; ++mu) {
        if (gate) {
            const int cb = mu & 1;
            if (mu + 1 < NA) {
#pragma unroll
                for (int k = 0; k < KK; ++k) buf[cb ^ 1][k] = abr[k * NAP + mu + 1];
            }
            if (mu == 0) {
                A[0] = T(1);
            } else {
                const T u = mt.axis[mu] == 0 ? ux : (mt.axis[mu] == 1 ? uy : uz);
                A[mu] = A[mt.par[mu]] * u;
            }
            T w1 = 0, w2 = 0;
#pragma unroll
            for (int k = 0; k < KK; ++k) {
                w1 += buf[cb][k] * dR[k];
                w2 += buf[cb][k] * R[k];
            }
            s1 += w1 * A[mu];
            // Euler sum n H_n and the gradient sums, each term weighted by its exponent
            const int dg = mt.deg[mu];
            if (dg == 1) eul += w2 * A[mu];
            else if (dg > 1) eul += (T(dg) * w2) * A[mu];
            T* gd[3] = {&g0, &g1, &g2};
#pragma unroll
            for (int dd = 0; dd < 3; ++dd) {
                if (mt.down[mu][dd] >= 0) {
                    const int e = mt.ex[mu][dd];
                    *gd[dd] += (e == 1 ? w2 : T(e) * w2) * A[mt.down[mu][dd]];
                }
            }
        }
    }
    const T a1 = s1 - eul * ri;
    gx = a1 * ux + ri * g0;
    gy = a1 * uy + ri * g1;
    gz = a1 * uz + ri * g2;
}

// Copy nbytes (a multiple of 16) from global memory into LDS with the
// direct global-to-LDS loads of gfx950: each lane moves 16 bytes, one
// instruction fills 1 KB of consecutive LDS.  Completion is awaited with
// lds_copy_wait.
__device__ __forceinline__ void lds_copy_issue(const void* src, void* dst, int nbytes, int lane) {
    typedef __attribute__((address_space(1))) void* gptr_t;
    typedef __attribute__((address_space(3))) void* lptr_t;
    const char* s = static_cast<const char*>(src);
    char* d = static_cast<char*>(dst);
    for (int off = 0; off < nbytes; off += 16 * WAVE) {
        if (off + 16 * lane < nbytes)
            __builtin_amdgcn_global_load_lds((gptr_t)(s + off + 16 * lane), (lptr_t)(d + off), 16, 0, 0);
    }
}

__device__ __forceinline__ void lds_copy_wait() {
    __builtin_amdgcn_s_waitcnt(0);
    wave_sync();
}

// Geometry and radial functions (with derivatives) of one pair.
template <typename T>
struct PairGeom {
    T d[3], r, ri, ux, uy, uz;
    T R[FAST_MAX_K], dR[FAST_MAX_K];
    bool ok;
};

template <typename T, int KK, bool FAST>
__device__ __forceinline__ void pair_setup(const PArgs<T>& g, bool valid, const T (&dv)[3], PairGeom<T>& q) {
    const ParamsT<T>* __restrict__ P = &g.prm;
    q.d[0] = dv[0]; q.d[1] = dv[1]; q.d[2] = dv[2];
    const T r2 = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2];
    // the atom kernel stored zero for a listed pair outside (rin, rcut)
    q.ok = valid && r2 > T(0);
    q.r = q.ok ? d_sqrt(r2) : T(0.5) * (P->rin + P->rcut);
    q.ri = T(1) / q.r;
    // Q from the parameter block (uniform addresses: scalar loads)
    radial_any<T, true, FAST, (KK > 0 ? KK : FAST_MAX_K)>(P, &P->Q[0][0], q.r, q.ri, q.R, q.dR);
    q.ux = q.d[0] * q.ri; q.uy = q.d[1] * q.ri; q.uz = q.d[2] * q.ri;
}

template <typename T, int PA, int KK>
__device__ __forceinline__ void pair_contract(const PArgs<T>& g, int K, const PairGeom<T>& q, const T* abr, T& gx,
                                              T& gy, T& gz) {
    constexpr MonoTable<PA> mt{};
    constexpr int NA = n_mono(PA);
    if constexpr (KK > 0) {
        pair_gradient_blocks<T, PA, KK>(abr, q.R, q.dR, q.ri, q.ux, q.uy, q.uz, g.gate, gx, gy, gz);
    } else {
        T A[NA];
        A[0] = T(1);
#pragma unroll
        for (int mu = 1; mu < NA; ++mu) {
            const T u = mt.axis[mu] == 0 ? q.ux : (mt.axis[mu] == 1 ? q.uy : q.uz);
            A[mu] = A[mt.par[mu]] * u;
        }
        pair_gradient_any<T, PA>(abr, K, A, q.R, q.dR, q.ri, q.ux, q.uy, q.uz, gx, gy, gz);
    }
}

// g_ij of pair p: stored at the pair's own slot and at its reverse slot (the
// finalize kernel gathers F_n = sum over n's slots of own - reverse), or
// added to both atoms with atomics.
template <typename T>
__device__ __forceinline__ void pair_store(const PArgs<T>& g, int p, int ci, int j, int rv, bool ok, T gx, T gy,
                                           T gz) {
    if (g.gbuf) {
        T* go = g.gown + 3 * static_cast<size_t>(p);
        go[0] = gx; go[1] = gy; go[2] = gz;
        if (rv >= 0 && rv < g.P) {
            T* gp3 = g.gbuf + 3 * static_cast<size_t>(rv);
            gp3[0] = gx; gp3[1] = gy; gp3[2] = gz;
        } else {
            atomicOr(g.err, ERR_NEIGH);
        }
    } else if (ok) {
        atomicAdd(&g.Facc[3 * j + 0], -static_cast<double>(gx));
        atomicAdd(&g.Facc[3 * j + 1], -static_cast<double>(gy));
        atomicAdd(&g.Facc[3 * j + 2], -static_cast<double>(gz));
        atomicAdd(&g.Facc[3 * ci + 0], static_cast<double>(gx));
        atomicAdd(&g.Facc[3 * ci + 1], static_cast<double>(gy));
        atomicAdd(&g.Facc[3 * ci + 2], static_cast<double>(gz));
    }
}

// One block of 64 consecutive pairs, one pair per lane.  The rows of the
// first acap atoms from the block's first centre atom are loaded into LDS
// while the radial functions are evaluated; a block whose pairs span more
// atoms takes the others in further chunks.  The virial of the lane's pair
// is added to vir.
template <typename T, int PA, int KK, bool FAST>
__device__ __forceinline__ void pair_block(const PArgs<T>& g, int blk, T* sAb, double (&vir)[9]) {
    constexpr int NA = n_mono(PA);
    const ParamsT<T>* __restrict__ P = &g.prm;
    const int K = KK > 0 ? KK : P->K;
    const int AST = abar_stride(K, NA, sizeof(T));
    const int acap = pair_acap(K, NA, sizeof(T));
    const int lane = threadIdx.x;
    const int p = blk * WAVE + lane;
    const bool valid = p < g.P;
    // everything the pair needs, requested at once: centre atom, pair vector,
    // reverse slot (gather path) or neighbour index (atomic path)
    // (issued on every lane: a lane past the end reads the last pair)
    const int pc = valid ? p : g.P - 1;
    int ci = g.centre[pc], rv = -1, j = -1;
    T dv[3] = {g.pdv[3 * static_cast<size_t>(pc) + 0], g.pdv[3 * static_cast<size_t>(pc) + 1],
               g.pdv[3 * static_cast<size_t>(pc) + 2]};
    if (g.gbuf) rv = g.rev[pc];
    else j = g.nbr_j[pc];
    int lo = g.centre[blk * WAVE];
    lo = lo < 0 ? 0 : (lo > g.N - 1 ? g.N - 1 : lo);
    const int na0 = (g.N - lo < acap) ? g.N - lo : acap;
    wave_sync();   // rows of a previous block are no longer read
    lds_copy_issue(g.abar + static_cast<size_t>(lo) * AST, sAb, na0 * AST * static_cast<int>(sizeof(T)), lane);
    ci = ci < 0 ? 0 : (ci > g.N - 1 ? g.N - 1 : ci);
    if (!g.gbuf && (j < 0 || j >= g.N)) j = ci;   // malformed list: reported by the atom kernel

    PairGeom<T> q;
    pair_setup<T, KK, FAST>(g, valid, dv, q);
    T gx = T(0), gy = T(0), gz = T(0);
    lds_copy_wait();
    if (q.ok && ci >= lo && ci < lo + na0)
        pair_contract<T, PA, KK>(g, K, q, sAb + static_cast<size_t>(ci - lo) * AST, gx, gy, gz);
    // further chunks, skipping atoms without pairs in this block
    constexpr int INF = 0x7fffffff;
    const int key = valid ? ci : INF;
    int base = wave_min(key >= lo + na0 ? key : INF);
    while (base != INF) {
        const int na = (g.N - base < acap) ? g.N - base : acap;
        wave_sync();
        lds_copy_issue(g.abar + static_cast<size_t>(base) * AST, sAb, na * AST * static_cast<int>(sizeof(T)), lane);
        lds_copy_wait();
        if (q.ok && ci >= base && ci < base + na)
            pair_contract<T, PA, KK>(g, K, q, sAb + static_cast<size_t>(ci - base) * AST, gx, gy, gz);
        base = wave_min(key >= base + na ? key : INF);
    }
    if (valid) pair_store<T>(g, p, ci, j, rv, q.ok, gx, gy, gz);
    if (q.ok) {
        const double dd[3] = {double(q.d[0]), double(q.d[1]), double(q.d[2])};
        const double gg[3] = {double(gx), double(gy), double(gz)};
#pragma unroll
        for (int x = 0; x < 3; ++x)
#pragma unroll
            for (int y = 0; y < 3; ++y) vir[3 * x + y] -= dd[x] * gg[y];
    }
}

// Workgroups are dealt to the eight XCDs of the chip in turn (workgroup i
// runs on XCD i mod 8).  The pair blocks are renumbered so that each XCD
// takes one contiguous range of them: neighbouring blocks share centre
// atoms, whose adjoint rows are then fetched once into that XCD's L2.
__device__ __forceinline__ int xcd_block(int i, int n) {
    constexpr int NX = 8;
    const int x = i % NX, k = i / NX;
    const int per = n / NX, rem = n % NX;
    return x * per + (x < rem ? x : rem) + k;
}

// KK: the radial count when fixed at compile time (4 or 6), 0 for any K.
// Wavefront w takes pairs 64 w .. 64 w + 63.
template <typename T, int PA, int KK, bool FAST>
__device__ __forceinline__ void pair_body(const PArgs<T>& g) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sAb = reinterpret_cast<T*>(smem_raw);
    const int lane = threadIdx.x;
    const int nblk = gridDim.x;
    const int w = xcd_block(blockIdx.x, nblk);
    double vir[9];
#pragma unroll
    for (int x = 0; x < 9; ++x) vir[x] = 0.0;
    pair_block<T, PA, KK, FAST>(g, w, sAb, vir);
    if (g.want_W) {
        // W_ab -= r_ij,a g_ij,b, summed over the wavefront's pairs
        int c;
        const double sw = wave_sum9(vir, lane, c);
        if (c < 9) g.wpart[static_cast<size_t>(c) * nblk + w] = sw;
    }
}

template <typename T, int PA, int KK, bool FAST>
__global__ __launch_bounds__(64) void pair_kernel(PArgs<T> g) {
    pair_body<T, PA, KK, FAST>(g);
}

// Totals and forces.  Blocks 0 .. 9 + M: column sums of the block partials
// in a fixed order (column 0 -> E and 10.. -> G from the atom kernel's
// blocks, 1..9 -> W from the pair kernel's blocks).  Remaining blocks, with
// a reverse index: F_n = sum over the slots p of n of gown[p] - gbuf[p],
// where gown[p] holds g of pair p and gbuf[p] g of its reverse (8 atoms x 32
// lanes per block, deterministic); without one: F = Facc (accumulated with
// atomics) and Facc cleared for the next call.
template <typename T>
struct FinArgs {
    const double* part;    // atom-kernel partials [10 + M][nblk]
    int nblk, ncol;
    const double* wpart;   // pair-kernel virial partials [9][nblk_p]
    int nblk_p;
    double* E;
    double* W;
    double* G;
    double* Facc;
    T* F;
    long n3;
    const T* gbuf;         // gather path: g stored at reverse slots
    const T* gown;         // gather path: g stored at own slots
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
                    // slot p of atom a: g of pair p (a -> j) and g of its reverse (j -> a)
                    for (int p = b + s0; p < e; p += 32) {
                        const size_t o = 3 * static_cast<size_t>(p);
                        f0 += static_cast<double>(f.gown[o + 0]) - static_cast<double>(f.gbuf[o + 0]);
                        f1 += static_cast<double>(f.gown[o + 1]) - static_cast<double>(f.gbuf[o + 1]);
                        f2 += static_cast<double>(f.gown[o + 2]) - static_cast<double>(f.gbuf[o + 2]);
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
                f.F[3 * a + 0] = static_cast<T>(f0);
                f.F[3 * a + 1] = static_cast<T>(f1);
                f.F[3 * a + 2] = static_cast<T>(f2);
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
    double* E = f.E;
    double* W = f.W;
    double* G = f.G;
    if ((col == 0 && !E) || (col >= 1 && col < 10 && !W) || (col >= 10 && !G)) return;
    const bool wcol = col >= 1 && col < 10;
    const int nb = wcol ? f.nblk_p : f.nblk;
    const double* src = wcol ? f.wpart + static_cast<size_t>(col - 1) * nb : f.part + static_cast<size_t>(col) * nb;
    // every thread adds b = t, t + 256, ... in order; eight loads in flight
    double s = 0.0;
    int b = threadIdx.x;
    for (; b + 7 * 256 < nb; b += 8 * 256) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = src[b + u * 256];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; b < nb; b += 256) s += src[b];
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
hipError_t launch_atom(const KArgs<T>& a, bool fast, int nblk, int nthr, size_t lds, hipStream_t st) {
    constexpr bool occ2 = sizeof(T) == 8 && PA <= 4;
    if constexpr (MODE == 2) {
        constexpr int WPE = sizeof(T) == 4 ? 3 : (occ2 ? 2 : 1);
        if (fast) hipLaunchKernelGGL((atom_net_kernel<T, PA, true, WPE>), dim3(nblk), dim3(nthr), lds, st, a);
        else hipLaunchKernelGGL((atom_net_kernel<T, PA, false, WPE>), dim3(nblk), dim3(nthr), lds, st, a);
    } else if constexpr (occ2) {
        if (fast) hipLaunchKernelGGL((atom_kernel_occ2<T, PA, MODE, true>), dim3(nblk), dim3(WAVE), lds, st, a);
        else hipLaunchKernelGGL((atom_kernel_occ2<T, PA, MODE, false>), dim3(nblk), dim3(WAVE), lds, st, a);
    } else {
        if (fast) hipLaunchKernelGGL((atom_kernel<T, PA, MODE, true>), dim3(nblk), dim3(WAVE), lds, st, a);
        else hipLaunchKernelGGL((atom_kernel<T, PA, MODE, false>), dim3(nblk), dim3(WAVE), lds, st, a);
    }
    return hipGetLastError();
}

template <typename T, int MODE>
hipError_t dispatch_pa(int PA, const KArgs<T>& a, bool fast, int nblk, int nthr, size_t lds, hipStream_t st) {
    switch (PA) {
        case 0: return launch_atom<T, 0, MODE>(a, fast, nblk, nthr, lds, st);
        case 1: return launch_atom<T, 1, MODE>(a, fast, nblk, nthr, lds, st);
        case 2: return launch_atom<T, 2, MODE>(a, fast, nblk, nthr, lds, st);
        case 3: return launch_atom<T, 3, MODE>(a, fast, nblk, nthr, lds, st);
        case 4: return launch_atom<T, 4, MODE>(a, fast, nblk, nthr, lds, st);
        case 5: return launch_atom<T, 5, MODE>(a, fast, nblk, nthr, lds, st);
        case 6: return launch_atom<T, 6, MODE>(a, fast, nblk, nthr, lds, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int PA, int KK>
void launch_pair_k(const PArgs<T>& a, bool fast, int nblk, size_t lds, hipStream_t st) {
    if (fast) hipLaunchKernelGGL((pair_kernel<T, PA, KK, true>), dim3(nblk), dim3(WAVE), lds, st, a);
    else hipLaunchKernelGGL((pair_kernel<T, PA, KK, false>), dim3(nblk), dim3(WAVE), lds, st, a);
}

template <typename T, int PA>
hipError_t launch_pair(const PArgs<T>& a, bool fast, int nblk, size_t lds, hipStream_t st) {
    const int K = a.prm.K;
    if (K == 6) launch_pair_k<T, PA, 6>(a, fast, nblk, lds, st);
    else if (K == 4) launch_pair_k<T, PA, 4>(a, fast, nblk, lds, st);
    else launch_pair_k<T, PA, 0>(a, fast, nblk, lds, st);
    return hipGetLastError();
}

template <typename T>
hipError_t dispatch_pair(int PA, const PArgs<T>& a, bool fast, int nblk, size_t lds, hipStream_t st) {
    switch (PA) {
        case 0: return launch_pair<T, 0>(a, fast, nblk, lds, st);
        case 1: return launch_pair<T, 1>(a, fast, nblk, lds, st);
        case 2: return launch_pair<T, 2>(a, fast, nblk, lds, st);
        case 3: return launch_pair<T, 3>(a, fast, nblk, lds, st);
        case 4: return launch_pair<T, 4>(a, fast, nblk, lds, st);
        case 5: return launch_pair<T, 5>(a, fast, nblk, lds, st);
        case 6: return launch_pair<T, 6>(a, fast, nblk, lds, st);
        default: return hipErrorInvalidValue;
    }
}

// LDS of one wavefront of the per-atom kernel
size_t lds_bytes(int K, int PA, size_t tsize, int M) {
    return atom_lds_layout(K, n_mono(PA), M, tsize, n_partitions(PA), PA).total;
}

// Wavefronts per workgroup of the mode-2 kernel: of 1 to 4, the count with
// the fewest network tiles per wavefront whose LDS (per_wave each, plus the
// tiles) fits 64 KB and allows at least as many wavefronts per compute unit
// (160 KB of LDS) as one wavefront per workgroup.
int net_waves(int K, size_t per_wave) {
    const int apw = WAVE / K;
    const auto bytes = [&](int w) { return w * per_wave + net_tiles(w, apw) * NET_LDS; };
    const auto waves_per_cu = [&](int w) { return static_cast<int>(163840 / bytes(w)) * w; };
    int best = 1;
    for (int w = 2; w <= 4; ++w) {
        if (bytes(w) > 65536 || waves_per_cu(w) < waves_per_cu(1)) continue;
        if (net_tiles(w, apw) * best < net_tiles(best, apw) * w) best = w;
    }
    return best;
}

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
    a.coef = nullptr; a.D = nullptr; a.E_atom = nullptr; a.abar = nullptr; a.centre = nullptr; a.pdv = nullptr; a.part = nullptr;
    a.want_G = 0; a.want_back = 0;
    a.netw = nullptr; a.n_net = 0;
    a.err = h->d_err;
    return POD_OK;
}

// Arguments of the wide-degree kernel from those of the per-atom kernel.
template <typename T>
WideArgs<T> wide_args(const KArgs<T>& a) {
    WideArgs<T> w;
    w.prm = a.prm; w.cell = a.cell;
    w.N = a.N; w.P = a.P;
    w.pos = a.pos; w.offsets = a.offsets; w.nbr_j = a.nbr_j; w.shift = a.shift;
    w.coef = a.coef; w.D = a.D; w.E_atom = a.E_atom;
    w.part = a.part; w.wpart = nullptr;
    w.gown = nullptr; w.gbuf = nullptr; w.rev = nullptr; w.Facc = nullptr;
    w.rec = nullptr; w.rs = 0;
    w.want_G = a.want_G; w.want_back = a.want_back; w.want_W = 0;
    w.err = a.err;
    return w;
}

template <typename T>
int descriptors_impl(pod_handle* h, int N, int P, const void* pos, const double* cell, const int* offsets,
                     const int* nbr_j, const int* shift, void* D) {
    if (N == 0) return POD_OK;
    KArgs<T> a;
    const int rc = fill_args<T>(h, a, N, P, pos, cell, offsets, nbr_j, shift);
    if (rc != POD_OK) return rc;
    a.D = static_cast<T*>(D);
    if (wide_path(h->K, h->PA)) {
        WideArgs<T> w = wide_args(a);
        w.rs = wide_rec_stride(h->K, false);
        const int rc2 = ensure_scratch(h, static_cast<size_t>(P > 0 ? P : 1) * w.rs * sizeof(T));
        if (rc2 != POD_OK) return rc2;
        w.rec = static_cast<T*>(h->d_scratch);
        timing_begin(h, 1);
        const hipError_t e = launch_wide<T>(w, 0, h->std_ok != 0, wide_blocks(N), h->stream);
        timing_end(h, 1);
        return e == hipSuccess ? POD_OK : POD_EHIP;
    }
    const int apw = WAVE / h->K;
    const int nblk = (N + apw - 1) / apw;
    timing_begin(h, 1);
    const hipError_t e = dispatch_pa<T, 0>(h->PA, a, h->std_ok != 0, nblk, WAVE, lds_bytes(h->K, h->PA, sizeof(T), h->M),
                                           h->stream);
    timing_end(h, 1);
    return e == hipSuccess ? POD_OK : POD_EHIP;
}

// Scratch of one energy call, carved from one device buffer (256-byte
// aligned pieces): atom-kernel partials [10 + M][nblk], pair-kernel virial
// partials [9][nblk_p], adjoint rows [N][K][NA] (per-atom stride padded to
// 16 bytes), centre atom and pair vector of each pair, on the gather path
// the pair gradients [P][3] at reverse and at own slots, and for the
// wide-degree kernel (no adjoint rows, centres or pair vectors) the pair
// records [P][4 + 2K].
struct EfScratch {
    size_t part, wpart, abar, centre, pdv, gbuf, gown, rec, total;
};

EfScratch ef_scratch_layout(int N, int P, int K, int PA, int M, size_t tsize, bool back, bool gather) {
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    const bool wide = wide_path(K, PA);   // one kernel, partials per persistent workgroup
    const int apw = WAVE / K;
    const size_t nblk = N <= 0 ? 0 : wide ? static_cast<size_t>(wide_blocks(N)) : (static_cast<size_t>(N) + apw - 1) / apw;
    const size_t nblk_p = !back ? 0 : wide ? nblk : (static_cast<size_t>(P) + PAIR_BLOCK - 1) / PAIR_BLOCK;
    EfScratch L;
    size_t o = 0;
    L.part = o; o += al(static_cast<size_t>(10 + M) * (nblk > 0 ? nblk : 1) * sizeof(double));
    L.wpart = o; o += al(9 * (nblk_p > 0 ? nblk_p : 1) * sizeof(double));
    L.abar = o;
    o += (back && !wide) ? al(static_cast<size_t>(N) * abar_stride(K, n_mono(PA), static_cast<int>(tsize)) * tsize) : 0;
    L.centre = o; o += wide ? 0 : al((static_cast<size_t>(P) + 1) * sizeof(int));   // entry P: spare for empty slots
    L.pdv = o; o += wide ? 0 : al((static_cast<size_t>(P) + 1) * 3 * tsize);
    L.gbuf = o; o += gather ? al(static_cast<size_t>(P > 0 ? P : 1) * 3 * tsize) : 0;
    L.gown = o; o += gather ? al(static_cast<size_t>(P > 0 ? P : 1) * 3 * tsize) : 0;
    L.rec = o; o += wide ? al(static_cast<size_t>(P > 0 ? P : 1) * wide_rec_stride(K, true) * tsize) : 0;
    L.total = o;
    return L;
}

// The energy path on a given scratch buffer (at least the layout's total)
// and, for the atomic force path, a zeroed FP64 accumulator of 3 N doubles.
template <typename T, int MODE = 1>
int energy_forces_run(pod_handle* h, char* scratch, double* facc, int N, int P, const void* pos, const double* cell,
                      const int* offsets, const int* nbr_j, const int* shift, const int* rev, const void* c,
                      void* E_atom, double* E, void* F, double* W, double* G,
                      const net::Packed* netw = nullptr, int n_net = 0) {
    KArgs<T> a;
    int rc = fill_args<T>(h, a, N, P, pos, cell, offsets, nbr_j, shift);
    if (rc != POD_OK) return rc;
    const int apw = WAVE / h->K;
    const int nblk = (N + apw - 1) / apw;
    const int ncol = 10 + h->M;
    const bool back = (F != nullptr) || (W != nullptr);
    const bool gather = rev != nullptr && F != nullptr;
    const int nblk_p = back ? (P + PAIR_BLOCK - 1) / PAIR_BLOCK : 0;
    const EfScratch L = ef_scratch_layout(N, P, h->K, h->PA, h->M, sizeof(T), back, gather);
    a.coef = static_cast<const T*>(c);
    a.E_atom = static_cast<T*>(E_atom);
    a.part = reinterpret_cast<double*>(scratch + L.part);
    a.abar = back ? reinterpret_cast<T*>(scratch + L.abar) : nullptr;
    a.centre = reinterpret_cast<int*>(scratch + L.centre);
    a.pdv = reinterpret_cast<T*>(scratch + L.pdv);
    a.want_G = G != nullptr;
    a.want_back = back;
    a.netw = netw; a.n_net = n_net;
    if (wide_path(h->K, h->PA)) {
        if constexpr (MODE != 1) return POD_ENOTSUP;
        // wide-degree kernel: energy, G and pair gradients in one launch
        WideArgs<T> w = wide_args(a);
        const int nblk_w = wide_blocks(N);
        w.wpart = reinterpret_cast<double*>(scratch + L.wpart);
        w.gbuf = gather ? reinterpret_cast<T*>(scratch + L.gbuf) : nullptr;
        w.gown = gather ? reinterpret_cast<T*>(scratch + L.gown) : nullptr;
        w.rev = gather ? rev : nullptr;
        w.Facc = (back && !gather) ? facc : nullptr;
        w.rec = reinterpret_cast<T*>(scratch + L.rec);
        w.rs = wide_rec_stride(h->K, true);
        w.want_W = W != nullptr;
        timing_begin(h, 1);
        const hipError_t e = launch_wide<T>(w, 1, h->std_ok != 0, nblk_w, h->stream);
        timing_end(h, 1);
        if (e != hipSuccess) return POD_EHIP;
        FinArgs<T> fa;
        fa.part = a.part;
        fa.nblk = nblk_w; fa.ncol = ncol;
        fa.wpart = w.wpart; fa.nblk_p = back ? nblk_w : 0;
        fa.E = E; fa.W = back ? W : nullptr; fa.G = G;
        fa.Facc = facc; fa.F = static_cast<T*>(F);
        fa.n3 = (back && !gather) ? 3L * N : 0L;
        fa.gbuf = w.gbuf; fa.gown = w.gown; fa.rev = gather ? rev : nullptr; fa.offsets = offsets;
        fa.N = N; fa.P = P; fa.err = h->d_err;
        const int nfb = gather ? (N + 7) / 8 : static_cast<int>((fa.n3 + 255) / 256);
        if (E || W || G || nfb > 0) {
            timing_begin(h, 0);
            hipLaunchKernelGGL((finalize_kernel<T>), dim3(ncol + nfb), dim3(256), 0, h->stream, fa);
            timing_end(h, 0);
            if (hipGetLastError() != hipSuccess) return POD_EHIP;
        }
        return POD_OK;
    }
    if (nblk > 0) {
        const size_t pw = lds_bytes(h->K, h->PA, sizeof(T), h->M);
        const int nw = MODE == 2 ? net_waves(h->K, pw) : 1;
        const size_t lds = nw * pw + (MODE == 2 ? net_tiles(nw, apw) * NET_LDS : 0);
        timing_begin(h, 1);
        const hipError_t e = dispatch_pa<T, MODE>(h->PA, a, h->std_ok != 0, (nblk + nw - 1) / nw, nw * WAVE, lds,
                                               h->stream);
        timing_end(h, 1);
        if (e != hipSuccess) return POD_EHIP;
    }
    PArgs<T> b;
    b.prm = a.prm; b.N = N; b.P = P; b.pos = a.pos; b.cell = a.cell;
    b.offsets = offsets; b.nbr_j = nbr_j; b.shift = shift;
    b.rev = gather ? rev : nullptr;
    b.abar = a.abar; b.centre = a.centre; b.pdv = a.pdv;
    b.gbuf = gather ? reinterpret_cast<T*>(scratch + L.gbuf) : nullptr;
    b.gown = gather ? reinterpret_cast<T*>(scratch + L.gown) : nullptr;
    b.Facc = facc;
    b.wpart = reinterpret_cast<double*>(scratch + L.wpart);
    b.want_W = W != nullptr;
    b.gate = 1;
    b.err = h->d_err;
    if (nblk_p > 0) {
        timing_begin(h, 4);
        const hipError_t e = dispatch_pair<T>(h->PA, b, h->std_ok != 0, nblk_p,
                                              pair_lds_bytes(h->K, n_mono(h->PA), sizeof(T)), h->stream);
        timing_end(h, 4);
        if (e != hipSuccess) return POD_EHIP;
    }
    // totals, and the forces: gathered from the per-pair gradients, or copied
    // out of the atomic accumulator (which is re-zeroed)
    FinArgs<T> fa;
    fa.part = a.part;
    fa.nblk = nblk; fa.ncol = ncol;
    fa.wpart = b.wpart; fa.nblk_p = nblk_p;
    fa.E = E; fa.W = back ? W : nullptr; fa.G = G;
    fa.Facc = facc; fa.F = static_cast<T*>(F);
    fa.n3 = (back && !gather) ? 3L * N : 0L;
    fa.gbuf = b.gbuf; fa.gown = b.gown; fa.rev = gather ? rev : nullptr; fa.offsets = offsets;
    fa.N = N; fa.P = P; fa.err = h->d_err;
    const int nfb = gather ? (N + 7) / 8 : static_cast<int>((fa.n3 + 255) / 256);
    if (E || W || G || nfb > 0) {
        timing_begin(h, 0);
        hipLaunchKernelGGL((finalize_kernel<T>), dim3(ncol + nfb), dim3(256), 0, h->stream, fa);
        timing_end(h, 0);
        if (hipGetLastError() != hipSuccess) return POD_EHIP;
    }
    return POD_OK;
}

template <typename T, int MODE = 1>
int energy_forces_impl(pod_handle* h, int N, int P, const void* pos, const double* cell, const int* offsets,
                       const int* nbr_j, const int* shift, const int* rev, const void* c, void* E_atom, double* E,
                       void* F, double* W, double* G, const net::Packed* netw = nullptr,
                       int n_net = 0) {
    const bool back = (F != nullptr) || (W != nullptr);
    const bool gather = rev != nullptr && F != nullptr;
    const EfScratch L = ef_scratch_layout(N, P, h->K, h->PA, h->M, sizeof(T), back, gather);
    int rc = ensure_scratch(h, L.total);
    if (rc != POD_OK) return rc;
    rc = ensure_force_acc(h, N);
    if (rc != POD_OK) return rc;
    rc = energy_forces_run<T, MODE>(h, static_cast<char*>(h->d_scratch), h->d_facc, N, P, pos, cell, offsets, nbr_j,
                                    shift, rev, c, E_atom, E, F, W, G, netw, n_net);
    if (rc == POD_EHIP && back && !gather) h->facc_dirty = 1;
    return rc;
}

// Network surrogate of the 4-body term: the weights packed once (one small
// kernel), then the per-atom kernel in mode 2 runs the network on its own
// 2/3-body descriptors and takes the energy and the adjoint weights
// c + dy/dD_i from it; pair and finalize kernels as for the linear model.
template <typename T>
int surrogate_impl(pod_handle* h, int N, int P, const void* pos, const double* cell, const int* offsets,
                   const int* nbr_j, const int* shift, const int* rev, const void* c, const float* theta,
                   const float* mu, const float* isg, void* E_atom, double* E, void* F, double* W) {
    const int n_in = h->M - 1;
    net::Packed* pk = nullptr;
    if (N > 0) {
        const int rc = ensure_mscratch(h, sizeof(net::Packed));
        if (rc != POD_OK) return rc;
        pk = static_cast<net::Packed*>(h->d_mscratch);
        const int rc2 = mlp_pack_launch(h, n_in, theta, mu, isg, pk);
        if (rc2 != POD_OK) return rc2;
    }
    return energy_forces_impl<T, 2>(h, N, P, pos, cell, offsets, nbr_j, shift, rev, c, E_atom, E, F, W, nullptr,
                                    pk, n_in);
}

__global__ __launch_bounds__(256) void zero_kernel(double* p, long n) {
    const long i = static_cast<long>(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// The energy path on the static scratch of this device: no allocation.
template <typename T>
int energy_forces_noalloc_impl(pod_handle* h, int N, int P, const void* pos, const double* cell,
                               const int* offsets, const int* nbr_j, const int* shift, const int* rev, const void* c,
                               void* E_atom, double* E, void* F, double* W, double* G) {
    const bool back = (F != nullptr) || (W != nullptr);
    const bool gather = rev != nullptr && F != nullptr;
    const EfScratch L = ef_scratch_layout(N, P, h->K, h->PA, h->M, sizeof(T), back, gather);
    const size_t facc_bytes = (back && !gather) ? ((static_cast<size_t>(N) * 3 * sizeof(double) + 255) & ~size_t(255))
                                                : 0;
    if (L.total + facc_bytes > static_cast<size_t>(POD_STATIC_SCRATCH_BYTES)) return POD_ETOOBIG;
    if (h->device < 0 || h->device >= MAX_DEVICES) return POD_EHIP;
    char* base;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        base = static_cast<char*>(g_scratch_ptr[h->device]);
    }
    if (!base) return POD_EHIP;
    double* facc = nullptr;
    if (facc_bytes > 0) {
        // the atomic force path adds into a zeroed accumulator (a fill kernel,
        // so that the call can be captured in a graph)
        facc = reinterpret_cast<double*>(base + L.total);
        const long n3 = 3L * N;
        if (n3 > 0) {
            hipLaunchKernelGGL(zero_kernel, dim3(static_cast<unsigned>((n3 + 255) / 256)), dim3(256), 0, h->stream, facc,
                               n3);
            if (hipGetLastError() != hipSuccess) return POD_EHIP;
        }
    }
    return energy_forces_run<T, 1>(h, base, facc, N, P, pos, cell, offsets, nbr_j, shift, rev, c, E_atom, E, F, W, G);
}

bool bad_common(pod_handle* h, int N, int P, const void* pos, const int* offsets, const int* nbr_j,
                const int* shift) {
    if (!h || N < 0 || P < 0) return true;
    if (N > 0 && (!pos || !offsets)) return true;
    if (P > 0 && (!nbr_j || !shift)) return true;
    return false;
}

}  // namespace

int resolve_static_scratch(int dev) {
    if (dev < 0 || dev >= MAX_DEVICES) return POD_EHIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return POD_OK;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return POD_EHIP;
    g_scratch_ptr[dev] = ptr;
    return POD_OK;
}

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

int pod_energy_forces_noalloc(pod_handle* h, int N, int P, const void* pos, const double* cell, const int* offsets,
                              const int* nbr_j, const int* shift, const int* rev, const void* c, void* E_atom,
                              double* E, void* F, double* W, double* G) {
    if (pod::bad_common(h, N, P, pos, offsets, nbr_j, shift)) return POD_EINVAL;
    if (!c) return POD_EINVAL;
    if (h->dtype == POD_F64)
        return pod::energy_forces_noalloc_impl<double>(h, N, P, pos, cell, offsets, nbr_j, shift, rev, c, E_atom, E,
                                                       F, W, G);
    return pod::energy_forces_noalloc_impl<float>(h, N, P, pos, cell, offsets, nbr_j, shift, rev, c, E_atom, E, F,
                                                  W, G);
}

int pod_energy_forces_surrogate(pod_handle* h, int N, int P, const void* pos, const double* cell,
                                const int* offsets, const int* nbr_j, const int* shift, const int* rev, const void* c,
                                const float* theta, const float* mu, const float* inv_sigma, void* E_atom, double* E,
                                void* F, double* W) {
    if (pod::bad_common(h, N, P, pos, offsets, nbr_j, shift)) return POD_EINVAL;
    if (!c || !theta || !mu || !inv_sigma) return POD_EINVAL;
    if (h->K4 != 0) return POD_EINVAL;
    if (h->M - 1 < 1 || h->M - 1 > POD_MLP_MAX_IN || pod::wide_path(h->K, h->PA)) return POD_ENOTSUP;
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
