// Batched descriptor-matrix assembly for fitting (Sec. IV.A, eqs. (58a),
// (63a)): for many small periodic cells, the per-atom descriptors D, the
// global descriptors G = sum_i D_i of each cell and their derivatives
// dG/dr_n (Sec. II.G, eqs. (26c), (24c), product rule for the 2- and 4-body
// terms), in FP64, in one persistent launch.
//
// One workgroup processes one cell at a time; cells are dealt to workgroups
// in order of decreasing pair count.  Per cell:
//   1. pair records (rhat, 1/r, R_k, R'_k) for every pair of the cell, in the
//      workgroup's scratch region (cache-resident);
//   2. forward: lanes (atom, m) accumulate the atomic-basis rows (eq. (24b)),
//      contract them (eqs. (25)-(30a)), write D, sum G in LDS, keep B;
//   3. dG/dR: for each radial index m and each chunk of at most `cw` of its
//      descriptor columns, the cell's dG/dR block [N_c][3][cw] is held in LDS.
//      Work items are (atom i, column): the lane forms the Jacobian row
//      dD_col/dB_{i m .} in registers, walks the pairs of atom i, contracts
//      the row with each pair's basis derivative (eq. (24c)) into v = dD_i/dr_ij,
//      adds +v to the LDS row of the neighbour (atomic) and keeps -v for atom
//      i in registers, added once at the end.  The chunk is then written out.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "pod.h"
#include "pod_device.h"
#include "pod_internal.h"
#include "pod_plan.h"
#include "pod_tables.h"

namespace pod {
namespace {

using namespace dev;

constexpr int MAX_THREADS = BATCH_MAX_THREADS;

struct BArgs {
    ParamsT<double> prm;  // by value: read with scalar loads
    int n_cfg;
    const int* order;     // processing order of the cells
    const int* cfg_off;   // n_cfg + 1 atom offsets
    const double* pos;
    const double* cells;  // n_cfg x 9, lattice vectors as rows
    const int* offsets;
    const int* nbr_j;
    const int* shift;
    int N, P;
    double* D;
    double* G;
    double* dGdR;
    double* scratch;      // per workgroup: rec_cap * (4 + 2K) + b_cap * K * NA doubles
    long rec_cap, b_cap;
    int cw, nc_max;
    int* err;
};

// Global column of local column lc of radial index m, laid out per m as
// [D2_m] [D3_m,0..P3] [D4_m,0..Ka4-1] (each present when m is below K2, K3, K4).
__device__ __forceinline__ int column_of(const ParamsT<double>* P, int m, int lc, int* kind, int* idx) {
    if (m < P->K2) {
        if (lc == 0) { *kind = 2; *idx = 0; return 1 + m; }
        --lc;
    }
    if (m < P->K3) {
        if (lc <= P->P3) { *kind = 3; *idx = lc; return P->off3 + m * (P->P3 + 1) + lc; }
        lc -= P->P3 + 1;
    }
    *kind = 4; *idx = lc;
    return P->off4 + m * P->Ka4 + lc;
}

// Row J_mu = dD/dB_{i m mu} of one descriptor of radial index m, from the
// atomic-basis row b = B_{i m .}.  All indices are compile-time, so b and J
// stay in registers.
template <int PA>
__device__ __forceinline__ void jacobian_row(int kind, int idx, const double (&b)[n_mono(PA)],
                                             double (&J)[n_mono(PA)]) {
    constexpr MonoTable<PA> mt{};
    constexpr int NA = n_mono(PA);
    using Tab = D4Table<PA>;
#pragma unroll
    for (int mu = 0; mu < NA; ++mu) J[mu] = 0.0;
    if (kind == 2) {                       // eq. (25): D2 = B_m0
        J[0] = 1.0;
    } else if (kind == 3) {                // eq. (26c): D3_n = sum_{|mu|=n} c_mu B_mu^2
#pragma unroll
        for (int mu = 0; mu < NA; ++mu)
            if (mt.deg[mu] == idx) J[mu] = 2.0 * mt.mult[mu] * b[mu];
    } else if (Tab::build.pb[idx] == 0) {  // eq. (27a): D4_(a,0,0) = B_0 D3_a
        const int aa = Tab::build.pa[idx];
        double d3a = 0.0;
#pragma unroll
        for (int mu = 0; mu < NA; ++mu)
            if (mt.deg[mu] == aa) {
                d3a += mt.mult[mu] * b[mu] * b[mu];
                J[mu] = 2.0 * mt.mult[mu] * b[0] * b[mu];
            }
        J[0] += d3a;
    } else {                               // eq. (30a): sum_t c_t B_x B_y B_z
#pragma unroll
        for (int t = 0; t < Tab::NT; ++t)
            if (Tab::build.tp[t] == idx) {
                const int x = Tab::build.tx[t], y = Tab::build.ty[t], z = Tab::build.tz[t];
                const double cf = Tab::build.tc[t];
                J[x] += cf * b[y] * b[z];
                J[y] += cf * b[x] * b[z];
                J[z] += cf * b[x] * b[y];
            }
    }
}

template <int PA, bool FAST>
__global__ __launch_bounds__(MAX_THREADS) void batch_kernel(BArgs g) {
    constexpr MonoTable<PA> mt{};
    constexpr int NA = n_mono(PA);
    using Tab = D4Table<PA>;
    constexpr int KA = Tab::KA;
    constexpr int NT = Tab::NT;

    const ParamsT<double>* __restrict__ P = &g.prm;
    const int K = P->K, M = P->M;
    const int SR = 4 + 2 * K;
    const int nth = blockDim.x;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6, nwv = nth >> 6;
    const int apw = WAVE / K;
    const int al = lane / K, q = lane - al * K;
    const int cw = g.cw;

    extern __shared__ __align__(16) unsigned char smem[];
    const BatchLds LY = batch_lds(M, cw, g.nc_max);
    double* sQ = reinterpret_cast<double*>(smem + LY.q);
    double* sG = reinterpret_cast<double*>(smem + LY.gsum);
    double* sAcc = reinterpret_cast<double*>(smem + LY.acc);
    int* sOff = reinterpret_cast<int*>(smem + LY.off);

    if (FAST)
        for (int i = tid; i < POD_MAX_L * POD_MAX_K; i += nth) sQ[i] = (&P->Q[0][0])[i];
    double* rec = g.scratch + static_cast<size_t>(blockIdx.x) * (g.rec_cap * SR + g.b_cap * K * NA);
    double* Bs = rec + g.rec_cap * SR;
    const double rin = P->rin, rcut = P->rcut;

    for (int w = blockIdx.x; w < g.n_cfg; w += gridDim.x) {
        const int c = g.order[w];
        const int a0 = g.cfg_off[c], a1 = g.cfg_off[c + 1];
        const int Nc = a1 - a0;
        for (int i = tid; i <= Nc; i += nth) sOff[i] = g.offsets[a0 + i];
        double cell[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) cell[k] = g.cells[9 * static_cast<size_t>(c) + k];
        __syncthreads();
        const int p0 = sOff[0];
        const int Pc = sOff[Nc] - p0;

        // ---- 1. pair records ----
        for (int pp = tid; pp < Pc; pp += nth) {
            int lo = 0, hi = Nc;   // sOff[lo] - p0 <= pp < sOff[hi] - p0
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (sOff[mid] - p0 <= pp) lo = mid; else hi = mid;
            }
            const int i = a0 + lo;
            const int p = p0 + pp;
            const int j = g.nbr_j[p];
            const int sh = g.shift[p];
            double d0 = 0, d1 = 0, d2 = 0, r = 0.5 * (rin + rcut);
            bool ok = false;
            if (j < a0 || j >= a1) {
                atomicOr(g.err, ERR_NEIGH);
            } else {
                const double sx = unpack_shift(sh, 0), sy = unpack_shift(sh, 1), sz = unpack_shift(sh, 2);
                d0 = g.pos[3 * j + 0] - g.pos[3 * i + 0] + sx * cell[0] + sy * cell[3] + sz * cell[6];
                d1 = g.pos[3 * j + 1] - g.pos[3 * i + 1] + sx * cell[1] + sy * cell[4] + sz * cell[7];
                d2 = g.pos[3 * j + 2] - g.pos[3 * i + 2] + sx * cell[2] + sy * cell[5] + sz * cell[8];
                const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
                if (!isfinite(r2)) {
                    atomicOr(g.err, ERR_NONFINITE);
                } else {
                    const double rr = sqrt(r2);
                    if (rr <= rin) atomicOr(g.err, ERR_RANGE);
                    else if (rr < rcut) { r = rr; ok = true; }   // beyond rcut: not a neighbour
                }
            }
            const double ri = 1.0 / r;
            double R[FAST_MAX_K], dR[FAST_MAX_K];
            if constexpr (FAST) radial_std<double, true>(P, sQ, r, ri, R, dR);
            else radial<double, true>(P, r, ri, R, dR);
            const double z = ok ? 1.0 : 0.0;
            double* row = rec + static_cast<size_t>(pp) * SR;
            row[0] = d0 * ri * z; row[1] = d1 * ri * z; row[2] = d2 * ri * z; row[3] = ri;
#pragma unroll
            for (int k = 0; k < FAST_MAX_K; ++k)
                if (k < K) { row[4 + k] = R[k] * z; row[4 + K + k] = dR[k] * z; }
        }
        for (int k = tid; k < M; k += nth) sG[k] = 0.0;
        __syncthreads();

        // ---- 2. forward: atomic basis, descriptors, G ----
        for (int base = 0; base < Nc; base += nwv * apw) {
            const int a = base + wv * apw + al;
            const bool act = al < apw && a < Nc;
            const int m = q;
            double acc[NA];
#pragma unroll
            for (int mu = 0; mu < NA; ++mu) acc[mu] = 0.0;
            if (act) {
                const int pe = sOff[a + 1] - p0;
                for (int pp = sOff[a] - p0; pp < pe; ++pp) {
                    const double* row = rec + static_cast<size_t>(pp) * SR;
                    accumulate_basis<double, PA>(acc, row[4 + m], row[0], row[1], row[2]);
                }
            }
            double d3[PA + 1];
#pragma unroll
            for (int n = 0; n <= PA; ++n) d3[n] = 0.0;
#pragma unroll
            for (int mu = 0; mu < NA; ++mu) d3[mt.deg[mu]] += double(mt.mult[mu]) * acc[mu] * acc[mu];
            double d4[KA];
#pragma unroll
            for (int p = 0; p < KA; ++p) d4[p] = (Tab::build.pb[p] == 0) ? acc[0] * d3[Tab::build.pa[p]] : 0.0;
#pragma unroll
            for (int t = 0; t < NT; ++t)
                d4[Tab::build.tp[t]] += double(Tab::build.tc[t]) * acc[Tab::build.tx[t]] * acc[Tab::build.ty[t]] *
                                        acc[Tab::build.tz[t]];
            if (act) {
#pragma unroll
                for (int mu = 0; mu < NA; ++mu) Bs[(static_cast<size_t>(a) * K + m) * NA + mu] = acc[mu];
                double* Drow = g.D ? g.D + static_cast<size_t>(a0 + a) * M : nullptr;
                if (q == 0) { if (Drow) Drow[0] = 1.0; atomicAdd(&sG[0], 1.0); }
                if (m < P->K2) { if (Drow) Drow[1 + m] = acc[0]; atomicAdd(&sG[1 + m], acc[0]); }
                if (m < P->K3) {
#pragma unroll
                    for (int n = 0; n <= PA; ++n)
                        if (n <= P->P3) {
                            const int col = P->off3 + m * (P->P3 + 1) + n;
                            if (Drow) Drow[col] = d3[n];
                            atomicAdd(&sG[col], d3[n]);
                        }
                }
                if (m < P->K4) {
#pragma unroll
                    for (int p = 0; p < KA; ++p)
                        if (p < P->Ka4) {
                            const int col = P->off4 + m * P->Ka4 + p;
                            if (Drow) Drow[col] = d4[p];
                            atomicAdd(&sG[col], d4[p]);
                        }
                }
            }
        }
        __syncthreads();
        if (g.G)
            for (int k = tid; k < M; k += nth) g.G[static_cast<size_t>(c) * M + k] = sG[k];

        // ---- 3. dG/dR ----
        if (g.dGdR) {
            for (int m = 0; m < K; ++m) {
                const int ncol_m = (m < P->K2 ? 1 : 0) + (m < P->K3 ? P->P3 + 1 : 0) + (m < P->K4 ? P->Ka4 : 0);
                for (int cs = 0; cs < ncol_m; cs += cw) {
                    const int nc = min(cw, ncol_m - cs);
                    for (int t = tid; t < Nc * 3 * cw; t += nth) sAcc[t] = 0.0;
                    __syncthreads();
                    for (int it = tid; it < Nc * nc; it += nth) {
                        const int a = it / nc, cl = it - a * nc;
                        int kind, idx;
                        column_of(P, m, cs + cl, &kind, &idx);
                        double J[NA];
                        {
                            double b[NA];
                            const double* brow = Bs + (static_cast<size_t>(a) * K + m) * NA;
#pragma unroll
                            for (int mu = 0; mu < NA; ++mu) b[mu] = brow[mu];
                            jacobian_row<PA>(kind, idx, b, J);
                        }
                        double s0 = 0.0, s1 = 0.0, s2 = 0.0;   // -sum_j v_ij, the centre's own row
                        const int pb = sOff[a] - p0, pe = sOff[a + 1] - p0;
                        // the next pair's record is requested before this pair's
                        // arithmetic (the loop is bound by these loads' latency otherwise)
                        int nj = 0;
                        double nux = 0, nuy = 0, nuz = 0, nri = 0, nRm = 0, ndRm = 0;
                        if (pb < pe) {
                            const double* row = rec + static_cast<size_t>(pb) * SR;
                            nj = g.nbr_j[p0 + pb];
                            nux = row[0]; nuy = row[1]; nuz = row[2]; nri = row[3];
                            nRm = row[4 + m]; ndRm = row[4 + K + m];
                        }
                        for (int pp = pb; pp < pe; ++pp) {
                            const int jl = nj - a0;
                            const double ux = nux, uy = nuy, uz = nuz, ri = nri;
                            const double Rm = nRm, dRm = ndRm;
                            if (pp + 1 < pe) {
                                const double* row = rec + static_cast<size_t>(pp + 1) * SR;
                                nj = g.nbr_j[p0 + pp + 1];
                                nux = row[0]; nuy = row[1]; nuz = row[2]; nri = row[3];
                                nRm = row[4 + m]; ndRm = row[4 + K + m];
                            }
                            double A[NA];
                            A[0] = 1.0;
#pragma unroll
                            for (int mu = 1; mu < NA; ++mu) {
                                const double u = mt.axis[mu] == 0 ? ux : (mt.axis[mu] == 1 ? uy : uz);
                                A[mu] = A[mt.par[mu]] * u;
                            }
                            // h = sum_mu J_mu A_mu(u), its u-gradient q and the Euler sum
                            // u . grad h = sum_mu deg(mu) J_mu A_mu (A_mu homogeneous)
                            double hn[PA + 1];
#pragma unroll
                            for (int n = 0; n <= PA; ++n) hn[n] = 0.0;
                            // grad_u h by exponent groups: q_d = sum_n n gq[d][n], one FMA per term
                            double gq[3][PA + 1];
#pragma unroll
                            for (int n = 0; n <= PA; ++n) { gq[0][n] = 0.0; gq[1][n] = 0.0; gq[2][n] = 0.0; }
#pragma unroll
                            for (int mu = 0; mu < NA; ++mu) {
                                hn[mt.deg[mu]] += J[mu] * A[mu];
#pragma unroll
                                for (int dd = 0; dd < 3; ++dd)
                                    if (mt.down[mu][dd] >= 0) gq[dd][mt.ex[mu][dd]] += J[mu] * A[mt.down[mu][dd]];
                            }
                            double q0 = 0, q1 = 0, q2 = 0;
#pragma unroll
                            for (int n = 1; n <= PA; ++n) {
                                q0 += double(n) * gq[0][n];
                                q1 += double(n) * gq[1][n];
                                q2 += double(n) * gq[2][n];
                            }
                            double hsum = 0.0, eul = 0.0;
#pragma unroll
                            for (int n = 0; n <= PA; ++n) { hsum += hn[n]; eul += double(n) * hn[n]; }
                            // eq. (24c): R'_m h rhat + R_m (grad_u h - (rhat . grad_u h) rhat) / r
                            const double c1 = dRm * hsum - Rm * eul * ri;
                            const double c2 = Rm * ri;
                            const double v0 = c1 * ux + c2 * q0, v1 = c1 * uy + c2 * q1, v2 = c1 * uz + c2 * q2;
                            if (jl >= 0 && jl < Nc) {
                                atomicAdd(&sAcc[(jl * 3 + 0) * cw + cl], v0);
                                atomicAdd(&sAcc[(jl * 3 + 1) * cw + cl], v1);
                                atomicAdd(&sAcc[(jl * 3 + 2) * cw + cl], v2);
                            }
                            s0 -= v0; s1 -= v1; s2 -= v2;
                        }
                        atomicAdd(&sAcc[(a * 3 + 0) * cw + cl], s0);
                        atomicAdd(&sAcc[(a * 3 + 1) * cw + cl], s1);
                        atomicAdd(&sAcc[(a * 3 + 2) * cw + cl], s2);
                    }
                    __syncthreads();
                    // write the chunk out
                    for (int t = tid; t < Nc * 3 * nc; t += nth) {
                        const int n = t / (3 * nc), r3 = t - n * 3 * nc;
                        const int d = r3 / nc, cl = r3 - d * nc;
                        int kind, idx;
                        const int col = column_of(P, m, cs + cl, &kind, &idx);
                        g.dGdR[(static_cast<size_t>(a0 + n) * 3 + d) * M + col] = sAcc[(n * 3 + d) * cw + cl];
                    }
                    __syncthreads();
                }
            }
            for (int t = tid; t < Nc * 3; t += nth) g.dGdR[(static_cast<size_t>(a0) * 3 + t) * M] = 0.0;
        }
        __syncthreads();
    }
}

template <int PA>
hipError_t launch_batch(const BArgs& a, bool fast, int nblk, int nth, size_t lds, hipStream_t st) {
    const void* fn = fast ? reinterpret_cast<const void*>(&batch_kernel<PA, true>)
                          : reinterpret_cast<const void*>(&batch_kernel<PA, false>);
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)) != hipSuccess)
        return hipErrorInvalidValue;
    if (fast) hipLaunchKernelGGL((batch_kernel<PA, true>), dim3(nblk), dim3(nth), lds, st, a);
    else hipLaunchKernelGGL((batch_kernel<PA, false>), dim3(nblk), dim3(nth), lds, st, a);
    return hipGetLastError();
}

hipError_t dispatch_batch(int PA, const BArgs& a, bool fast, int nblk, int nth, size_t lds, hipStream_t st) {
    switch (PA) {
        case 0: return launch_batch<0>(a, fast, nblk, nth, lds, st);
        case 1: return launch_batch<1>(a, fast, nblk, nth, lds, st);
        case 2: return launch_batch<2>(a, fast, nblk, nth, lds, st);
        case 3: return launch_batch<3>(a, fast, nblk, nth, lds, st);
        case 4: return launch_batch<4>(a, fast, nblk, nth, lds, st);
        case 5: return launch_batch<5>(a, fast, nblk, nth, lds, st);
        case 6: return launch_batch<6>(a, fast, nblk, nth, lds, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace
}  // namespace pod

extern "C" {

int pod_batch_assemble(pod_handle* h, int n_cfg, int N, int P, const int* cfg_atom_off, const void* pos,
                       const double* cells, const int* offsets, const int* nbr_j, const int* shift, double* D,
                       double* G, double* dGdR, const pod_tune* tune) {
    using namespace pod;
    if (!h || n_cfg < 0 || N < 0 || P < 0) return POD_EINVAL;
    if (h->dtype != POD_F64 || h->PA > FAST_MAX_PA || h->K > FAST_MAX_K) return POD_ENOTSUP;
    if (n_cfg == 0 || N == 0) return POD_OK;
    if (!cfg_atom_off || !pos || !cells || !offsets || (P > 0 && (!nbr_j || !shift))) return POD_EINVAL;
    // plan on the host: cell sizes and pair counts
    std::vector<int> coff(n_cfg + 1), off(N + 1);
    if (hipMemcpyAsync(coff.data(), cfg_atom_off, sizeof(int) * (n_cfg + 1), hipMemcpyDeviceToHost, h->stream) !=
            hipSuccess ||
        hipMemcpyAsync(off.data(), offsets, sizeof(int) * (N + 1), hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
        return POD_EHIP;
    BatchPlan plan;
    int rc = plan_batch(n_cfg, N, P, coff.data(), off.data(), h->M, h->lds_max, tune, &plan);
    if (rc != POD_OK) return rc;
    const int NA = n_mono(h->PA);
    const int nblk = plan.nblk, nth = plan.nth;
    const size_t lds = plan.lds;
    const std::vector<int>& order = plan.order;
    const int SR = 4 + 2 * h->K;
    const long rec_cap = std::max(plan.max_pc, 1), b_cap = std::max(plan.max_nc, 1);
    const size_t per_blk = static_cast<size_t>(rec_cap) * SR + static_cast<size_t>(b_cap) * h->K * NA;
    const size_t order_bytes = ((sizeof(int) * n_cfg + 255) / 256) * 256;
    rc = ensure_scratch(h, order_bytes + per_blk * nblk * sizeof(double));
    if (rc != POD_OK) return rc;
    int* d_order = static_cast<int*>(h->d_scratch);
    if (hipMemcpyAsync(d_order, order.data(), sizeof(int) * n_cfg, hipMemcpyHostToDevice, h->stream) != hipSuccess)
        return POD_EHIP;
    BArgs a;
    a.prm = h->hp_d;
    a.n_cfg = n_cfg; a.order = d_order; a.cfg_off = cfg_atom_off;
    a.pos = static_cast<const double*>(pos); a.cells = cells;
    a.offsets = offsets; a.nbr_j = nbr_j; a.shift = shift;
    a.N = N; a.P = P;
    a.D = D; a.G = G; a.dGdR = dGdR;
    a.scratch = reinterpret_cast<double*>(static_cast<char*>(h->d_scratch) + order_bytes);
    a.rec_cap = rec_cap; a.b_cap = b_cap;
    a.cw = plan.cw; a.nc_max = plan.nc_max;
    a.err = h->d_err;
    timing_begin(h, 1);
    const hipError_t e = dispatch_batch(h->PA, a, h->std_ok != 0, nblk, nth, lds, h->stream);
    timing_end(h, 1);
    return e == hipSuccess ? POD_OK : POD_EHIP;
}

}  // extern "C"
