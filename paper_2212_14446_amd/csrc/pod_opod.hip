// Exclusive-sum descriptors: the earlier POD form that the paper compares
// its fast descriptors with, evaluated by their defining sums.
//   3-body  eq. (15b): sum over neighbour pairs j < k        O(N_i^2)
//   4-body  eq. (20a): sum over neighbour triples j < k < l  O(N_i^3), with
//           the cyclic angular functions g_p of eq. (19a) / Table 2
// and the linear 2/3-body model built on them (OPOD of Table 6) with its
// forces, up to the largest sizes of Table 6 (K = 12, 3-body degree 10,
// 4-body degree 6).  One wavefront per atom; the atom's neighbours (unit vectors,
// distances, R_m and R'_m) are staged in LDS once, then the pair and triple
// loops read them from there.  FP64.
#include <hip/hip_runtime.h>

#include <cmath>

#include "pod.h"
#include "pod_device.h"
#include "pod_internal.h"
#include "pod_tables.h"

namespace pod {
namespace {

using namespace dev;

constexpr int OPOD_NMAX = 128;   // neighbours within rcut per atom (else POD_ENEIGH)

// 4-body descriptor instances: angular degree up to 4 (Table 2, 11 functions
// g_p, four radial indices per accumulator pass) and up to 6 (eq. (19a) for
// n = 5, 6 as well: 23 functions, two radial indices per pass).
template <int P4MAX>
struct OpodD4 {
    static constexpr int KA = n_partitions(P4MAX);
    static constexpr int MC = P4MAX <= 4 ? 4 : 2;
};

// g_p terms (eq. (19a), Table 2 for n <= 4): for each p in Table-1 order the
// distinct members of the cyclic orbit {(a,b,c), (c,a,b), (b,c,a)} of the
// exponents of (w_ijk, w_ijl, w_ikl).
template <int P4MAX>
struct GTable {
    static constexpr int KA = n_partitions(P4MAX);
    int nterm[KA];
    int e[KA][3][3];
    constexpr GTable() : nterm{}, e{} {
        int p = 0;
        for (int n = 0; n <= P4MAX; ++n)
            for (int a = n; a >= 0; --a)
                for (int b = (a < n - a ? a : n - a); b >= 0; --b) {
                    const int c = n - a - b;
                    if (c < 0 || c > b) continue;
                    const int rot[3][3] = {{a, b, c}, {c, a, b}, {b, c, a}};
                    int t = 0;
                    for (int r = 0; r < 3; ++r) {
                        bool dup = false;
                        for (int q = 0; q < t; ++q)
                            dup = dup || (e[p][q][0] == rot[r][0] && e[p][q][1] == rot[r][1] && e[p][q][2] == rot[r][2]);
                        if (!dup) {
                            e[p][t][0] = rot[r][0];
                            e[p][t][1] = rot[r][1];
                            e[p][t][2] = rot[r][2];
                            ++t;
                        }
                    }
                    nterm[p] = t;
                    ++p;
                }
    }
};

struct OArgs {
    ParamsT<double> prm;
    CellT<double> cell;
    int N;
    const double* pos;
    const int* offsets;
    const int* nbr_j;
    const int* shift;
    const double* coef;   // M coefficients (energy kernel)
    double* D;            // N x M (descriptor kernel)
    double* E_atom;       // N or null
    double* Facc;         // 3N FP64 accumulator (zero on entry, energy kernel)
    double* part;         // [N][10]: E_i and the atom's virial share (energy kernel)
    int* err;
};

// Neighbour staging: unit vector, distance, R_m, R'_m of every neighbour of
// atom i (absent pairs -- r >= rcut -- get R = R' = 0 and u = 0).  KS radial
// slots: FAST_MAX_K for models with K up to 8 (less LDS, more workgroups per
// CU), POD_MAX_K otherwise.
template <int KS>
struct Stage {
    double u[OPOD_NMAX][3];
    double r[OPOD_NMAX];
    double R[OPOD_NMAX][KS];
    double dR[OPOD_NMAX][KS];
    int ok[OPOD_NMAX];   // a neighbour within rcut with a valid index
};

template <int KS>
__device__ __forceinline__ void stage_neighbours(const OArgs& a, int i, int p0, int n, int lane, Stage<KS>& s) {
    const double pi0 = a.pos[3 * i], pi1 = a.pos[3 * i + 1], pi2 = a.pos[3 * i + 2];
    for (int t = lane; t < n; t += WAVE) {
        const int p = p0 + t;
        const int j = a.nbr_j[p];
        const int sh = a.shift[p];
        double u[3] = {0.0, 0.0, 0.0}, r = 0.5 * (a.prm.rin + a.prm.rcut);
        double R[KS], dR[KS];
        bool ok = false;
        if (j < 0 || j >= a.N || (!a.cell.periodic && (sh & 0xFFFFFF) != 0)) {
            atomicOr(a.err, ERR_NEIGH);
        } else {
            const double sx = unpack_shift(sh, 0), sy = unpack_shift(sh, 1), sz = unpack_shift(sh, 2);
            const double* c = a.cell.a;
            const double d0 = a.pos[3 * j] - pi0 + sx * c[0] + sy * c[3] + sz * c[6];
            const double d1 = a.pos[3 * j + 1] - pi1 + sx * c[1] + sy * c[4] + sz * c[7];
            const double d2 = a.pos[3 * j + 2] - pi2 + sx * c[2] + sy * c[5] + sz * c[8];
            const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
            if (!isfinite(r2)) {
                atomicOr(a.err, ERR_NONFINITE);
            } else {
                const double rr = sqrt(r2);
                if (rr <= a.prm.rin) {
                    atomicOr(a.err, ERR_RANGE);
                } else if (rr < a.prm.rcut) {
                    ok = true;
                    r = rr;
                    u[0] = d0 / rr;
                    u[1] = d1 / rr;
                    u[2] = d2 / rr;
                }
            }
        }
        radial<double, true>(&a.prm, r, 1.0 / r, R, dR);
        s.u[t][0] = u[0];
        s.u[t][1] = u[1];
        s.u[t][2] = u[2];
        s.r[t] = r;
        s.ok[t] = ok ? 1 : 0;
#pragma unroll
        for (int m = 0; m < KS; ++m) {
            s.R[t][m] = ok ? R[m] : 0.0;
            s.dR[t][m] = ok ? dR[m] : 0.0;
        }
    }
}

// Exclusive descriptors [1 | D2 | D3 (eq. (15b)) | D4 (eq. (20a))].
template <int P4MAX, int KS, int P3MAX>
__global__ __launch_bounds__(WAVE) void opod_desc_kernel(OArgs a) {
    constexpr GTable<P4MAX> gt{};
    constexpr int OPOD_KA = OpodD4<P4MAX>::KA;
    constexpr int OPOD_MC = OpodD4<P4MAX>::MC;
    constexpr int OPOD_P4MAX = P4MAX;
    __shared__ Stage<KS> s;
    const int i = blockIdx.x;
    const int lane = threadIdx.x;
    const int p0 = a.offsets[i], n = a.offsets[i + 1] - p0;
    double* Drow = a.D + static_cast<long>(i) * a.prm.M;
    if (n < 0 || n > OPOD_NMAX) {
        if (lane == 0) atomicOr(a.err, ERR_NEIGH);
        for (int k = lane; k < a.prm.M; k += WAVE) Drow[k] = k == 0 ? 1.0 : 0.0;
        return;
    }
    stage_neighbours(a, i, p0, n, lane, s);
    __syncthreads();
    const int K2 = a.prm.K2, K3 = a.prm.K3, P3 = a.prm.P3, K4 = a.prm.K4;
    if (lane == 0) Drow[0] = 1.0;
    // 2-body (eq. (12b))
    for (int k = 0; k < K2; ++k) {
        double v = 0.0;
        for (int t = lane; t < n; t += WAVE) v += s.R[t][k];
        v = wave_sum(v);
        if (lane == 0) Drow[1 + k] = v;
    }
    // 3-body: lane j sums over k > j (eq. (15b))
    for (int m = 0; m < K3; ++m) {
        double acc[P3MAX + 1];
#pragma unroll
        for (int q = 0; q <= P3MAX; ++q) acc[q] = 0.0;
        for (int j = lane; j < n; j += WAVE) {
            const double Rj = s.R[j][m];
            for (int k = j + 1; k < n; ++k) {
                const double w = s.u[j][0] * s.u[k][0] + s.u[j][1] * s.u[k][1] + s.u[j][2] * s.u[k][2];
                double x = Rj * s.R[k][m];
#pragma unroll
                for (int q = 0; q <= P3MAX; ++q) {
                    if (q <= P3) acc[q] += x;
                    x *= w;
                }
            }
        }
#pragma unroll
        for (int q = 0; q <= P3MAX; ++q) {
            const double v = wave_sum(acc[q]);
            if (lane == 0 && q <= P3) Drow[a.prm.off3 + m * (P3 + 1) + q] = v;
        }
    }
    if (K4 == 0) return;
    // 4-body: pairs (j, k), j < k, dealt to the lanes; each walks l > k (eq. (20a))
    const int KA = a.prm.Ka4;
    const int npair = n * (n - 1) / 2;
    for (int m0 = 0; m0 < K4; m0 += OPOD_MC) {
        double acc[OPOD_MC][OPOD_KA];
#pragma unroll
        for (int mm = 0; mm < OPOD_MC; ++mm)
#pragma unroll
            for (int q = 0; q < OPOD_KA; ++q) acc[mm][q] = 0.0;
        for (int pi = lane; pi < npair; pi += WAVE) {
            // pair index -> (j, k): pairs ordered by k, then j < k
            int k = static_cast<int>((1.0 + sqrt(1.0 + 8.0 * pi)) * 0.5);
            while (k * (k - 1) / 2 > pi) --k;
            while ((k + 1) * k / 2 <= pi) ++k;
            const int j = pi - k * (k - 1) / 2;
            const double w1 = s.u[j][0] * s.u[k][0] + s.u[j][1] * s.u[k][1] + s.u[j][2] * s.u[k][2];
            double rjk[OPOD_MC];
#pragma unroll
            for (int mm = 0; mm < OPOD_MC; ++mm)
                rjk[mm] = m0 + mm < K4 ? s.R[j][m0 + mm] * s.R[k][m0 + mm] : 0.0;
            double p1[OPOD_P4MAX + 1];
            p1[0] = 1.0;
#pragma unroll
            for (int e = 1; e <= OPOD_P4MAX; ++e) p1[e] = p1[e - 1] * w1;
            for (int l = k + 1; l < n; ++l) {
                const double w2 = s.u[j][0] * s.u[l][0] + s.u[j][1] * s.u[l][1] + s.u[j][2] * s.u[l][2];
                const double w3 = s.u[k][0] * s.u[l][0] + s.u[k][1] * s.u[l][1] + s.u[k][2] * s.u[l][2];
                double p2[OPOD_P4MAX + 1], p3[OPOD_P4MAX + 1];
                p2[0] = p3[0] = 1.0;
#pragma unroll
                for (int e = 1; e <= OPOD_P4MAX; ++e) {
                    p2[e] = p2[e - 1] * w2;
                    p3[e] = p3[e - 1] * w3;
                }
                double g[OPOD_KA];
#pragma unroll
                for (int q = 0; q < OPOD_KA; ++q) {
                    double v = 0.0;
#pragma unroll
                    for (int t = 0; t < 3; ++t)
                        if (t < gt.nterm[q]) v += p1[gt.e[q][t][0]] * p2[gt.e[q][t][1]] * p3[gt.e[q][t][2]];
                    g[q] = v;
                }
#pragma unroll
                for (int mm = 0; mm < OPOD_MC; ++mm) {
                    const double x = rjk[mm] * (m0 + mm < K4 ? s.R[l][m0 + mm] : 0.0);
#pragma unroll
                    for (int q = 0; q < OPOD_KA; ++q) acc[mm][q] += x * g[q];
                }
            }
        }
#pragma unroll
        for (int mm = 0; mm < OPOD_MC; ++mm)
#pragma unroll
            for (int q = 0; q < OPOD_KA; ++q) {
                const double v = wave_sum(acc[mm][q]);   // uniform guards: every lane reduces
                if (lane == 0 && m0 + mm < K4 && q < KA) Drow[a.prm.off4 + (m0 + mm) * KA + q] = v;
            }
    }
}

// Energy and forces of the 2/3-body exclusive model: lane j takes neighbour
// j (and j + 64, ...), walks every k != j, and accumulates half of each
// pair's energy and the whole of dE_i/dr_ij:
//   X_jk = R_m(r_ij) R_m(r_ik) P_m(w),  P_m(w) = sum_n c3_mn w^n
//   dE_i/dr_ij = sum_k sum_m [R'_m(r_ij) R_m(r_ik) P_m u_j
//                             + R_m R_m P'_m (u_k - w u_j) / r_ij]
template <int KS>
__global__ __launch_bounds__(WAVE) void opod_energy_kernel(OArgs a) {
    __shared__ Stage<KS> s;
    __shared__ double cf[1 + POD_MAX_K + POD_MAX_K * (POD_MAX_P + 1)];
    const int i = blockIdx.x;
    const int lane = threadIdx.x;
    const int M = a.prm.M;
    for (int k = lane; k < M; k += WAVE) cf[k] = a.coef[k];
    const int p0 = a.offsets[i], n = a.offsets[i + 1] - p0;
    const bool too_many = n < 0 || n > OPOD_NMAX;
    if (!too_many) stage_neighbours(a, i, p0, too_many ? 0 : n, lane, s);
    __syncthreads();
    const int K2 = a.prm.K2, K3 = a.prm.K3, P3 = a.prm.P3;
    const double* c2 = cf + 1;
    const double* c3 = cf + a.prm.off3;
    double e = 0.0, fo[3] = {0.0, 0.0, 0.0}, vir[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) vir[q] = 0.0;
    if (too_many) {
        if (lane == 0) atomicOr(a.err, ERR_NEIGH);
    } else {
        for (int j = lane; j < n; j += WAVE) {
            const double uj0 = s.u[j][0], uj1 = s.u[j][1], uj2 = s.u[j][2], rj = s.r[j];
            double gr = 0.0, ga0 = 0.0, ga1 = 0.0, ga2 = 0.0;
            for (int k = 0; k < n; ++k) {
                if (k == j) continue;
                const double uk0 = s.u[k][0], uk1 = s.u[k][1], uk2 = s.u[k][2];
                const double w = uj0 * uk0 + uj1 * uk1 + uj2 * uk2;
                double er = 0.0, ea = 0.0;
                for (int m = 0; m < K3; ++m) {
                    // Horner for P_m(w) and P'_m(w)
                    const double* cm = c3 + m * (P3 + 1);
                    double P = cm[P3], dP = 0.0;
                    for (int q = P3 - 1; q >= 0; --q) {
                        dP = dP * w + P;
                        P = P * w + cm[q];
                    }
                    const double Rk = s.R[k][m];
                    e += 0.5 * s.R[j][m] * Rk * P;
                    er += s.dR[j][m] * Rk * P;
                    ea += s.R[j][m] * Rk * dP;
                }
                gr += er;
                ga0 += ea * (uk0 - w * uj0);
                ga1 += ea * (uk1 - w * uj1);
                ga2 += ea * (uk2 - w * uj2);
            }
            for (int k = 0; k < K2; ++k) {
                e += c2[k] * s.R[j][k];
                gr += c2[k] * s.dR[j][k];
            }
            const double inv = 1.0 / rj;
            const double g0 = gr * uj0 + ga0 * inv, g1 = gr * uj1 + ga1 * inv, g2 = gr * uj2 + ga2 * inv;
            const double d[3] = {uj0 * rj, uj1 * rj, uj2 * rj};
            const double g[3] = {g0, g1, g2};
            if (s.ok[j] && a.Facc) {   // only valid indices reach the scatter
                const int jn = a.nbr_j[p0 + j];
                atomicAdd(&a.Facc[3 * jn], -g0);
                atomicAdd(&a.Facc[3 * jn + 1], -g1);
                atomicAdd(&a.Facc[3 * jn + 2], -g2);
            }
            fo[0] += g0;
            fo[1] += g1;
            fo[2] += g2;
#pragma unroll
            for (int x = 0; x < 3; ++x)
#pragma unroll
                for (int y = 0; y < 3; ++y) vir[3 * x + y] -= d[x] * g[y];
        }
    }
    e = wave_sum(e);
    fo[0] = wave_sum(fo[0]);
    fo[1] = wave_sum(fo[1]);
    fo[2] = wave_sum(fo[2]);
#pragma unroll
    for (int q = 0; q < 9; ++q) vir[q] = wave_sum(vir[q]);
    if (lane == 0) {
        const double Ei = cf[0] + e;
        if (a.E_atom) a.E_atom[i] = Ei;
        if (a.Facc) {
            atomicAdd(&a.Facc[3 * i], fo[0]);
            atomicAdd(&a.Facc[3 * i + 1], fo[1]);
            atomicAdd(&a.Facc[3 * i + 2], fo[2]);
        }
        double* pr = a.part + static_cast<long>(i) * 10;
        pr[0] = Ei;
#pragma unroll
        for (int q = 0; q < 9; ++q) pr[1 + q] = vir[q];
    }
}

// Totals E, W (fixed order over atoms, block 0) and the forces out of the
// accumulator, which is re-zeroed (other blocks).
__global__ __launch_bounds__(256) void opod_finalize_kernel(const double* __restrict__ part, int N, double* E,
                                                            double* W, double* Facc, double* F, long n3) {
    if (blockIdx.x == 0) {
        // each thread sums all ten columns over its atoms, then one tree
        // reduction per column (fixed order)
        __shared__ double red[10][256];
        double v[10];
#pragma unroll
        for (int col = 0; col < 10; ++col) v[col] = 0.0;
        for (int i = threadIdx.x; i < N; i += 256) {
#pragma unroll
            for (int col = 0; col < 10; ++col) v[col] += part[static_cast<long>(i) * 10 + col];
        }
#pragma unroll
        for (int col = 0; col < 10; ++col) red[col][threadIdx.x] = v[col];
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (static_cast<int>(threadIdx.x) < o) {
#pragma unroll
                for (int col = 0; col < 10; ++col) red[col][threadIdx.x] += red[col][threadIdx.x + o];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0 && E) *E = red[0][0];
        if (threadIdx.x < 9 && W) W[threadIdx.x] = red[1 + threadIdx.x][0];
        return;
    }
    const long k = static_cast<long>(blockIdx.x - 1) * 256 + threadIdx.x;
    if (k < n3) {
        if (F) F[k] = Facc[k];
        Facc[k] = 0.0;
    }
}

int fill(pod_handle* h, OArgs& a, int N, const void* pos, const double* cell, const int* offsets, const int* nbr_j,
         const int* shift) {
    a.prm = h->hp_d;
    a.N = N;
    a.pos = static_cast<const double*>(pos);
    a.cell.periodic = cell != nullptr;
    for (int k = 0; k < 9; ++k) {
        const double v = cell ? cell[k] : 0.0;
        if (!std::isfinite(v)) return POD_EINVAL;
        a.cell.a[k] = v;
    }
    a.offsets = offsets;
    a.nbr_j = nbr_j;
    a.shift = shift;
    a.coef = nullptr;
    a.D = nullptr;
    a.E_atom = nullptr;
    a.Facc = nullptr;
    a.part = nullptr;
    a.err = h->d_err;
    return POD_OK;
}

}  // namespace
}  // namespace pod

extern "C" {

int pod_opod_descriptors(pod_handle* h, int N, int P, const void* pos, const double* cell, const int* offsets,
                         const int* nbr_j, const int* shift, void* D) {
    using namespace pod;
    if (!h || N < 0 || P < 0) return POD_EINVAL;
    if (N > 0 && (!pos || !offsets || !D || (P > 0 && (!nbr_j || !shift)))) return POD_EINVAL;
    if (h->dtype != POD_F64) return POD_ENOTSUP;
    if (h->K4 > 0 && h->P4 > POD_MAX_P4) return POD_ENOTSUP;
    if (N == 0) return POD_OK;
    OArgs a;
    const int rc = fill(h, a, N, pos, cell, offsets, nbr_j, shift);
    if (rc != POD_OK) return rc;
    a.D = static_cast<double*>(D);
    timing_begin(h, 1);
    // instances: 4-body degree up to 4 or 6; K up to 8 with 3-body degree up
    // to 6, or the largest sizes
    const bool p6 = h->K4 > 0 && h->P4 > 4;
    const bool big = h->K > FAST_MAX_K || (h->K3 > 0 && h->P3 > FAST_MAX_PA);
    if (p6 && big)
        hipLaunchKernelGGL((opod_desc_kernel<POD_MAX_P4, POD_MAX_K, POD_MAX_P>), dim3(N), dim3(WAVE), 0, h->stream, a);
    else if (p6)
        hipLaunchKernelGGL((opod_desc_kernel<POD_MAX_P4, FAST_MAX_K, FAST_MAX_PA>), dim3(N), dim3(WAVE), 0, h->stream, a);
    else if (big)
        hipLaunchKernelGGL((opod_desc_kernel<4, POD_MAX_K, POD_MAX_P>), dim3(N), dim3(WAVE), 0, h->stream, a);
    else
        hipLaunchKernelGGL((opod_desc_kernel<4, FAST_MAX_K, FAST_MAX_PA>), dim3(N), dim3(WAVE), 0, h->stream, a);
    timing_end(h, 1);
    return hipGetLastError() == hipSuccess ? POD_OK : POD_EHIP;
}

int pod_opod_energy_forces(pod_handle* h, int N, int P, const void* pos, const double* cell, const int* offsets,
                           const int* nbr_j, const int* shift, const void* c, void* E_atom, double* E, void* F,
                           double* W) {
    using namespace pod;
    if (!h || N < 0 || P < 0) return POD_EINVAL;
    if (N > 0 && (!pos || !offsets || !c || (P > 0 && (!nbr_j || !shift)))) return POD_EINVAL;
    if (h->dtype != POD_F64 || h->K4 != 0) return POD_ENOTSUP;
    OArgs a;
    int rc = fill(h, a, N, pos, cell, offsets, nbr_j, shift);
    if (rc != POD_OK) return rc;
    const size_t part_bytes = sizeof(double) * 10 * static_cast<size_t>(N > 0 ? N : 1);
    rc = ensure_scratch(h, part_bytes);
    if (rc != POD_OK) return rc;
    rc = ensure_force_acc(h, N);
    if (rc != POD_OK) return rc;
    a.coef = static_cast<const double*>(c);
    a.E_atom = static_cast<double*>(E_atom);
    a.Facc = F ? h->d_facc : nullptr;
    a.part = static_cast<double*>(h->d_scratch);
    if (N > 0) {
        timing_begin(h, 1);
        if (h->K > FAST_MAX_K) hipLaunchKernelGGL(opod_energy_kernel<POD_MAX_K>, dim3(N), dim3(WAVE), 0, h->stream, a);
        else hipLaunchKernelGGL(opod_energy_kernel<FAST_MAX_K>, dim3(N), dim3(WAVE), 0, h->stream, a);
        timing_end(h, 1);
    }
    const long n3 = F ? 3L * N : 0L;
    const int nfb = static_cast<int>((n3 + 255) / 256);
    timing_begin(h, 0);
    hipLaunchKernelGGL(opod_finalize_kernel, dim3(1 + nfb), dim3(256), 0, h->stream, a.part, N, E, W, h->d_facc,
                       static_cast<double*>(F), n3);
    timing_end(h, 0);
    if (hipGetLastError() != hipSuccess) {
        h->facc_dirty = 1;
        return POD_EHIP;
    }
    return POD_OK;
}

}  // extern "C"
