// Linear fit of the POD coefficients (Sec. IV.A, eq. (63a)): the normal
// equations of the weighted, regularised least-squares problem, accumulated
// on the FP64 matrix cores, and their solution by a Cholesky factorisation
// in one workgroup.
//
// Rows of the problem: one energy row per configuration (G_c, E_ref_c) with
// weight w_e and one force row per atom coordinate (-dG/dr_{n,d}, F_ref_{n,d})
// with weight w_f; the weights multiply the squared residuals as in the loss
// of eq. (63b).  With every row augmented by its label, x = [a | b], the
// Gram matrix Z = sum_r w_r x_r^T x_r holds A^T W A, A^T W b and b^T W b in
// one (M+1) x (M+1) block.  The Gram sum is a dense contraction, so it runs
// on v_mfma_f64_16x16x4_f64: one MFMA adds the outer products of four rows
// for one 16 x 16 tile of Z.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "pod.h"
#include "pod_internal.h"

namespace pod {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int GRAM_WAVES = 4;          // waves per workgroup
constexpr int GRAM_THREADS = GRAM_WAVES * WAVE;
constexpr int GRAM_BLOCKS = 512;       // persistent: two workgroups per CU
constexpr int GRAM_ROWS = 32;          // rows per LDS chunk (8 MFMA k-steps)
constexpr int RED_SLICES = 16;         // first reduction pass: workgroup partials in 16 slices
constexpr int FIT_MAX_TILES = 8;       // M + 1 <= 128
constexpr int SOLVE_THREADS = 256;      // a 16 x 16 grid in the Cholesky update
static_assert(SOLVE_THREADS == 256, "solve_kernel maps its threads to a 16 x 16 grid");

// Upper-triangle tile pairs (ti <= tj) of a T x T tiling, row by row; pair
// p belongs to wave p % GRAM_WAVES.
template <int T>
struct TilePairs {
    static constexpr int n = T * (T + 1) / 2;
    int ti[n], tj[n];
    constexpr TilePairs() : ti{}, tj{} {
        int p = 0;
        for (int i = 0; i < T; ++i)
            for (int j = i; j < T; ++j) {
                ti[p] = i;
                tj[p] = j;
                ++p;
            }
    }
};

struct GramArgs {
    const double* X;   // R x M, leading dimension ldx
    const double* y;   // R labels (column M of the augmented rows), or null
    double ysign;      // label sign: +1 energy rows, -1 force rows (a = -dG/dr)
    long ldx;
    long R;
    int M;
    int vec;           // X is 16-byte aligned and ldx == M: 16-byte loads
    double* part;      // [gridDim.x][n pairs][256] workgroup partial tiles
};

// Value of a double held by lane `src` (uniform) of the wave.
__device__ __forceinline__ double lane_value(double x, int src) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane(static_cast<int>(b & 0xffffffffLL), src);
    const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), src);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// One wave's share of a chunk: for every k-step of four rows, the T tile
// operands of the rows (lane l: row k0 + l / 16, column 16 t + l % 16) from
// LDS, then one MFMA per owned tile pair.
template <int T, int W>
__device__ __forceinline__ void gram_chunk(const double* __restrict__ buf, int lane,
                                           f64x4 (&acc)[(TilePairs<T>::n + GRAM_WAVES - 1) / GRAM_WAVES]) {
    constexpr TilePairs<T> tp{};
    constexpr int NP = TilePairs<T>::n;
    constexpr int LDW = 16 * T + 2;
    const int rl = lane >> 4, cl = lane & 15;
#pragma unroll 1
    for (int k0 = 0; k0 < GRAM_ROWS; k0 += 4) {
        double v[T];
#pragma unroll
        for (int t = 0; t < T; ++t) v[t] = buf[(k0 + rl) * LDW + 16 * t + cl];
#pragma unroll
        for (int q = 0; W + GRAM_WAVES * q < NP; ++q) {
            const int p = W + GRAM_WAVES * q;
            acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[tp.ti[p]], v[tp.tj[p]], acc[q], 0, 0, 0);
        }
    }
}

// Gram partials of the augmented rows [X | ysign y]: chunks of GRAM_ROWS
// rows are dealt round-robin to the workgroups; the rows of a chunk are one
// contiguous block of GRAM_ROWS x M doubles, loaded in 16-byte pieces (T per
// thread) two chunks ahead of the products (register double-buffering, so
// two chunks per workgroup are in flight), then stored into a double-
// buffered LDS tile with padded rows; each wave accumulates its own tile
// pairs in registers.
template <int T>
__global__ __launch_bounds__(GRAM_THREADS, 2) void gram_kernel(GramArgs a) {
    constexpr int NP = TilePairs<T>::n;
    constexpr int QP = (NP + GRAM_WAVES - 1) / GRAM_WAVES;
    constexpr int LDW = 16 * T + 2;
    static_assert(GRAM_ROWS * 16 * T / 2 <= GRAM_THREADS * T, "T pieces of 16 bytes per thread cover a chunk");
    __shared__ double buf[2][GRAM_ROWS * LDW];
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const int M = a.M;
    const long nchunks = (a.R + GRAM_ROWS - 1) / GRAM_ROWS;
    const long nfull = a.R / GRAM_ROWS;           // chunks without a ragged end
    const int npc = GRAM_ROWS * M / 2;            // 16-byte pieces per chunk
    const bool vec = a.vec != 0;                  // X 16-byte aligned with ldx == M

    for (int e = tid; e < 2 * GRAM_ROWS * LDW; e += GRAM_THREADS) (&buf[0][0])[e] = 0.0;
    // LDS position (row << 8 | column) of the first double of each piece
    int rc[T];
#pragma unroll
    for (int e = 0; e < T; ++e) {
        const int p = tid + GRAM_THREADS * e;
        rc[e] = p < npc ? (((2 * p) / M) << 8) | ((2 * p) % M) : -1;
    }
    f64x4 acc[QP];
#pragma unroll
    for (int q = 0; q < QP; ++q) acc[q] = f64x4{0.0, 0.0, 0.0, 0.0};
    struct Regs {
        double2 x[T];
        double yv;
    };
    auto load = [&](long c, Regs& g) {
        const long r0 = c * GRAM_ROWS;
        if (vec && c < nfull) {
            const double2* base = reinterpret_cast<const double2*>(a.X + r0 * M);
#pragma unroll
            for (int e = 0; e < T; ++e) g.x[e] = rc[e] >= 0 ? base[tid + GRAM_THREADS * e] : double2{0.0, 0.0};
        } else {
#pragma unroll
            for (int e = 0; e < T; ++e) {
                double v0 = 0.0, v1 = 0.0;
                if (rc[e] >= 0) {
                    const int row = rc[e] >> 8, col = rc[e] & 255;
                    const int row1 = col + 1 < M ? row : row + 1, col1 = col + 1 < M ? col + 1 : 0;
                    if (r0 + row < a.R) v0 = a.X[(r0 + row) * a.ldx + col];
                    if (r0 + row1 < a.R) v1 = a.X[(r0 + row1) * a.ldx + col1];
                }
                g.x[e] = double2{v0, v1};
            }
        }
        g.yv = (tid < GRAM_ROWS && a.y && r0 + tid < a.R) ? a.ysign * a.y[r0 + tid] : 0.0;
    };
    auto store = [&](const Regs& g, double* b) {
#pragma unroll
        for (int e = 0; e < T; ++e) {
            if (rc[e] >= 0) {
                const int row = rc[e] >> 8, col = rc[e] & 255;
                b[row * LDW + col] = g.x[e].x;
                if (col + 1 < M) b[row * LDW + col + 1] = g.x[e].y;
                else b[(row + 1) * LDW] = g.x[e].y;
            }
        }
        if (tid < GRAM_ROWS) b[tid * LDW + M] = g.yv;
    };
    auto compute = [&](const double* b) {
        switch (wave) {
            case 0: gram_chunk<T, 0>(b, lane, acc); break;
            case 1: gram_chunk<T, 1>(b, lane, acc); break;
            case 2: gram_chunk<T, 2>(b, lane, acc); break;
            default: gram_chunk<T, 3>(b, lane, acc); break;
        }
    };
    const long G = gridDim.x;
    Regs ga, gb;
    long c = blockIdx.x;
    if (c < nchunks) load(c, ga);
    if (c + G < nchunks) load(c + G, gb);
    __syncthreads();
    int cur = 0;
    for (; c < nchunks; c += 2 * G) {
        store(ga, buf[cur]);
        __syncthreads();
        if (c + 2 * G < nchunks) load(c + 2 * G, ga);
        compute(buf[cur]);
        cur ^= 1;
        if (c + G >= nchunks) break;
        store(gb, buf[cur]);
        __syncthreads();
        if (c + 3 * G < nchunks) load(c + 3 * G, gb);
        compute(buf[cur]);
        cur ^= 1;
    }

    // result layout of the 16 x 16 x 4 FP64 product (checked on the device
    // with an in-bounds probe): lane l, element e holds tile entry
    // (row l / 16 + 4 e, column l % 16)
#pragma unroll
    for (int q = 0; q < QP; ++q) {
        const int p = wave + GRAM_WAVES * q;
        if (p < NP) {
            double* out = a.part + (static_cast<long>(blockIdx.x) * NP + p) * 256;
#pragma unroll
            for (int e = 0; e < 4; ++e) out[((lane >> 4) + 4 * e) * 16 + (lane & 15)] = acc[q][e];
        }
    }
}

// First reduction pass: slice s of tile pair p sums the partials of
// workgroups s, s + S, s + 2S, ... (fixed order).
__global__ __launch_bounds__(256) void gram_slice_kernel(const double* __restrict__ part, int nb, int NP,
                                                         double* __restrict__ sl) {
    const int p = blockIdx.x, s = blockIdx.y, k = threadIdx.x;
    double v = 0.0;
    for (int b = s; b < nb; b += RED_SLICES) v += part[(static_cast<long>(b) * NP + p) * 256 + k];
    sl[(static_cast<long>(s) * NP + p) * 256 + k] = v;
}

struct ReduceArgs {
    const double* sl_e;     // [RED_SLICES][NP][256] energy-row slices
    const double* sl_f;     // [RED_SLICES][NP][256] force-row slices
    int has_e, has_f, NP, M, T;
    double w_e, w_f;
    int accumulate;
    double* Z;              // (M+1) x (M+1), row-major
};

// Z = w_e sum(energy slices) + w_f sum(force slices) (+ Z), fixed order;
// each element is written from its upper-triangle tile entry and mirrored.
__global__ __launch_bounds__(256) void gram_reduce_kernel(ReduceArgs a) {
    const int p = blockIdx.x;
    const int k = threadIdx.x;
    int ti = 0, rem = p;
    while (rem >= a.T - ti) {
        rem -= a.T - ti;
        ++ti;
    }
    const int tj = ti + rem;
    const int row = 16 * ti + k / 16, col = 16 * tj + k % 16;
    const int D = a.M + 1;
    if (row >= D || col >= D || row > col) return;
    double se = 0.0, sf = 0.0;
    for (int s = 0; s < RED_SLICES; ++s) {
        if (a.has_e) se += a.sl_e[(static_cast<long>(s) * a.NP + p) * 256 + k];
        if (a.has_f) sf += a.sl_f[(static_cast<long>(s) * a.NP + p) * 256 + k];
    }
    double v = a.w_e * se + a.w_f * sf;
    if (a.accumulate) v += a.Z[static_cast<long>(row) * D + col];
    a.Z[static_cast<long>(row) * D + col] = v;
    if (row != col) a.Z[static_cast<long>(col) * D + row] = v;
}

// (Z_AA + gamma I) c = Z_Ab by Cholesky on the symmetrically scaled matrix
// (unit diagonal, same solution), one workgroup with the matrix in LDS;
// loss = c^T Z_AA c - 2 c^T Z_Ab + Z_bb + gamma c^T c, the value of eq. (63a).
//
// Factorisation: blocked right-looking Cholesky with panels of 16 columns
// (three barriers per panel).  The two triangular solves run in wave 0 with
// the right-hand side in registers (lane l holds rows l and l + 64) and the
// pivot value broadcast by readlane, so they need no barriers.
__global__ __launch_bounds__(SOLVE_THREADS) void solve_kernel(int M, const double* __restrict__ Z, double gamma,
                                                              double* __restrict__ c, double* __restrict__ loss,
                                                              int* err) {
    extern __shared__ double lds[];
    const int D = M + 1;             // Z is D x D; S keeps Z's row stride
    double* S = lds;                 // D x D
    double* sc = S + D * D;          // M: 1 / sqrt(diag of the unscaled matrix)
    double* ipiv = sc + M;           // M: 1 / sqrt(pivot)
    double* cv = ipiv + M;           // M: solution
    __shared__ int bad;
    const int tid = threadIdx.x;
    const int ty = tid >> 4, tx = tid & 15;
    if (tid == 0) bad = 0;
#pragma unroll 4
    for (int e = tid; e < M * D; e += SOLVE_THREADS) S[e] = Z[e];
    __syncthreads();
    for (int i = tid; i < M; i += SOLVE_THREADS) {
        const double d = S[i * D + i] + gamma;
        if (!(d > 0.0) || !isfinite(d)) {
            bad = 1;
            sc[i] = 0.0;
        } else {
            sc[i] = 1.0 / sqrt(d);
        }
    }
    __syncthreads();
    // scaled lower triangle and right-hand side (column M)
    for (int i = ty; i < M; i += 16) {
        const double si = sc[i];
        for (int j = tx; j <= i; j += 16) S[i * D + j] = (S[i * D + j] + (i == j ? gamma : 0.0)) * si * sc[j];
        if (tx == 0) S[i * D + M] *= si;
    }
    __syncthreads();
    // blocked right-looking Cholesky, panels of 16 columns, lower triangle:
    // (1) wave 0 factors the diagonal block (its LDS operations execute in
    // order, so wavefront fences suffice between the steps), (2) one thread
    // per row below solves the panel against it, (3) the trailing triangle
    // takes the rank-16 update -- three barriers per panel
    for (int k0 = 0; k0 < M; k0 += 16) {
        const int kb = M - k0 < 16 ? M - k0 : 16;
        if (tid < WAVE) {
            const int r = tid & 15, cg = tid >> 4;   // row r of the block, columns 4 cg .. 4 cg + 3
            for (int k = 0; k < kb; ++k) {
                const double d = S[(k0 + k) * D + k0 + k];
                if (!(d > 0.0) || !isfinite(d)) {   // the same value in every lane
                    if (tid == 0) bad = 1;
                    break;
                }
                const double lkk = sqrt(d), ilkk = 1.0 / lkk;
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                if (cg == 0 && r >= k && r < kb) {
                    const int at = (k0 + r) * D + k0 + k;
                    S[at] = r == k ? lkk : S[at] * ilkk;
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                if (r > k && r < kb) {
                    const double lrk = S[(k0 + r) * D + k0 + k];
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        const int j = 4 * cg + jj;
                        if (j > k && j <= r) S[(k0 + r) * D + k0 + j] -= lrk * S[(k0 + j) * D + k0 + k];
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            }
        }
        __syncthreads();
        if (bad) break;
        const int b0 = k0 + kb;
        if (tid < kb) ipiv[k0 + tid] = 1.0 / S[(k0 + tid) * D + k0 + tid];
        __syncthreads();
        for (int i = b0 + tid; i < M; i += SOLVE_THREADS) {
            double x[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) x[q] = q < kb ? S[i * D + k0 + q] : 0.0;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                if (q < kb) {
                    double v = x[q];
#pragma unroll
                    for (int pp = 0; pp < q; ++pp) v -= x[pp] * S[(k0 + q) * D + k0 + pp];
                    x[q] = v * ipiv[k0 + q];
                }
            }
#pragma unroll
            for (int q = 0; q < 16; ++q)
                if (q < kb) S[i * D + k0 + q] = x[q];
        }
        __syncthreads();
        for (int i = b0 + ty; i < M; i += 16) {
            double li[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) li[q] = q < kb ? S[i * D + k0 + q] : 0.0;
            for (int j = b0 + tx; j <= i; j += 16) {
                double v = 0.0;
#pragma unroll
                for (int q = 0; q < 16; ++q) v += q < kb ? li[q] * S[j * D + k0 + q] : 0.0;
                S[i * D + j] -= v;
            }
        }
        __syncthreads();
    }
    __syncthreads();
    if (bad) {
        if (tid == 0) atomicOr(err, ERR_SINGULAR);
        for (int i = tid; i < M; i += SOLVE_THREADS) c[i] = 0.0;
        if (loss && tid == 0) *loss = NAN;
        return;
    }
    // a mirrored copy of the factor's columns in the upper triangle
    // (S[j][i] = S[i][j], i > j), so both sweeps read rows; ipiv holds 1 / L_kk
    for (int i = ty; i < M; i += 16)
        for (int j = tx; j < i; j += 16) S[j * D + i] = S[i * D + j];
    __syncthreads();
    if (tid < WAVE) {
        const int l = tid;
        const bool in0 = l < M, in1 = l + WAVE < M;
        double r0 = in0 ? S[l * D + M] : 0.0;
        double r1 = in1 ? S[(l + WAVE) * D + M] : 0.0;
        // L u = r: u_j = r_j / L_jj, r_i -= L_ij u_j (L_ij mirrored at S[j][i]);
        // row j + 1 and its pivot are read while step j runs
        double a0 = in0 ? S[l] : 0.0, a1 = in1 ? S[l + WAVE] : 0.0, pj = ipiv[0];
        for (int j = 0; j < M; ++j) {
            const int jn = j + 1 < M ? j + 1 : j;
            const double n0 = in0 ? S[jn * D + l] : 0.0, n1 = in1 ? S[jn * D + l + WAVE] : 0.0, pn = ipiv[jn];
            const double uj = lane_value(j < WAVE ? r0 : r1, j & (WAVE - 1)) * pj;
            if (l == (j & (WAVE - 1))) {
                if (j < WAVE) r0 = uj;
                else r1 = uj;
            }
            if (l > j && in0) r0 -= a0 * uj;
            if (l + WAVE > j && in1) r1 -= a1 * uj;
            a0 = n0;
            a1 = n1;
            pj = pn;
        }
        // L^T w = u: w_j = u_j / L_jj, u_i -= L_ji w_j for i < j
        a0 = in0 ? S[(M - 1) * D + l] : 0.0;
        a1 = in1 ? S[(M - 1) * D + l + WAVE] : 0.0;
        pj = ipiv[M - 1];
        for (int j = M - 1; j >= 0; --j) {
            const int jn = j > 0 ? j - 1 : 0;
            const double n0 = in0 ? S[jn * D + l] : 0.0, n1 = in1 ? S[jn * D + l + WAVE] : 0.0, pn = ipiv[jn];
            const double wj = lane_value(j < WAVE ? r0 : r1, j & (WAVE - 1)) * pj;
            if (l == (j & (WAVE - 1))) {
                if (j < WAVE) r0 = wj;
                else r1 = wj;
            }
            if (l < j) r0 -= a0 * wj;
            if (l + WAVE < j) r1 -= a1 * wj;
            a0 = n0;
            a1 = n1;
            pj = pn;
        }
        if (in0) {
            cv[l] = r0 * sc[l];
            c[l] = cv[l];
        }
        if (in1) {
            cv[l + WAVE] = r1 * sc[l + WAVE];
            c[l + WAVE] = cv[l + WAVE];
        }
    }
    if (!loss) return;
    __syncthreads();
    // objective from the unmodified Gram blocks, reloaded into LDS
#pragma unroll 4
    for (int e = tid; e < D * D; e += SOLVE_THREADS) S[e] = Z[e];
    __syncthreads();
    double* part = sc;   // M values; the scales are no longer needed
    for (int i = tid; i < M; i += SOLVE_THREADS) {
        double q = 0.0;
        for (int j = 0; j < M; ++j) q += S[i * D + j] * cv[j];
        part[i] = cv[i] * (q - 2.0 * S[i * D + M] + gamma * cv[i]);
    }
    __syncthreads();
    if (tid == 0) {
        double s = S[M * D + M];
        for (int i = 0; i < M; ++i) s += part[i];
        *loss = s;
    }
}

template <int T>
void launch_gram(const GramArgs& a, int nblk, hipStream_t s) {
    hipLaunchKernelGGL((gram_kernel<T>), dim3(nblk), dim3(GRAM_THREADS), 0, s, a);
}

void launch_gram_t(int T, const GramArgs& a, int nblk, hipStream_t s) {
    switch (T) {
        case 1: launch_gram<1>(a, nblk, s); break;
        case 2: launch_gram<2>(a, nblk, s); break;
        case 3: launch_gram<3>(a, nblk, s); break;
        case 4: launch_gram<4>(a, nblk, s); break;
        case 5: launch_gram<5>(a, nblk, s); break;
        case 6: launch_gram<6>(a, nblk, s); break;
        case 7: launch_gram<7>(a, nblk, s); break;
        default: launch_gram<8>(a, nblk, s); break;
    }
}

// Workgroups for R rows: one per chunk, at most GRAM_BLOCKS.
int gram_blocks(long R) {
    if (R <= 0) return 0;
    return static_cast<int>(std::min<long>(GRAM_BLOCKS, (R + GRAM_ROWS - 1) / GRAM_ROWS));
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace
}  // namespace pod

extern "C" {

int pod_fit_gram(pod_handle* h, int M, int n_cfg, const double* G, const double* E_ref, double w_e, long n_frows,
                 const double* dGdR, const double* F_ref, double w_f, int accumulate, double* Z) {
    using namespace pod;
    if (!h || M < 1 || n_cfg < 0 || n_frows < 0 || !Z) return POD_EINVAL;
    if (M + 1 > 16 * FIT_MAX_TILES) return POD_ENOTSUP;
    if ((n_cfg > 0 && (!G || !E_ref)) || (n_frows > 0 && (!dGdR || !F_ref))) return POD_EINVAL;
    if (!std::isfinite(w_e) || !std::isfinite(w_f) || w_e < 0.0 || w_f < 0.0) return POD_EINVAL;
    const int T = (M + 1 + 15) / 16;
    const int NP = T * (T + 1) / 2;
    const int nb_e = gram_blocks(n_cfg), nb_f = gram_blocks(n_frows);
    const size_t tile_bytes = sizeof(double) * 256 * NP;
    const size_t be = align256(tile_bytes * nb_e), bf = align256(tile_bytes * nb_f);
    const size_t bs = align256(tile_bytes * RED_SLICES);
    const int rc = ensure_scratch(h, be + bf + 2 * bs);
    if (rc != POD_OK) return rc;
    char* base = static_cast<char*>(h->d_scratch);
    double* part_e = reinterpret_cast<double*>(base);
    double* part_f = reinterpret_cast<double*>(base + be);
    double* sl_e = reinterpret_cast<double*>(base + be + bf);
    double* sl_f = reinterpret_cast<double*>(base + be + bf + bs);
    timing_begin(h, 3);
    const int vec_e = (reinterpret_cast<uintptr_t>(G) & 15) == 0;
    const int vec_f = (reinterpret_cast<uintptr_t>(dGdR) & 15) == 0;
    if (nb_e > 0) launch_gram_t(T, GramArgs{G, E_ref, 1.0, M, n_cfg, M, vec_e, part_e}, nb_e, h->stream);
    if (nb_f > 0) launch_gram_t(T, GramArgs{dGdR, F_ref, -1.0, M, n_frows, M, vec_f, part_f}, nb_f, h->stream);
    timing_end(h, 3);
    if (nb_e > 0)
        hipLaunchKernelGGL(gram_slice_kernel, dim3(NP, RED_SLICES), dim3(256), 0, h->stream, part_e, nb_e, NP, sl_e);
    if (nb_f > 0)
        hipLaunchKernelGGL(gram_slice_kernel, dim3(NP, RED_SLICES), dim3(256), 0, h->stream, part_f, nb_f, NP, sl_f);
    ReduceArgs r{sl_e, sl_f, nb_e > 0, nb_f > 0, NP, M, T, w_e, w_f, accumulate ? 1 : 0, Z};
    hipLaunchKernelGGL(gram_reduce_kernel, dim3(NP), dim3(256), 0, h->stream, r);
    return hipGetLastError() == hipSuccess ? POD_OK : POD_EHIP;
}

int pod_fit_solve(pod_handle* h, int M, const double* Z, double gamma, double* c, double* loss) {
    using namespace pod;
    if (!h || M < 1 || !Z || !c) return POD_EINVAL;
    if (!std::isfinite(gamma) || gamma < 0.0) return POD_EINVAL;
    const size_t lds = sizeof(double) * (static_cast<size_t>(M + 1) * (M + 1) + 3 * static_cast<size_t>(M));
    if (M > 2 * WAVE) return POD_ENOTSUP;   // two right-hand-side rows per lane
    if (lds > h->lds_max) return POD_ENOTSUP;
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(solve_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                            static_cast<int>(lds)) != hipSuccess)
        return POD_EHIP;
    hipLaunchKernelGGL(solve_kernel, dim3(1), dim3(SOLVE_THREADS), lds, h->stream, M, Z, gamma, c, loss, h->d_err);
    return hipGetLastError() == hipSuccess ? POD_OK : POD_EHIP;
}

}  // extern "C"
