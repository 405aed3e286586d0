// Full neighbour list on the device (Sec. II.A: the neighbours of atom i are
// the atoms, and periodic images, closer to atom i than the cut-off radius).
//
// Cell list in fractional coordinates of the (possibly triclinic) cell: a
// bin spans at least r_list perpendicular to each lattice plane, atoms are
// ordered by bin with a stable radix sort (positions copied into bin order,
// so a bin scan reads contiguous memory), and every atom scans the bins
// within ns_d bins of its own.  The bin offset carries the periodic image,
// so small cells produce their multiple images and self-images and no image
// is visited twice.  A count pass and a prefix sum give the offsets; a fill
// pass writes (j, packed image shift) in the same fixed order.
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include <algorithm>
#include <cmath>
#include <vector>

#include "pod.h"
#include "pod_internal.h"
#include "pod_plan.h"

namespace pod {
namespace {

constexpr int NB_THREADS = 256;
constexpr int NB_MAX_WRAP = 1 << 20;   // |lattice vectors| between an atom and its home cell

__device__ __forceinline__ int floor_div(int a, int b) {
    const int q = a / b;
    return (a % b != 0 && (a < 0)) ? q - 1 : q;   // b > 0
}

// Bin of every atom; its position moved into the home cell (periodic) and
// the number of lattice vectors removed.
template <typename T>
__global__ __launch_bounds__(NB_THREADS) void bin_kernel(int N, const T* __restrict__ pos, NbGeom g,
                                                         int* __restrict__ key, int* __restrict__ idx,
                                                         double* __restrict__ wpos, int* __restrict__ wrap, int* err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double r[3] = {static_cast<double>(pos[3 * i]), static_cast<double>(pos[3 * i + 1]),
                         static_cast<double>(pos[3 * i + 2])};
    int c[3] = {0, 0, 0}, w[3] = {0, 0, 0};
    double rw[3] = {r[0], r[1], r[2]};
    if (!(isfinite(r[0]) && isfinite(r[1]) && isfinite(r[2]))) {
        atomicOr(err, ERR_NONFINITE);
    } else if (g.periodic) {
        double sw[3];
        for (int d = 0; d < 3; ++d) {
            const double s = r[0] * g.inv[0 * 3 + d] + r[1] * g.inv[1 * 3 + d] + r[2] * g.inv[2 * 3 + d];
            double f = floor(s);
            if (fabs(f) > NB_MAX_WRAP) {
                atomicOr(err, ERR_NEIGH);
                f = 0.0;
            }
            w[d] = static_cast<int>(f);
            sw[d] = s - f;
            c[d] = min(max(static_cast<int>(sw[d] * g.nb[d]), 0), g.nb[d] - 1);
        }
        for (int e = 0; e < 3; ++e) rw[e] = r[e] - (w[0] * g.a[0 * 3 + e] + w[1] * g.a[1 * 3 + e] + w[2] * g.a[2 * 3 + e]);
    } else {
        for (int d = 0; d < 3; ++d) c[d] = min(max(static_cast<int>((r[d] - g.lo[d]) / g.bw[d]), 0), g.nb[d] - 1);
    }
    key[i] = (c[2] * g.nb[1] + c[1]) * g.nb[0] + c[0];
    idx[i] = i;
    for (int d = 0; d < 3; ++d) {
        wpos[3 * i + d] = rw[d];
        wrap[3 * i + d] = w[d];
    }
}

__global__ __launch_bounds__(NB_THREADS) void fill_int_kernel(int* __restrict__ x, long n, int v) {
    const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

// Bin ranges [start, end) in sorted order and the positions in sorted order.
__global__ __launch_bounds__(NB_THREADS) void order_kernel(int N, const int* __restrict__ ks,
                                                           const int* __restrict__ sidx,
                                                           const double* __restrict__ wpos, int* __restrict__ start,
                                                           int* __restrict__ end, double* __restrict__ spos) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int b = ks[k];
    if (k == 0 || ks[k - 1] != b) start[b] = k;
    if (k == N - 1 || ks[k + 1] != b) end[b] = k + 1;
    const int j = sidx[k];
    for (int d = 0; d < 3; ++d) spos[3 * k + d] = wpos[3 * j + d];
}

// FILL = false: number of neighbours of every atom into cnt[i];
// FILL = true: the neighbours themselves from offsets[i] on (same order).
// The rows of a workgroup's atoms are one contiguous range of the list:
// when it fits the workgroup's LDS (FILL_CAP entries) the rows are built
// there and copied out with consecutive threads on consecutive entries
// (each thread's own row would otherwise be written with one scattered
// 4-byte store per entry and lane).
constexpr int FILL_CAP = 4096;
constexpr int FILL_THREADS = 128;   // workgroup of the fill pass

// The search of one atom; with `stage`, its row goes to stage[out ..] and
// stage[FILL_CAP + out ..] (LDS) instead of nbr_j / shift.
template <bool FILL>
__device__ __forceinline__ void search_atom(int i, const NbGeom& g, const int* __restrict__ key,
                                            const int* __restrict__ sidx, const int* __restrict__ start,
                                            const int* __restrict__ end, const double* __restrict__ wpos,
                                            const double* __restrict__ spos, const int* __restrict__ wrap,
                                            long* __restrict__ cnt, const int* __restrict__ offsets,
                                            int* __restrict__ nbr_j, int* __restrict__ shift, int* err,
                                            int* stage) {
    const int b = key[i];
    const int ci[3] = {b % g.nb[0], (b / g.nb[0]) % g.nb[1], b / (g.nb[0] * g.nb[1])};
    const double ri[3] = {wpos[3 * i], wpos[3 * i + 1], wpos[3 * i + 2]};
    int n = 0;
    const int out = FILL ? offsets[i] : 0;
    const int room = FILL ? offsets[i + 1] - out : 0;
    for (int dz = -g.ns[2]; dz <= g.ns[2]; ++dz)
        for (int dy = -g.ns[1]; dy <= g.ns[1]; ++dy)
            for (int dx = -g.ns[0]; dx <= g.ns[0]; ++dx) {
                const int bp[3] = {ci[0] + dx, ci[1] + dy, ci[2] + dz};
                int S[3] = {0, 0, 0}, bb[3] = {bp[0], bp[1], bp[2]};
                if (g.periodic) {
                    for (int d = 0; d < 3; ++d) {
                        S[d] = floor_div(bp[d], g.nb[d]);
                        bb[d] = bp[d] - S[d] * g.nb[d];
                    }
                } else if (bp[0] < 0 || bp[0] >= g.nb[0] || bp[1] < 0 || bp[1] >= g.nb[1] || bp[2] < 0 ||
                           bp[2] >= g.nb[2]) {
                    continue;
                }
                const bool home = S[0] == 0 && S[1] == 0 && S[2] == 0;
                double q[3];
                for (int e = 0; e < 3; ++e) {
                    double o = 0.0;
                    if (g.periodic)
                        o = __dadd_rn(__dadd_rn(__dmul_rn(S[0], g.a[0 * 3 + e]), __dmul_rn(S[1], g.a[1 * 3 + e])),
                                      __dmul_rn(S[2], g.a[2 * 3 + e]));
                    q[e] = __dsub_rn(ri[e], o);
                }
                const int bin = (bb[2] * g.nb[1] + bb[1]) * g.nb[0] + bb[0];
                const int k1 = end[bin];
                for (int k = start[bin]; k < k1; ++k) {
                    // explicit roundings: the count and fill passes take the
                    // same decision for every pair
                    const double d0 = __dsub_rn(spos[3 * k], q[0]);
                    const double d1 = __dsub_rn(spos[3 * k + 1], q[1]);
                    const double d2 = __dsub_rn(spos[3 * k + 2], q[2]);
                    const double r2 = __dadd_rn(__dadd_rn(__dmul_rn(d0, d0), __dmul_rn(d1, d1)), __dmul_rn(d2, d2));
                    if (!(r2 < g.rl2)) continue;
                    const int j = sidx[k];
                    if (home && j == i) continue;
                    if (FILL) {
                        if (n >= room) {   // the count pass saw fewer pairs: never write past the row
                            atomicOr(err, ERR_NEIGH);
                            continue;
                        }
                        // image in the caller's coordinates: r_ij = pos_j + n a - pos_i
                        const int n0 = S[0] - wrap[3 * j] + wrap[3 * i];
                        const int n1 = S[1] - wrap[3 * j + 1] + wrap[3 * i + 1];
                        const int n2 = S[2] - wrap[3 * j + 2] + wrap[3 * i + 2];
                        if (n0 < -127 || n0 > 127 || n1 < -127 || n1 > 127 || n2 < -127 || n2 > 127)
                            atomicOr(err, ERR_NEIGH);   // beyond the signed-byte shift
                        const int sh = (n0 & 0xFF) | ((n1 & 0xFF) << 8) | ((n2 & 0xFF) << 16);
                        if (stage) {
                            stage[out + n] = j;
                            stage[FILL_CAP + out + n] = sh;
                        } else {
                            nbr_j[out + n] = j;
                            shift[out + n] = sh;
                        }
                    }
                    ++n;
                }
            }
    if (!FILL) cnt[i] = n;
}

template <bool FILL>
__global__ __launch_bounds__(NB_THREADS) void search_kernel(int N, NbGeom g, const int* __restrict__ key,
                                                            const int* __restrict__ sidx,
                                                            const int* __restrict__ start, const int* __restrict__ end,
                                                            const double* __restrict__ wpos,
                                                            const double* __restrict__ spos,
                                                            const int* __restrict__ wrap, long* __restrict__ cnt,
                                                            const int* __restrict__ offsets, int* __restrict__ nbr_j,
                                                            int* __restrict__ shift, int* err) {
    extern __shared__ int sfill[];   // FILL: [FILL_CAP] neighbour indices, [FILL_CAP] shifts
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int base = 0, total = 0;
    bool staged = false;
    if (FILL) {
        const int i0 = min(static_cast<int>(blockIdx.x * blockDim.x), N);
        const int i1 = min(i0 + static_cast<int>(blockDim.x), N);
        base = offsets[i0];
        total = offsets[i1] - base;
        staged = total >= 0 && total <= FILL_CAP;
    }
    if (i < N) search_atom<FILL>(i, g, key, sidx, start, end, wpos, spos, wrap, cnt, offsets, nbr_j, shift, err,
                                 staged ? sfill - base : nullptr);
    if (FILL && staged) {
        __syncthreads();
        for (int t = threadIdx.x; t < total; t += blockDim.x) {
            nbr_j[base + t] = sfill[t];
            shift[base + t] = sfill[FILL_CAP + t];
        }
    }
}



// int32 offsets from the 64-bit prefix sum; total[0] = number of pairs.
__global__ __launch_bounds__(NB_THREADS) void offsets_kernel(int N, const long* __restrict__ off64,
                                                             int* __restrict__ offsets, long* __restrict__ total) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > N) return;
    const long v = off64[i];
    offsets[i] = v > 0x7fffffffL ? 0x7fffffff : static_cast<int>(v);
    if (i == N) total[0] = v;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Bounding box of an open system (host copy of the positions).
int open_geometry_dev(pod_handle* h, int N, const void* pos, double rlist, NbGeom* g) {
    std::vector<double> hp(3 * static_cast<size_t>(N));
    if (h->dtype == POD_F64) {
        if (hipMemcpyAsync(hp.data(), pos, hp.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream) !=
                hipSuccess ||
            hipStreamSynchronize(h->stream) != hipSuccess)
            return POD_EHIP;
    } else {
        std::vector<float> hf(hp.size());
        if (hipMemcpyAsync(hf.data(), pos, hf.size() * sizeof(float), hipMemcpyDeviceToHost, h->stream) !=
                hipSuccess ||
            hipStreamSynchronize(h->stream) != hipSuccess)
            return POD_EHIP;
        for (size_t k = 0; k < hf.size(); ++k) hp[k] = hf[k];
    }
    return open_geometry(hp.data(), N, rlist, g);
}

}  // namespace
}  // namespace pod

extern "C" {

int pod_build_neighbors(pod_handle* h, int N, const void* pos, const double* cell, double rlist, int* offsets,
                        int* nbr_j, int* shift, long capacity, long* n_pairs) {
    using namespace pod;
    if (!h || N < 0 || !offsets || !n_pairs || capacity < 0) return POD_EINVAL;
    if (N > 0 && !pos) return POD_EINVAL;
    if (capacity > 0 && (!nbr_j || !shift)) return POD_EINVAL;
    if (rlist == 0.0) rlist = h->rcut;
    if (!(rlist > 0.0) || !std::isfinite(rlist)) return POD_EINVAL;
    *n_pairs = 0;
    const dim3 tb(NB_THREADS);
    const dim3 gb(static_cast<unsigned>((static_cast<long>(N) + NB_THREADS) / NB_THREADS));   // N + 1 threads
    if (N == 0) {
        hipLaunchKernelGGL(fill_int_kernel, dim3(1), tb, 0, h->stream, offsets, 1L, 0);
        return hipStreamSynchronize(h->stream) == hipSuccess ? POD_OK : POD_EHIP;
    }
    NbGeom g{};
    {
        const int rc = cell ? periodic_geometry(cell, rlist, &g) : open_geometry_dev(h, N, pos, rlist, &g);
        if (rc != POD_OK) return rc;
    }
    const long nbins = static_cast<long>(g.nb[0]) * g.nb[1] * g.nb[2];
    int key_bits = 1;
    while ((1L << key_bits) < nbins) ++key_bits;

    size_t sort_bytes = 0, scan_bytes = 0;
    if (rocprim::radix_sort_pairs(nullptr, sort_bytes, static_cast<int*>(nullptr), static_cast<int*>(nullptr),
                                  static_cast<int*>(nullptr), static_cast<int*>(nullptr), N, 0u,
                                  static_cast<unsigned>(key_bits), h->stream) != hipSuccess ||
        rocprim::exclusive_scan(nullptr, scan_bytes, static_cast<long*>(nullptr), static_cast<long*>(nullptr), 0L,
                                static_cast<size_t>(N) + 1, rocprim::plus<long>(), h->stream) != hipSuccess)
        return POD_EHIP;
    const size_t n1 = static_cast<size_t>(N) + 1;
    const size_t sI = align256(sizeof(int) * n1), sL = align256(sizeof(long) * n1);
    const size_t sP = align256(sizeof(double) * 3 * n1), sW = align256(sizeof(int) * 3 * n1);
    const size_t sB = align256(sizeof(int) * static_cast<size_t>(nbins)), sT = align256(std::max(sort_bytes, scan_bytes));
    const int rc = ensure_scratch(h, 4 * sI + 2 * sL + 2 * sP + sW + 2 * sB + sT);
    if (rc != POD_OK) return rc;
    char* base = static_cast<char*>(h->d_scratch);
    auto take = [&base](size_t bytes) { char* p = base; base += bytes; return p; };
    int* key = reinterpret_cast<int*>(take(sI));
    int* key_s = reinterpret_cast<int*>(take(sI));
    int* idx = reinterpret_cast<int*>(take(sI));
    int* idx_s = reinterpret_cast<int*>(take(sI));
    long* cnt = reinterpret_cast<long*>(take(sL));
    long* off64 = reinterpret_cast<long*>(take(sL));
    double* wpos = reinterpret_cast<double*>(take(sP));
    double* spos = reinterpret_cast<double*>(take(sP));
    int* wrap = reinterpret_cast<int*>(take(sW));
    int* start = reinterpret_cast<int*>(take(sB));
    int* end = reinterpret_cast<int*>(take(sB));
    void* tmp = take(sT);

    if (h->dtype == POD_F64)
        hipLaunchKernelGGL((bin_kernel<double>), gb, tb, 0, h->stream, N, static_cast<const double*>(pos), g, key, idx,
                           wpos, wrap, h->d_err);
    else
        hipLaunchKernelGGL((bin_kernel<float>), gb, tb, 0, h->stream, N, static_cast<const float*>(pos), g, key, idx,
                           wpos, wrap, h->d_err);
    size_t tbytes = sT;
    if (rocprim::radix_sort_pairs(tmp, tbytes, key, key_s, idx, idx_s, N, 0u, static_cast<unsigned>(key_bits),
                                  h->stream) != hipSuccess)
        return POD_EHIP;
    const dim3 gbins(static_cast<unsigned>((nbins + NB_THREADS - 1) / NB_THREADS));
    hipLaunchKernelGGL(fill_int_kernel, gbins, tb, 0, h->stream, start, nbins, 0);
    hipLaunchKernelGGL(fill_int_kernel, gbins, tb, 0, h->stream, end, nbins, 0);
    hipLaunchKernelGGL(order_kernel, gb, tb, 0, h->stream, N, key_s, idx_s, wpos, start, end, spos);
    hipLaunchKernelGGL((search_kernel<false>), gb, tb, 0, h->stream, N, g, key, idx_s, start, end, wpos, spos, wrap,
                       cnt, nullptr, nullptr, nullptr, h->d_err);
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), tb, 0, h->stream, reinterpret_cast<int*>(cnt + N), 2L, 0);
    tbytes = sT;
    if (rocprim::exclusive_scan(tmp, tbytes, cnt, off64, 0L, static_cast<size_t>(N) + 1, rocprim::plus<long>(),
                                h->stream) != hipSuccess)
        return POD_EHIP;
    hipLaunchKernelGGL(offsets_kernel, gb, tb, 0, h->stream, N, off64, offsets, cnt);
    long P = 0;
    if (hipMemcpyAsync(&P, cnt, sizeof(long), hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
        return POD_EHIP;
    *n_pairs = P;
    if (P > 0x7fffffffL) return POD_ENOTSUP;   // int32 offsets
    if (P > 0 && capacity >= P) {
        const dim3 gf(static_cast<unsigned>((static_cast<long>(N) + FILL_THREADS - 1) / FILL_THREADS));
        hipLaunchKernelGGL((search_kernel<true>), gf, dim3(FILL_THREADS), 2 * FILL_CAP * sizeof(int), h->stream, N, g,
                           key, idx_s, start, end, wpos, spos, wrap, nullptr, offsets, nbr_j, shift, h->d_err);
        if (hipStreamSynchronize(h->stream) != hipSuccess) return POD_EHIP;
    }
    return hipGetLastError() == hipSuccess ? POD_OK : POD_EHIP;
}

}  // extern "C"
