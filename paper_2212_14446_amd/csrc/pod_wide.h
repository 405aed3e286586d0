// Energy path for models whose angular degree is above FAST_MAX_PA or whose
// radial-function count is above FAST_MAX_K (up to POD_MAX_P = 10 and
// POD_MAX_K = 12): one
// 256-thread workgroup per atom at a time, the atom's basis rows and their
// adjoint in LDS.  Internal to libpod; the host side of the energy path
// chooses it by the model's degree.
#pragma once

#include <hip/hip_runtime.h>

#include "pod_internal.h"
#include "pod_tables.h"

namespace pod {

constexpr int WIDE_THREADS = 256;
constexpr int WIDE_CHUNK = 32;          // pairs staged per step
constexpr int WIDE_MAX_BLOCKS = 2048;   // persistent workgroups

template <typename T>
struct WideArgs {
    ParamsT<T> prm;      // by value: read with scalar loads
    CellT<T> cell;
    int N, P;
    const T* pos;
    const int* offsets;
    const int* nbr_j;
    const int* shift;
    const T* coef;       // energy coefficients (mode 1)
    T* D;                // descriptors N x M (mode 0)
    T* E_atom;           // per-atom energy or null (mode 1)
    double* part;        // block partials [10 + M][nblk]: column 0 E, 10.. G (mode 1)
    double* wpart;       // block virial partials [9][nblk]
    T* gown;             // gather path: g of pair p at slot p
    T* gbuf;             // gather path: g of pair p at slot rev[p]
    const int* rev;
    double* Facc;        // atomic path: FP64 force accumulator (zero on entry)
    T* rec;              // pair records, P x rs (scratch)
    int rs;              // record stride: 4 + K, or 4 + 2 K with R'_k (mode 1)
    int want_G, want_back, want_W;
    int* err;
};

// LDS layout of one wide_kernel workgroup, in bytes: the energy coefficients
// (M), the monomial codes (NA ints), with 4-body terms the packed eq. (30a)
// tables (wide_tab_ints ints), the basis rows [K][NA] (later the adjoint
// rows), the degree sums [K][PA + 1], the staged R_k and R'_k
// [2][WIDE_CHUNK][POD_MAX_K], unit vectors and distances [WIDE_CHUNK][4],
// the powers of the unit vectors' components [WIDE_CHUNK][3][PA + 1], and a
// reduction area.
struct WideLds {
    size_t coef, code, tab, b, s, r, u, pw, red, total;
};

__host__ __device__ constexpr size_t wide_align(size_t b) { return (b + 15) & ~size_t(15); }

// ints of the packed 4-body tables: per index p its triple and term range
// (3 KA4), the terms (NT4), the occurrence ranges (NA4 + 1), the
// occurrences (3 NT4) and the index of (a, 0, 0) per degree a
__host__ __device__ constexpr int wide_tab_ints() {
    return 3 * n_partitions(POD_MAX_P4) + 4 * D4Table<POD_MAX_P4>::NT + n_mono(POD_MAX_P4) + 1 + POD_MAX_P4 + 1;
}

__host__ __device__ constexpr WideLds wide_lds(int K, int PA, int M, bool four, int tsize) {
    const size_t ts = static_cast<size_t>(tsize);
    const size_t NA = static_cast<size_t>(n_mono(PA));
    WideLds L{};
    L.coef = 0;
    L.code = wide_align(L.coef + static_cast<size_t>(M) * ts);
    L.tab = wide_align(L.code + NA * sizeof(int));
    L.b = wide_align(L.tab + (four ? static_cast<size_t>(wide_tab_ints()) * sizeof(int) : 0));
    L.s = wide_align(L.b + static_cast<size_t>(K) * NA * ts);
    L.r = wide_align(L.s + static_cast<size_t>(K) * (PA + 1) * ts);
    L.u = wide_align(L.r + 2 * static_cast<size_t>(WIDE_CHUNK) * POD_MAX_K * ts);
    L.pw = wide_align(L.u + 4 * static_cast<size_t>(WIDE_CHUNK) * ts);
    L.red = wide_align(L.pw + static_cast<size_t>(WIDE_CHUNK) * 3 * (PA + 1) * ts);
    L.total = wide_align(L.red + 16 * sizeof(double));
    return L;
}

inline int wide_blocks(int N) { return N < WIDE_MAX_BLOCKS ? N : WIDE_MAX_BLOCKS; }

// The energy path of a model with K radial functions and angular degree PA
// runs here when either exceeds what the register-resident kernels hold.
inline bool wide_path(int K, int PA) { return PA > FAST_MAX_PA || K > FAST_MAX_K; }

// Pair-record stride and bytes for P pairs.
inline int wide_rec_stride(int K, bool deriv) { return 4 + (deriv ? 2 : 1) * K; }

// mode 0: descriptors; mode 1: energy, and with want_back the pair
// gradients.  The pair records go to a.rec (P x a.rs values); then nblk
// workgroups take the atoms i = blk, blk + nblk, ...
template <typename T>
hipError_t launch_wide(const WideArgs<T>& a, int mode, bool fast, int nblk, hipStream_t st);

}  // namespace pod
