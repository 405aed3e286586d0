// Host-only planning logic of libpod: parameter validation, the POD radial
// basis, the neighbour-list bin geometry and the batch-assembly plan.  Plain
// C++ with no HIP types, so that it also builds on its own with g++ for the
// host-code sanitizer tests; the kernels' sources use the plain structs and
// constexpr layouts declared here.
#pragma once

#include <cstddef>
#include <vector>

#include "pod.h"

namespace pod {

// Parameter checks of pod_init / pod_compute_basis (POD_OK, POD_EINVAL, POD_ENOTSUP).
int validate_params(const pod_params* p);

// Snapshot l of the family at distance r, eqs. (3)-(8), in double.
double snapshot_value(const pod_params* p, int l, double r);

// POD basis of the snapshot family (Sec. II.B, eqs. (9)-(12)): midpoint rule
// on (rin, rcut) with n_quad points (2000 when zero), eigenvectors of the L x L
// covariance by cyclic Jacobi, sorted by decreasing eigenvalue, each column's
// largest component made positive.  Q: L x L row-major (column k = mode k).
int compute_basis(const pod_params* p, std::vector<double>& Q, std::vector<double>& eig);

// Neighbour-list bin geometry, passed by value to the neighbour kernels.
constexpr int NB_MAX_BINS = 256;   // per direction (wider bins stay correct)
constexpr int NB_MAX_SPAN = 64;    // search half-width in bins

struct NbGeom {
    double a[9];     // periodic: lattice vectors as rows
    double inv[9];   // periodic: inverse of a, fractional s = r inv
    double lo[3];    // open: bounding-box origin
    double bw[3];    // open: bin width
    double rl2;      // r_list^2
    int nb[3];       // bins per direction
    int ns[3];       // search half-width in bins
    int periodic;
};

// Periodic cell (lattice vectors as rows): bins at least r_list apart
// perpendicular to each lattice plane and the search half-width that covers
// r_list.  POD_EINVAL for a singular or non-finite cell or r_list,
// POD_ENOTSUP when the search would span more than NB_MAX_SPAN bins.
int periodic_geometry(const double* cell, double rlist, NbGeom* g);

// Open system from a host copy of the positions (N x 3): bounding box of the
// finite coordinates, bins of at least r_list, search half-width 1.
int open_geometry(const double* pos, int N, double rlist, NbGeom* g);

// LDS layout of one batch-assembly workgroup: Q, the cell's G row, the
// dG/dR chunk accumulator (nc_max atoms x 3 x cw columns) and the atom offsets.
struct BatchLds {
    size_t q, gsum, acc, off, total;
};

constexpr BatchLds batch_lds(int M, int cw, int nc_max) {
    BatchLds L{};
    const size_t d = sizeof(double);
    L.q = 0;
    L.gsum = L.q + static_cast<size_t>(POD_MAX_L) * POD_MAX_K * d;
    L.acc = L.gsum + static_cast<size_t>(M + 1) * d;
    L.off = L.acc + static_cast<size_t>(nc_max) * 3 * cw * d;
    L.total = L.off + static_cast<size_t>(nc_max + 1) * sizeof(int);
    return L;
}

constexpr int BATCH_MAX_THREADS = 512;

// Launch plan of pod_batch_assemble from host copies of the cell atom
// offsets coff[n_cfg + 1] and the pair offsets off[N + 1]: the chunk width
// (largest that fits lds_max, from the tuning value or 17 down), the
// workgroup count, the LDS bytes, the largest cell and pair count, and the
// processing order of the cells (decreasing pair count, stable).
struct BatchPlan {
    int cw, nblk, nth, nc_max, max_nc, max_pc;
    size_t lds;
    std::vector<int> order;
};

// POD_EINVAL for offsets that do not start at 0, end at N / P or decrease
// between cells or for a bad thread count, POD_ENEIGH for pair offsets that
// decrease within a cell, POD_ENOTSUP when even one column does not fit LDS.
int plan_batch(int n_cfg, int N, int P, const int* coff, const int* off, int M, size_t lds_max,
               const pod_tune* tune, BatchPlan* plan);

}  // namespace pod
