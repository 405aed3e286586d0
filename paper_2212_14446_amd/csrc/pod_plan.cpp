// Host-only planning logic of libpod (declarations and contracts in
// pod_plan.h): parameter validation, the POD radial basis (Sec. II.B),
// neighbour-list bin geometry, the batch-assembly plan, and the two pure-host
// entry points pod_compute_basis and pod_strerror.  No HIP calls.
#include "pod_plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

namespace pod {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kEpsCut = 1e-6;  // epsilon of the cut-off function, eq. (8)

bool finite(double v) { return std::isfinite(v); }

// Cyclic Jacobi eigensolver for a small symmetric matrix (row-major, n x n).
// On return A's diagonal holds the eigenvalues and V (row-major) the
// eigenvectors as columns.
void jacobi_eigen(std::vector<double>& A, std::vector<double>& V, int n) {
    V.assign(static_cast<size_t>(n) * n, 0.0);
    for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += A[i * n + j] * A[i * n + j];
                if (i != j) off += A[i * n + j] * A[i * n + j];
            }
        if (off <= 1e-30 * tot) break;
        for (int pidx = 0; pidx < n - 1; ++pidx)
            for (int q = pidx + 1; q < n; ++q) {
                const double apq = A[pidx * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                const double app = A[pidx * n + pidx], aqq = A[q * n + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {  // A <- A J (columns p, q)
                    const double akp = A[k * n + pidx], akq = A[k * n + q];
                    A[k * n + pidx] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // A <- J^T A (rows p, q)
                    const double apk = A[pidx * n + k], aqk = A[q * n + k];
                    A[pidx * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = V[k * n + pidx], vkq = V[k * n + q];
                    V[k * n + pidx] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
    }
}

double det3(const double* a) {
    return a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) + a[2] * (a[3] * a[7] - a[4] * a[6]);
}

void invert3(const double* a, double* inv, double det) {
    const double id = 1.0 / det;
    inv[0] = (a[4] * a[8] - a[5] * a[7]) * id;
    inv[1] = (a[2] * a[7] - a[1] * a[8]) * id;
    inv[2] = (a[1] * a[5] - a[2] * a[4]) * id;
    inv[3] = (a[5] * a[6] - a[3] * a[8]) * id;
    inv[4] = (a[0] * a[8] - a[2] * a[6]) * id;
    inv[5] = (a[2] * a[3] - a[0] * a[5]) * id;
    inv[6] = (a[3] * a[7] - a[4] * a[6]) * id;
    inv[7] = (a[1] * a[6] - a[0] * a[7]) * id;
    inv[8] = (a[0] * a[4] - a[1] * a[3]) * id;
}

}  // namespace

int validate_params(const pod_params* p) {
    if (!p) return POD_EINVAL;
    if (!finite(p->rin) || !finite(p->rcut) || p->rin < 0.0 || !(p->rin < p->rcut)) return POD_EINVAL;
    if (p->L < 1) return POD_EINVAL;
    if (p->L > POD_MAX_L) return POD_ENOTSUP;
    if (!p->alpha || !p->beta || !p->gamma || !p->kappa) return POD_EINVAL;
    for (int l = 0; l < p->L; ++l) {
        if (!finite(p->alpha[l]) || !finite(p->beta[l]) || !finite(p->gamma[l]) || !finite(p->kappa[l]))
            return POD_EINVAL;
        if (p->kappa[l] < 0.0 || p->kappa[l] > 1.0 || p->beta[l] < 0.0) return POD_EINVAL;
    }
    if (p->K2 < 0 || p->K3 < 0 || p->K4 < 0 || p->P3 < 0 || p->P4 < 0) return POD_EINVAL;
    const int K = std::max(p->K2, std::max(p->K3, p->K4));
    if (K < 1 || K > p->L) return POD_EINVAL;
    if (K > POD_MAX_K) return POD_ENOTSUP;
    if (p->P3 > POD_MAX_P || p->P4 > POD_MAX_P4) return POD_ENOTSUP;
    if (p->dtype != POD_F64 && p->dtype != POD_F32) return POD_EINVAL;
    if (p->n_quad != 0 && p->n_quad < 2 * p->L) return POD_EINVAL;
    if (p->Q) {
        for (int i = 0; i < p->L * K; ++i)
            if (!finite(p->Q[i])) return POD_EINVAL;
    }
    return POD_OK;
}

double snapshot_value(const pod_params* p, int l, double r) {
    const double h = p->rcut - p->rin;
    const double t = (r - p->rin) / h;
    const double y = 1.0 - t * t * t;
    const double fc = std::exp(1.0 - 1.0 / std::sqrt(y * y + kEpsCut));
    double psi = 0.0;
    const double kap = p->kappa[l];
    if (kap != 0.0) {
        const double b = p->beta[l];
        const double x = (b == 0.0) ? t : std::expm1(-b * t) / std::expm1(-b);
        psi += kap * std::sin(p->alpha[l] * kPi * x) / (r - p->rin);
    }
    if (kap != 1.0) psi += (1.0 - kap) * std::pow(r, -p->gamma[l]);
    return fc * psi;
}

int compute_basis(const pod_params* p, std::vector<double>& Q, std::vector<double>& eig) {
    const int L = p->L;
    const int nq = p->n_quad > 0 ? p->n_quad : 2000;
    const double h = (p->rcut - p->rin) / nq;
    std::vector<double> C(static_cast<size_t>(L) * L, 0.0), phi(L);
    for (int s = 0; s < nq; ++s) {
        const double r = p->rin + (s + 0.5) * h;
        for (int l = 0; l < L; ++l) phi[l] = snapshot_value(p, l, r);
        for (int a = 0; a < L; ++a)
            for (int b = 0; b < L; ++b) C[a * L + b] += phi[a] * phi[b];
    }
    for (double& v : C) v /= nq;
    std::vector<double> V;
    jacobi_eigen(C, V, L);
    std::vector<int> order(L);
    for (int i = 0; i < L; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return C[a * L + a] > C[b * L + b]; });
    Q.assign(static_cast<size_t>(L) * L, 0.0);
    eig.assign(L, 0.0);
    for (int k = 0; k < L; ++k) {
        const int src = order[k];
        eig[k] = C[src * L + src];
        int big = 0;
        for (int l = 1; l < L; ++l)
            if (std::fabs(V[l * L + src]) > std::fabs(V[big * L + src])) big = l;
        const double sgn = V[big * L + src] < 0 ? -1.0 : 1.0;
        for (int l = 0; l < L; ++l) Q[l * L + k] = sgn * V[l * L + src];
        for (int l = 0; l < L; ++l)
            if (!std::isfinite(Q[l * L + k])) return POD_EINVAL;
    }
    return POD_OK;
}

int periodic_geometry(const double* cell, double rlist, NbGeom* g) {
    if (!cell || !g || !(rlist > 0.0) || !std::isfinite(rlist)) return POD_EINVAL;
    *g = NbGeom{};
    g->rl2 = rlist * rlist;
    g->periodic = 1;
    for (int k = 0; k < 9; ++k) {
        if (!std::isfinite(cell[k])) return POD_EINVAL;
        g->a[k] = cell[k];
    }
    const double det = det3(g->a);
    if (!(std::fabs(det) > 0.0) || !std::isfinite(det)) return POD_EINVAL;
    invert3(g->a, g->inv, det);
    for (int d = 0; d < 3; ++d) {
        // spacing of the lattice planes normal to direction d: V / |a_e x a_f|
        const double* ae = g->a + 3 * ((d + 1) % 3);
        const double* af = g->a + 3 * ((d + 2) % 3);
        const double cx = ae[1] * af[2] - ae[2] * af[1], cy = ae[2] * af[0] - ae[0] * af[2],
                     cz = ae[0] * af[1] - ae[1] * af[0];
        const double hd = std::fabs(det) / std::sqrt(cx * cx + cy * cy + cz * cz);
        if (!std::isfinite(hd) || !(hd > 0.0)) return POD_EINVAL;
        g->nb[d] = static_cast<int>(std::max(1.0, std::min<double>(NB_MAX_BINS, std::floor(hd / rlist))));
        const double span = std::ceil(rlist * g->nb[d] / hd * (1.0 + 1e-12));
        if (!(span <= NB_MAX_SPAN)) return POD_ENOTSUP;
        g->ns[d] = static_cast<int>(span);
    }
    return POD_OK;
}

int open_geometry(const double* pos, int N, double rlist, NbGeom* g) {
    if (!g || N < 0 || (N > 0 && !pos) || !(rlist > 0.0) || !std::isfinite(rlist)) return POD_EINVAL;
    *g = NbGeom{};
    g->rl2 = rlist * rlist;
    g->periodic = 0;
    for (int d = 0; d < 3; ++d) {
        double lo = 0.0, hi = 0.0;
        bool any = false;
        for (int i = 0; i < N; ++i) {
            const double v = pos[3 * static_cast<size_t>(i) + d];
            if (!std::isfinite(v)) continue;   // latched by the bin kernel
            lo = any ? std::min(lo, v) : v;
            hi = any ? std::max(hi, v) : v;
            any = true;
        }
        const double ext = hi - lo;
        const double nbf = std::floor(ext / rlist) + 1.0;
        const int nbd = std::isfinite(nbf) ? static_cast<int>(std::min<double>(NB_MAX_BINS, nbf)) : NB_MAX_BINS;
        g->lo[d] = lo;
        g->nb[d] = std::max(1, nbd);
        g->bw[d] = std::max(rlist, ext / g->nb[d] * (1.0 + 1e-12));
        g->ns[d] = 1;
    }
    return POD_OK;
}

int plan_batch(int n_cfg, int N, int P, const int* coff, const int* off, int M, size_t lds_max,
               const pod_tune* tune, BatchPlan* plan) {
    if (n_cfg < 1 || N < 0 || P < 0 || !coff || !off || !plan || M < 1) return POD_EINVAL;
    if (coff[0] != 0 || coff[n_cfg] != N || off[0] != 0 || off[N] != P) return POD_EINVAL;
    std::vector<int> npair(n_cfg);
    int max_nc = 0, max_pc = 0;
    for (int c = 0; c < n_cfg; ++c) {
        if (coff[c + 1] < coff[c] || coff[c + 1] > N) return POD_EINVAL;
        const int nc = coff[c + 1] - coff[c];
        for (int a = coff[c]; a < coff[c + 1]; ++a)
            if (off[a + 1] < off[a]) return POD_ENEIGH;
        npair[c] = off[coff[c + 1]] - off[coff[c]];
        max_nc = std::max(max_nc, nc);
        max_pc = std::max(max_pc, npair[c]);
    }
    int cw = tune && tune->cw > 0 ? tune->cw : 17;
    int nblk = tune && tune->nblocks > 0 ? tune->nblocks : 512;
    const int nth = tune && tune->threads > 0 ? tune->threads : 512;
    if (nth % 64 != 0 || nth > BATCH_MAX_THREADS) return POD_EINVAL;
    nblk = std::min(nblk, n_cfg);
    const int nc_max = ((max_nc + 15) / 16) * 16;
    while (cw > 1 && batch_lds(M, cw, nc_max).total > lds_max) --cw;
    const size_t lds = batch_lds(M, cw, nc_max).total;
    if (lds > lds_max) return POD_ENOTSUP;   // a cell too large for the LDS accumulator
    plan->cw = cw;
    plan->nblk = nblk;
    plan->nth = nth;
    plan->nc_max = nc_max;
    plan->max_nc = max_nc;
    plan->max_pc = max_pc;
    plan->lds = lds;
    plan->order.resize(n_cfg);
    std::iota(plan->order.begin(), plan->order.end(), 0);
    std::stable_sort(plan->order.begin(), plan->order.end(), [&](int x, int y) { return npair[x] > npair[y]; });
    return POD_OK;
}

}  // namespace pod

extern "C" {

int pod_compute_basis(const pod_params* p, double* Q, double* eigvals) {
    const int rc = pod::validate_params(p);
    if (rc != POD_OK) return rc;
    std::vector<double> q, e;
    const int r2 = pod::compute_basis(p, q, e);
    if (r2 != POD_OK) return r2;
    if (Q) std::memcpy(Q, q.data(), q.size() * sizeof(double));
    if (eigvals) std::memcpy(eigvals, e.data(), e.size() * sizeof(double));
    return POD_OK;
}

const char* pod_strerror(int code) {
    switch (code) {
        case POD_OK: return "ok";
        case POD_EINVAL: return "invalid argument";
        case POD_ERANGE: return "pair distance at or below rin";
        case POD_ENONFINITE: return "non-finite coordinate";
        case POD_ENOMEM: return "device allocation failed";
        case POD_EHIP: return "HIP runtime error";
        case POD_ENOTSUP: return "parameters beyond the compiled kernel limits";
        case POD_ENEIGH: return "malformed neighbour list";
        case POD_ESINGULAR: return "fit matrix not positive definite";
        case POD_ETOOBIG: return "problem larger than the static scratch of the allocation-free entry point";
        default: return "unknown error";
    }
}

}  // extern "C"
