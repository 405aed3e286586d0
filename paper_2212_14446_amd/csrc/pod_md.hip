// Molecular dynamics with a linear POD potential: velocity Verlet steps
// (Swope et al., J. Chem. Phys. 76, 637 (1982)) around the energy and force
// evaluation, all on the handle's stream -- the use by which the paper
// measures the cost of its potentials (Sec. V, Fig. 4).
//
// Units: angstrom, femtosecond, atomic mass unit, electronvolt; an
// acceleration F/m in eV/(A amu) is ACC A/fs^2.  Position and velocity
// updates are computed in FP64 and stored in the handle's dtype.
#include <hip/hip_runtime.h>

#include <cmath>

#include "pod.h"
#include "pod_internal.h"

namespace pod {
namespace {

// 1 eV / (1 A * 1 amu) in A / fs^2 (CODATA: e = 1.602176634e-19 C, u = 1.66053906660e-27 kg)
constexpr double ACC = 1.602176634e-19 / 1e-10 / 1.66053906660e-27 * 1e-20;
constexpr int MD_THREADS = 256;
constexpr int MD_BLOCKS = 512;   // grid-stride kernels; partial sums per block
constexpr int KE_RING = 64;      // steps of kinetic-energy partials folded together

// v += dt/2 a F, x += dt v, one atom per thread; with a reference, the
// block's running maximum of |x - x_ref| over the steps in its own slot of
// `part` (a NaN displacement wins)
template <typename T>
__global__ __launch_bounds__(MD_THREADS) void kick_drift_kernel(int N, T* __restrict__ x, T* __restrict__ v,
                                                                const T* __restrict__ F, const T* __restrict__ xr,
                                                                double hka, double dt, double* __restrict__ part) {
    __shared__ double red[MD_THREADS];
    double mx = 0.0;
    for (long i = static_cast<long>(blockIdx.x) * MD_THREADS + threadIdx.x; i < N;
         i += static_cast<long>(gridDim.x) * MD_THREADS) {
        double d2 = 0.0;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const long k = 3 * i + e;
            const double vh = static_cast<double>(v[k]) + hka * static_cast<double>(F[k]);
            v[k] = static_cast<T>(vh);
            const T xn = static_cast<T>(static_cast<double>(x[k]) + dt * vh);
            x[k] = xn;
            if (xr) {
                const double dd = static_cast<double>(xn) - static_cast<double>(xr[k]);
                d2 += dd * dd;
            }
        }
        const double d = sqrt(d2);
        mx = (d > mx || d != d) ? d : mx;
    }
    if (!part) return;
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int o = MD_THREADS / 2; o > 0; o >>= 1) {
        if (static_cast<int>(threadIdx.x) < o) {
            const double b = red[threadIdx.x + o];
            if (b > red[threadIdx.x] || b != b) red[threadIdx.x] = b;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double r = red[0], o = part[blockIdx.x];
        part[blockIdx.x] = (r > o || r != r) ? r : o;
    }
}

// One atom per thread: the second half-kick of a step with its forces (the
// block's partial sum of m v^2 / 2 in ke_part) and, with DRIFT, the first
// half-kick and drift of the next step with the same forces (the running
// displacement maximum as in kick_drift_kernel).  Per component the
// arithmetic is a half kick rounded to the stored type followed by
// kick_drift_kernel's, as with two launches; one launch per step is saved.
template <typename T, bool DRIFT>
__global__ __launch_bounds__(MD_THREADS) void kick_atoms_kernel(int N, T* __restrict__ x, T* __restrict__ v,
                                                                const T* __restrict__ F, const T* __restrict__ xr,
                                                                double hka, double dt, double half_m_over_acc,
                                                                double* __restrict__ ke_part,
                                                                double* __restrict__ disp_part) {
    __shared__ double red[MD_THREADS];
    double ke = 0.0, mx = 0.0;
    for (long i = static_cast<long>(blockIdx.x) * MD_THREADS + threadIdx.x; i < N;
         i += static_cast<long>(gridDim.x) * MD_THREADS) {
        double d2 = 0.0;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const long k = 3 * i + e;
            const double f = static_cast<double>(F[k]);
            const double vn = static_cast<double>(v[k]) + hka * f;
            const double vs = static_cast<double>(static_cast<T>(vn));
            ke += vs * vs;
            if constexpr (DRIFT) {
                const double vh = vs + hka * f;
                v[k] = static_cast<T>(vh);
                const T xn = static_cast<T>(static_cast<double>(x[k]) + dt * vh);
                x[k] = xn;
                if (xr) {
                    const double dd = static_cast<double>(xn) - static_cast<double>(xr[k]);
                    d2 += dd * dd;
                }
            } else {
                v[k] = static_cast<T>(vn);
            }
        }
        if constexpr (DRIFT) {
            const double d = sqrt(d2);
            mx = (d > mx || d != d) ? d : mx;
        }
    }
    red[threadIdx.x] = ke * half_m_over_acc;
    __syncthreads();
    for (int o = MD_THREADS / 2; o > 0; o >>= 1) {
        if (static_cast<int>(threadIdx.x) < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) ke_part[blockIdx.x] = red[0];
    if (!DRIFT || !disp_part) return;
    __syncthreads();
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int o = MD_THREADS / 2; o > 0; o >>= 1) {
        if (static_cast<int>(threadIdx.x) < o) {
            const double b = red[threadIdx.x + o];
            if (b > red[threadIdx.x] || b != b) red[threadIdx.x] = b;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double r = red[0], o = disp_part[blockIdx.x];
        disp_part[blockIdx.x] = (r > o || r != r) ? r : o;
    }
}

// max_n |x_n - x_ref_n| per block
template <typename T>
__global__ __launch_bounds__(MD_THREADS) void disp_kernel(int N, const T* __restrict__ x, const T* __restrict__ xr,
                                                          double* __restrict__ part) {
    __shared__ double red[MD_THREADS];
    double mx = 0.0;
    for (long i = static_cast<long>(blockIdx.x) * MD_THREADS + threadIdx.x; i < N;
         i += static_cast<long>(gridDim.x) * MD_THREADS) {
        const double d0 = static_cast<double>(x[3 * i]) - static_cast<double>(xr[3 * i]);
        const double d1 = static_cast<double>(x[3 * i + 1]) - static_cast<double>(xr[3 * i + 1]);
        const double d2 = static_cast<double>(x[3 * i + 2]) - static_cast<double>(xr[3 * i + 2]);
        const double d = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        mx = (d > mx || d != d) ? d : mx;   // a NaN displacement wins
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int o = MD_THREADS / 2; o > 0; o >>= 1) {
        if (static_cast<int>(threadIdx.x) < o) {
            const double b = red[threadIdx.x + o];
            if (b > red[threadIdx.x] || b != b) red[threadIdx.x] = b;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Block b: out[b] = sum of the nb partials at part + b * stride (mode 0),
// their maximum (1), or the maximum of out[b] and the partials (2), a NaN
// winning every maximum; fixed order (each thread folds a strided subset,
// then a tree in LDS)
__global__ __launch_bounds__(MD_THREADS) void fold_kernel(const double* __restrict__ part, int nb, int mode,
                                                          double* __restrict__ out, long stride) {
    __shared__ double red[MD_THREADS];
    part += blockIdx.x * stride;
    out += blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += MD_THREADS) {
        const double x = part[b];
        s = mode ? ((x > s || x != x) ? x : s) : s + x;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = MD_THREADS / 2; o > 0; o >>= 1) {
        if (static_cast<int>(threadIdx.x) < o) {
            const double b = red[threadIdx.x + o];
            const double a = red[threadIdx.x];
            red[threadIdx.x] = mode ? ((b > a || b != b) ? b : a) : a + b;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double r = red[0];
        if (mode == 2) {
            const double a = *out;
            *out = (r > a || r != r) ? r : a;
        } else {
            *out = r;
        }
    }
}

__global__ __launch_bounds__(MD_THREADS) void zero_kernel(double* out, int n) {
    for (int k = threadIdx.x; k < n; k += MD_THREADS) out[k] = 0.0;
}

int md_blocks(long n) {
    const long b = (n + MD_THREADS - 1) / MD_THREADS;
    return static_cast<int>(b < 1 ? 1 : (b > MD_BLOCKS ? MD_BLOCKS : b));
}

template <typename T>
int verlet_impl(pod_handle* h, int N, int P, void* pos, void* vel, void* F, const double* cell, const int* offsets,
                const int* nbr_j, const int* shift, const int* rev, const void* c, double mass, double dt, int nsteps,
                double* E_pot, double* E_kin, const void* pos_ref, double* max_disp) {
    const int nb1 = md_blocks(N);
    int rc = ensure_mscratch(h, sizeof(double) * (KE_RING + 1) * MD_BLOCKS);
    if (rc != POD_OK) return rc;
    double* partd = static_cast<double*>(h->d_mscratch);   // running displacement maxima
    double* ring = partd + MD_BLOCKS;                       // kinetic-energy partials, KE_RING steps
    const double hka = 0.5 * dt * ACC / mass;
    const double half_m_over_acc = 0.5 * mass / ACC;
    T* x = static_cast<T*>(pos);
    T* v = static_cast<T*>(vel);
    T* f = static_cast<T*>(F);
    const T* xr = max_disp ? static_cast<const T*>(pos_ref) : nullptr;
    if (max_disp) {
        hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(MD_THREADS), 0, h->stream, max_disp, 1);
        hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(MD_THREADS), 0, h->stream, partd, MD_BLOCKS);
    }
    // step s: half kick + drift, forces, half kick; the closing half kick of
    // step s and the opening half kick and drift of step s + 1 share one
    // launch (same forces)
    if (N > 0 && nsteps > 0)
        hipLaunchKernelGGL((kick_drift_kernel<T>), dim3(nb1), dim3(MD_THREADS), 0, h->stream, N, x, v, f, xr, hka, dt,
                           xr ? partd : nullptr);
    for (int s = 0; s < nsteps; ++s) {
        rc = pod_energy_forces(h, N, P, pos, cell, offsets, nbr_j, shift, rev, c, nullptr, E_pot ? E_pot + s : nullptr,
                               F, nullptr, nullptr);
        if (rc != POD_OK) return rc;
        double* ke = ring + static_cast<long>(s % KE_RING) * MD_BLOCKS;
        if (N > 0) {
            if (s + 1 < nsteps)
                hipLaunchKernelGGL((kick_atoms_kernel<T, true>), dim3(nb1), dim3(MD_THREADS), 0, h->stream, N, x, v, f,
                                   xr, hka, dt, half_m_over_acc, ke, xr ? partd : nullptr);
            else
                hipLaunchKernelGGL((kick_atoms_kernel<T, false>), dim3(nb1), dim3(MD_THREADS), 0, h->stream, N, x, v,
                                   f, xr, hka, dt, half_m_over_acc, ke, nullptr);
        }
        // kinetic energies of up to KE_RING steps in one launch, one block per step
        if (E_kin && (s % KE_RING == KE_RING - 1 || s == nsteps - 1)) {
            const int cnt = s % KE_RING + 1;
            hipLaunchKernelGGL(fold_kernel, dim3(cnt), dim3(MD_THREADS), 0, h->stream, ring, N > 0 ? nb1 : 0, 0,
                               E_kin + (s + 1 - cnt), static_cast<long>(MD_BLOCKS));
        }
    }
    if (max_disp && N > 0)
        hipLaunchKernelGGL(fold_kernel, dim3(1), dim3(MD_THREADS), 0, h->stream, partd, nb1, 2, max_disp, 0L);
    return hipGetLastError() == hipSuccess ? POD_OK : POD_EHIP;
}

}  // namespace
}  // namespace pod

extern "C" {

int pod_md_verlet(pod_handle* h, int N, int P, void* pos, void* vel, void* F, const double* cell, const int* offsets,
                  const int* nbr_j, const int* shift, const int* rev, const void* c, double mass, double dt,
                  int nsteps, double* E_pot, double* E_kin, const void* pos_ref, double* max_disp) {
    using namespace pod;
    if (!h || N < 0 || P < 0 || nsteps < 0) return POD_EINVAL;
    if (N > 0 && (!pos || !vel || !F || !offsets || !c || (P > 0 && (!nbr_j || !shift)))) return POD_EINVAL;
    if (!(mass > 0.0) || !std::isfinite(mass) || !std::isfinite(dt)) return POD_EINVAL;
    if (max_disp && N > 0 && !pos_ref) return POD_EINVAL;
    if (h->dtype == POD_F64)
        return verlet_impl<double>(h, N, P, pos, vel, F, cell, offsets, nbr_j, shift, rev, c, mass, dt, nsteps, E_pot,
                                   E_kin, pos_ref, max_disp);
    return verlet_impl<float>(h, N, P, pos, vel, F, cell, offsets, nbr_j, shift, rev, c, mass, dt, nsteps, E_pot,
                              E_kin, pos_ref, max_disp);
}

int pod_md_max_displacement(pod_handle* h, int N, const void* pos, const void* pos_ref, double* out) {
    using namespace pod;
    if (!h || N < 0 || !out || (N > 0 && (!pos || !pos_ref))) return POD_EINVAL;
    const int nb = md_blocks(N);
    const int rc = ensure_mscratch(h, sizeof(double) * MD_BLOCKS);
    if (rc != POD_OK) return rc;
    double* part = static_cast<double*>(h->d_mscratch);
    if (N > 0) {
        if (h->dtype == POD_F64)
            hipLaunchKernelGGL((disp_kernel<double>), dim3(nb), dim3(MD_THREADS), 0, h->stream, N,
                               static_cast<const double*>(pos), static_cast<const double*>(pos_ref), part);
        else
            hipLaunchKernelGGL((disp_kernel<float>), dim3(nb), dim3(MD_THREADS), 0, h->stream, N,
                               static_cast<const float*>(pos), static_cast<const float*>(pos_ref), part);
    }
    hipLaunchKernelGGL(fold_kernel, dim3(1), dim3(MD_THREADS), 0, h->stream, part, N > 0 ? nb : 0, 1, out, 0L);
    return hipGetLastError() == hipSuccess ? POD_OK : POD_EHIP;
}

}  // extern "C"
