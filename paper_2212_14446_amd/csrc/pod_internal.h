// Internal declarations shared by the host code and the kernels of libpod.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "pod.h"

namespace pod {

constexpr int WAVE = 64;

// Largest angular degree and radial-function count of the kernels that keep
// an atom's basis rows in registers (energy path, batch assembly, surrogate,
// five-body terms); beyond either the energy path runs on the kernel with
// the basis in LDS.
constexpr int FAST_MAX_PA = 6;
constexpr int FAST_MAX_K = 8;

// Device error word bits (latched with atomicOr, read and cleared by pod_check).
constexpr int ERR_RANGE = 1;
constexpr int ERR_NONFINITE = 2;
constexpr int ERR_NEIGH = 4;
constexpr int ERR_SINGULAR = 8;   // fit matrix not positive definite

// Kernel kinds with their own timing events: 0 finalize kernels, 1 per-atom
// and batch kernels, 2 network, 3 fit Gram, 4 pair-gradient kernel.
constexpr int TIMING_KINDS = 5;

// One snapshot tuple as the kernels evaluate it (Sec. II.B, eqs. (3)-(6)).
//   bessel  : kappa != 0; phi = sin(alpha pi x)/(r - rin)
//   newbeta : x(r) must be (re)computed for this snapshot's beta
//   steps   : >= 0 -> sin/cos(alpha pi x) reached from the previous integer
//             multiple of pi x by `steps` angle-addition steps; -1 -> direct
//   power   : kappa != 1; 1 = integer gamma (igamma), 2 = general gamma
template <typename T>
struct SnapT {
    T kappa;
    T apix;     // alpha * pi
    T bh;       // beta / (rcut - rin)
    T inv_em1;  // 1 / expm1(-beta)
    T gamma;
    int bessel;
    int newbeta;
    int steps;
    int power;
    int igamma;
};

template <typename T>
struct ParamsT {
    T rin, rcut, inv_h;
    int L, K, K2, K3, K4, P3, P4, Ka4, M, PA;
    int off3, off4;             // first column of the 3- and 4-body blocks in D
    // Standard family fast path (std_nb + std_ni == L): snapshots 0..nb-1 are
    // Bessel with kappa = 1, alpha = 1..nb and one beta; the rest are inverse
    // powers with kappa = 0, gamma = 1..ni.  std_ok = 0 -> generic path.
    int std_ok, std_nb, std_ni;
    T std_bh, std_inv_em1;
    SnapT<T> s[POD_MAX_L];
    T Q[POD_MAX_L][POD_MAX_K];  // zero-padded beyond K
};

// Periodic cell passed by value to the kernels.
template <typename T>
struct CellT {
    T a[9];
    int periodic;
};

}  // namespace pod

struct pod_handle {
    int dtype;
    int device;                // HIP device current at pod_init
    hipStream_t stream;
    double rin, rcut;
    int L, K2, K3, K4, P3, P4, K, PA, Ka4, M;
    int m_by_order[4];
    int std_ok;                // standard snapshot family: fast radial path
    std::vector<double> alpha, beta, gamma, kappa;
    std::vector<double> Q;     // L x K row-major
    std::vector<double> eig;   // L
    // parameter block of the kernels, passed by value in their arguments
    // (scalar loads through the constant cache); the member for the dtype
    pod::ParamsT<double> hp_d;
    pod::ParamsT<float> hp_f;
    int* d_err;
    void* d_scratch;           // block partial sums
    double* d_facc;            // force accumulator, 3 x facc_n doubles, zero between calls
    int facc_n;
    int facc_dirty;            // a call failed between accumulation and copy-out
    size_t scratch_bytes;
    size_t lds_max;            // LDS bytes a workgroup may use on this device
    void* d_mscratch;          // network outputs and gradient partials (separate from d_scratch,
    size_t mscratch_bytes;     // which the energy kernels reuse within one call)
    // kernel timing per kernel kind (0 finalize, 1 per-atom and batch, 2 network,
    // 3 fit Gram, 4 pair gradients), 2 events per launch
    std::vector<hipEvent_t> ev[pod::TIMING_KINDS];
    int ev_used[pod::TIMING_KINDS];
};

namespace pod {
// Device address of the static scratch array of pod_energy_forces_noalloc on
// device `dev` (the current device): looked up once per device, POD_OK /
// POD_EHIP.
int resolve_static_scratch(int dev);
// Grow the handle's scratch buffer to at least `bytes` (POD_OK / POD_ENOMEM).
int ensure_scratch(pod_handle* h, size_t bytes);
// Same for the network scratch buffer.
int ensure_mscratch(pod_handle* h, size_t bytes);
// Force accumulator for N atoms, zero on return (POD_OK / POD_ENOMEM / POD_EHIP).
int ensure_force_acc(pod_handle* h, int N);
// Kernel timing around the main per-atom launch (no-ops unless enabled).
void timing_begin(pod_handle* h, int kind);
void timing_end(pod_handle* h, int kind);
// Network forward + input gradient on the handle's stream (x_dtype: POD_F64 / POD_F32).
int mlp_forward_launch(pod_handle* h, int n, int n_in, const void* X, long ldx, int x_dtype, const float* theta,
                       const float* mu, const float* isg, float* y, float* dydx);
namespace net {
struct Packed;
}
// The network weights packed for the per-atom energy kernel (one small
// kernel on the handle's stream); out: device memory of sizeof(net::Packed).
int mlp_pack_launch(pod_handle* h, int n_in, const float* theta, const float* mu, const float* isg,
                    net::Packed* out);
}  // namespace pod
