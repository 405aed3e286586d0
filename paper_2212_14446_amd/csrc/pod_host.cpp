// Host side of libpod: handle set-up (kernel parameter block, device buffers),
// error-word readout, kernel timing and teardown.  Validation and the POD basis
// live in pod_plan.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "pod.h"
#include "pod_internal.h"
#include "pod_plan.h"
#include "pod_tables.h"

namespace {

constexpr double kPi = 3.14159265358979323846;

template <typename T>
void fill_params(const pod_handle* h, pod::ParamsT<T>& d) {
    std::memset(&d, 0, sizeof(d));
    d.rin = static_cast<T>(h->rin);
    d.rcut = static_cast<T>(h->rcut);
    d.inv_h = static_cast<T>(1.0 / (h->rcut - h->rin));
    d.L = h->L; d.K = h->K; d.K2 = h->K2; d.K3 = h->K3; d.K4 = h->K4;
    d.P3 = h->P3; d.P4 = h->P4; d.Ka4 = h->Ka4; d.M = h->M; d.PA = h->PA;
    d.off3 = 1 + h->K2;
    d.off4 = 1 + h->K2 + h->K3 * (h->P3 + 1) * (h->K3 > 0);
    // angle-addition plan: within a run of snapshots sharing beta, an integer
    // alpha not below the previous one is reached by stepping sin/cos(k pi x)
    double cur_beta = -1.0;
    int cur_k = 0;
    for (int l = 0; l < h->L; ++l) {
        pod::SnapT<T>& s = d.s[l];
        const double kap = h->kappa[l];
        s.kappa = static_cast<T>(kap);
        s.apix = static_cast<T>(h->alpha[l] * kPi);
        s.gamma = static_cast<T>(h->gamma[l]);
        s.bessel = kap != 0.0;
        if (s.bessel) {
            const double b = h->beta[l];
            s.bh = static_cast<T>(b / (h->rcut - h->rin));
            s.inv_em1 = static_cast<T>(b == 0.0 ? 0.0 : 1.0 / std::expm1(-b));
            if (b != cur_beta) { s.newbeta = 1; cur_beta = b; cur_k = 0; }
            const double a = h->alpha[l];
            const bool is_int = a >= 0 && a == std::floor(a) && a <= 64.0;
            if (is_int && static_cast<int>(a) >= cur_k) {
                s.steps = static_cast<int>(a) - cur_k;
                cur_k = static_cast<int>(a);
            } else {
                s.steps = -1;
            }
        }
        s.power = 0;
        if (kap != 1.0) {
            const double g = h->gamma[l];
            if (g == std::floor(g) && g >= 1.0 && g <= 16.0) { s.power = 1; s.igamma = static_cast<int>(g); }
            else s.power = 2;
        }
    }
    for (int l = 0; l < h->L; ++l)
        for (int k = 0; k < h->K; ++k) d.Q[l][k] = static_cast<T>(h->Q[l * h->K + k]);
    // standard family: Bessel alpha = 1..nb at one beta (kappa = 1), then
    // inverse powers gamma = 1..ni (kappa = 0)
    int nb = 0;
    while (nb < h->L && h->kappa[nb] == 1.0 && h->alpha[nb] == nb + 1.0 && h->beta[nb] == h->beta[0]) ++nb;
    int ni = 0;
    while (nb + ni < h->L && h->kappa[nb + ni] == 0.0 && h->gamma[nb + ni] == ni + 1.0) ++ni;
    if (nb + ni == h->L) {
        d.std_ok = 1; d.std_nb = nb; d.std_ni = ni;
        const double b = nb > 0 ? h->beta[0] : 0.0;
        d.std_bh = static_cast<T>(b / (h->rcut - h->rin));
        d.std_inv_em1 = static_cast<T>(b == 0.0 ? 0.0 : 1.0 / std::expm1(-b));
    }
}

}  // namespace

int pod::ensure_force_acc(pod_handle* h, int N) {
    if (N > h->facc_n || !h->d_facc) {
        if (h->d_facc) {
            if (hipStreamSynchronize(h->stream) != hipSuccess) return POD_EHIP;
            (void)hipFree(h->d_facc);
            h->d_facc = nullptr;
            h->facc_n = 0;
        }
        const int want = N > 0 ? N + N / 4 + 64 : 64;
        if (hipMalloc(reinterpret_cast<void**>(&h->d_facc), sizeof(double) * 3 * static_cast<size_t>(want)) !=
            hipSuccess) {
            h->d_facc = nullptr;
            return POD_ENOMEM;
        }
        if (hipMemset(h->d_facc, 0, sizeof(double) * 3 * static_cast<size_t>(want)) != hipSuccess) return POD_EHIP;
        h->facc_n = want;
        h->facc_dirty = 0;
    }
    if (h->facc_dirty) {
        if (hipStreamSynchronize(h->stream) != hipSuccess) return POD_EHIP;
        if (hipMemset(h->d_facc, 0, sizeof(double) * 3 * static_cast<size_t>(h->facc_n)) != hipSuccess)
            return POD_EHIP;
        h->facc_dirty = 0;
    }
    return POD_OK;
}

int pod::ensure_scratch(pod_handle* h, size_t bytes) {
    if (bytes <= h->scratch_bytes) return POD_OK;
    if (h->d_scratch) {
        if (hipStreamSynchronize(h->stream) != hipSuccess) return POD_EHIP;
        (void)hipFree(h->d_scratch);
        h->d_scratch = nullptr;
        h->scratch_bytes = 0;
    }
    size_t want = bytes + bytes / 4 + 4096;
    if (hipMalloc(&h->d_scratch, want) != hipSuccess) {
        h->d_scratch = nullptr;
        return POD_ENOMEM;
    }
    h->scratch_bytes = want;
    return POD_OK;
}

int pod::ensure_mscratch(pod_handle* h, size_t bytes) {
    if (bytes <= h->mscratch_bytes) return POD_OK;
    if (h->d_mscratch) {
        if (hipStreamSynchronize(h->stream) != hipSuccess) return POD_EHIP;
        (void)hipFree(h->d_mscratch);
        h->d_mscratch = nullptr;
        h->mscratch_bytes = 0;
    }
    size_t want = bytes + bytes / 4 + 4096;
    if (hipMalloc(&h->d_mscratch, want) != hipSuccess) {
        h->d_mscratch = nullptr;
        return POD_ENOMEM;
    }
    h->mscratch_bytes = want;
    return POD_OK;
}

void pod::timing_begin(pod_handle* h, int kind) {
    auto& ev = h->ev[kind];
    const int u = h->ev_used[kind];
    if (2 * (u + 1) <= static_cast<int>(ev.size())) (void)hipEventRecord(ev[2 * u], h->stream);
}

void pod::timing_end(pod_handle* h, int kind) {
    auto& ev = h->ev[kind];
    const int u = h->ev_used[kind];
    if (2 * (u + 1) <= static_cast<int>(ev.size())) {
        (void)hipEventRecord(ev[2 * u + 1], h->stream);
        ++h->ev_used[kind];
    }
}

namespace {
void release_events(pod_handle* h) {
    bool any = false;
    for (int k = 0; k < pod::TIMING_KINDS; ++k) any = any || !h->ev[k].empty();
    if (any) (void)hipStreamSynchronize(h->stream);
    for (int k = 0; k < pod::TIMING_KINDS; ++k) {
        for (hipEvent_t e : h->ev[k]) (void)hipEventDestroy(e);
        h->ev[k].clear();
        h->ev_used[k] = 0;
    }
}
}  // namespace

extern "C" {

int pod_set_kernel_timing(pod_handle* h, int n) {
    if (!h || n < 0 || n > (1 << 20)) return POD_EINVAL;
    release_events(h);
    for (int k = 0; k < pod::TIMING_KINDS; ++k) {
        h->ev[k].reserve(2 * static_cast<size_t>(n));
        for (int i = 0; i < 2 * n; ++i) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) { release_events(h); return POD_EHIP; }
            h->ev[k].push_back(e);
        }
    }
    return POD_OK;
}

int pod_get_kernel_time(pod_handle* h, int kind, double* total_ms, int* launches) {
    if (!h || kind < 0 || kind >= pod::TIMING_KINDS) return POD_EINVAL;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return POD_EHIP;
    double tot = 0.0;
    for (int i = 0; i < h->ev_used[kind]; ++i) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, h->ev[kind][2 * i], h->ev[kind][2 * i + 1]) != hipSuccess) return POD_EHIP;
        tot += ms;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = h->ev_used[kind];
    h->ev_used[kind] = 0;
    return POD_OK;
}

int pod_init(const pod_params* p, void* hip_stream, pod_handle** out) {
    if (!out) return POD_EINVAL;
    *out = nullptr;
    int rc = pod::validate_params(p);
    if (rc != POD_OK) return rc;
    pod_handle* h = new (std::nothrow) pod_handle();
    if (!h) return POD_ENOMEM;
    h->dtype = p->dtype;
    h->stream = static_cast<hipStream_t>(hip_stream);
    h->lds_max = 64 * 1024;
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) { delete h; return POD_EHIP; }
        h->device = dev;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.sharedMemPerBlock > 0)
            h->lds_max = prop.sharedMemPerBlock;
        // address of the allocation-free entry point's scratch on this device
        if (pod::resolve_static_scratch(dev) != POD_OK) { delete h; return POD_EHIP; }
    }
    h->rin = p->rin; h->rcut = p->rcut; h->L = p->L;
    h->K2 = p->K2; h->K3 = p->K3; h->K4 = p->K4; h->P3 = p->P3; h->P4 = p->P4;
    h->K = std::max(p->K2, std::max(p->K3, p->K4));
    h->PA = std::max(p->K3 > 0 ? p->P3 : 0, p->K4 > 0 ? p->P4 : 0);
    h->Ka4 = p->K4 > 0 ? pod::n_partitions(p->P4) : 0;
    h->m_by_order[0] = 1;
    h->m_by_order[1] = p->K2;
    h->m_by_order[2] = p->K3 * (p->P3 + 1);
    h->m_by_order[3] = p->K4 * h->Ka4;
    h->M = 1 + h->m_by_order[1] + h->m_by_order[2] + h->m_by_order[3];
    h->alpha.assign(p->alpha, p->alpha + p->L);
    h->beta.assign(p->beta, p->beta + p->L);
    h->gamma.assign(p->gamma, p->gamma + p->L);
    h->kappa.assign(p->kappa, p->kappa + p->L);
    if (p->Q) {
        h->Q.assign(p->Q, p->Q + static_cast<size_t>(p->L) * h->K);
        h->eig.assign(p->L, 0.0);
    } else {
        std::vector<double> qfull;
        rc = pod::compute_basis(p, qfull, h->eig);
        if (rc != POD_OK) { delete h; return rc; }
        h->Q.assign(static_cast<size_t>(p->L) * h->K, 0.0);
        for (int l = 0; l < p->L; ++l)
            for (int k = 0; k < h->K; ++k) h->Q[l * h->K + k] = qfull[l * p->L + k];
    }
    if (hipMalloc(reinterpret_cast<void**>(&h->d_err), sizeof(int)) != hipSuccess) {
        delete h; return POD_ENOMEM;
    }
    if (h->dtype == POD_F64) {
        fill_params(h, h->hp_d);
        h->std_ok = h->hp_d.std_ok;
    } else {
        fill_params(h, h->hp_f);
        h->std_ok = h->hp_f.std_ok;
    }
    if (hipMemset(h->d_err, 0, sizeof(int)) != hipSuccess) { pod_free(h); return POD_EHIP; }
    *out = h;
    return POD_OK;
}

int pod_num_descriptors(const pod_handle* h, int* M, int* M_by_order) {
    if (!h) return POD_EINVAL;
    if (M) *M = h->M;
    if (M_by_order)
        for (int i = 0; i < 4; ++i) M_by_order[i] = h->m_by_order[i];
    return POD_OK;
}

int pod_get_basis(const pod_handle* h, double* Q, double* eigvals) {
    if (!h) return POD_EINVAL;
    if (Q) std::memcpy(Q, h->Q.data(), h->Q.size() * sizeof(double));
    if (eigvals) std::memcpy(eigvals, h->eig.data(), h->eig.size() * sizeof(double));
    return POD_OK;
}

int pod_check(pod_handle* h) {
    if (!h) return POD_EINVAL;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return POD_EHIP;
    int word = 0;
    if (hipMemcpy(&word, h->d_err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return POD_EHIP;
    if (word != 0 && hipMemset(h->d_err, 0, sizeof(int)) != hipSuccess) return POD_EHIP;
    if (word & pod::ERR_NEIGH) return POD_ENEIGH;
    if (word & pod::ERR_SINGULAR) return POD_ESINGULAR;
    if (word & pod::ERR_NONFINITE) return POD_ENONFINITE;
    if (word & pod::ERR_RANGE) return POD_ERANGE;
    return POD_OK;
}

void pod_free(pod_handle* h) {
    if (!h) return;
    release_events(h);
    (void)hipStreamSynchronize(h->stream);
    if (h->d_err) (void)hipFree(h->d_err);
    if (h->d_scratch) (void)hipFree(h->d_scratch);
    if (h->d_mscratch) (void)hipFree(h->d_mscratch);
    if (h->d_facc) (void)hipFree(h->d_facc);
    delete h;
}

}  // extern "C"
