// Network surrogate of the 4-body energy (Sec. IV.D, eqs. (671a)-(673a)):
// a 2-hidden-layer SiLU network of width 64 on the standardised 2/3-body
// descriptors, with bfloat16 MFMA products accumulated in FP32.
//
// Layout of the parameter vector theta (FP32): W1 [64][n_in], b1 [64],
// W2 [64][64], b2 [64], w3 [64], b3, row-major and concatenated.
//
// All matrix products use v_mfma_f32_16x16x16_bf16 on tiles of 16 atoms;
// the arithmetic of a tile (forward, output, input gradient) is shared with
// the per-atom energy kernel through pod_net.h.  Here the weights sit in
// LDS; training adds the weight gradients of every tile.
#include <hip/hip_runtime.h>

#include <cmath>

#include "pod.h"
#include "pod_internal.h"
#include "pod_net.h"

namespace pod {
namespace {

using net::bf4;
using net::f4;
using net::from_bf16;
using net::Layout;
using net::layout;
using net::mfma;
using net::silu;
using net::silu_d;
using net::to_bf16;

constexpr int H = POD_MLP_HIDDEN;     // 64
constexpr int MAX_IN = POD_MLP_MAX_IN;  // 64
constexpr int WS = H + 4;             // padded LDS row stride of the weight tiles (bf16 elements)
constexpr int TS = 20;                // padded row stride of the per-wave transpose tiles

__device__ __forceinline__ bf4 lds4(const unsigned short* p) { return *reinterpret_cast<const bf4*>(p); }

// Weights as the products read them, in LDS.
struct alignas(16) Weights {
    unsigned short W1[H * WS];       // [h][k], zero for k >= n_in
    unsigned short W1T[MAX_IN * WS]; // [k][h]
    unsigned short W2[H * WS];       // [h2][h1]
    unsigned short W2T[H * WS];      // [h1][h2]
    float b1[H], b2[H], w3[H], mu[MAX_IN], isg[MAX_IN];
    float b3;
};

__device__ void load_weights(Weights& L, const float* __restrict__ theta, const float* __restrict__ mu,
                             const float* __restrict__ isg, int n_in) {
    const Layout o = layout(n_in);
    const int tid = threadIdx.x, nth = blockDim.x;
    for (int i = tid; i < H * MAX_IN; i += nth) {
        const int h = i / MAX_IN, k = i - h * MAX_IN;
        const unsigned short b = to_bf16(k < n_in ? theta[h * n_in + k] : 0.0f);
        L.W1[h * WS + k] = b;
        L.W1T[k * WS + h] = b;
    }
    for (int i = tid; i < H * H; i += nth) {
        const int h2 = i / H, h1 = i - h2 * H;
        const unsigned short b = to_bf16(theta[o.o_W2 + i]);
        L.W2[h2 * WS + h1] = b;
        L.W2T[h1 * WS + h2] = b;
    }
    for (int i = tid; i < H; i += nth) {
        L.b1[i] = theta[o.o_b1 + i];
        L.b2[i] = theta[o.o_b2 + i];
        L.w3[i] = theta[o.o_w3 + i];
    }
    for (int i = tid; i < MAX_IN; i += nth) {
        L.mu[i] = i < n_in ? mu[i] : 0.0f;
        L.isg[i] = i < n_in ? isg[i] : 0.0f;
    }
    if (tid == 0) L.b3 = theta[o.o_b3];
}

// Accessor of the LDS weights for the shared tile arithmetic (pod_net.h).
struct LdsW {
    const Weights& L;
    __device__ __forceinline__ bf4 w1(int h, int k) const { return lds4(&L.W1[h * WS + k]); }
    __device__ __forceinline__ bf4 w1t(int k, int h) const { return lds4(&L.W1T[k * WS + h]); }
    __device__ __forceinline__ bf4 w2(int a, int b) const { return lds4(&L.W2[a * WS + b]); }
    __device__ __forceinline__ bf4 w2t(int a, int b) const { return lds4(&L.W2T[a * WS + b]); }
    __device__ __forceinline__ float b1(int i) const { return L.b1[i]; }
    __device__ __forceinline__ float b2(int i) const { return L.b2[i]; }
    __device__ __forceinline__ float w3(int i) const { return L.w3[i]; }
    __device__ __forceinline__ float b3() const { return L.b3; }
};

// Forward pass of one tile of 16 atoms.  Lane l: atom r = l % 16 of the tile,
// feature group g = l / 16.  xb[s]: standardised inputs 16 s + 4 g + i;
// z1[t], z2[u]: pre-activations of hidden units 16 t + 4 g + i.
template <typename TX>
__device__ __forceinline__ void forward_tile(const Weights& L, const TX* __restrict__ X, long ldx, int atom, bool ok,
                                             int n_in, int ns, int r, int g, bf4 (&xb)[4], f4 (&z1)[4], bf4 (&h1b)[4],
                                             f4 (&z2)[4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = 16 * s + 4 * g + i;
            float v = 0.0f;
            // standardise in the precision of the input: low-variance
            // descriptors lose their spread if rounded before the subtraction
            if (ok && s < ns && k < n_in)
                v = static_cast<float>((X[atom * ldx + k] - static_cast<TX>(L.mu[k])) * static_cast<TX>(L.isg[k]));
            xb[s][i] = static_cast<short>(to_bf16(v));
        }
    }
    net::layers(LdsW{L}, xb, r, g, z1, h1b, z2);
}

// y of the tile's atoms: every lane of column r ends with the same value.
__device__ __forceinline__ float output_tile(const Weights& L, const f4 (&z2)[4], int g) {
    return net::output(LdsW{L}, z2, g);
}

template <typename TX>
struct InferArgs {
    int n, n_in;
    const TX* X;
    long ldx;
    const float* theta;
    const float* mu;
    const float* isg;
    float* y;
    float* dydx;
};

// Forward and input gradient dy/dX, 4 waves per workgroup, one tile of 16
// atoms per wave and step; held to four wavefronts per SIMD, which the LDS
// of its weights allows.
template <typename TX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void infer_kernel(InferArgs<TX> a) {
    __shared__ Weights L;
    load_weights(L, a.theta, a.mu, a.isg, a.n_in);
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int ns = (a.n_in + 15) / 16;
    const int ntile = (a.n + 15) / 16;
    for (int tile = blockIdx.x * 4 + wv; tile < ntile; tile += gridDim.x * 4) {
        const int atom = tile * 16 + r;
        const bool ok = atom < a.n;
        bf4 xb[4], h1b[4];
        f4 z1[4], z2[4];
        forward_tile<TX>(L, a.X, a.ldx, atom, ok, a.n_in, ns, r, g, xb, z1, h1b, z2);
        const float y = output_tile(L, z2, g);
        if (ok && g == 0 && a.y) a.y[atom] = y;
        if (!a.dydx) continue;
        // back-propagation to the inputs (eq. (673a))
        f4 dx[4];
        net::input_grad(LdsW{L}, z1, z2, r, g, dx);
        if (ok) {
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int k = 16 * s + 4 * g + i;
                    if (s < ns && k < a.n_in) a.dydx[static_cast<long>(atom) * a.n_in + k] = dx[s][i] * L.isg[k];
                }
        }
    }
}

struct TrainArgs {
    int n, n_in;
    const float* X;
    long ldx;
    const float* target;
    const float* theta;
    const float* mu;
    const float* isg;
    float dscale;     // 2 / n: d(mean squared error)/dy per unit residual
    float* part;      // per-wave partial gradients, rows of pstride floats
    int pstride;
};

constexpr int TRAIN_WAVES = 2;

// Forward and backward of the per-atom energy loss; every wave accumulates
// its gradient in registers and writes one row of partial sums.  The tile
// sequence of every wave is fixed by the launch shape, so the result is
// deterministic.
__global__ __launch_bounds__(64 * TRAIN_WAVES) void train_kernel(TrainArgs a) {
    __shared__ Weights L;
    __shared__ __align__(16) unsigned short T[TRAIN_WAVES][4][MAX_IN * TS];  // x, h1, dz2, dz1: [feature][atom]
    load_weights(L, a.theta, a.mu, a.isg, a.n_in);
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int ns = (a.n_in + 15) / 16;
    const int ntile = (a.n + 15) / 16;
    unsigned short* sX = T[wv][0];
    unsigned short* sH1 = T[wv][1];
    unsigned short* sD2 = T[wv][2];
    unsigned short* sD1 = T[wv][3];

    f4 gW2[4][4], gW1[4][4];
    float gb1[4][4], gb2[4][4], gw3[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            gW2[u][t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
            gW1[u][t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
            gb1[u][t] = 0.0f; gb2[u][t] = 0.0f; gw3[u][t] = 0.0f;
        }
    float gb3 = 0.0f, lsum = 0.0f;

    // every wave of the workgroup runs the same number of steps (tiles past
    // the end are fully masked), so the workgroup barriers below are uniform
    for (int base = blockIdx.x * TRAIN_WAVES; base < ntile; base += gridDim.x * TRAIN_WAVES) {
        const int tile = base + wv;
        const int atom = tile * 16 + r;
        const bool ok = tile < ntile && atom < a.n;
        bf4 xb[4], h1b[4];
        f4 z1[4], z2[4];
        forward_tile<float>(L, a.X, a.ldx, atom, ok, a.n_in, ns, r, g, xb, z1, h1b, z2);
        const float y = output_tile(L, z2, g);
        const float res = ok ? y - a.target[atom] : 0.0f;
        if (g == 0) lsum += res * res;
        const float dy = res * a.dscale;
        if (g == 0) gb3 += dy;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int i = 0; i < 4; ++i) sX[(16 * s + 4 * g + i) * TS + r] = static_cast<unsigned short>(xb[s][i]);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) sH1[(16 * t + 4 * g + i) * TS + r] = static_cast<unsigned short>(h1b[t][i]);
        bf4 dz2b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int h = 16 * u + 4 * g + i;
                gw3[u][i] += dy * silu(z2[u][i]);
                const unsigned short b = to_bf16(dy * L.w3[h] * silu_d(z2[u][i]));
                dz2b[u][i] = static_cast<short>(b);
                gb2[u][i] += from_bf16(b);
                sD2[h * TS + r] = b;
            }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int u = 0; u < 4; ++u) acc = mfma(lds4(&L.W2T[(16 * t + r) * WS + 16 * u + 4 * g]), dz2b[u], acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const unsigned short b = to_bf16(acc[i] * silu_d(z1[t][i]));
                gb1[t][i] += from_bf16(b);
                sD1[(16 * t + 4 * g + i) * TS + r] = b;
            }
        }
        __syncthreads();
        // dW2[h2][h1] += sum_atoms dz2[h2][atom] h1[h1][atom]
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int t = 0; t < 4; ++t)
                gW2[u][t] = mfma(lds4(&sD2[(16 * u + r) * TS + 4 * g]), lds4(&sH1[(16 * t + r) * TS + 4 * g]), gW2[u][t]);
        // dW1[h1][k] += sum_atoms dz1[h1][atom] x[k][atom]
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int s = 0; s < 4; ++s)
                if (s < ns)
                    gW1[t][s] = mfma(lds4(&sD1[(16 * t + r) * TS + 4 * g]), lds4(&sX[(16 * s + r) * TS + 4 * g]),
                                     gW1[t][s]);
        __syncthreads();
    }

    // sums over the 16 atom lanes of each feature group
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                gb1[u][i] += __shfl_xor(gb1[u][i], off);
                gb2[u][i] += __shfl_xor(gb2[u][i], off);
                gw3[u][i] += __shfl_xor(gw3[u][i], off);
            }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        gb3 += __shfl_xor(gb3, off);
        lsum += __shfl_xor(lsum, off);
    }
    const Layout o = layout(a.n_in);
    float* row = a.part + static_cast<long>(blockIdx.x * TRAIN_WAVES + wv) * a.pstride;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int h1 = 16 * t + 4 * g + i, k = 16 * s + r;
                if (s < ns && k < a.n_in) row[h1 * a.n_in + k] = gW1[t][s][i];
            }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) row[o.o_W2 + (16 * u + 4 * g + i) * H + 16 * t + r] = gW2[u][t][i];
    if (r == 0) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int h = 16 * u + 4 * g + i;
                row[o.o_b1 + h] = gb1[u][i];
                row[o.o_b2 + h] = gb2[u][i];
                row[o.o_w3 + h] = gw3[u][i];
            }
    }
    if (lane == 0) {
        row[o.o_b3] = gb3;
        row[o.n] = lsum;
    }
}

struct AdamArgs {
    int np, rows, pstride;
    const float* part;
    float* theta;
    float* m;
    float* v;
    float lr, beta1, beta2, eps, bc1, bc2, inv_n;
    float* loss;
};

// Sum of the partial rows in a fixed order, then one Adam update
// (Kingma and Ba, 2015, Algorithm 1) per parameter; the parameter past the
// last one carries the batch loss.  A workgroup takes 16 parameters; its 16
// row groups each sum every 16th row, and the group sums are added in a
// fixed order.
constexpr int ADAM_P = 16, ADAM_G = 16;

__global__ __launch_bounds__(ADAM_P * ADAM_G) void adam_kernel(AdamArgs a) {
    __shared__ float red[ADAM_G][ADAM_P];
    const int lp = threadIdx.x % ADAM_P, grp = threadIdx.x / ADAM_P;
    const int p = blockIdx.x * ADAM_P + lp;
    float s = 0.0f;
    if (p <= a.np)
        for (int q = grp; q < a.rows; q += ADAM_G) s += a.part[static_cast<long>(q) * a.pstride + p];
    red[grp][lp] = s;
    __syncthreads();
    if (grp != 0 || p > a.np) return;
    s = 0.0f;
    for (int k = 0; k < ADAM_G; ++k) s += red[k][lp];
    if (p == a.np) {
        if (a.loss) *a.loss = s * a.inv_n;
        return;
    }
    const float m = a.beta1 * a.m[p] + (1.0f - a.beta1) * s;
    const float v = a.beta2 * a.v[p] + (1.0f - a.beta2) * s * s;
    a.m[p] = m;
    a.v[p] = v;
    a.theta[p] -= a.lr * (m / a.bc1) / (sqrtf(v / a.bc2) + a.eps);
}

int grid_for(int tiles, int per_block, int cap) {
    int b = (tiles + per_block - 1) / per_block;
    return b < 1 ? 1 : (b > cap ? cap : b);
}

// The weights packed for the per-atom kernel (net::Packed): one element of
// W1 / W2 (and its transposed copy) per thread, the vectors by the first
// workgroup.
constexpr int PACK_THREADS = 256;
constexpr int PACK_BLOCKS = (H * MAX_IN + H * H) / PACK_THREADS;

__global__ __launch_bounds__(PACK_THREADS) void pack_kernel(const float* __restrict__ theta,
                                                            const float* __restrict__ mu,
                                                            const float* __restrict__ isg, int n_in,
                                                            net::Packed* out) {
    const Layout o = layout(n_in);
    const int i = blockIdx.x * PACK_THREADS + threadIdx.x;
    if (i < H * MAX_IN) {
        const int h = i / MAX_IN, k = i - h * MAX_IN;
        const unsigned short b = to_bf16(k < n_in ? theta[h * n_in + k] : 0.0f);
        out->W1[net::packed_index(h, k)] = b;
        out->W1T[net::packed_index(k, h)] = b;
    } else if (i < H * MAX_IN + H * H) {
        const int j = i - H * MAX_IN;
        const int h2 = j / H, h1 = j - h2 * H;
        const unsigned short b = to_bf16(theta[o.o_W2 + j]);
        out->W2[net::packed_index(h2, h1)] = b;
        out->W2T[net::packed_index(h1, h2)] = b;
    }
    if (blockIdx.x == 0) {
        const int t = threadIdx.x;
        if (t < H) {
            out->b1[t] = theta[o.o_b1 + t];
            out->b2[t] = theta[o.o_b2 + t];
            out->w3[t] = theta[o.o_w3 + t];
        }
        if (t < MAX_IN) {
            out->mu[t] = t < n_in ? mu[t] : 0.0f;
            out->isg[t] = t < n_in ? isg[t] : 0.0f;
        }
        if (t == 0) {
            out->b3 = theta[o.o_b3];
            out->pad[0] = out->pad[1] = out->pad[2] = 0.0f;
        }
    }
}

static_assert((H * MAX_IN + H * H) % PACK_THREADS == 0, "pack grid");
static_assert(H <= PACK_THREADS && MAX_IN <= PACK_THREADS, "pack vectors");

}  // namespace

int mlp_pack_launch(pod_handle* h, int n_in, const float* theta, const float* mu, const float* isg,
                    net::Packed* out) {
    timing_begin(h, 2);
    hipLaunchKernelGGL(pack_kernel, dim3(PACK_BLOCKS), dim3(PACK_THREADS), 0, h->stream, theta, mu, isg, n_in, out);
    timing_end(h, 2);
    return hipGetLastError() == hipSuccess ? POD_OK : POD_EHIP;
}

int mlp_forward_launch(pod_handle* h, int n, int n_in, const void* X, long ldx, int x_dtype, const float* theta,
                       const float* mu, const float* isg, float* y, float* dydx) {
    if (n == 0) return POD_OK;
    const int nblk = grid_for((n + 15) / 16, 4, 2048);
    timing_begin(h, 2);
    if (x_dtype == POD_F64) {
        InferArgs<double> a{n, n_in, static_cast<const double*>(X), ldx, theta, mu, isg, y, dydx};
        hipLaunchKernelGGL(infer_kernel<double>, dim3(nblk), dim3(256), 0, h->stream, a);
    } else {
        InferArgs<float> a{n, n_in, static_cast<const float*>(X), ldx, theta, mu, isg, y, dydx};
        hipLaunchKernelGGL(infer_kernel<float>, dim3(nblk), dim3(256), 0, h->stream, a);
    }
    timing_end(h, 2);
    return hipGetLastError() == hipSuccess ? POD_OK : POD_EHIP;
}

}  // namespace pod

extern "C" {

int pod_mlp_num_params(int n_in) {
    if (n_in < 1 || n_in > POD_MLP_MAX_IN) return POD_EINVAL;
    return pod::layout(n_in).n;
}

int pod_mlp_forward(pod_handle* h, int n, int n_in, const void* X, long ldx, const float* theta, const float* mu,
                    const float* inv_sigma, float* y, float* dydx) {
    if (!h || n < 0 || n_in < 1 || n_in > POD_MLP_MAX_IN || ldx < n_in) return POD_EINVAL;
    if (n > 0 && (!X || !theta || !mu || !inv_sigma || (!y && !dydx))) return POD_EINVAL;
    return pod::mlp_forward_launch(h, n, n_in, X, ldx, h->dtype, theta, mu, inv_sigma, y, dydx);
}

int pod_mlp_train_step(pod_handle* h, int n, int n_in, const float* X, long ldx, const float* target,
                       const float* mu, const float* inv_sigma, float* theta, float* adam_m, float* adam_v, int step,
                       float lr, float beta1, float beta2, float eps, float* loss) {
    using namespace pod;
    if (!h || n < 1 || n_in < 1 || n_in > POD_MLP_MAX_IN || ldx < n_in || step < 1) return POD_EINVAL;
    if (!X || !target || !mu || !inv_sigma || !theta || !adam_m || !adam_v) return POD_EINVAL;
    if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return POD_EINVAL;
    const Layout o = layout(n_in);
    const int pstride = ((o.n + 1 + 63) / 64) * 64;
    const int nblk = grid_for((n + 15) / 16, TRAIN_WAVES, 128);
    const int rows = nblk * TRAIN_WAVES;
    const int rc = ensure_mscratch(h, static_cast<size_t>(rows) * pstride * sizeof(float));
    if (rc != POD_OK) return rc;
    TrainArgs ta{n, n_in, X, ldx, target, theta, mu, inv_sigma, 2.0f / static_cast<float>(n),
                 static_cast<float*>(h->d_mscratch), pstride};
    timing_begin(h, 2);
    hipLaunchKernelGGL(train_kernel, dim3(nblk), dim3(64 * TRAIN_WAVES), 0, h->stream, ta);
    timing_end(h, 2);
    if (hipGetLastError() != hipSuccess) return POD_EHIP;
    AdamArgs aa{o.n, rows, pstride, static_cast<const float*>(h->d_mscratch), theta, adam_m, adam_v, lr, beta1, beta2,
                eps, static_cast<float>(1.0 - std::pow(static_cast<double>(beta1), step)),
                static_cast<float>(1.0 - std::pow(static_cast<double>(beta2), step)), 1.0f / static_cast<float>(n),
                loss};
    hipLaunchKernelGGL(adam_kernel, dim3((o.n + 1 + ADAM_P - 1) / ADAM_P), dim3(ADAM_P * ADAM_G), 0, h->stream, aa);
    return hipGetLastError() == hipSuccess ? POD_OK : POD_EHIP;
}

}  // extern "C"
