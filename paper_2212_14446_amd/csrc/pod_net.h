// Network surrogate of the 4-body energy (Sec. IV.D, eqs. (671a)-(673a)):
// the arithmetic of one tile of 16 atoms, shared by the network kernels
// (pod_mlp.hip, weights in LDS) and the per-atom energy kernel that runs the
// network on its own descriptors (pod_kernels.hip, weights packed in global
// memory).  Both read the weights through an accessor with the same
// members, so the two paths evaluate the same products in the same order.
//
// A 2-hidden-layer SiLU network of width 64 on standardised descriptors;
// products are v_mfma_f32_16x16x16_bf16 (bfloat16 operands, FP32
// accumulation).  Activations are kept transposed (feature x atom): the
// product Z^T = W X^T leaves lane l holding atom l % 16 and features
// 4 (l / 16) + i, which is the B-operand layout of the next product, so the
// layers chain in registers.  Rounding to bfloat16 (nearest even) happens
// where a value enters a product: standardised inputs, W1, W2, the first
// hidden activation, and the back-propagated pre-activation gradients.
#pragma once

#include <hip/hip_runtime.h>

#include "pod.h"

namespace pod {
namespace net {

constexpr int H = POD_MLP_HIDDEN;       // 64
constexpr int MAX_IN = POD_MLP_MAX_IN;  // 64

typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short to_bf16(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return static_cast<unsigned short>(u >> 16);
}
__device__ __forceinline__ float from_bf16(unsigned short b) { return __uint_as_float(static_cast<unsigned>(b) << 16); }

__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigm(z); }
__device__ __forceinline__ float silu_d(float z) {
    const float s = sigm(z);
    return s * (1.0f + z * (1.0f - s));
}

__device__ __forceinline__ f4 mfma(bf4 a, bf4 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }

// Scheduling fence between output groups: the weight operands of a group
// are requested one group ahead (during the previous group's products), not
// all at the top of the network (which would hold every operand of the
// network in registers at once).
__device__ __forceinline__ void tile_fence() { __builtin_amdgcn_sched_barrier(0); }

// Offsets of the parameter vector theta (FP32): W1 [64][n_in], b1 [64],
// W2 [64][64], b2 [64], w3 [64], b3, row-major and concatenated.
struct Layout {
    int o_b1, o_W2, o_b2, o_w3, o_b3, n;
};
__host__ __device__ inline Layout layout(int n_in) {
    Layout L;
    L.o_b1 = H * n_in;
    L.o_W2 = L.o_b1 + H;
    L.o_b2 = L.o_W2 + H * H;
    L.o_w3 = L.o_b2 + H;
    L.o_b3 = L.o_w3 + H;
    L.n = L.o_b3 + 1;
    return L;
}

// Place of element (a, b) of a 64 x 64 weight matrix in its packed block.
// The products of output group a / 16 read, in lane (r, g), the elements
// (16 A + r, 16 B + 4 g + i) of the four input groups B: they are stored
// together, 32 bytes per lane and output group, so that a lane's operands
// for one output group come in two 16-byte loads and a wavefront's loads
// cover 2 KB contiguously (rows of 64 elements would spread each load over
// 16 cache lines).
__host__ __device__ constexpr int packed_index(int a, int b) {
    return (((a >> 4) * 64 + ((b & 15) >> 2) * 16 + (a & 15)) * 4 + (b >> 4)) * 4 + (b & 3);
}

// The weights as the products read them, packed once per call in global
// memory for the per-atom kernel: bfloat16 W1 [h][k] (zero for k >= n_in),
// its transpose, W2 [h2][h1] and its transpose, each in the order of
// packed_index; FP32 biases, output weights and the standardisation.
struct alignas(16) Packed {
    unsigned short W1[H * MAX_IN];
    unsigned short W1T[MAX_IN * H];
    unsigned short W2[H * H];
    unsigned short W2T[H * H];
    float b1[H], b2[H], w3[H], mu[MAX_IN], isg[MAX_IN];
    float b3, pad[3];
};

// Accessor of a Packed block.
struct PackedW {
    const Packed* __restrict__ p;
    __device__ __forceinline__ bf4 w1(int h, int k) const { return *reinterpret_cast<const bf4*>(&p->W1[packed_index(h, k)]); }
    __device__ __forceinline__ bf4 w1t(int k, int h) const { return *reinterpret_cast<const bf4*>(&p->W1T[packed_index(k, h)]); }
    __device__ __forceinline__ bf4 w2(int a, int b) const { return *reinterpret_cast<const bf4*>(&p->W2[packed_index(a, b)]); }
    __device__ __forceinline__ bf4 w2t(int a, int b) const { return *reinterpret_cast<const bf4*>(&p->W2T[packed_index(a, b)]); }
    __device__ __forceinline__ float b1(int i) const { return p->b1[i]; }
    __device__ __forceinline__ float b2(int i) const { return p->b2[i]; }
    __device__ __forceinline__ float w3(int i) const { return p->w3[i]; }
    __device__ __forceinline__ float b3() const { return p->b3; }
};

// Hidden layers of one tile.  Lane l: atom r = l % 16, feature group
// g = l / 16; xb[s]: standardised inputs 16 s + 4 g + i (bfloat16, zero at
// and beyond n_in, where W1 is zero as well: all four input groups enter
// every product, so the code has no branches and each tile's operand loads
// go out together); z1[t], z2[u]: pre-activations of hidden units
// 16 t + 4 g + i; h1b: the first activation rounded for the product.
template <class W>
__device__ __forceinline__ void layers(const W& w, const bf4 (&xb)[4], int r, int g, f4 (&z1)[4], bf4 (&h1b)[4],
                                       f4 (&z2)[4]) {
    // eight output groups (four of each layer); the operands of group q + 1
    // are requested before the products of group q
    bf4 op[4], nx[4];
    f4 bias, nb;
#pragma unroll
    for (int s = 0; s < 4; ++s) op[s] = w.w1(r, 16 * s + 4 * g);
#pragma unroll
    for (int i = 0; i < 4; ++i) bias[i] = w.b1(4 * g + i);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        if (q + 1 < 4) {
#pragma unroll
            for (int s = 0; s < 4; ++s) nx[s] = w.w1(16 * (q + 1) + r, 16 * s + 4 * g);
#pragma unroll
            for (int i = 0; i < 4; ++i) nb[i] = w.b1(16 * (q + 1) + 4 * g + i);
        } else if (q + 1 < 8) {
#pragma unroll
            for (int s = 0; s < 4; ++s) nx[s] = w.w2(16 * (q - 3) + r, 16 * s + 4 * g);
#pragma unroll
            for (int i = 0; i < 4; ++i) nb[i] = w.b2(16 * (q - 3) + 4 * g + i);
        }
        f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        if (q < 4) {
#pragma unroll
            for (int s = 0; s < 4; ++s) acc = mfma(op[s], xb[s], acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                z1[q][i] = acc[i] + bias[i];
                h1b[q][i] = static_cast<short>(to_bf16(silu(z1[q][i])));
            }
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) acc = mfma(op[t], h1b[t], acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) z2[q - 4][i] = acc[i] + bias[i];
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) op[s] = nx[s];
        bias = nb;
        tile_fence();
    }
}

// y of the tile's atoms: every lane of column r ends with the same value.
template <class W>
__device__ __forceinline__ float output(const W& w, const f4 (&z2)[4], int g) {
    float p = 0.0f;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int i = 0; i < 4; ++i) p += w.w3(16 * u + 4 * g + i) * silu(z2[u][i]);
    p += __shfl_xor(p, 16);
    p += __shfl_xor(p, 32);
    return p + w.b3();
}

// Back-propagation to the standardised inputs (eq. (673a)): dx[s][i] =
// dy/dx_k for k = 16 s + 4 g + i (the caller applies inv_sigma), from the
// first layer's pre-activations z1 (bias included) and the second's z2 kept
// from the forward pass.
template <class W>
__device__ __forceinline__ void input_grad(const W& w, const f4 (&z1)[4], const f4 (&z2)[4], int r, int g,
                                           f4 (&dx)[4]) {
    // eight output groups (four of W2^T, four of W1^T); the operands of
    // group q + 1 are requested before the products of group q
    bf4 op[4], nx[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) op[u] = w.w2t(r, 16 * u + 4 * g);
    bf4 dz2b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            dz2b[u][i] = static_cast<short>(to_bf16(w.w3(16 * u + 4 * g + i) * silu_d(z2[u][i])));
    tile_fence();
    bf4 dz1b[4];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        if (q + 1 < 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) nx[u] = w.w2t(16 * (q + 1) + r, 16 * u + 4 * g);
        } else if (q + 1 < 8) {
#pragma unroll
            for (int t = 0; t < 4; ++t) nx[t] = w.w1t(16 * (q - 3) + r, 16 * t + 4 * g);
        }
        f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        if (q < 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) acc = mfma(op[u], dz2b[u], acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) dz1b[q][i] = static_cast<short>(to_bf16(acc[i] * silu_d(z1[q][i])));
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) acc = mfma(op[t], dz1b[t], acc);
            dx[q - 4] = acc;
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) op[s] = nx[s];
        tile_fence();
    }
}

}  // namespace net
}  // namespace pod
