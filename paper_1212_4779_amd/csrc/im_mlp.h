// im_mlp.h -- the candidate-scoring network of the learned lazy order.
//
// 5 -> 64 -> 64 -> 1 with ReLU after both hidden layers. Weights are stored
// as bfloat16 (with FP32 master copies for training); every product is
// accumulated in FP32. Parameter vector layout (MLP_NP values):
//   W1[64][5], b1[64], W2[64][64], b2[64], w3[64], b3.
// Features of node u (each ln(1 + .)): in-degree, out-degree, sum of the
// out-arc probabilities, sum over the out-arcs (u, v) of out-degree(v), and
// the last exact gain of u divided by R. The network predicts ln(1 + g/R) of
// the current exact gain g; the lazy evaluation uses it only as an order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define MLP_IN 5
#define MLP_H 64
#define MLP_OFF_W1 0
#define MLP_OFF_B1 (MLP_OFF_W1 + MLP_H * MLP_IN)
#define MLP_OFF_W2 (MLP_OFF_B1 + MLP_H)
#define MLP_OFF_B2 (MLP_OFF_W2 + MLP_H * MLP_H)
#define MLP_OFF_W3 (MLP_OFF_B2 + MLP_H)
#define MLP_OFF_B3 (MLP_OFF_W3 + MLP_H)
#define MLP_NP (MLP_OFF_B3 + 1)

// device state of one network (owned by the library)
struct im_mlp {
    int device = -1;
    float *w = nullptr;      // [MLP_NP] FP32 master weights
    uint16_t *wb = nullptr;  // [MLP_NP] bfloat16 copies used by every forward pass
    float *am = nullptr;     // [MLP_NP] Adam first moments
    float *av = nullptr;     // [MLP_NP] Adam second moments
    uint32_t step = 0;       // Adam steps taken
    float *part = nullptr;   // [cap_part][MLP_NP + 1] per-workgroup partial gradients and loss
    uint32_t cap_part = 0;
};

__device__ __forceinline__ float bf16_bits_to_f32(uint16_t h)
{
    return __uint_as_float((uint32_t)h << 16);
}

// nearest bfloat16, ties to even (finite inputs)
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Stage the bfloat16 weights as FP32 in LDS (all threads of the block call).
__device__ __forceinline__ void mlp_stage(const uint16_t *wb, float *sw)
{
    for (int i = threadIdx.x; i < MLP_NP; i += blockDim.x) sw[i] = bf16_bits_to_f32(wb[i]);
    __syncthreads();
}

// Forward pass of one input with the weights staged in LDS.
__device__ __forceinline__ float mlp_eval(const float *sw, const float *x)
{
    float h1[MLP_H];
#pragma unroll
    for (int j = 0; j < MLP_H; j++) {
        float z = sw[MLP_OFF_B1 + j];
#pragma unroll
        for (int i = 0; i < MLP_IN; i++) z = fmaf(sw[MLP_OFF_W1 + j * MLP_IN + i], x[i], z);
        h1[j] = fmaxf(z, 0.0f);
    }
    float y = sw[MLP_OFF_B3];
    for (int j = 0; j < MLP_H; j++) {
        float z = sw[MLP_OFF_B2 + j];
#pragma unroll
        for (int i = 0; i < MLP_H; i++) z = fmaf(sw[MLP_OFF_W2 + j * MLP_H + i], h1[i], z);
        y = fmaf(sw[MLP_OFF_W3 + j], fmaxf(z, 0.0f), y);
    }
    return y;
}

// Forward pass of one input by a whole wavefront (all 64 lanes call it with
// the same x): lane j computes hidden unit j of both layers; the second
// layer takes the first layer's units lane by lane (uniform index: a scalar
// read of that lane), the output is a wavefront sum. Every lane returns y.
__device__ __forceinline__ float mlp_eval_wave(const float *sw, const float *x)
{
    static_assert(MLP_H == 64, "one hidden unit per lane");
    const int j = threadIdx.x & 63;
    float z = sw[MLP_OFF_B1 + j];
#pragma unroll
    for (int i = 0; i < MLP_IN; i++) z = fmaf(sw[MLP_OFF_W1 + j * MLP_IN + i], x[i], z);
    const float h1 = fmaxf(z, 0.0f);
    float z2 = sw[MLP_OFF_B2 + j];
#pragma unroll 16
    for (int i = 0; i < MLP_H; i++) {
        const float hi = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(h1), i));
        z2 = fmaf(sw[MLP_OFF_W2 + j * MLP_H + i], hi, z2);
    }
    float y = sw[MLP_OFF_W3 + j] * fmaxf(z2, 0.0f);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) y += __shfl_xor(y, d, 64);
    return y + sw[MLP_OFF_B3];
}
