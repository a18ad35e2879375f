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

// ---------------------------------------------------------------------------
// Forward pass of 16 inputs per wavefront on the matrix cores. The second
// layer, H2 = H1 W2^T with H1 [16 nodes][64] and W2 [64][64], is a dense
// contraction: 4 column tiles x 4 k-steps of v_mfma_f32_16x16x16_bf16
// (16 x 16 outputs, k = 16, FP32 accumulation). Lane layout of that
// instruction (A: 16 x 16, B: 16 x 16, D: 16 x 16): lane l supplies row l % 16
// of A and column l % 16 of B at k = 4 (l / 16) .. 4 (l / 16) + 3, and holds
// D rows 4 (l / 16) .. + 3 of column l % 16. So lane l computes the first-
// layer units it feeds to A itself (node l % 16, units 16 s + 4 (l / 16) + q)
// and no data moves between lanes before the multiply. The weights are
// bfloat16 already; an activation h enters as hi + lo, both bfloat16
// (hi = bf16(h), lo = bf16(h - hi)), two products per step, so the result is
// the FP32 network's to about 2^-16 relative.
// ---------------------------------------------------------------------------
typedef short mlp_v4s __attribute__((ext_vector_type(4)));
typedef float mlp_v4f __attribute__((ext_vector_type(4)));

struct MlpFrag {
    mlp_v4s b[4][4];        // W2 fragments: [column tile][k-step]
    float w1[16][MLP_IN];   // first-layer rows of this lane's 16 units
    float b1[16];
    float b2[4], w3[4];     // second-layer bias and output weight of column 16 t + l % 16
    float b3;
};

__device__ __forceinline__ uint32_t mlp_unit(int s, int q)   // k index of (k-step s, element q)
{
    return 16u * (uint32_t)s + 4u * ((threadIdx.x & 63u) >> 4) + (uint32_t)q;
}

__device__ __forceinline__ void mlp_frag_load(const uint16_t *wb, MlpFrag &f)
{
    const uint32_t c = threadIdx.x & 15u;
#pragma unroll
    for (int t = 0; t < 4; t++) {
        const uint32_t j = 16u * t + c;
#pragma unroll
        for (int s = 0; s < 4; s++) {
            mlp_v4s v;
#pragma unroll
            for (int q = 0; q < 4; q++) v[q] = (short)wb[MLP_OFF_W2 + j * MLP_H + mlp_unit(s, q)];
            f.b[t][s] = v;
        }
        f.b2[t] = bf16_bits_to_f32(wb[MLP_OFF_B2 + j]);
        f.w3[t] = bf16_bits_to_f32(wb[MLP_OFF_W3 + j]);
    }
#pragma unroll
    for (int s = 0; s < 4; s++)
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const uint32_t k = mlp_unit(s, q);
            f.b1[4 * s + q] = bf16_bits_to_f32(wb[MLP_OFF_B1 + k]);
#pragma unroll
            for (int i = 0; i < MLP_IN; i++)
                f.w1[4 * s + q][i] = bf16_bits_to_f32(wb[MLP_OFF_W1 + k * MLP_IN + i]);
        }
    f.b3 = bf16_bits_to_f32(wb[MLP_OFF_B3]);
}

// x: the input of node l % 16 (every lane of the wavefront calls, with its
// node's input). Returns, on lanes with l % 16 == 0, the outputs of nodes
// 4 (l / 16) .. 4 (l / 16) + 3 in y[0..3] (other lanes: partial sums).
__device__ __forceinline__ void mlp_tile_mfma(const MlpFrag &f, const float *x, float y[4])
{
    mlp_v4s ahi[4], alo[4];
#pragma unroll
    for (int s = 0; s < 4; s++)
#pragma unroll
        for (int q = 0; q < 4; q++) {
            float z = f.b1[4 * s + q];
#pragma unroll
            for (int i = 0; i < MLP_IN; i++) z = fmaf(f.w1[4 * s + q][i], x[i], z);
            const float h = fmaxf(z, 0.0f);
            const uint16_t hi = f32_to_bf16_bits(h);
            const uint16_t lo = f32_to_bf16_bits(h - bf16_bits_to_f32(hi));
            ahi[s][q] = (short)hi;
            alo[s][q] = (short)lo;
        }
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int t = 0; t < 4; t++) {
        mlp_v4f d = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < 4; s++) {
            d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi[s], f.b[t][s], d, 0, 0, 0);
            d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo[s], f.b[t][s], d, 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < 4; q++) acc[q] = fmaf(f.w3[t], fmaxf(d[q] + f.b2[t], 0.0f), acc[q]);
    }
    // sum over the 16 columns held by the 16 lanes of this row group
#pragma unroll
    for (int q = 0; q < 4; q++) {
        float v = acc[q];
#pragma unroll
        for (int m = 8; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
        y[q] = v + f.b3;
    }
}
