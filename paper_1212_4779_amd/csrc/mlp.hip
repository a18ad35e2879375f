// mlp.hip -- forward, backward and Adam kernels of the candidate-scoring
// network (im_mlp.h), and the training-sample gather.
//
// Training minimises L = (1 / (2N)) * sum_s (y_s - t_s)^2 over a batch of N
// samples. The gradient kernel gives every workgroup 64 samples (one per
// lane); the hidden activations and the back-propagated errors of those 64
// samples sit in LDS, so each weight gradient is a 64-term sum read from
// LDS. Workgroups write partial gradients that a second kernel sums in a
// fixed order, so a gradient never depends on scheduling.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "im.h"
#include "im_host.h"
#include "im_mlp.h"

constexpr int MG_S = 64;           // samples per gradient workgroup
constexpr int MG_LD = MLP_H + 1;   // padded LDS row (conflict-free column reads)

__global__ void k_mlp_to_bf16(const float *w, uint16_t *wb)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < MLP_NP) wb[i] = f32_to_bf16_bits(w[i]);
}

// 16 inputs per wavefront and step on the matrix cores (mlp_tile_mfma)
__global__ __launch_bounds__(256) void k_mlp_forward(const uint16_t *wb, const float *x, uint32_t N,
                                                     float *y)
{
    MlpFrag f;
    mlp_frag_load(wb, f);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = (blockIdx.x * 256u + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * 256u) >> 6;
    for (uint32_t base = wave * 16u; base < N; base += nwaves * 16u) {
        const uint32_t i = base + (lane & 15u);
        float xi[MLP_IN];
#pragma unroll
        for (int c = 0; c < MLP_IN; c++) xi[c] = i < N ? x[(uint64_t)i * MLP_IN + c] : 0.0f;
        float yo[4];
        mlp_tile_mfma(f, xi, yo);
        if ((lane & 15u) == 0)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const uint32_t o = base + 4u * (lane >> 4) + (uint32_t)q;
                if (o < N) y[o] = yo[q];
            }
    }
}

// One workgroup of MG_S lanes, lane s owns sample blockIdx.x * MG_S + s
// (taken through idx when idx != nullptr; an index >= nx contributes
// nothing). Writes this workgroup's share of
// dL/dparams and of L to part[blockIdx.x][0 .. MLP_NP].
__global__ __launch_bounds__(MG_S) void k_mlp_grad(const uint16_t *wb, const float *x,
                                                   const float *t, uint32_t nx, const uint32_t *idx,
                                                   uint32_t N, float *part)
{
    __shared__ float sw[MLP_NP];
    __shared__ float H1[MG_S * MG_LD];   // relu(z1), later dL/dz1
    __shared__ float D2[MG_S * MG_LD];   // relu(z2), later dL/dz2
    __shared__ float X[MG_S * MLP_IN];
    __shared__ float dd[MG_S];           // dL/dy per sample
    __shared__ float red[MG_S];
    mlp_stage(wb, sw);
    const int s = threadIdx.x;
    const uint32_t gs = blockIdx.x * MG_S + s;
    uint64_t src = gs < N ? (idx ? idx[gs] : gs) : 0;
    const bool valid = gs < N && src < nx;
    if (!valid) src = 0;
    float xs[MLP_IN];
#pragma unroll
    for (int c = 0; c < MLP_IN; c++) {
        xs[c] = valid ? x[src * MLP_IN + c] : 0.0f;
        X[s * MLP_IN + c] = xs[c];
    }
    // forward
    for (int j = 0; j < MLP_H; j++) {
        float z = sw[MLP_OFF_B1 + j];
#pragma unroll
        for (int c = 0; c < MLP_IN; c++) z = fmaf(sw[MLP_OFF_W1 + j * MLP_IN + c], xs[c], z);
        H1[s * MG_LD + j] = fmaxf(z, 0.0f);
    }
    float y = sw[MLP_OFF_B3];
    for (int j = 0; j < MLP_H; j++) {
        float z = sw[MLP_OFF_B2 + j];
        for (int i = 0; i < MLP_H; i++) z = fmaf(sw[MLP_OFF_W2 + j * MLP_H + i], H1[s * MG_LD + i], z);
        const float h = fmaxf(z, 0.0f);
        D2[s * MG_LD + j] = h;
        y = fmaf(sw[MLP_OFF_W3 + j], h, y);
    }
    const float r = valid ? y - t[src] : 0.0f;
    const float invN = 1.0f / (float)N;
    dd[s] = r * invN;
    red[s] = 0.5f * r * r * invN;
    __syncthreads();
    float *out = part + (uint64_t)blockIdx.x * (MLP_NP + 1);
    // output layer: lane j owns w3[j]
    {
        const int j = s;
        float g = 0.0f;
        for (int q = 0; q < MG_S; q++) g = fmaf(dd[q], D2[q * MG_LD + j], g);
        out[MLP_OFF_W3 + j] = g;
        if (s == 0) {
            float gb = 0.0f, l = 0.0f;
            for (int q = 0; q < MG_S; q++) { gb += dd[q]; l += red[q]; }
            out[MLP_OFF_B3] = gb;
            out[MLP_NP] = l;
        }
    }
    __syncthreads();
    // dL/dz2 of this lane's sample
    for (int j = 0; j < MLP_H; j++) {
        const float h = D2[s * MG_LD + j];
        D2[s * MG_LD + j] = h > 0.0f ? dd[s] * sw[MLP_OFF_W3 + j] : 0.0f;
    }
    __syncthreads();
    // second layer: lane j owns row j of W2 and b2[j]
    {
        const int j = s;
        float acc[MLP_H];
#pragma unroll
        for (int i = 0; i < MLP_H; i++) acc[i] = 0.0f;
        float gb = 0.0f;
        for (int q = 0; q < MG_S; q++) {
            const float d = D2[q * MG_LD + j];
            gb += d;
#pragma unroll
            for (int i = 0; i < MLP_H; i++) acc[i] = fmaf(d, H1[q * MG_LD + i], acc[i]);
        }
#pragma unroll
        for (int i = 0; i < MLP_H; i++) out[MLP_OFF_W2 + j * MLP_H + i] = acc[i];
        out[MLP_OFF_B2 + j] = gb;
    }
    __syncthreads();
    // dL/dz1 of this lane's sample (in place of relu(z1))
    for (int i = 0; i < MLP_H; i++) {
        float d1 = 0.0f;
        if (H1[s * MG_LD + i] > 0.0f)
            for (int j = 0; j < MLP_H; j++) d1 = fmaf(sw[MLP_OFF_W2 + j * MLP_H + i], D2[s * MG_LD + j], d1);
        H1[s * MG_LD + i] = d1;
    }
    __syncthreads();
    // first layer: lane i owns row i of W1 and b1[i]
    {
        const int i = s;
        float acc[MLP_IN] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        float gb = 0.0f;
        for (int q = 0; q < MG_S; q++) {
            const float d = H1[q * MG_LD + i];
            gb += d;
#pragma unroll
            for (int c = 0; c < MLP_IN; c++) acc[c] = fmaf(d, X[q * MLP_IN + c], acc[c]);
        }
#pragma unroll
        for (int c = 0; c < MLP_IN; c++) out[MLP_OFF_W1 + i * MLP_IN + c] = acc[c];
        out[MLP_OFF_B1 + i] = gb;
    }
}

// grad[p] = sum over workgroups b (in order) of part[b][p]; p = MLP_NP is the loss
__global__ void k_mlp_reduce(const float *part, uint32_t nblk, float *grad, float *loss)
{
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > MLP_NP) return;
    float g = 0.0f;
    for (uint32_t b = 0; b < nblk; b++) g += part[(uint64_t)b * (MLP_NP + 1) + p];
    if (p < MLP_NP) {
        if (grad) grad[p] = g;
    } else if (loss) {
        *loss = g;
    }
}

__global__ void k_mlp_adam(float *w, uint16_t *wb, float *am, float *av, const float *grad, float lr,
                           float b1, float b2, float eps, float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NP) return;
    const float g = grad[p];
    const float m = b1 * am[p] + (1.0f - b1) * g;
    const float v = b2 * av[p] + (1.0f - b2) * g * g;
    am[p] = m;
    av[p] = v;
    const float nw = w[p] - lr * (m / c1) / (sqrtf(v / c2) + eps);
    w[p] = nw;
    wb[p] = f32_to_bf16_bits(nw);
}

// x[s] = (feat[u][0..3], ln(1 + trace[tp][u] / R)), t[s] = ln(1 + trace[tc][u] / R);
// a sample whose node or rounds are out of range gets NaN everywhere
__global__ void k_mlp_samples(const float *feat, const uint32_t *trace, uint32_t n, uint32_t T,
                              float invR, const uint32_t *node, const uint32_t *tprev,
                              const uint32_t *tcur, uint32_t N, float *x, float *t)
{
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    const uint32_t u = node[s];
    if (u >= n || tprev[s] >= T || tcur[s] >= T) {
        for (int c = 0; c < MLP_IN; c++) x[(uint64_t)s * MLP_IN + c] = __builtin_nanf("");
        t[s] = __builtin_nanf("");
        return;
    }
#pragma unroll
    for (int c = 0; c < 4; c++) x[(uint64_t)s * MLP_IN + c] = feat[(uint64_t)u * 4 + c];
    x[(uint64_t)s * MLP_IN + 4] = log1pf((float)trace[(uint64_t)tprev[s] * n + u] * invR);
    t[s] = log1pf((float)trace[(uint64_t)tcur[s] * n + u] * invR);
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" int im_mlp_create(im_mlp **out)
{
    if (!out) return im_fail(IM_EINVAL, "im_mlp_create: null output pointer");
    im_mlp *m = new im_mlp();
    hipError_t e = hipGetDevice(&m->device);
    if (e == hipSuccess) e = hipMalloc((void **)&m->w, MLP_NP * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void **)&m->wb, MLP_NP * sizeof(uint16_t));
    if (e == hipSuccess) e = hipMalloc((void **)&m->am, MLP_NP * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void **)&m->av, MLP_NP * sizeof(float));
    if (e == hipSuccess) e = hipMemset(m->w, 0, MLP_NP * sizeof(float));
    if (e == hipSuccess) e = hipMemset(m->wb, 0, MLP_NP * sizeof(uint16_t));
    if (e == hipSuccess) e = hipMemset(m->am, 0, MLP_NP * sizeof(float));
    if (e == hipSuccess) e = hipMemset(m->av, 0, MLP_NP * sizeof(float));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (m->w) (void)hipFree(m->w);
        if (m->wb) (void)hipFree(m->wb);
        if (m->am) (void)hipFree(m->am);
        if (m->av) (void)hipFree(m->av);
        delete m;
        return im_fail(IM_ENOMEM, "im_mlp_create: %s", hipGetErrorString(e));
    }
    *out = m;
    return IM_OK;
}

extern "C" int im_mlp_destroy(im_mlp *m)
{
    if (!m) return IM_OK;
    (void)hipDeviceSynchronize();
    (void)hipFree(m->w);
    (void)hipFree(m->wb);
    (void)hipFree(m->am);
    (void)hipFree(m->av);
    if (m->part) (void)hipFree(m->part);
    delete m;
    return IM_OK;
}

extern "C" int im_mlp_set_params(im_mlp *m, const float *host_params)
{
    if (!m || !host_params) return im_fail(IM_EINVAL, "im_mlp_set_params: null argument");
    for (int i = 0; i < MLP_NP; i++)
        if (!std::isfinite(host_params[i]))
            return im_fail(IM_EINVAL, "im_mlp_set_params: parameter %d is not finite", i);
    HIPCHK(hipMemcpy(m->w, host_params, MLP_NP * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(hipMemset(m->am, 0, MLP_NP * sizeof(float)));
    HIPCHK(hipMemset(m->av, 0, MLP_NP * sizeof(float)));
    k_mlp_to_bf16<<<(MLP_NP + 255) / 256, 256>>>(m->w, m->wb);
    HIPCHK(hipGetLastError());
    HIPCHK(hipDeviceSynchronize());
    m->step = 0;
    return IM_OK;
}

extern "C" int im_mlp_get_params(const im_mlp *m, float *host_master, uint16_t *host_bf16)
{
    if (!m) return im_fail(IM_EINVAL, "im_mlp_get_params: null model");
    HIPCHK(hipDeviceSynchronize());
    if (host_master)
        HIPCHK(hipMemcpy(host_master, m->w, MLP_NP * sizeof(float), hipMemcpyDeviceToHost));
    if (host_bf16)
        HIPCHK(hipMemcpy(host_bf16, m->wb, MLP_NP * sizeof(uint16_t), hipMemcpyDeviceToHost));
    return IM_OK;
}

extern "C" int im_mlp_forward(const im_mlp *m, const float *x, uint32_t N, float *y, void *stream)
{
    if (!m) return im_fail(IM_EINVAL, "im_mlp_forward: null model");
    if (N == 0) return IM_OK;
    if (!x || !y) return im_fail(IM_EINVAL, "im_mlp_forward: null input or output");
    const unsigned g = (unsigned)std::min<uint64_t>(((uint64_t)N + 63) / 64, 8192);
    k_mlp_forward<<<g, 256, 0, (hipStream_t)stream>>>(m->wb, x, N, y);
    HIPCHK(hipGetLastError());
    return IM_OK;
}

static int mlp_grad(im_mlp *m, const float *x, const float *t, uint32_t nx, const uint32_t *idx,
                    uint32_t N, float *grad, float *loss, hipStream_t s)
{
    const uint32_t nblk = (N + MG_S - 1) / MG_S;
    if (nblk > m->cap_part) {
        HIPCHK(hipStreamSynchronize(s));
        if (m->part) (void)hipFree(m->part);
        m->part = nullptr;
        m->cap_part = 0;
        HIPCHK(hipMalloc((void **)&m->part, (uint64_t)nblk * (MLP_NP + 1) * sizeof(float)));
        m->cap_part = nblk;
    }
    k_mlp_grad<<<nblk, MG_S, 0, s>>>(m->wb, x, t, nx, idx, N, m->part);
    k_mlp_reduce<<<(MLP_NP + 1 + 255) / 256, 256, 0, s>>>(m->part, nblk, grad, loss);
    HIPCHK(hipGetLastError());
    return IM_OK;
}

extern "C" int im_mlp_loss_grad(im_mlp *m, const float *x, const float *t, uint32_t N, float *grad,
                                float *loss, void *stream)
{
    if (!m || !x || !t || N == 0) return im_fail(IM_EINVAL, "im_mlp_loss_grad: bad argument");
    return mlp_grad(m, x, t, N, nullptr, N, grad, loss, (hipStream_t)stream);
}

static int mlp_adam(im_mlp *m, const float *grad, float lr, float b1, float b2, float eps,
                    hipStream_t s)
{
    if (!(lr > 0.0f) || !(b1 >= 0.0f && b1 < 1.0f) || !(b2 >= 0.0f && b2 < 1.0f) || !(eps > 0.0f))
        return im_fail(IM_EINVAL, "Adam: need lr > 0, 0 <= beta1, beta2 < 1, eps > 0");
    m->step++;
    const float c1 = (float)(1.0 - std::pow((double)b1, (double)m->step));
    const float c2 = (float)(1.0 - std::pow((double)b2, (double)m->step));
    k_mlp_adam<<<(MLP_NP + 255) / 256, 256, 0, s>>>(m->w, m->wb, m->am, m->av, grad, lr, b1, b2, eps,
                                                    c1, c2);
    HIPCHK(hipGetLastError());
    return IM_OK;
}

extern "C" int im_mlp_adam(im_mlp *m, const float *grad, float lr, float beta1, float beta2,
                           float eps, void *stream)
{
    if (!m || !grad) return im_fail(IM_EINVAL, "im_mlp_adam: null argument");
    return mlp_adam(m, grad, lr, beta1, beta2, eps, (hipStream_t)stream);
}

extern "C" int im_mlp_train_step(im_mlp *m, const float *x, const float *t, uint32_t nsamples,
                                 const uint32_t *idx, uint32_t nbatch, float *grad_scratch,
                                 float *loss_out, float lr, float beta1, float beta2, float eps,
                                 void *stream)
{
    if (!m || !x || !t || !idx || !grad_scratch || nbatch == 0 || nsamples == 0)
        return im_fail(IM_EINVAL, "im_mlp_train_step: bad argument");
    int rc;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = mlp_grad(m, x, t, nsamples, idx, nbatch, grad_scratch, loss_out, s))) return rc;
    return mlp_adam(m, grad_scratch, lr, beta1, beta2, eps, s);
}

extern "C" int im_mlp_samples(const float *feat, const uint32_t *trace, uint32_t n, uint32_t T,
                              uint32_t R, const uint32_t *node, const uint32_t *tprev,
                              const uint32_t *tcur, uint32_t N, float *x_out, float *t_out,
                              void *stream)
{
    if (N == 0) return IM_OK;
    if (!feat || !trace || !node || !tprev || !tcur || !x_out || !t_out || R == 0 || n == 0 || T == 0)
        return im_fail(IM_EINVAL, "im_mlp_samples: bad argument");
    k_mlp_samples<<<(N + 255) / 256, 256, 0, (hipStream_t)stream>>>(
        feat, trace, n, T, 1.0f / (float)R, node, tprev, tcur, N, x_out, t_out);
    HIPCHK(hipGetLastError());
    return IM_OK;
}
