/*
 * mlp.c -- FP64 reference of the candidate-scoring network of the learned
 * lazy evaluation order, its training gradients and its optimiser step.
 *
 * TEST INFRASTRUCTURE ONLY, like oracle.c: the GPU path never loads it.
 *
 * The paper's lazy variant (StaticGreedyCELF, Sec. 5) re-evaluates stale
 * upper bounds in bound order. The learned order replaces only that order
 * with the score of a small network; exact gains still decide every pick.
 * What this file fixes:
 *
 * Node features (static part, per node u of the out-CSR):
 *   f0 = ln(1 + in-degree(u))
 *   f1 = ln(1 + out-degree(u))
 *   f2 = ln(1 + sum of p over the out-arcs of u)
 *   f3 = ln(1 + sum over the out-arcs (u, v) of out-degree(v))
 * and the dynamic part f4 = ln(1 + g / R), g the last exact gain of u
 * (summed over R snapshots). The regression target is ln(1 + g_t / R) for
 * the exact gain g_t of a later round.
 *
 * Network 5 -> 64 -> 64 -> 1 with ReLU after both hidden layers:
 *   h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = w3 . h2 + b3.
 * Parameter vector (4609 values, this order): W1[64][5], b1[64], W2[64][64],
 * b2[64], w3[64], b3.
 * Loss over N samples: L = (1 / (2N)) * sum_s (y_s - t_s)^2; gradients by
 * the chain rule (backpropagation), all in double.
 *
 * bfloat16 rounding (the stored precision of the weights): a finite binary32
 * value is rounded to the nearest value with 8 significant bits, ties to the
 * one with an even last bit (IEEE-754 round-to-nearest-even), written here
 * through frexp / nearbyint.
 *
 * Adam (Kingma & Ba, ICLR 2015, Algorithm 1), step t >= 1:
 *   m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2;
 *   theta -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 */
#include <fenv.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MLP_IN 5
#define MLP_H 64
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + MLP_H * MLP_IN)
#define OFF_W2 (OFF_B1 + MLP_H)
#define OFF_B2 (OFF_W2 + MLP_H * MLP_H)
#define OFF_W3 (OFF_B2 + MLP_H)
#define OFF_B3 (OFF_W3 + MLP_H)
#define MLP_NP (OFF_B3 + 1)

int oracle_mlp_nparams(void) { return MLP_NP; }

static double round_bf16(double x)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    (void)frexp(x, &e);              /* x = f * 2^e, 0.5 <= |f| < 1 */
    const double scale = ldexp(1.0, 8 - e);
    return nearbyint(x * scale) / scale;  /* 8 significant bits, ties to even */
}

void oracle_bf16_round(uint64_t cnt, const float *in, float *out)
{
    fesetround(FE_TONEAREST);
    for (uint64_t i = 0; i < cnt; i++) out[i] = (float)round_bf16((double)in[i]);
}

int oracle_node_features(uint32_t n, uint64_t m, const uint64_t *row_ptr, const uint32_t *col,
                         const float *prob, double *feat)
{
    uint64_t *indeg = calloc(n ? n : 1, sizeof(uint64_t));
    if (!indeg) return -1;
    for (uint64_t e = 0; e < m; e++) indeg[col[e]]++;
    for (uint32_t u = 0; u < n; u++) {
        double psum = 0.0, two = 0.0;
        for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
            psum += prob[e];
            two += (double)(row_ptr[col[e] + 1] - row_ptr[col[e]]);
        }
        feat[4 * (uint64_t)u + 0] = log1p((double)indeg[u]);
        feat[4 * (uint64_t)u + 1] = log1p((double)(row_ptr[u + 1] - row_ptr[u]));
        feat[4 * (uint64_t)u + 2] = log1p(psum);
        feat[4 * (uint64_t)u + 3] = log1p(two);
    }
    free(indeg);
    return 0;
}

static double relu(double z) { return z > 0.0 ? z : 0.0; }

/* forward pass of one sample; h1, z2 receive the hidden pre/post values */
static double forward1(const double *p, const double *x, double *z1, double *z2)
{
    for (int j = 0; j < MLP_H; j++) {
        double z = p[OFF_B1 + j];
        for (int i = 0; i < MLP_IN; i++) z += p[OFF_W1 + j * MLP_IN + i] * x[i];
        z1[j] = z;
    }
    double y = p[OFF_B3];
    for (int j = 0; j < MLP_H; j++) {
        double z = p[OFF_B2 + j];
        for (int i = 0; i < MLP_H; i++) z += p[OFF_W2 + j * MLP_H + i] * relu(z1[i]);
        z2[j] = z;
        y += p[OFF_W3 + j] * relu(z);
    }
    return y;
}

void oracle_mlp_forward(const double *params, uint64_t N, const double *x, double *y)
{
    double z1[MLP_H], z2[MLP_H];
    for (uint64_t s = 0; s < N; s++) y[s] = forward1(params, x + MLP_IN * s, z1, z2);
}

/* L and dL/dparams (grad: MLP_NP values, overwritten) */
double oracle_mlp_loss_grad(const double *params, uint64_t N, const double *x, const double *t,
                            double *grad)
{
    memset(grad, 0, MLP_NP * sizeof(double));
    if (N == 0) return 0.0;
    double loss = 0.0;
    double z1[MLP_H], z2[MLP_H], d2[MLP_H];
    for (uint64_t s = 0; s < N; s++) {
        const double *xs = x + MLP_IN * s;
        const double y = forward1(params, xs, z1, z2);
        const double r = y - t[s];
        loss += 0.5 * r * r / (double)N;
        const double dy = r / (double)N;           /* dL/dy */
        grad[OFF_B3] += dy;
        for (int j = 0; j < MLP_H; j++) {
            grad[OFF_W3 + j] += dy * relu(z2[j]);
            d2[j] = z2[j] > 0.0 ? dy * params[OFF_W3 + j] : 0.0;   /* dL/dz2 */
        }
        for (int j = 0; j < MLP_H; j++) {
            grad[OFF_B2 + j] += d2[j];
            for (int i = 0; i < MLP_H; i++) grad[OFF_W2 + j * MLP_H + i] += d2[j] * relu(z1[i]);
        }
        for (int i = 0; i < MLP_H; i++) {
            if (!(z1[i] > 0.0)) continue;
            double d1 = 0.0;                         /* dL/dz1 */
            for (int j = 0; j < MLP_H; j++) d1 += params[OFF_W2 + j * MLP_H + i] * d2[j];
            grad[OFF_B1 + i] += d1;
            for (int c = 0; c < MLP_IN; c++) grad[OFF_W1 + i * MLP_IN + c] += d1 * xs[c];
        }
    }
    return loss;
}

void oracle_adam_step(uint64_t cnt, double *theta, double *m, double *v, const double *g,
                      double lr, double b1, double b2, double eps, uint32_t t)
{
    const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (uint64_t i = 0; i < cnt; i++) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        theta[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}
