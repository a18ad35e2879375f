/*
 * sanitize_oracle.c -- drives every function of the CPU oracle on random
 * small graphs, built with AddressSanitizer and UndefinedBehaviorSanitizer
 * by tests/test_oracle_sanitized.py (CPU only). Besides the sanitizers'
 * own checks it asserts the equalities the oracle's three selection
 * algorithms must satisfy (Algorithm 1 = Algorithm 2 = lazy CELF, seeds and
 * gains), the pair-coin dynamic update = the component method on symmetric
 * graphs, and that spread prefixes of the selected seeds equal their gains.
 * Exit status 0: all held; 1: a mismatch (printed).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

uint64_t oracle_splitmix64_output(uint64_t state, uint64_t i);
int oracle_live_bits(uint64_t m, const float *prob, uint32_t R, uint64_t seed, uint64_t *bits);
int oracle_live_bits_lt(uint32_t n, uint64_t m, const uint64_t *row_ptr, const uint32_t *col,
                        const float *prob, uint32_t R, uint64_t seed, uint64_t *bits);
int oracle_initial_gains(uint32_t n, uint64_t m, const uint64_t *row_ptr, const uint32_t *col,
                         const float *prob, uint32_t R, uint64_t seed, uint32_t *gain_out,
                         uint64_t *stats);
int oracle_select_du(uint32_t n, uint64_t m, const uint64_t *row_ptr, const uint32_t *col,
                     const float *prob, uint32_t R, uint32_t k, uint64_t seed, uint32_t *seeds,
                     uint64_t *gains, uint32_t *trace, uint64_t *stats);
int oracle_select_du_lt(uint32_t n, uint64_t m, const uint64_t *row_ptr, const uint32_t *col,
                        const float *prob, uint32_t R, uint32_t k, uint64_t seed, uint32_t *seeds,
                        uint64_t *gains, uint32_t *trace, uint64_t *stats);
int oracle_select_alg1(uint32_t n, uint64_t m, const uint64_t *row_ptr, const uint32_t *col,
                       const float *prob, uint32_t R, uint32_t k, uint64_t seed, uint32_t *seeds,
                       uint64_t *gains);
int oracle_select_celf(uint32_t n, uint64_t m, const uint64_t *row_ptr, const uint32_t *col,
                       const float *prob, uint32_t R, uint32_t k, uint64_t seed, uint32_t *seeds,
                       uint64_t *gains, uint64_t *stats);
int oracle_spread_prefix(uint32_t n, uint64_t m, const uint64_t *row_ptr, const uint32_t *col,
                         const float *prob, uint32_t R, uint64_t seed, const uint32_t *S,
                         uint32_t nS, uint64_t *marg, uint32_t *per);
int oracle_pair_ids(uint32_t n, uint64_t m, const uint64_t *row_ptr, const uint32_t *col,
                    const float *prob, uint32_t *pair);
int oracle_select_du_pairs(uint32_t n, uint64_t m, const uint64_t *row_ptr, const uint32_t *col,
                           const float *prob, uint32_t R, uint32_t k, uint64_t seed,
                           uint32_t *seeds, uint64_t *gains, uint32_t *trace, uint64_t *stats);
int oracle_select_components(uint32_t n, uint64_t m, const uint64_t *row_ptr, const uint32_t *col,
                             const float *prob, uint32_t R, uint32_t k, uint64_t seed,
                             uint32_t *seeds, uint64_t *gains, uint32_t *trace);
int oracle_mlp_nparams(void);
void oracle_bf16_round(uint64_t cnt, const float *in, float *out);
int oracle_node_features(uint32_t n, uint64_t m, const uint64_t *row_ptr, const uint32_t *col,
                         const float *prob, double *feat);
void oracle_mlp_forward(const double *params, uint64_t N, const double *x, double *y);
double oracle_mlp_loss_grad(const double *params, uint64_t N, const double *x, const double *t,
                            double *grad);
void oracle_adam_step(uint64_t cnt, double *theta, double *m, double *v, const double *g,
                      double lr, double b1, double b2, double eps, uint32_t t);

static uint64_t rng_state = 12345;
static uint32_t rnd(uint32_t bound)   /* a plain LCG: test inputs only */
{
    rng_state = rng_state * 6364136223846793005ULL + 1442695040888963407ULL;
    return (uint32_t)((rng_state >> 33) % bound);
}

/* CSR of n nodes and m arcs (u, v), u != v; symmetric: both directions, equal p */
static int make_graph(uint32_t n, uint32_t m, int symmetric, uint64_t **row_ptr, uint32_t **col,
                      float **prob, uint64_t *m_out)
{
    uint32_t cap = symmetric ? 2 * m : m;
    uint32_t *src = malloc(cap * sizeof(uint32_t)), *dst = malloc(cap * sizeof(uint32_t));
    float *p = malloc(cap * sizeof(float));
    uint32_t cnt = 0;
    for (uint32_t i = 0; i < m; i++) {
        uint32_t u = rnd(n), v = rnd(n);
        if (u == v) continue;
        int dup = 0;   /* no pair twice (in either direction when symmetric) */
        for (uint32_t j = 0; j < cnt && !dup; j++)
            dup = (src[j] == u && dst[j] == v) || (symmetric && src[j] == v && dst[j] == u);
        if (dup) continue;
        float pr = (float)(rnd(1000) + 1) / 1000.0f;
        src[cnt] = u; dst[cnt] = v; p[cnt] = pr; cnt++;
        if (symmetric) { src[cnt] = v; dst[cnt] = u; p[cnt] = pr; cnt++; }
    }
    *row_ptr = calloc((size_t)n + 1, sizeof(uint64_t));
    *col = malloc((cnt ? cnt : 1) * sizeof(uint32_t));
    *prob = malloc((cnt ? cnt : 1) * sizeof(float));
    for (uint32_t i = 0; i < cnt; i++) (*row_ptr)[src[i] + 1]++;
    for (uint32_t u = 0; u < n; u++) (*row_ptr)[u + 1] += (*row_ptr)[u];
    uint64_t *cur = malloc(((size_t)n + 1) * sizeof(uint64_t));
    memcpy(cur, *row_ptr, ((size_t)n + 1) * sizeof(uint64_t));
    for (uint32_t i = 0; i < cnt; i++) {
        uint64_t at = cur[src[i]]++;
        (*col)[at] = dst[i];
        (*prob)[at] = p[i];
    }
    free(cur); free(src); free(dst); free(p);
    *m_out = cnt;
    return 0;
}

static int fail(const char *what, int c) { printf("mismatch: %s (case %d)\n", what, c); return 1; }

int main(void)
{
    int bad = 0;
    for (int c = 0; c < 24 && !bad; c++) {
        uint32_t n = 3 + rnd(14), R = (uint32_t[]){1, 5, 64, 70, 130}[rnd(5)];
        uint32_t k = 1 + rnd(n);
        uint64_t seed = ((uint64_t)rnd(1u << 30) << 20) ^ (uint64_t)c, m;
        uint64_t *row; uint32_t *col; float *prob;
        make_graph(n, 3 * n, 0, &row, &col, &prob, &m);
        uint32_t W = (R + 63) / 64;
        uint64_t *bits = malloc((m ? m : 1) * W * sizeof(uint64_t));
        if (oracle_live_bits(m, prob, R, seed, bits)) bad |= fail("live_bits", c);
        uint32_t *gain = malloc(n * sizeof(uint32_t));
        uint64_t st[8], st2[8], st3[8];
        if (oracle_initial_gains(n, m, row, col, prob, R, seed, gain, st)) bad |= fail("initial", c);
        uint32_t *s1 = malloc(k * sizeof(uint32_t)), *s2 = malloc(k * sizeof(uint32_t)),
                 *s3 = malloc(k * sizeof(uint32_t));
        uint64_t *g1 = malloc(k * sizeof(uint64_t)), *g2 = malloc(k * sizeof(uint64_t)),
                 *g3 = malloc(k * sizeof(uint64_t));
        uint32_t *trace = malloc((size_t)(k + 1) * n * sizeof(uint32_t));
        if (oracle_select_du(n, m, row, col, prob, R, k, seed, s1, g1, trace, st2)) bad |= fail("du", c);
        if (oracle_select_alg1(n, m, row, col, prob, R, k, seed, s2, g2)) bad |= fail("alg1", c);
        if (oracle_select_celf(n, m, row, col, prob, R, k, seed, s3, g3, st3)) bad |= fail("celf", c);
        for (uint32_t i = 0; i < k; i++)
            if (s1[i] != s2[i] || s1[i] != s3[i] || g1[i] != g2[i] || g1[i] != g3[i])
                bad |= fail("alg1 = du = celf", c);
        for (uint32_t u = 0; u < n; u++)
            if (trace[u] != gain[u]) bad |= fail("trace[0] = initial gains", c);
        uint64_t *marg = malloc(k * sizeof(uint64_t));
        uint32_t *per = malloc(R * sizeof(uint32_t));
        if (oracle_spread_prefix(n, m, row, col, prob, R, seed, s1, k, marg, per))
            bad |= fail("spread", c);
        for (uint32_t i = 0; i < k; i++)
            if (marg[i] != g1[i]) bad |= fail("spread prefix = gains", c);
        /* linear threshold */
        uint64_t *lbits = malloc((m ? m : 1) * W * sizeof(uint64_t));
        if (oracle_live_bits_lt(n, m, row, col, prob, R, seed, lbits)) bad |= fail("lt bits", c);
        if (oracle_select_du_lt(n, m, row, col, prob, R, k, seed, s2, g2, NULL, NULL))
            bad |= fail("lt du", c);
        /* network */
        double *feat = malloc((size_t)n * 4 * sizeof(double));
        if (oracle_node_features(n, m, row, col, prob, feat)) bad |= fail("features", c);
        free(bits); free(gain); free(s1); free(s2); free(s3); free(g1); free(g2); free(g3);
        free(trace); free(marg); free(per); free(lbits); free(feat);
        free(row); free(col); free(prob);
        /* undirected: pair coins = component method */
        make_graph(n, 2 * n, 1, &row, &col, &prob, &m);
        uint32_t *pair = malloc((m ? m : 1) * sizeof(uint32_t));
        if (oracle_pair_ids(n, m, row, col, prob, pair)) bad |= fail("pair ids", c);
        s1 = malloc(k * sizeof(uint32_t)); s2 = malloc(k * sizeof(uint32_t));
        g1 = malloc(k * sizeof(uint64_t)); g2 = malloc(k * sizeof(uint64_t));
        if (oracle_select_du_pairs(n, m, row, col, prob, R, k, seed, s1, g1, NULL, NULL))
            bad |= fail("du pairs", c);
        if (oracle_select_components(n, m, row, col, prob, R, k, seed, s2, g2, NULL))
            bad |= fail("components", c);
        for (uint32_t i = 0; i < k; i++)
            if (s1[i] != s2[i] || g1[i] != g2[i]) bad |= fail("pairs du = components", c);
        free(pair); free(s1); free(s2); free(g1); free(g2);
        free(row); free(col); free(prob);
    }
    /* network reference: forward, loss gradient, Adam, bf16 rounding */
    const int np = oracle_mlp_nparams();
    double *prm = malloc(np * sizeof(double)), *grad = malloc(np * sizeof(double));
    double *mm = calloc(np, sizeof(double)), *vv = calloc(np, sizeof(double));
    float *f32 = malloc(np * sizeof(float)), *b16 = malloc(np * sizeof(float));
    for (int i = 0; i < np; i++) { prm[i] = ((double)rnd(2001) - 1000.0) / 4000.0; f32[i] = (float)prm[i]; }
    oracle_bf16_round((uint64_t)np, f32, b16);
    double x[40 * 5], t[40], y[40];
    for (int i = 0; i < 40 * 5; i++) x[i] = (double)rnd(1000) / 250.0;
    for (int i = 0; i < 40; i++) t[i] = (double)rnd(1000) / 500.0;
    oracle_mlp_forward(prm, 40, x, y);
    const double loss = oracle_mlp_loss_grad(prm, 40, x, t, grad);
    oracle_adam_step((uint64_t)np, prm, mm, vv, grad, 1e-3, 0.9, 0.999, 1e-8, 1);
    if (!(loss >= 0.0)) bad |= fail("loss", -1);
    free(prm); free(grad); free(mm); free(vv); free(f32); free(b16);
    if (oracle_splitmix64_output(0, 1) != 0xE220A8397B1DCDAFULL) bad |= fail("splitmix64", -1);
    printf(bad ? "FAILED\n" : "ok\n");
    return bad;
}
