/*
 * oracle.c -- plain, slow, single-threaded CPU StaticGreedy.
 *
 * TEST INFRASTRUCTURE ONLY. The test suite, the smoke check and the
 * benchmark's CPU-baseline leg are the only code that loads this library.
 * The GPU product path never calls it, and the two share no code, header,
 * table or helper.
 *
 * What it computes follows Cheng et al., "StaticGreedy: Solving the
 * Scalability-Accuracy Dilemma in Influence Maximization" (CIKM 2013,
 * arXiv 1212.4779):
 *   - the independent cascade (IC) model and the snapshot estimator
 *     (Sec. 3.1): a snapshot keeps arc <u,v> with probability p(u,v); the
 *     spread of S in a snapshot is the number of nodes reachable from S;
 *   - StaticGreedy (Sec. 3.3, Algorithm 1): sample R snapshots once, then
 *     k greedy rounds, each adding the node with the largest summed spread;
 *   - StaticGreedyDU (Sec. 4, Algorithm 2): per-node gains kept current by
 *     deleting every newly reached node w from R(G'_i,u) for all u in
 *     U(G'_i,w), one decrement each;
 *   - StaticGreedyCELF (Sec. 5, the compared lazy-evaluation variant):
 *     stale gains as upper bounds, exact re-evaluation on demand.
 * Every function below restates the paper's steps in its own order; none
 * of them blocks, fuses or reorders work beyond the definition.
 *
 * Readings of the paper used here (the paper is silent on each):
 *   R1  a node reaches itself: u is in R(G'_i,u), so initial s_u >= R
 *       (Sec. 3.1 counts seeds as activated; Algorithm 1 sums the spread
 *       of S u {v}, which includes v).
 *   R2  gains are integers summed over snapshots, not divided by R; the
 *       argmax is unchanged because R > 0 (Algorithm 1's s_v/R).
 *   R3  argmax ties go to the lowest node id; candidates are V \ S.
 *   R4  when every remaining gain is 0 the round still adds the lowest
 *       unselected id (Algorithm 1 always adds an argmax); k <= n.
 *   R5  coin flips: one Bernoulli(p) per (stored arc, snapshot), drawn by
 *       the counter-based generator below (Sec. 3.1 leaves the RNG open).
 *   R6  Algorithm 2's inner loop runs over the nodes newly reached from v*
 *       in snapshot i (the sets are the ones already shrunk by earlier
 *       deletions), iterated over a copy; the reverse sets U(G'_i,w) are
 *       taken on the whole snapshot.
 *
 * Counter-based edge generator (R5). SplitMix64, Steele, Lea & Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014: a
 * generator with state s returns, as its i-th output (i >= 1),
 * mix(s + i*gamma) with gamma = 0x9e3779b97f4a7c15 and mix the 64-bit
 * finaliser published with it (xor-shift 30, multiply, xor-shift 27,
 * multiply, xor-shift 31). Here:
 *   key_e   = output (e+1) of a generator with state seed
 *   draw_er = top 32 bits of output (r+1) of a generator with state key_e
 *   t_e     = floor(p_e * 2^32)          (exact in double for float p_e)
 *   arc e is live in snapshot r  <=>  draw_er < t_e
 * Snapshot r maps to bit (r mod 64) of word floor(r / 64); bits for
 * r >= R are zero.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)
#define ORACLE_EINTERNAL (-3)

/* ---------------- SplitMix64 (published definition) ---------------- */

static uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* i-th output (i >= 1) of a SplitMix64 generator whose state starts at s */
static uint64_t sm64_output(uint64_t s, uint64_t i)
{
    return sm64_mix(s + i * 0x9e3779b97f4a7c15ULL);
}

uint64_t oracle_splitmix64_output(uint64_t state, uint64_t i)
{
    return sm64_output(state, i);
}

/* Sec. 3.1 "Snapshot": arc e kept in snapshot r with probability p_e */
static int arc_live(uint64_t key, uint32_t r, uint64_t thr)
{
    uint64_t draw = sm64_output(key, (uint64_t)r + 1u) >> 32;
    return draw < thr;
}

static uint64_t arc_threshold(float p)
{
    /* p in [0,1]; float * 2^32 is exact in double; floor == truncation */
    return (uint64_t)floor((double)p * 4294967296.0);
}

/* live bits, arc-major: bits[e*W + w], bit b of word w is snapshot 64w+b.
 * The coin of arc e is drawn under the index key_of[e] (NULL: e itself), so
 * arcs that share an index share every coin (one coin per undirected pair). */
int oracle_live_bits_keyed(uint64_t m, const float *prob, uint32_t R, uint64_t seed,
                           const uint32_t *key_of, uint64_t *bits)
{
    uint32_t W = (R + 63u) / 64u;
    for (uint64_t e = 0; e < m; e++) {
        uint64_t key = sm64_output(seed, (key_of ? (uint64_t)key_of[e] : e) + 1u);
        uint64_t thr = arc_threshold(prob[e]);
        for (uint32_t w = 0; w < W; w++) bits[e * W + w] = 0;
        for (uint32_t r = 0; r < R; r++)
            if (arc_live(key, r, thr))
                bits[e * W + r / 64u] |= 1ULL << (r % 64u);
    }
    return ORACLE_OK;
}

int oracle_live_bits(uint64_t m, const float *prob, uint32_t R, uint64_t seed,
                     uint64_t *bits)
{
    return oracle_live_bits_keyed(m, prob, R, seed, NULL, bits);
}

/*
 * Linear threshold model in its live-edge form (the paper states that the
 * method extends to it): in each snapshot every node keeps at most one of
 * its in-arcs, arc e with probability b_e, none with the rest.
 * Reading: b_e is prob[e]; the in-arcs of v, in increasing arc id, own
 * consecutive sub-intervals of [0, 2^32) of lengths floor(b_e * 2^32) (the
 * part of an interval past 2^32 is cut off); in snapshot r the node's draw,
 * the top 32 bits of output r+1 of SplitMix64 seeded with output v+1 of
 * SplitMix64(seed), keeps the arc whose sub-interval holds it.
 * bits: arc-major as oracle_live_bits.
 */
int oracle_live_bits_lt(uint32_t n, uint64_t m, const uint64_t *row_ptr, const uint32_t *col,
                        const float *prob, uint32_t R, uint64_t seed, uint64_t *bits)
{
    uint32_t W = (R + 63u) / 64u;
    /* in-arcs of every node in increasing arc id (a stable counting sort) */
    uint64_t *start = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    uint64_t *in_arc = (uint64_t *)malloc((m ? m : 1) * sizeof(uint64_t));
    if (!start || !in_arc) { free(start); free(in_arc); return ORACLE_ENOMEM; }
    for (uint64_t e = 0; e < m; e++) start[col[e] + 1]++;
    for (uint32_t v = 0; v < n; v++) start[v + 1] += start[v];
    uint64_t *cur = (uint64_t *)malloc(((size_t)n + 1) * sizeof(uint64_t));
    if (!cur) { free(start); free(in_arc); return ORACLE_ENOMEM; }
    memcpy(cur, start, ((size_t)n + 1) * sizeof(uint64_t));
    for (uint32_t u = 0; u < n; u++)
        for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) in_arc[cur[col[e]]++] = e;
    free(cur);
    memset(bits, 0, (m ? m : 1) * W * sizeof(uint64_t));
    for (uint32_t v = 0; v < n; v++) {
        uint64_t key = sm64_output(seed, (uint64_t)v + 1u);
        for (uint32_t r = 0; r < R; r++) {
            uint64_t d = sm64_output(key, (uint64_t)r + 1u) >> 32;
            uint64_t lo = 0;
            for (uint64_t i = start[v]; i < start[v + 1]; i++) {
                uint64_t e = in_arc[i];
                uint64_t hi = lo + arc_threshold(prob[e]);
                if (d >= lo && d < hi) {
                    bits[e * W + r / 64u] |= 1ULL << (r % 64u);
                    break;
                }
                lo = hi;
            }
        }
    }
    free(start); free(in_arc);
    return ORACLE_OK;
}

/* ---------------- input checks ---------------- */

static int check_graph(uint32_t n, uint64_t m, const uint64_t *row_ptr,
                       const uint32_t *col, const float *prob, uint32_t R)
{
    if (R == 0 || R > 4096u) return ORACLE_EINVAL;
    if (m >= (1ULL << 32)) return ORACLE_EINVAL;
    if ((uint64_t)n * (uint64_t)R >= (1ULL << 32)) return ORACLE_EINVAL;
    if (row_ptr[0] != 0 || row_ptr[n] != m) return ORACLE_EINVAL;
    for (uint32_t u = 0; u < n; u++)
        if (row_ptr[u + 1] < row_ptr[u]) return ORACLE_EINVAL;
    for (uint64_t e = 0; e < m; e++) {
        if (col[e] >= n) return ORACLE_EINVAL;
        if (!(prob[e] >= 0.0f && prob[e] <= 1.0f)) return ORACLE_EINVAL;
    }
    return ORACLE_OK;
}

/* ---------------- the R static snapshots (Algorithm 1, sampling loop) ---- */

typedef struct {
    uint32_t n, R;
    uint64_t *fbase, *rbase;   /* [R] start of snapshot r's arc list   */
    uint32_t *fptr, *rptr;     /* [R][n+1] offsets inside snapshot r    */
    uint32_t *fadj, *radj;     /* live heads (forward) / tails (reverse) */
    uint64_t nlive;            /* total (arc, snapshot) pairs kept      */
} snaps_t;

static void snaps_free(snaps_t *g)
{
    free(g->fbase); free(g->rbase); free(g->fptr); free(g->rptr);
    free(g->fadj); free(g->radj);
    memset(g, 0, sizeof(*g));
}

/* lt = 1: linear-threshold snapshots (key_of unused) */
static int snaps_build_keyed(snaps_t *g, uint32_t n, uint64_t m, const uint64_t *row_ptr,
                             const uint32_t *col, const float *prob, uint32_t R,
                             uint64_t seed, const uint32_t *key_of, int lt)
{
    uint32_t W = (R + 63u) / 64u;
    uint64_t stride = (uint64_t)n + 1u;
    memset(g, 0, sizeof(*g));
    g->n = n; g->R = R;
    uint64_t *bits = (uint64_t *)malloc((m ? m : 1) * W * sizeof(uint64_t));
    g->fbase = (uint64_t *)calloc(R, sizeof(uint64_t));
    g->rbase = (uint64_t *)calloc(R, sizeof(uint64_t));
    g->fptr = (uint32_t *)calloc((size_t)R * stride, sizeof(uint32_t));
    g->rptr = (uint32_t *)calloc((size_t)R * stride, sizeof(uint32_t));
    if (!bits || !g->fbase || !g->rbase || !g->fptr || !g->rptr) {
        free(bits); snaps_free(g); return ORACLE_ENOMEM;
    }
    if (lt) {
        if (oracle_live_bits_lt(n, m, row_ptr, col, prob, R, seed, bits)) {
            free(bits); snaps_free(g); return ORACLE_ENOMEM;
        }
    } else {
        oracle_live_bits_keyed(m, prob, R, seed, key_of, bits);
    }

    /* count live out-arcs and in-arcs per (snapshot, node) */
    for (uint32_t u = 0; u < n; u++)
        for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++)
            for (uint32_t w = 0; w < W; w++) {
                uint64_t b = bits[e * W + w];
                while (b) {
                    uint32_t r = w * 64u + (uint32_t)__builtin_ctzll(b);
                    b &= b - 1;
                    g->fptr[(uint64_t)r * stride + u + 1]++;
                    g->rptr[(uint64_t)r * stride + col[e] + 1]++;
                    g->nlive++;
                }
            }
    uint64_t tot = 0;
    for (uint32_t r = 0; r < R; r++) {
        uint32_t *fp = g->fptr + (uint64_t)r * stride;
        uint32_t *rp = g->rptr + (uint64_t)r * stride;
        for (uint32_t x = 0; x < n; x++) { fp[x + 1] += fp[x]; rp[x + 1] += rp[x]; }
        g->fbase[r] = tot;
        g->rbase[r] = tot;
        tot += fp[n];
    }
    g->fadj = (uint32_t *)malloc((tot ? tot : 1) * sizeof(uint32_t));
    g->radj = (uint32_t *)malloc((tot ? tot : 1) * sizeof(uint32_t));
    if (!g->fadj || !g->radj) { free(bits); snaps_free(g); return ORACLE_ENOMEM; }
    /* fill, using the offsets as cursors, then shift them back */
    for (uint32_t u = 0; u < n; u++)
        for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++)
            for (uint32_t w = 0; w < W; w++) {
                uint64_t b = bits[e * W + w];
                while (b) {
                    uint32_t r = w * 64u + (uint32_t)__builtin_ctzll(b);
                    b &= b - 1;
                    uint32_t *fp = g->fptr + (uint64_t)r * stride;
                    uint32_t *rp = g->rptr + (uint64_t)r * stride;
                    g->fadj[g->fbase[r] + fp[u]++] = col[e];
                    g->radj[g->rbase[r] + rp[col[e]]++] = u;
                }
            }
    for (uint32_t r = 0; r < R; r++) {
        uint32_t *fp = g->fptr + (uint64_t)r * stride;
        uint32_t *rp = g->rptr + (uint64_t)r * stride;
        for (uint32_t x = n; x > 0; x--) { fp[x] = fp[x - 1]; rp[x] = rp[x - 1]; }
        fp[0] = 0; rp[0] = 0;
    }
    free(bits);
    return ORACLE_OK;
}

static int snaps_build(snaps_t *g, uint32_t n, uint64_t m, const uint64_t *row_ptr,
                       const uint32_t *col, const float *prob, uint32_t R,
                       uint64_t seed)
{
    return snaps_build_keyed(g, n, m, row_ptr, col, prob, R, seed, NULL, 0);
}

/* ---------------- reachability inside one snapshot ---------------- */

typedef struct {
    uint32_t *stamp;  /* [n] visit stamps */
    uint32_t cur;     /* current stamp    */
    uint32_t *queue;  /* [n] visit order  */
} bfs_ws;

static int ws_init(bfs_ws *ws, uint32_t n)
{
    ws->stamp = (uint32_t *)calloc(n ? n : 1, sizeof(uint32_t));
    ws->queue = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    ws->cur = 0;
    return (ws->stamp && ws->queue) ? ORACLE_OK : ORACLE_ENOMEM;
}

static void ws_free(bfs_ws *ws) { free(ws->stamp); free(ws->queue); }

static void ws_next(bfs_ws *ws, uint32_t n)
{
    if (++ws->cur == 0) {  /* wrapped: clear all stamps */
        memset(ws->stamp, 0, (size_t)n * sizeof(uint32_t));
        ws->cur = 1;
    }
}

static int bit_get(const uint64_t *b, uint32_t i) { return (int)((b[i / 64u] >> (i % 64u)) & 1u); }
static void bit_set(uint64_t *b, uint32_t i) { b[i / 64u] |= 1ULL << (i % 64u); }

/*
 * Nodes reachable from the sources in snapshot r (forward; R(G'_r, src)).
 * A node set in `blocked` (may be NULL) is neither entered nor expanded.
 * Leaves the visited nodes in ws->queue[0..ret). *trav gets the number
 * of (arc, snapshot) pairs examined: the full out-degree of every node
 * expanded, whether or not the arc is live.
 */
static uint32_t reach_fwd(const snaps_t *g, uint32_t r, const uint32_t *src,
                          uint32_t nsrc, const uint64_t *blocked, bfs_ws *ws,
                          const uint64_t *row_ptr, uint64_t *trav)
{
    uint64_t stride = (uint64_t)g->n + 1u;
    const uint32_t *ptr = g->fptr + (uint64_t)r * stride;
    const uint32_t *adj = g->fadj + g->fbase[r];
    uint32_t head = 0, tail = 0;
    ws_next(ws, g->n);
    for (uint32_t i = 0; i < nsrc; i++) {
        uint32_t s = src[i];
        if (blocked && bit_get(blocked, s)) continue;
        if (ws->stamp[s] == ws->cur) continue;
        ws->stamp[s] = ws->cur;
        ws->queue[tail++] = s;
    }
    while (head < tail) {
        uint32_t x = ws->queue[head++];
        if (trav) *trav += row_ptr[x + 1] - row_ptr[x];
        for (uint32_t j = ptr[x]; j < ptr[x + 1]; j++) {
            uint32_t v = adj[j];
            if (ws->stamp[v] == ws->cur) continue;
            if (blocked && bit_get(blocked, v)) continue;
            ws->stamp[v] = ws->cur;
            ws->queue[tail++] = v;
        }
    }
    return tail;
}

/* Nodes from which w is reachable in snapshot r (U(G'_r, w)), w included. */
static uint32_t reach_rev(const snaps_t *g, uint32_t r, uint32_t w, bfs_ws *ws,
                          const uint64_t *indeg, uint64_t *trav)
{
    uint64_t stride = (uint64_t)g->n + 1u;
    const uint32_t *ptr = g->rptr + (uint64_t)r * stride;
    const uint32_t *adj = g->radj + g->rbase[r];
    uint32_t head = 0, tail = 0;
    ws_next(ws, g->n);
    ws->stamp[w] = ws->cur;
    ws->queue[tail++] = w;
    while (head < tail) {
        uint32_t x = ws->queue[head++];
        if (trav) *trav += indeg[x];
        for (uint32_t j = ptr[x]; j < ptr[x + 1]; j++) {
            uint32_t v = adj[j];
            if (ws->stamp[v] == ws->cur) continue;
            ws->stamp[v] = ws->cur;
            ws->queue[tail++] = v;
        }
    }
    return tail;
}

/* argmax over u not in S of (s_u, then lowest id)  (R3, R4) */
static uint32_t argmax_unselected(uint32_t n, const int64_t *s, const uint8_t *sel)
{
    uint32_t best = UINT32_MAX;
    for (uint32_t u = 0; u < n; u++) {
        if (sel[u]) continue;
        if (best == UINT32_MAX || s[u] > s[best]) best = u;
    }
    return best;
}

/*
 * Stats layout (uint64[8]):
 *  [0] traversals in the initial counts   (sum over u, r, x in R_r(u) of outdeg x)
 *  [1] traversals of the forward steps    (sum over rounds, r, x in N_r of outdeg x)
 *  [2] traversals of the reverse steps    (sum over rounds, r, w in N_r, x in U_r(w) of indeg x)
 *  [3] exact gain evaluations (lazy CELF only)
 *  [4] live (arc, snapshot) pairs
 *  [5] word-level reach: sum over (u, word) of sum of outdeg x over the union of R_r(u), r in word
 *  [6] word-level reach: sum over (u, word) of the size of that union
 *  [7] decrements applied (DU only)
 */
#define NSTATS 8

/* Algorithm 2, initial loop: s_v = sum_i |R(G'_i, v)| (R1). Also fills stats[0,5,6]. */
static int initial_gains(const snaps_t *g, const uint64_t *row_ptr, int64_t *s,
                         uint64_t *stats)
{
    uint32_t n = g->n, R = g->R, W = (R + 63u) / 64u;
    bfs_ws ws = {0}, wu = {0};
    if (ws_init(&ws, n) || ws_init(&wu, n)) { ws_free(&ws); ws_free(&wu); return ORACLE_ENOMEM; }
    for (uint32_t u = 0; u < n; u++) s[u] = 0;
    for (uint32_t u = 0; u < n; u++) {
        for (uint32_t w = 0; w < W; w++) {
            /* union of the reach sets over the snapshots of word w (stats only) */
            ws_next(&wu, n);
            for (uint32_t r = w * 64u; r < R && r < w * 64u + 64u; r++) {
                uint32_t c = reach_fwd(g, r, &u, 1, NULL, &ws, row_ptr, &stats[0]);
                s[u] += c;
                for (uint32_t i = 0; i < c; i++) {
                    uint32_t x = ws.queue[i];
                    if (wu.stamp[x] != wu.cur) {
                        wu.stamp[x] = wu.cur;
                        stats[5] += row_ptr[x + 1] - row_ptr[x];
                        stats[6] += 1;
                    }
                }
            }
        }
    }
    ws_free(&ws); ws_free(&wu);
    return ORACLE_OK;
}

/* initial per-node reach counts s_u = sum_r |R_r(u)| */
int oracle_initial_gains(uint32_t n, uint64_t m, const uint64_t *row_ptr,
                         const uint32_t *col, const float *prob, uint32_t R,
                         uint64_t seed, uint32_t *gain_out, uint64_t *stats)
{
    int rc = check_graph(n, m, row_ptr, col, prob, R);
    if (rc) return rc;
    snaps_t g;
    uint64_t st[NSTATS] = {0};
    int64_t *s = (int64_t *)malloc((n ? n : 1) * sizeof(int64_t));
    if (!s) return ORACLE_ENOMEM;
    if ((rc = snaps_build(&g, n, m, row_ptr, col, prob, R, seed))) { free(s); return rc; }
    st[4] = g.nlive;
    rc = initial_gains(&g, row_ptr, s, st);
    if (!rc)
        for (uint32_t u = 0; u < n; u++) gain_out[u] = (uint32_t)s[u];
    if (stats) memcpy(stats, st, sizeof(st));
    snaps_free(&g); free(s);
    return rc;
}

/*
 * StaticGreedyDU (Sec. 4, Algorithm 2), with readings R1-R6.
 * seeds[k], gains[k]: the chosen nodes and their marginal gains (summed
 * over snapshots). trace (nullable, [k+1][n]): the gain vector s at the
 * start of every round and after the last one.
 */
static int select_du_keyed(uint32_t n, uint64_t m, const uint64_t *row_ptr,
                           const uint32_t *col, const float *prob, uint32_t R,
                           uint32_t k, uint64_t seed, const uint32_t *key_of, int lt,
                           uint32_t *seeds, uint64_t *gains, uint32_t *trace, uint64_t *stats)
{
    int rc = check_graph(n, m, row_ptr, col, prob, R);
    if (rc) return rc;
    if (k > n) return ORACLE_EINVAL;
    uint64_t st[NSTATS] = {0};
    uint64_t nw = ((uint64_t)n + 63u) / 64u;
    snaps_t g;
    if ((rc = snaps_build_keyed(&g, n, m, row_ptr, col, prob, R, seed, key_of, lt))) return rc;
    st[4] = g.nlive;
    int64_t *s = (int64_t *)malloc((n ? n : 1) * sizeof(int64_t));
    uint8_t *sel = (uint8_t *)calloc(n ? n : 1, 1);
    uint64_t *covered = (uint64_t *)calloc((size_t)R * (nw ? nw : 1), sizeof(uint64_t));
    uint64_t *indeg = (uint64_t *)calloc(n ? n : 1, sizeof(uint64_t));
    uint32_t *newly = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    bfs_ws ws;
    int wsok = ws_init(&ws, n);
    if (!s || !sel || !covered || !indeg || !newly || wsok) { rc = ORACLE_ENOMEM; goto out; }
    for (uint64_t e = 0; e < m; e++) indeg[col[e]]++;

    if ((rc = initial_gains(&g, row_ptr, s, st))) goto out;

    for (uint32_t t = 0; t < k; t++) {
        if (trace)
            for (uint32_t u = 0; u < n; u++) trace[(uint64_t)t * n + u] = (uint32_t)s[u];
        uint32_t best = argmax_unselected(n, s, sel);         /* v* = argmax s_v */
        seeds[t] = best;
        gains[t] = (uint64_t)s[best];
        sel[best] = 1;                                        /* S = S u {v*} */
        for (uint32_t r = 0; r < R; r++) {
            uint64_t *cov = covered + (uint64_t)r * nw;
            /* the part of R(G'_r, v*) not yet deleted: reachable, not covered */
            uint32_t c = reach_fwd(&g, r, &best, 1, cov, &ws, row_ptr, &st[1]);
            memcpy(newly, ws.queue, (size_t)c * sizeof(uint32_t));
            for (uint32_t i = 0; i < c; i++) bit_set(cov, newly[i]);
            for (uint32_t i = 0; i < c; i++) {
                uint32_t w = newly[i];
                uint32_t cu = reach_rev(&g, r, w, &ws, indeg, &st[2]);
                for (uint32_t j = 0; j < cu; j++) {
                    s[ws.queue[j]] -= 1;   /* delete w from R(G'_r,u); s_u -= 1 */
                    if (s[ws.queue[j]] < 0) { rc = ORACLE_EINTERNAL; goto out; }
                }
                st[7] += cu;
            }
        }
    }
    if (trace)
        for (uint32_t u = 0; u < n; u++) trace[(uint64_t)k * n + u] = (uint32_t)s[u];
out:
    if (stats) memcpy(stats, st, sizeof(st));
    ws_free(&ws);
    free(s); free(sel); free(covered); free(indeg); free(newly);
    snaps_free(&g);
    return rc;
}

int oracle_select_du(uint32_t n, uint64_t m, const uint64_t *row_ptr,
                     const uint32_t *col, const float *prob, uint32_t R,
                     uint32_t k, uint64_t seed, uint32_t *seeds, uint64_t *gains,
                     uint32_t *trace, uint64_t *stats)
{
    return select_du_keyed(n, m, row_ptr, col, prob, R, k, seed, NULL, 0, seeds, gains, trace,
                           stats);
}

/* Algorithm 2 on linear-threshold snapshots (prob[e] = the weight b_e) */
int oracle_select_du_lt(uint32_t n, uint64_t m, const uint64_t *row_ptr,
                        const uint32_t *col, const float *prob, uint32_t R,
                        uint32_t k, uint64_t seed, uint32_t *seeds, uint64_t *gains,
                        uint32_t *trace, uint64_t *stats)
{
    return select_du_keyed(n, m, row_ptr, col, prob, R, k, seed, NULL, 1, seeds, gains, trace,
                           stats);
}

/*
 * StaticGreedy, literally (Sec. 3.3, Algorithm 1): every round recomputes
 * s_v = sum_j |R(G'_j, S u {v})| for every v not in S and adds the argmax.
 * gains[t] is the marginal gain f(S u {v*}) - f(S), with
 * f(S) = sum_j |R(G'_j, S)|.
 */
int oracle_select_alg1(uint32_t n, uint64_t m, const uint64_t *row_ptr,
                       const uint32_t *col, const float *prob, uint32_t R,
                       uint32_t k, uint64_t seed, uint32_t *seeds, uint64_t *gains)
{
    int rc = check_graph(n, m, row_ptr, col, prob, R);
    if (rc) return rc;
    if (k > n) return ORACLE_EINVAL;
    snaps_t g;
    if ((rc = snaps_build(&g, n, m, row_ptr, col, prob, R, seed))) return rc;
    int64_t *s = (int64_t *)malloc((n ? n : 1) * sizeof(int64_t));
    uint8_t *sel = (uint8_t *)calloc(n ? n : 1, 1);
    uint32_t *src = (uint32_t *)malloc(((uint64_t)k + 1u) * sizeof(uint32_t));
    bfs_ws ws;
    int wsok = ws_init(&ws, n);
    if (!s || !sel || !src || wsok) { rc = ORACLE_ENOMEM; goto out; }
    int64_t fS = 0;                         /* f(S), S empty */
    for (uint32_t t = 0; t < k; t++) {
        for (uint32_t v = 0; v < n; v++) {
            s[v] = 0;
            if (sel[v]) continue;
            src[t] = v;                     /* sources S u {v}: seeds[0..t) then v */
            for (uint32_t j = 0; j < R; j++)
                s[v] += reach_fwd(&g, j, src, t + 1u, NULL, &ws, row_ptr, NULL);
        }
        uint32_t best = argmax_unselected(n, s, sel);
        seeds[t] = best;
        src[t] = best;
        sel[best] = 1;
        gains[t] = (uint64_t)(s[best] - fS);
        fS = s[best];
    }
out:
    ws_free(&ws);
    free(s); free(sel); free(src);
    snaps_free(&g);
    return rc;
}

/* ---------------- lazy CELF on the static snapshots ---------------- */

typedef struct { int64_t key; uint32_t id; } hent;

/* heap order: larger key first, then smaller id (R3 applied to bounds) */
static int hbefore(hent a, hent b) { return a.key > b.key || (a.key == b.key && a.id < b.id); }

static void hpush(hent *h, uint32_t *len, hent x)
{
    uint32_t i = (*len)++;
    h[i] = x;
    while (i > 0) {
        uint32_t p = (i - 1u) / 2u;
        if (!hbefore(h[i], h[p])) break;
        hent t = h[i]; h[i] = h[p]; h[p] = t; i = p;
    }
}

static hent hpop(hent *h, uint32_t *len)
{
    hent top = h[0];
    h[0] = h[--(*len)];
    uint32_t i = 0;
    for (;;) {
        uint32_t a = 2u * i + 1u, b = a + 1u, best = i;
        if (a < *len && hbefore(h[a], h[best])) best = a;
        if (b < *len && hbefore(h[b], h[best])) best = b;
        if (best == i) break;
        hent t = h[i]; h[i] = h[best]; h[best] = t; i = best;
    }
    return top;
}

/*
 * StaticGreedyCELF: the gain of u from an earlier round bounds its current
 * gain (submodularity, Sec. 3.2), so a node is re-evaluated exactly only
 * when it reaches the top of the queue with a stale bound. The exact gain
 * is sum_r |R(G'_r,u) \ covered_r|. stats[3] counts exact evaluations
 * after the initial counts.
 */
int oracle_select_celf(uint32_t n, uint64_t m, const uint64_t *row_ptr,
                       const uint32_t *col, const float *prob, uint32_t R,
                       uint32_t k, uint64_t seed, uint32_t *seeds, uint64_t *gains,
                       uint64_t *stats)
{
    int rc = check_graph(n, m, row_ptr, col, prob, R);
    if (rc) return rc;
    if (k > n) return ORACLE_EINVAL;
    uint64_t st[NSTATS] = {0};
    uint64_t nw = ((uint64_t)n + 63u) / 64u;
    snaps_t g;
    if ((rc = snaps_build(&g, n, m, row_ptr, col, prob, R, seed))) return rc;
    st[4] = g.nlive;
    int64_t *s = (int64_t *)malloc((n ? n : 1) * sizeof(int64_t));
    uint32_t *when = (uint32_t *)calloc(n ? n : 1, sizeof(uint32_t));
    uint64_t *covered = (uint64_t *)calloc((size_t)R * (nw ? nw : 1), sizeof(uint64_t));
    hent *heap = (hent *)malloc((n ? n : 1) * sizeof(hent));
    uint32_t hlen = 0;
    bfs_ws ws;
    int wsok = ws_init(&ws, n);
    if (!s || !when || !covered || !heap || wsok) { rc = ORACLE_ENOMEM; goto out; }
    if ((rc = initial_gains(&g, row_ptr, s, st))) goto out;
    for (uint32_t u = 0; u < n; u++) {
        hent x = { s[u], u };
        hpush(heap, &hlen, x);     /* when[u] = 0: exact for round 0 */
    }
    for (uint32_t t = 0; t < k; t++) {
        hent top;
        for (;;) {
            top = hpop(heap, &hlen);
            if (when[top.id] == t) break;
            int64_t gsum = 0;
            for (uint32_t r = 0; r < R; r++) {
                const uint64_t *cov = covered + (uint64_t)r * nw;
                gsum += reach_fwd(&g, r, &top.id, 1, cov, &ws, row_ptr, NULL);
            }
            st[3]++;
            when[top.id] = t;
            top.key = gsum;
            hpush(heap, &hlen, top);
        }
        seeds[t] = top.id;
        gains[t] = (uint64_t)top.key;
        for (uint32_t r = 0; r < R; r++) {
            uint64_t *cov = covered + (uint64_t)r * nw;
            uint32_t c = reach_fwd(&g, r, &top.id, 1, cov, &ws, row_ptr, &st[1]);
            for (uint32_t i = 0; i < c; i++) bit_set(cov, ws.queue[i]);
        }
    }
out:
    if (stats) memcpy(stats, st, sizeof(st));
    ws_free(&ws);
    free(s); free(when); free(covered); free(heap);
    snaps_free(&g);
    return rc;
}

/* f(S) = sum_r |R(G'_r, S)|  (Sec. 3.1, snapshot estimator, times R) */
int oracle_spread(uint32_t n, uint64_t m, const uint64_t *row_ptr,
                  const uint32_t *col, const float *prob, uint32_t R,
                  uint64_t seed, const uint32_t *S, uint32_t nS, uint64_t *out)
{
    int rc = check_graph(n, m, row_ptr, col, prob, R);
    if (rc) return rc;
    for (uint32_t i = 0; i < nS; i++) if (S[i] >= n) return ORACLE_EINVAL;
    snaps_t g;
    if ((rc = snaps_build(&g, n, m, row_ptr, col, prob, R, seed))) return rc;
    bfs_ws ws;
    if (ws_init(&ws, n)) { snaps_free(&g); return ORACLE_ENOMEM; }
    uint64_t tot = 0;
    for (uint32_t r = 0; r < R; r++)
        tot += reach_fwd(&g, r, S, nS, NULL, &ws, row_ptr, NULL);
    *out = tot;
    ws_free(&ws);
    snaps_free(&g);
    return ORACLE_OK;
}

/* Prefix spreads (Sec. 3.1 estimator, used to score seed sets on snapshots
 * independent of the ones that chose them, Sec. 5.2):
 *   marg[i] = f(S[0..i]) - f(S[0..i-1]),  per[r] = |R(G'_r, S)|.
 * Every prefix is searched from scratch, straight from the definition of f.
 * marg or per may be NULL. */
int oracle_spread_prefix(uint32_t n, uint64_t m, const uint64_t *row_ptr,
                         const uint32_t *col, const float *prob, uint32_t R,
                         uint64_t seed, const uint32_t *S, uint32_t nS,
                         uint64_t *marg, uint32_t *per)
{
    /* an evaluation may use more snapshots than a selection: up to 2^20 */
    if (R == 0 || R > (1u << 20) || (uint64_t)n * R >= (1ULL << 32)) return ORACLE_EINVAL;
    int rc = check_graph(n, m, row_ptr, col, prob, 1);
    if (rc) return rc;
    for (uint32_t i = 0; i < nS; i++) if (S[i] >= n) return ORACLE_EINVAL;
    snaps_t g;
    if ((rc = snaps_build(&g, n, m, row_ptr, col, prob, R, seed))) return rc;
    bfs_ws ws;
    if (ws_init(&ws, n)) { snaps_free(&g); return ORACLE_ENOMEM; }
    if (marg) memset(marg, 0, (size_t)nS * sizeof(uint64_t));
    for (uint32_t r = 0; r < R; r++) {
        if (marg) {
            uint32_t prev = 0;
            for (uint32_t i = 0; i < nS; i++) {
                uint32_t cur = reach_fwd(&g, r, S, i + 1, NULL, &ws, row_ptr, NULL);
                marg[i] += cur - prev;
                prev = cur;
            }
        }
        if (per) per[r] = nS ? reach_fwd(&g, r, S, nS, NULL, &ws, row_ptr, NULL) : 0;
    }
    ws_free(&ws);
    snaps_free(&g);
    return ORACLE_OK;
}

/* ======================================================================
 * Undirected graphs with one coin per undirected pair (Sec. 4: in an
 * undirected snapshot R(G'_i,v) = U(G'_i,v), so the connected components
 * of each snapshot carry all the information; the update after a pick is
 * a subtraction over the picked node's components).
 * Reading: the caller's CSR stores both directions of every pair with the
 * same probability and no parallel arcs; the pair's coin is drawn under the
 * index of its canonical arc (the direction whose tail is the smaller id);
 * a self-loop is its own pair and never changes a component.
 * ====================================================================== */

typedef struct { uint32_t lo, hi, tail; uint64_t e; } pair_rec;

static int pair_cmp(const void *a, const void *b)
{
    const pair_rec *x = (const pair_rec *)a, *y = (const pair_rec *)b;
    if (x->lo != y->lo) return x->lo < y->lo ? -1 : 1;
    if (x->hi != y->hi) return x->hi < y->hi ? -1 : 1;
    if (x->tail != y->tail) return x->tail < y->tail ? -1 : 1;
    return 0;
}

/* pair[e] = the canonical arc of e's undirected pair; ORACLE_EINVAL unless
 * every arc's reverse is stored exactly once with the same probability */
int oracle_pair_ids(uint32_t n, uint64_t m, const uint64_t *row_ptr, const uint32_t *col,
                    const float *prob, uint32_t *pair)
{
    int rc = check_graph(n, m, row_ptr, col, prob, 1);
    if (rc) return rc;
    pair_rec *a = (pair_rec *)malloc((m ? m : 1) * sizeof(pair_rec));
    if (!a) return ORACLE_ENOMEM;
    for (uint32_t u = 0; u < n; u++)
        for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
            uint32_t v = col[e];
            a[e].lo = u < v ? u : v;
            a[e].hi = u < v ? v : u;
            a[e].tail = u;
            a[e].e = e;
        }
    qsort(a, m, sizeof(pair_rec), pair_cmp);
    rc = ORACLE_OK;
    for (uint64_t i = 0; i < m && rc == ORACLE_OK;) {
        if (a[i].lo == a[i].hi) {                       /* self-loop: its own pair */
            if (i + 1 < m && a[i + 1].lo == a[i].lo && a[i + 1].hi == a[i].hi) rc = ORACLE_EINVAL;
            pair[a[i].e] = (uint32_t)a[i].e;
            i += 1;
            continue;
        }
        /* exactly two arcs: lo -> hi (canonical), then hi -> lo */
        if (i + 1 >= m || a[i + 1].lo != a[i].lo || a[i + 1].hi != a[i].hi ||
            a[i].tail != a[i].lo || a[i + 1].tail != a[i].hi ||
            (i + 2 < m && a[i + 2].lo == a[i].lo && a[i + 2].hi == a[i].hi) ||
            prob[a[i].e] != prob[a[i + 1].e]) {
            rc = ORACLE_EINVAL;
            break;
        }
        pair[a[i].e] = (uint32_t)a[i].e;
        pair[a[i + 1].e] = (uint32_t)a[i].e;
        i += 2;
    }
    free(a);
    return rc;
}

/* Algorithm 2 on the pair-coin snapshots (the directed machinery, for
 * cross-checking the component method) */
int oracle_select_du_pairs(uint32_t n, uint64_t m, const uint64_t *row_ptr,
                           const uint32_t *col, const float *prob, uint32_t R,
                           uint32_t k, uint64_t seed, uint32_t *seeds, uint64_t *gains,
                           uint32_t *trace, uint64_t *stats)
{
    uint32_t *pair = (uint32_t *)malloc((m ? m : 1) * sizeof(uint32_t));
    if (!pair) return ORACLE_ENOMEM;
    int rc = oracle_pair_ids(n, m, row_ptr, col, prob, pair);
    if (rc == ORACLE_OK)
        rc = select_du_keyed(n, m, row_ptr, col, prob, R, k, seed, pair, 0, seeds, gains, trace,
                             stats);
    free(pair);
    return rc;
}

static uint32_t uf_find(uint32_t *parent, uint32_t x)
{
    while (parent[x] != x) {
        parent[x] = parent[parent[x]];   /* path halving */
        x = parent[x];
    }
    return x;
}

/*
 * The component method. Per snapshot r: union-find over the live pairs
 * gives comp_r(u); s_u = sum_r |comp_r(u)| (every node of a component
 * reaches every other, itself included). A pick v* covers, in every
 * snapshot where it is still uncovered, its whole component C; each member
 * u loses |C| (the decrements of Algorithm 2 for the |C| newly covered
 * nodes, each of which every member reaches).
 */
int oracle_select_components(uint32_t n, uint64_t m, const uint64_t *row_ptr,
                             const uint32_t *col, const float *prob, uint32_t R,
                             uint32_t k, uint64_t seed, uint32_t *seeds, uint64_t *gains,
                             uint32_t *trace)
{
    int rc = check_graph(n, m, row_ptr, col, prob, R);
    if (rc) return rc;
    if (k > n) return ORACLE_EINVAL;
    uint64_t nR = (uint64_t)n * R;
    uint32_t *pair = (uint32_t *)malloc((m ? m : 1) * sizeof(uint32_t));
    uint32_t *root = (uint32_t *)malloc((nR ? nR : 1) * sizeof(uint32_t));   /* [R][n] */
    uint32_t *size = (uint32_t *)calloc(nR ? nR : 1, sizeof(uint32_t));     /* [R][n] by root */
    uint32_t *start = (uint32_t *)malloc((nR ? nR : 1) * sizeof(uint32_t)); /* [R][n] by root */
    uint32_t *member = (uint32_t *)malloc((nR ? nR : 1) * sizeof(uint32_t));/* [R][n] */
    uint8_t *covered = (uint8_t *)calloc(nR ? nR : 1, 1);                   /* [R][n] by root */
    int64_t *s = (int64_t *)calloc(n ? n : 1, sizeof(int64_t));
    uint8_t *sel = (uint8_t *)calloc(n ? n : 1, 1);
    if (!pair || !root || !size || !start || !member || !covered || !s || !sel) {
        rc = ORACLE_ENOMEM;
        goto out;
    }
    if ((rc = oracle_pair_ids(n, m, row_ptr, col, prob, pair))) goto out;
    for (uint32_t r = 0; r < R; r++) {
        uint32_t *par = root + (uint64_t)r * n;
        uint32_t *sz = size + (uint64_t)r * n, *st = start + (uint64_t)r * n;
        uint32_t *mem = member + (uint64_t)r * n;
        for (uint32_t u = 0; u < n; u++) par[u] = u;
        /* the live pairs of snapshot r (Sec. 3.1, one coin per pair) */
        for (uint32_t u = 0; u < n; u++)
            for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
                if (pair[e] != e || col[e] == u) continue;
                if (!arc_live(sm64_output(seed, e + 1u), r, arc_threshold(prob[e]))) continue;
                uint32_t a = uf_find(par, u), b = uf_find(par, col[e]);
                if (a != b) par[a < b ? b : a] = a < b ? a : b;
            }
        for (uint32_t u = 0; u < n; u++) par[u] = uf_find(par, u);
        for (uint32_t u = 0; u < n; u++) sz[par[u]]++;
        /* members of each component, grouped by root (counting sort) */
        uint32_t acc = 0;
        for (uint32_t x = 0; x < n; x++) { st[x] = acc; acc += sz[x]; }
        for (uint32_t u = 0; u < n; u++) mem[st[par[u]]++] = u;
        for (uint32_t x = 0; x < n; x++) st[x] -= sz[x];
        for (uint32_t u = 0; u < n; u++) s[u] += sz[par[u]];
    }
    for (uint32_t t = 0; t < k; t++) {
        if (trace)
            for (uint32_t u = 0; u < n; u++) trace[(uint64_t)t * n + u] = (uint32_t)s[u];
        uint32_t best = argmax_unselected(n, s, sel);
        seeds[t] = best;
        gains[t] = (uint64_t)s[best];
        sel[best] = 1;
        for (uint32_t r = 0; r < R; r++) {
            uint64_t o = (uint64_t)r * n;
            uint32_t c = root[o + best];
            if (covered[o + c]) continue;
            covered[o + c] = 1;
            uint32_t csz = size[o + c];
            for (uint32_t i = 0; i < csz; i++) {
                uint32_t u = member[o + start[o + c] + i];
                s[u] -= csz;
                if (s[u] < 0) { rc = ORACLE_EINTERNAL; goto out; }
            }
        }
    }
    if (trace)
        for (uint32_t u = 0; u < n; u++) trace[(uint64_t)k * n + u] = (uint32_t)s[u];
out:
    free(pair); free(root); free(size); free(start); free(member); free(covered);
    free(s); free(sel);
    return rc;
}
