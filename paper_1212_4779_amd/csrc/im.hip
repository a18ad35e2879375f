// im.hip -- StaticGreedy influence maximisation on one MI355X (gfx950).
//
// Paper: Cheng et al., "StaticGreedy: Solving the Scalability-Accuracy
// Dilemma in Influence Maximization", CIKM 2013 (arXiv 1212.4779).
//
// Pipeline of one im_select call, all on one HIP stream:
//   A1  validate the caller's CSR, build the reverse CSR (counting sort)
//   A2  snapshot masks: 64 snapshots per uint64 word, word-major [W][m],
//       for the forward arcs and (gathered) for the reverse arcs
//       (Sec. 3.3, Algorithm 1, sampling loop; Sec. 3.1 snapshot definition)
//   A3  initial gains s_u = sum_r |R_r(u)|, one reachability task per
//       (node, word) (Sec. 4, Algorithm 2, initial loop)
//   per round (Sec. 4, Algorithm 2, greedy loop):
//   A4  argmax over unselected nodes of (gain, lowest id)
//   A5  forward search from the new seed v*, pruned at covered nodes:
//       newly covered bits N[w][x]; covered |= N
//   A6  for every (x, word) with N != 0: reverse search from x carrying
//       N[w][x]; every node y reached loses popcount(bits of y) from its gain
//       (delete x from R(G'_i,y) once per snapshot i, s_y -= 1)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "im.h"
#include "im_bfs.h"

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(call)                                                               \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess)                                                      \
            return fail(IM_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));   \
    } while (0)

extern "C" const char *im_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// generic kernels
// ---------------------------------------------------------------------------
template <typename Tv>
__global__ void k_fill(Tv *p, uint64_t cnt, Tv v)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < cnt;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static unsigned grid_for(uint64_t work, unsigned nt, unsigned cap = 8192)
{
    uint64_t g = (work + nt - 1) / nt;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

template <typename Tv>
static void fill(Tv *p, uint64_t cnt, Tv v, hipStream_t s)
{
    if (cnt == 0) return;
    k_fill<Tv><<<grid_for(cnt, 256), 256, 0, s>>>(p, cnt, v);
}

// ---------------------------------------------------------------------------
// A1: validation and reverse CSR
// ---------------------------------------------------------------------------
enum { ERR_ROW0 = 1, ERR_ROWN = 2, ERR_ROWDEC = 4, ERR_ROWBIG = 8, ERR_COL = 16, ERR_PROB = 32 };

__global__ void k_validate(const uint64_t *row_ptr, const uint32_t *col, const float *prob,
                           uint32_t n, uint64_t m, uint32_t *err, uint32_t *row32)
{
    uint64_t lim = (uint64_t)n + 1 > m ? (uint64_t)n + 1 : m;
    uint32_t e = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < lim;
         i += (uint64_t)gridDim.x * blockDim.x) {
        if (i <= n) {
            uint64_t r = row_ptr[i];
            if (i == 0 && r != 0) e |= ERR_ROW0;
            if (i == n && r != m) e |= ERR_ROWN;
            if (i < n && row_ptr[i + 1] < r) e |= ERR_ROWDEC;
            if (r > m) e |= ERR_ROWBIG;
            if (row32) row32[i] = (uint32_t)r;
        }
        if (i < m) {
            if (col[i] >= n) e |= ERR_COL;
            float p = prob[i];
            if (!(p >= 0.0f && p <= 1.0f)) e |= ERR_PROB;
        }
    }
    if (e) atomicOr(err, e);
}

__global__ void k_hist(const uint32_t *col, uint64_t m, uint32_t *cnt)
{
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < m;
         e += (uint64_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[col[e]], 1u);
}

constexpr int SCAN_NT = 256, SCAN_IPT = 8, SCAN_TILE = SCAN_NT * SCAN_IPT;

// exclusive scan, pass 1: per-tile scan and tile totals
__global__ __launch_bounds__(SCAN_NT) void k_scan_tiles(const uint32_t *in, uint32_t *out,
                                                        uint64_t len, uint32_t *sums)
{
    __shared__ uint32_t wsum[SCAN_NT / 64 + 1];
    uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_IPT;
    uint32_t v[SCAN_IPT], s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_IPT; j++) {
        v[j] = base + j < len ? in[base + j] : 0u;
        s += v[j];
    }
    uint32_t total;
    uint32_t ex = block_excl_scan<SCAN_NT>(s, wsum, &total);
#pragma unroll
    for (int j = 0; j < SCAN_IPT; j++) {
        if (base + j < len) out[base + j] = ex;
        ex += v[j];
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// pass 2: one block scans the tile totals in place, carrying across chunks
__global__ __launch_bounds__(SCAN_NT) void k_scan_sums(uint32_t *sums, uint32_t ntiles)
{
    __shared__ uint32_t wsum[SCAN_NT / 64 + 1];
    uint32_t carry = 0;
    for (uint32_t c = 0; c < ntiles; c += SCAN_TILE) {
        uint32_t base = c + threadIdx.x * SCAN_IPT;
        uint32_t v[SCAN_IPT], s = 0;
#pragma unroll
        for (int j = 0; j < SCAN_IPT; j++) {
            v[j] = base + j < ntiles ? sums[base + j] : 0u;
            s += v[j];
        }
        uint32_t total;
        uint32_t ex = block_excl_scan<SCAN_NT>(s, wsum, &total) + carry;
#pragma unroll
        for (int j = 0; j < SCAN_IPT; j++) {
            if (base + j < ntiles) sums[base + j] = ex;
            ex += v[j];
        }
        carry += total;
    }
}

// pass 3: add tile offsets
__global__ void k_scan_add(uint32_t *out, uint64_t len, const uint32_t *sums)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < len;
         i += (uint64_t)gridDim.x * blockDim.x)
        out[i] += sums[i / SCAN_TILE];
}

// tail of arc e: largest u with row32[u] <= e
__device__ __forceinline__ uint32_t arc_tail(const uint32_t *row32, uint32_t n, uint32_t e)
{
    uint32_t lo = 0, hi = n;  // row32[lo] <= e < row32[hi] (row32[n] = m > e)
    while (hi - lo > 1) {
        uint32_t mid = lo + (hi - lo) / 2;
        if (row32[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void k_scatter(const uint32_t *row32, const uint32_t *col, uint32_t n, uint64_t m,
                          const uint32_t *in_row, uint32_t *cursor, uint32_t *in_col,
                          uint32_t *in2out)
{
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < m;
         e += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t u = arc_tail(row32, n, (uint32_t)e);
        uint32_t v = col[e];
        uint32_t pos = in_row[v] + atomicAdd(&cursor[v], 1u);
        in_col[pos] = u;
        in2out[pos] = (uint32_t)e;
    }
}

// ---------------------------------------------------------------------------
// A2: snapshot masks
// ---------------------------------------------------------------------------
// Arc e is live in snapshot r iff the top 32 bits of output r+1 of a
// SplitMix64 generator seeded with key_e (output e+1 of SplitMix64(seed))
// are below floor(p_e * 2^32). One thread per (arc, word).
__global__ __launch_bounds__(256) void k_mask_gen(const float *prob, uint64_t m, uint32_t R,
                                                  uint64_t seed, uint64_t *mask)
{
    uint64_t e = blockIdx.x * 256ull + threadIdx.x;
    uint32_t w = blockIdx.y;
    if (e >= m) return;
    uint64_t thr = (uint64_t)((double)prob[e] * 4294967296.0);
    uint32_t r0 = w * 64u;
    uint32_t cnt = min(64u, R - r0);
    uint64_t word = 0;
    if (thr >= (1ull << 32)) {
        word = im_valid_bits(R, w);
    } else if (thr) {
        uint64_t key = sm64_finalise(seed + (e + 1ull) * IM_GOLDEN);
        uint64_t z = key + (uint64_t)(r0 + 1u) * IM_GOLDEN;
        for (uint32_t b = 0; b < cnt; b++) {
            uint64_t d = sm64_finalise(z) >> 32;
            word |= (uint64_t)(d < thr) << b;
            z += IM_GOLDEN;
        }
    }
    mask[(uint64_t)w * m + e] = word;
}

__global__ __launch_bounds__(256) void k_mask_gather(const uint32_t *in2out, uint64_t m,
                                                     const uint64_t *mask_out, uint64_t *mask_in)
{
    uint64_t e = blockIdx.x * 256ull + threadIdx.x;
    uint64_t w = blockIdx.y;
    if (e >= m) return;
    mask_in[w * m + e] = mask_out[w * m + in2out[e]];
}

// ---------------------------------------------------------------------------
// A4: argmax of (gain, lowest id) over unselected nodes
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_argmax(const uint32_t *gain, const uint8_t *sel,
                                                uint32_t n, unsigned long long *key)
{
    __shared__ unsigned long long red[4];
    unsigned long long best = 0;
    for (uint32_t u = blockIdx.x * 256u + threadIdx.x; u < n; u += gridDim.x * 256u)
        if (!sel[u]) {
            unsigned long long k = ((unsigned long long)gain[u] << 32) | (0xFFFFFFFFu - u);
            best = k > best ? k : best;
        }
    best = wave_max_u64(best);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 4; i++) best = red[i] > best ? red[i] : best;
        if (best) atomicMax(key, best);
    }
}

// ---------------------------------------------------------------------------
// A5: forward search from the chosen seed, pruned at covered nodes
// ---------------------------------------------------------------------------
struct FwdArgs {
    const uint32_t *row, *col;
    const uint64_t *mask;
    uint64_t m;
    uint32_t n, R, W;
    uint64_t *covered, *newly, *pend, *fdel;
    uint32_t *qa, *qb, *tnodes, *tcounts;
    const unsigned long long *key;
    uint32_t *seeds_out;
    uint64_t *gains_out;
    uint8_t *sel;
    unsigned long long *stats;
};

constexpr int FWD_NT = 1024;

__global__ __launch_bounds__(FWD_NT) void k_forward(FwdArgs a, uint32_t t)
{
    __shared__ BlockLds<FWD_NT> L;
    const int tid = threadIdx.x;
    const unsigned long long key = a.key[t];
    if (key == 0) return;  // no unselected node (cannot happen for k <= n)
    const uint32_t v = 0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull);
    const uint32_t w = blockIdx.x;
    const uint64_t off = (uint64_t)w * a.n;
    if (w == 0 && tid == 0) {
        a.seeds_out[t] = v;
        a.gains_out[t] = key >> 32;
        a.sel[v] = 1;
    }
    const uint64_t start = im_valid_bits(a.R, w) & ~a.covered[off + v];
    if (!start) {
        if (tid == 0) a.tcounts[w] = 0;
        return;
    }
    uint64_t arcs = 0;
    block_bfs_run<FWD_NT, true>(L, v, start, a.row, a.col, a.mask + (uint64_t)w * a.m,
                                a.covered + off, a.newly + off, a.pend + off, a.fdel + off,
                                a.qa + off, a.qb + off, a.tnodes + off, arcs);
    const uint32_t nvis = L.nvis;
    uint64_t relax = 0, trav = 0;
    for (uint32_t i = tid; i < nvis; i += FWD_NT) {
        uint32_t x = a.tnodes[off + i];
        uint64_t b = a.newly[off + x];
        a.covered[off + x] |= b;
        uint32_t dg = a.row[x + 1] - a.row[x];
        relax += dg;
        trav += (uint64_t)__popcll(b) * dg;
    }
    relax = wave_sum_u64(relax);
    trav = wave_sum_u64(trav);
    if ((tid & 63) == 0) {
        atomicAdd(&a.stats[ST_RELAX_FWD], (unsigned long long)relax);
        atomicAdd(&a.stats[ST_TRAV_FWD], (unsigned long long)trav);
    }
    if (tid == 0) {
        a.tcounts[w] = nvis;
        atomicAdd(&a.stats[ST_TASKS_REV], (unsigned long long)nvis);
    }
}

// reset the newly-covered words after the reverse step consumed them
__global__ void k_clear_newly(uint64_t *newly, const uint32_t *tnodes, const uint32_t *tcounts,
                              uint32_t n, uint32_t W)
{
    for (uint32_t w = 0; w < W; w++) {
        uint32_t c = tcounts[w];
        uint64_t off = (uint64_t)w * n;
        for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < c; i += gridDim.x * blockDim.x)
            newly[off + tnodes[off + i]] = 0;
    }
}

__global__ void k_copy_u32(const uint32_t *src, uint32_t *dst, uint64_t cnt)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < cnt;
         i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// engine configuration
// ---------------------------------------------------------------------------
// wavefront engine: T tasks per wavefront, CS table entries per task,
// LIM entries before hand-over, DMAX largest degree expanded in LDS
constexpr int WV_T = 8, WV_CS = 32, WV_LIM = 24, WV_DMAX = 1024;
constexpr int BLK_NT = 256;
constexpr int PH_CTRS = 4;  // per-phase counters: grab, ovf_n, bgrab, spare

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
struct im_workspace {
    int device = -1;
    int num_cu = 256;
    uint32_t cap_n = 0, cap_W = 0, cap_k = 0, slots = 0;
    uint64_t cap_m = 0;
    // graph-derived
    uint32_t *row32 = nullptr, *in_row = nullptr, *in_col = nullptr, *in2out = nullptr;
    uint32_t *cnt = nullptr, *scan_sums = nullptr;
    uint64_t *mask_out = nullptr, *mask_in = nullptr;
    // selection state
    uint32_t *gain = nullptr;
    uint8_t *sel = nullptr;
    uint64_t *covered = nullptr, *newly = nullptr, *fpend = nullptr, *ffdel = nullptr;
    uint32_t *fqa = nullptr, *fqb = nullptr, *tnodes = nullptr, *tcounts = nullptr;
    unsigned long long *keys = nullptr;
    uint32_t *ovf_q = nullptr;
    uint32_t *ctrs = nullptr;
    // block engine slots
    uint64_t *b_reach = nullptr, *b_pend = nullptr, *b_fdel = nullptr;
    uint32_t *b_qa = nullptr, *b_qb = nullptr, *b_vis = nullptr;
    // misc
    unsigned long long *stats = nullptr;
    uint32_t *err = nullptr;
    uint32_t *host_err = nullptr;
    unsigned long long *host_stats = nullptr;
    hipStream_t last_stream = nullptr;
};

template <typename Tv>
static int dalloc(Tv **p, uint64_t cnt)
{
    if (*p) { (void)hipFree(*p); *p = nullptr; }
    if (cnt == 0) cnt = 1;
    hipError_t e = hipMalloc((void **)p, cnt * sizeof(Tv));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(IM_ENOMEM, "hipMalloc of %llu bytes failed: %s",
                    (unsigned long long)(cnt * sizeof(Tv)), hipGetErrorString(e));
    }
    return IM_OK;
}

template <typename Tv>
static void dfree(Tv *&p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

extern "C" int im_workspace_create(im_workspace **out)
{
    if (!out) return fail(IM_EINVAL, "im_workspace_create: null output pointer");
    im_workspace *ws = new im_workspace();
    HIPCHK(hipGetDevice(&ws->device));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, ws->device));
    ws->num_cu = prop.multiProcessorCount;
    int rc;
    if ((rc = dalloc(&ws->stats, ST_COUNT))) { delete ws; return rc; }
    if ((rc = dalloc(&ws->err, 1))) { delete ws; return rc; }
    HIPCHK(hipHostMalloc((void **)&ws->host_err, sizeof(uint32_t), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&ws->host_stats, ST_COUNT * sizeof(unsigned long long),
                         hipHostMallocDefault));
    HIPCHK(hipMemset(ws->stats, 0, ST_COUNT * sizeof(unsigned long long)));
    *out = ws;
    return IM_OK;
}

extern "C" int im_workspace_destroy(im_workspace *ws)
{
    if (!ws) return IM_OK;
    (void)hipDeviceSynchronize();
    dfree(ws->row32); dfree(ws->in_row); dfree(ws->in_col); dfree(ws->in2out);
    dfree(ws->cnt); dfree(ws->scan_sums); dfree(ws->mask_out); dfree(ws->mask_in);
    dfree(ws->gain); dfree(ws->sel); dfree(ws->covered); dfree(ws->newly);
    dfree(ws->fpend); dfree(ws->ffdel); dfree(ws->fqa); dfree(ws->fqb);
    dfree(ws->tnodes); dfree(ws->tcounts); dfree(ws->keys); dfree(ws->ovf_q); dfree(ws->ctrs);
    dfree(ws->b_reach); dfree(ws->b_pend); dfree(ws->b_fdel);
    dfree(ws->b_qa); dfree(ws->b_qb); dfree(ws->b_vis);
    dfree(ws->stats); dfree(ws->err);
    if (ws->host_err) (void)hipHostFree(ws->host_err);
    if (ws->host_stats) (void)hipHostFree(ws->host_stats);
    delete ws;
    return IM_OK;
}

static uint32_t slots_for(uint32_t n)
{
    // dense block-engine state: 36 bytes per node per slot, about 8 GB total
    uint64_t per = 36ull * (n ? n : 1);
    uint64_t s = (8ull << 30) / per;
    if (s > 256) s = 256;
    if (s < 8) s = 8;
    return (uint32_t)s;
}

// grow the workspace to hold a graph with n nodes, m arcs, W words, k rounds
static int ws_reserve(im_workspace *ws, uint32_t n, uint64_t m, uint32_t W, uint32_t k)
{
    int rc;
    const bool grow_n = n > ws->cap_n || W > ws->cap_W || ws->gain == nullptr;
    const bool grow_m = m > ws->cap_m || W > ws->cap_W || ws->mask_out == nullptr;
    const uint32_t cn = std::max(n, ws->cap_n), cW = std::max(W, ws->cap_W);
    const uint64_t cm = std::max(m, ws->cap_m);
    if (grow_n) {
        uint64_t nn = (uint64_t)cn + 1, nW = (uint64_t)cn * cW;
        if ((rc = dalloc(&ws->row32, nn)) || (rc = dalloc(&ws->in_row, nn)) ||
            (rc = dalloc(&ws->cnt, nn)) || (rc = dalloc(&ws->scan_sums, nn / SCAN_TILE + 2)) ||
            (rc = dalloc(&ws->gain, cn)) || (rc = dalloc(&ws->sel, cn)) ||
            (rc = dalloc(&ws->covered, nW)) || (rc = dalloc(&ws->newly, nW)) ||
            (rc = dalloc(&ws->fpend, nW)) || (rc = dalloc(&ws->ffdel, nW)) ||
            (rc = dalloc(&ws->fqa, nW)) || (rc = dalloc(&ws->fqb, nW)) ||
            (rc = dalloc(&ws->tnodes, nW)) || (rc = dalloc(&ws->tcounts, 64)) ||
            (rc = dalloc(&ws->ovf_q, nW)))
            return rc;
        HIPCHK(hipMemset(ws->newly, 0, nW * sizeof(uint64_t)));
        HIPCHK(hipMemset(ws->fpend, 0, nW * sizeof(uint64_t)));
        uint32_t slots = slots_for(cn);
        uint64_t sn = (uint64_t)slots * cn;
        if ((rc = dalloc(&ws->b_reach, sn)) || (rc = dalloc(&ws->b_pend, sn)) ||
            (rc = dalloc(&ws->b_fdel, sn)) || (rc = dalloc(&ws->b_qa, sn)) ||
            (rc = dalloc(&ws->b_qb, sn)) || (rc = dalloc(&ws->b_vis, sn)))
            return rc;
        HIPCHK(hipMemset(ws->b_reach, 0, sn * sizeof(uint64_t)));
        HIPCHK(hipMemset(ws->b_pend, 0, sn * sizeof(uint64_t)));
        ws->slots = slots;
        ws->cap_n = cn;
    }
    if (grow_m) {
        if ((rc = dalloc(&ws->in_col, cm)) || (rc = dalloc(&ws->in2out, cm)) ||
            (rc = dalloc(&ws->mask_out, cm * cW)) || (rc = dalloc(&ws->mask_in, cm * cW)))
            return rc;
        ws->cap_m = cm;
    }
    ws->cap_W = cW;
    if (k + 1 > ws->cap_k) {
        uint32_t ck = k + 1;
        if ((rc = dalloc(&ws->keys, ck)) || (rc = dalloc(&ws->ctrs, (uint64_t)(ck + 1) * PH_CTRS)))
            return rc;
        ws->cap_k = ck;
    }
    return IM_OK;
}

// ---------------------------------------------------------------------------
// host-side steps
// ---------------------------------------------------------------------------
static int check_args(const im_graph *g, uint32_t R)
{
    if (!g) return fail(IM_EINVAL, "null graph");
    if (g->m >= (1ull << 32)) return fail(IM_EINVAL, "m = %llu must be < 2^32", (unsigned long long)g->m);
    if (!g->row_ptr) return fail(IM_EINVAL, "null row_ptr");
    if (g->m && (!g->col || !g->prob)) return fail(IM_EINVAL, "null col or prob");
    if (R == 0 || R > IM_R_MAX) return fail(IM_EINVAL, "R = %u must be in [1, %u]", R, IM_R_MAX);
    if ((uint64_t)g->n * R >= (1ull << 32))
        return fail(IM_EOVERFLOW, "n * R = %llu must be < 2^32", (unsigned long long)g->n * R);
    return IM_OK;
}

static int validate(const im_graph *g, im_workspace *ws, hipStream_t s, uint32_t *row32)
{
    HIPCHK(hipMemsetAsync(ws->err, 0, sizeof(uint32_t), s));
    uint64_t lim = std::max<uint64_t>((uint64_t)g->n + 1, g->m);
    k_validate<<<grid_for(lim, 256), 256, 0, s>>>(g->row_ptr, g->col, g->prob, g->n, g->m,
                                                  ws->err, row32);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(ws->host_err, ws->err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    uint32_t e = *ws->host_err;
    if (e & ERR_ROW0) return fail(IM_EINVAL, "row_ptr[0] != 0");
    if (e & ERR_ROWN) return fail(IM_EINVAL, "row_ptr[n] != m");
    if (e & (ERR_ROWDEC | ERR_ROWBIG)) return fail(IM_EINVAL, "row_ptr is not non-decreasing within [0, m]");
    if (e & ERR_COL) return fail(IM_EINVAL, "col entry >= n");
    if (e & ERR_PROB) return fail(IM_EINVAL, "prob outside [0, 1] or NaN");
    return IM_OK;
}

static void exclusive_scan(const uint32_t *in, uint32_t *out, uint64_t len, uint32_t *sums,
                           hipStream_t s)
{
    uint64_t ntiles = (len + SCAN_TILE - 1) / SCAN_TILE;
    k_scan_tiles<<<(unsigned)ntiles, SCAN_NT, 0, s>>>(in, out, len, sums);
    k_scan_sums<<<1, SCAN_NT, 0, s>>>(sums, (uint32_t)ntiles);
    k_scan_add<<<grid_for(len, 256), 256, 0, s>>>(out, len, sums);
}

// A1: reverse CSR (row32 must already hold the 32-bit offsets)
static void build_reverse(const im_graph *g, im_workspace *ws, hipStream_t s)
{
    uint32_t n = g->n;
    uint64_t m = g->m;
    fill<uint32_t>(ws->cnt, (uint64_t)n + 1, 0u, s);
    if (m) k_hist<<<grid_for(m, 256), 256, 0, s>>>(g->col, m, ws->cnt);
    exclusive_scan(ws->cnt, ws->in_row, (uint64_t)n + 1, ws->scan_sums, s);
    fill<uint32_t>(ws->cnt, (uint64_t)n + 1, 0u, s);
    if (m) k_scatter<<<grid_for(m, 256), 256, 0, s>>>(ws->row32, g->col, n, m, ws->in_row, ws->cnt,
                                                      ws->in_col, ws->in2out);
}

// A2: masks for both directions
static void build_masks(const im_graph *g, uint32_t R, uint64_t seed, im_workspace *ws,
                        uint64_t *mask_out, bool reverse, hipStream_t s)
{
    uint32_t W = (R + 63) / 64;
    uint64_t m = g->m;
    if (m == 0) return;
    dim3 grid((unsigned)((m + 255) / 256), W);
    k_mask_gen<<<grid, 256, 0, s>>>(g->prob, m, R, seed, mask_out);
    if (reverse) k_mask_gather<<<grid, 256, 0, s>>>(ws->in2out, m, mask_out, ws->mask_in);
}

static BfsArgs bfs_args(im_workspace *ws, const uint32_t *row, const uint32_t *col,
                        const uint64_t *mask, uint64_t m, uint32_t n, uint32_t R, uint32_t W,
                        uint32_t *ctr)
{
    BfsArgs a;
    memset(&a, 0, sizeof(a));
    a.row = row; a.col = col; a.mask = mask; a.m = m; a.n = n; a.R = R; a.W = W;
    a.gain = ws->gain;
    a.grab = ctr + 0; a.ovf_n = ctr + 1; a.bgrab = ctr + 2;
    a.ovf_q = ws->ovf_q;
    a.b_reach = ws->b_reach; a.b_pend = ws->b_pend; a.b_fdel = ws->b_fdel;
    a.b_qa = ws->b_qa; a.b_qb = ws->b_qb; a.b_vis = ws->b_vis;
    a.stats = ws->stats;
    return a;
}

static unsigned wave_grid(im_workspace *ws) { return (unsigned)ws->num_cu * 12u; }

// A3: initial gains (gain must be zero on entry)
static void initial_gains(const im_graph *g, uint32_t R, im_workspace *ws, uint32_t *ctr,
                          hipStream_t s)
{
    uint32_t n = g->n, W = (R + 63) / 64;
    if (n == 0) return;
    BfsArgs a = bfs_args(ws, ws->row32, g->col, ws->mask_out, g->m, n, R, W, ctr);
    a.ntasks = n * W;
    a.st_trav = ST_TRAV_INIT; a.st_relax = ST_RELAX_INIT; a.st_reached = ST_REACHED_INIT;
    a.st_arcs = ST_ARCS_INIT; a.st_ovf = ST_OVF_INIT;
    k_wave_bfs<MODE_COUNT, WV_T, WV_CS, WV_LIM, WV_DMAX, false><<<wave_grid(ws), 64, 0, s>>>(a);
    k_block_bfs<MODE_COUNT, BLK_NT, false><<<ws->slots, BLK_NT, 0, s>>>(a);
}

// A4-A6: one greedy round
static void greedy_round(const im_graph *g, uint32_t R, uint32_t t, uint32_t *seeds_out,
                         uint64_t *gains_out, im_workspace *ws, uint32_t *ctr, hipStream_t s)
{
    uint32_t n = g->n, W = (R + 63) / 64;
    k_argmax<<<grid_for(n, 256, 2048), 256, 0, s>>>(ws->gain, ws->sel, n, ws->keys + t);

    FwdArgs f;
    f.row = ws->row32; f.col = g->col; f.mask = ws->mask_out; f.m = g->m;
    f.n = n; f.R = R; f.W = W;
    f.covered = ws->covered; f.newly = ws->newly; f.pend = ws->fpend; f.fdel = ws->ffdel;
    f.qa = ws->fqa; f.qb = ws->fqb; f.tnodes = ws->tnodes; f.tcounts = ws->tcounts;
    f.key = ws->keys; f.seeds_out = seeds_out; f.gains_out = gains_out; f.sel = ws->sel;
    f.stats = ws->stats;
    k_forward<<<W, FWD_NT, 0, s>>>(f, t);

    BfsArgs a = bfs_args(ws, ws->in_row, ws->in_col, ws->mask_in, g->m, n, R, W, ctr);
    a.tnodes = ws->tnodes; a.tcounts = ws->tcounts; a.tbits = ws->newly;
    a.st_trav = ST_TRAV_REV; a.st_relax = ST_RELAX_REV; a.st_reached = ST_REACHED_REV;
    a.st_arcs = ST_ARCS_REV; a.st_ovf = ST_OVF_REV;
    k_wave_bfs<MODE_DEC, WV_T, WV_CS, WV_LIM, WV_DMAX, false><<<wave_grid(ws), 64, 0, s>>>(a);
    k_block_bfs<MODE_DEC, BLK_NT, false><<<ws->slots, BLK_NT, 0, s>>>(a);
    k_clear_newly<<<grid_for(n, 256, 1024), 256, 0, s>>>(ws->newly, ws->tnodes, ws->tcounts, n, W);
}

// everything up to (and including) the initial gains
static int prepare(const im_graph *g, uint32_t R, uint64_t seed, uint32_t k, im_workspace *ws,
                   hipStream_t s)
{
    int rc;
    uint32_t n = g->n, W = (R + 63) / 64;
    if ((rc = ws_reserve(ws, n, g->m, W, k))) return rc;
    if ((rc = validate(g, ws, s, ws->row32))) return rc;
    HIPCHK(hipMemsetAsync(ws->stats, 0, ST_COUNT * sizeof(unsigned long long), s));
    fill<uint32_t>(ws->ctrs, (uint64_t)(k + 1) * PH_CTRS, 0u, s);
    fill<unsigned long long>(ws->keys, (uint64_t)k + 1, 0ull, s);
    fill<uint32_t>(ws->gain, n, 0u, s);
    fill<uint8_t>(ws->sel, n, (uint8_t)0, s);
    fill<uint64_t>(ws->covered, (uint64_t)n * W, 0ull, s);
    build_reverse(g, ws, s);
    build_masks(g, R, seed, ws, ws->mask_out, true, s);
    initial_gains(g, R, ws, ws->ctrs, s);
    HIPCHK(hipGetLastError());
    ws->last_stream = s;
    return IM_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" int im_validate(const im_graph *g, uint32_t R, void *stream)
{
    if (!g) return fail(IM_EINVAL, "null graph");
    int rc = R ? check_args(g, R) : (g->m >= (1ull << 32) ? fail(IM_EINVAL, "m >= 2^32") : IM_OK);
    if (rc) return rc;
    im_workspace *ws;
    if ((rc = im_workspace_create(&ws))) return rc;
    rc = validate(g, ws, (hipStream_t)stream, nullptr);
    im_workspace_destroy(ws);
    return rc;
}

extern "C" int im_stats_get(im_workspace *ws, im_stats *out)
{
    if (!ws || !out) return fail(IM_EINVAL, "null argument");
    HIPCHK(hipStreamSynchronize(ws->last_stream));
    HIPCHK(hipMemcpy(ws->host_stats, ws->stats, ST_COUNT * sizeof(unsigned long long),
                     hipMemcpyDeviceToHost));
    memset(out, 0, sizeof(*out));
    const unsigned long long *h = ws->host_stats;
    out->trav_init = h[ST_TRAV_INIT];
    out->trav_fwd = h[ST_TRAV_FWD];
    out->trav_rev = h[ST_TRAV_REV];
    out->relax_init = h[ST_RELAX_INIT];
    out->reached_init = h[ST_REACHED_INIT];
    out->relax_rev = h[ST_RELAX_REV];
    out->reached_rev = h[ST_REACHED_REV];
    out->relax_fwd = h[ST_RELAX_FWD];
    out->arcs_read_init = h[ST_ARCS_INIT];
    out->arcs_read_rev = h[ST_ARCS_REV];
    out->ovf_init = h[ST_OVF_INIT];
    out->ovf_rev = h[ST_OVF_REV];
    out->tasks_rev = h[ST_TASKS_REV];
    out->decrements = h[ST_DECREMENTS];
    out->celf_evals = h[ST_CELF_EVALS];
    return IM_OK;
}

extern "C" int im_snapshot_masks(const im_graph *g, uint32_t R, uint64_t seed, uint64_t *mask_out,
                                 im_workspace *ws, void *stream)
{
    int rc;
    if ((rc = check_args(g, R))) return rc;
    if (!ws || (g->m && !mask_out)) return fail(IM_EINVAL, "null workspace or output");
    hipStream_t s = (hipStream_t)stream;
    if ((rc = ws_reserve(ws, g->n, g->m, (R + 63) / 64, 0))) return rc;
    if ((rc = validate(g, ws, s, nullptr))) return rc;
    build_masks(g, R, seed, ws, mask_out, false, s);
    HIPCHK(hipGetLastError());
    ws->last_stream = s;
    return IM_OK;
}

extern "C" int im_transpose(const im_graph *g, uint32_t *in_row_ptr, uint32_t *in_col,
                            uint32_t *in2out, im_workspace *ws, void *stream)
{
    int rc;
    if ((rc = check_args(g, 1))) return rc;
    if (!ws || !in_row_ptr || (g->m && (!in_col || !in2out)))
        return fail(IM_EINVAL, "null workspace or output");
    hipStream_t s = (hipStream_t)stream;
    if ((rc = ws_reserve(ws, g->n, g->m, 1, 0))) return rc;
    if ((rc = validate(g, ws, s, ws->row32))) return rc;
    build_reverse(g, ws, s);
    HIPCHK(hipMemcpyAsync(in_row_ptr, ws->in_row, ((uint64_t)g->n + 1) * sizeof(uint32_t),
                          hipMemcpyDeviceToDevice, s));
    if (g->m) {
        HIPCHK(hipMemcpyAsync(in_col, ws->in_col, g->m * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(in2out, ws->in2out, g->m * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    }
    HIPCHK(hipGetLastError());
    ws->last_stream = s;
    return IM_OK;
}

extern "C" int im_initial_gains(const im_graph *g, uint32_t R, uint64_t seed, uint32_t *gain_out,
                                im_workspace *ws, void *stream)
{
    int rc;
    if ((rc = check_args(g, R))) return rc;
    if (!ws || (g->n && !gain_out)) return fail(IM_EINVAL, "null workspace or output");
    hipStream_t s = (hipStream_t)stream;
    if ((rc = prepare(g, R, seed, 0, ws, s))) return rc;
    if (g->n)
        k_copy_u32<<<grid_for(g->n, 256), 256, 0, s>>>(ws->gain, gain_out, g->n);
    HIPCHK(hipGetLastError());
    return IM_OK;
}

extern "C" int im_select(const im_graph *g, uint32_t R, uint32_t k, uint64_t seed,
                         uint32_t *seeds_out, uint64_t *gains_out, uint32_t *trace_out,
                         im_workspace *ws, void *stream)
{
    int rc;
    if ((rc = check_args(g, R))) return rc;
    if (!ws) return fail(IM_EINVAL, "null workspace");
    if (k > g->n) return fail(IM_EINVAL, "k = %u exceeds n = %u", k, g->n);
    if (k && (!seeds_out || !gains_out)) return fail(IM_EINVAL, "null seeds or gains output");
    hipStream_t s = (hipStream_t)stream;
    if ((rc = prepare(g, R, seed, k, ws, s))) return rc;
    uint32_t n = g->n;
    for (uint32_t t = 0; t < k; t++) {
        if (trace_out)
            k_copy_u32<<<grid_for(n, 256), 256, 0, s>>>(ws->gain, trace_out + (uint64_t)t * n, n);
        greedy_round(g, R, t, seeds_out, gains_out, ws, ws->ctrs + (uint64_t)(t + 1) * PH_CTRS, s);
    }
    if (trace_out && n)
        k_copy_u32<<<grid_for(n, 256), 256, 0, s>>>(ws->gain, trace_out + (uint64_t)k * n, n);
    HIPCHK(hipGetLastError());
    return IM_OK;
}
