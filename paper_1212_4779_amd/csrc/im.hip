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
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include <hip/hip_cooperative_groups.h>

#include "im.h"
#include "im_bfs.h"
#include "im_host.h"
#include "im_mlp.h"

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static_assert(IM_PH_COUNT <= IM_PH_MAX, "phase table too small");

static thread_local std::string g_err;

int im_fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

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

// 32-bit copy of the row offsets (a plan's replays re-read row_ptr with this)
__global__ void k_row32(const uint64_t *row_ptr, uint32_t n, uint32_t *row32)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i <= n;
         i += (uint64_t)gridDim.x * blockDim.x)
        row32[i] = (uint32_t)row_ptr[i];
}

// Reverse-CSR construction. Arcs into one high in-degree node are spread over
// the whole arc array, so plain per-arc global atomics on its counter
// serialise. Each workgroup therefore first aggregates its contiguous slice of
// arcs in an LDS hash table (head -> count) and touches each global counter
// once per distinct head.
constexpr int TR_NT = 256, TR_ARCS = 4096, TR_HT = 8192;

struct TrLds {
    uint32_t key[TR_HT];
    uint32_t cnt[TR_HT];
    uint32_t off[TR_HT];
};

__device__ __forceinline__ uint32_t tr_slot(TrLds &L, uint32_t v)
{
    uint32_t h = (v * 0x9E3779B1u) >> (32 - 13);
    for (;;) {
        uint32_t k = L.key[h];
        if (k == v) return h;
        if (k == IM_EMPTY) {
            uint32_t old = atomicCAS(&L.key[h], IM_EMPTY, v);
            if (old == IM_EMPTY || old == v) return h;
        }
        h = (h + 1) & (TR_HT - 1);
    }
}

// pass 1: in-degree histogram. pass 2 (scatter): positions.
template <bool SCATTER>
__global__ __launch_bounds__(TR_NT) void k_transpose(const uint32_t *row32, const uint32_t *col,
                                                     uint32_t n, uint64_t m, uint32_t *cnt,
                                                     const uint32_t *in_row, uint32_t *in_col,
                                                     uint32_t *in2out)
{
    __shared__ TrLds L;
    const int tid = threadIdx.x;
    const uint64_t e0 = (uint64_t)blockIdx.x * TR_ARCS;
    const uint64_t e1 = e0 + TR_ARCS < m ? e0 + TR_ARCS : m;
    for (int i = tid; i < TR_HT; i += TR_NT) { L.key[i] = IM_EMPTY; L.cnt[i] = 0; }
    __syncthreads();
    for (uint64_t e = e0 + tid; e < e1; e += TR_NT) atomicAdd(&L.cnt[tr_slot(L, col[e])], 1u);
    __syncthreads();
    for (int i = tid; i < TR_HT; i += TR_NT) {
        uint32_t v = L.key[i];
        if (v == IM_EMPTY) continue;
        uint32_t base = atomicAdd(&cnt[v], L.cnt[i]);
        if (SCATTER) { L.off[i] = in_row[v] + base; L.cnt[i] = 0; }
    }
    if constexpr (SCATTER) {
        // tails of the slice's arcs: tl[i] = the node whose row holds arc e0+i.
        // The nodes u_lo .. u_hi own the slice; each of them after u_lo with
        // arcs marks the position where its row starts, and an inclusive max
        // scan carries every mark forward over its row.
        __shared__ uint32_t tl[TR_ARCS];
        __shared__ uint32_t ends[2], wmax[TR_NT / 64];
        const uint32_t len = (uint32_t)(e1 - e0);
        for (uint32_t i = tid; i < TR_ARCS; i += TR_NT) tl[i] = 0;
        if (tid == 0 || tid == 64) {
            const uint32_t e = tid == 0 ? (uint32_t)e0 : (uint32_t)(e1 - 1);
            uint32_t lo = 0, hi = n;  // largest u with row32[u] <= e
            while (hi - lo > 1) {
                uint32_t mid = lo + (hi - lo) / 2;
                if (row32[mid] <= e) lo = mid; else hi = mid;
            }
            ends[tid / 64] = lo;
        }
        __syncthreads();
        const uint32_t u_lo = ends[0], u_hi = ends[1];
        if (tid == 0) tl[0] = u_lo;
        for (uint32_t u = u_lo + 1 + tid; u <= u_hi; u += TR_NT) {
            const uint32_t r0 = row32[u];   // e0 < r0 <= e1 - 1
            if (row32[u + 1] > r0) tl[r0 - (uint32_t)e0] = u;
        }
        __syncthreads();
        constexpr uint32_t PER = TR_ARCS / TR_NT;
        const uint32_t c0 = tid * PER;
        uint32_t run = 0;
        for (uint32_t i = 0; i < PER; i++) run = max(run, tl[c0 + i]);
        // exclusive max over the lower threads' chunks
        const int lane = tid & 63, wid = tid >> 6;
        uint32_t x = run;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off, 64);
            if (lane >= off) x = max(x, y);
        }
        if (lane == 63) wmax[wid] = x;
        const uint32_t below = __shfl_up(x, 1, 64);
        __syncthreads();
        uint32_t carry = lane > 0 ? below : 0u;
        for (int k = 0; k < wid; k++) carry = max(carry, wmax[k]);
        for (uint32_t i = 0; i < PER; i++) {
            carry = max(carry, tl[c0 + i]);
            tl[c0 + i] = carry;
        }
        __syncthreads();
        for (uint32_t i = tid; i < len; i += TR_NT) {
            const uint64_t e = e0 + i;
            uint32_t v = col[e];
            uint32_t h = tr_slot(L, v);
            uint32_t pos = L.off[h] + atomicAdd(&L.cnt[h], 1u);
            in_col[pos] = tl[i];
            in2out[pos] = (uint32_t)e;
        }
    }
}

// A batch's instances are copied side by side into one block-diagonal CSR
// (node ids shifted by the instance's node offset, arc ids by its arc
// offset) and validated on the way.
struct InstDesc {
    const uint64_t *row_ptr;
    const uint32_t *col;
    const float *prob;
    uint64_t m;
    uint64_t arc_off;
    uint32_t n;
    uint32_t node_off;
};

__global__ void k_batch_merge(const InstDesc *desc, uint32_t *err, uint32_t *row32, uint32_t *mcol,
                              float *mprob, uint32_t *node_inst)
{
    const uint32_t i = blockIdx.y;
    const InstDesc d = desc[i];
    const uint64_t lim = (uint64_t)d.n + 1 > d.m ? (uint64_t)d.n + 1 : d.m;
    uint32_t e = 0;
    for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < lim;
         j += (uint64_t)gridDim.x * blockDim.x) {
        if (j <= d.n) {
            const uint64_t r = d.row_ptr[j];
            if (j == 0 && r != 0) e |= ERR_ROW0;
            if (j == d.n && r != d.m) e |= ERR_ROWN;
            if (j < d.n && d.row_ptr[j + 1] < r) e |= ERR_ROWDEC;
            if (r > d.m) e |= ERR_ROWBIG;
            row32[d.node_off + j] = (uint32_t)(d.arc_off + r);
            if (j < d.n) node_inst[d.node_off + j] = i;
        }
        if (j < d.m) {
            const uint32_t c = d.col[j];
            if (c >= d.n) e |= ERR_COL;
            mcol[d.arc_off + j] = d.node_off + c;
            const float p = d.prob[j];
            if (!(p >= 0.0f && p <= 1.0f)) e |= ERR_PROB;
            mprob[d.arc_off + j] = p;
        }
    }
    if (e) atomicOr(err, e);
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

// ---------------------------------------------------------------------------
// A2: snapshot masks
// ---------------------------------------------------------------------------
// Arc e is live in snapshot r iff the top 32 bits of output r+1 of a
// SplitMix64 generator seeded with key_e (output e+1 of SplitMix64(seed))
// are below floor(p_e * 2^32). One thread per (arc, word).
// In a batch, arc e belongs to instance i and is arc e - arc_off[i] of it:
// the instance's own seed and R apply (its words beyond R are all zero).
// word w0 + blockIdx.y of every arc, stored at mask[blockIdx.y][e]
// key_of (single graphs): the index arc e's coins are drawn under (one coin
// per undirected pair: both directions use the canonical arc's index)
__global__ __launch_bounds__(256) void k_mask_gen(const float *prob, uint64_t m, uint32_t R,
                                                  uint64_t seed, uint64_t *mask, Batch b,
                                                  uint32_t w0 = 0, const uint32_t *key_of = nullptr)
{
    uint64_t e = blockIdx.x * 256ull + threadIdx.x;
    uint32_t w = w0 + blockIdx.y;
    if (e >= m) return;
    uint64_t el = key_of ? key_of[e] : e;
    if (b.arc_off) {
        const uint32_t i = find_instance<uint64_t>(b.arc_off, b.count, e);
        el = e - b.arc_off[i];
        R = b.R[i];
        seed = b.seed[i];
    }
    uint64_t word = 0;
    const uint32_t r0 = w * 64u;
    if (r0 < R) {
        const uint32_t cnt = min(64u, R - r0);
        const uint64_t thr = (uint64_t)((double)prob[e] * 4294967296.0);
        if (thr >= (1ull << 32)) {
            word = im_valid_bits(R, w);
        } else if (thr) {
            uint64_t key = sm64_finalise(seed + (el + 1ull) * IM_GOLDEN);
            uint64_t z = key + (uint64_t)(r0 + 1u) * IM_GOLDEN;
            for (uint32_t bt = 0; bt < cnt; bt++) {
                uint64_t d = sm64_finalise(z) >> 32;
                word |= (uint64_t)(d < thr) << bt;
                z += IM_GOLDEN;
            }
        }
    }
    mask[(uint64_t)blockIdx.y * m + e] = word;
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
// Hub lists: per-snapshot live adjacency of heavy nodes (see HubLists)
// ---------------------------------------------------------------------------
constexpr int HB_NT = 1024;

__global__ void k_hub_mark(const uint32_t *row, uint32_t n, uint32_t hub_deg, uint32_t *slot,
                           uint32_t *list, uint32_t *nhub)
{
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x) {
        uint32_t d = row[x + 1] - row[x];
        uint32_t h = IM_EMPTY;
        if (hub_deg && d >= hub_deg) {
            h = atomicAdd(nhub, 1u);
            list[h] = x;
        }
        slot[x] = h;
    }
}

// Count the live (arc, snapshot) pairs of hub h in word w per bit and reserve
// their range of adj. Each block takes hubs blockIdx.x, blockIdx.x + gridDim.x,
// ... in word blockIdx.y (the hub count is known only on the device). A hub
// whose lists would be denser than a quarter of its masks, or would not fit,
// is expanded through the masks instead (its slot is cleared).
__global__ __launch_bounds__(HB_NT) void k_hub_count(const uint32_t *row, const uint64_t *mask,
                                                     uint64_t m, uint32_t W, const uint32_t *list,
                                                     const uint32_t *nhub, uint32_t *slot,
                                                     uint32_t *hcnt, unsigned long long *hbase,
                                                     unsigned long long *alloc, uint64_t cap)
{
    constexpr int U = 8;
    __shared__ uint32_t cnt[64];
    const uint32_t w = blockIdx.y, nh = *nhub;
    const int tid = threadIdx.x;
    const uint64_t *mw = mask + (uint64_t)w * m;
    for (uint32_t h = blockIdx.x; h < nh; h += gridDim.x) {
        const uint32_t x = list[h], e0 = row[x], e1 = row[x + 1];
        if (tid < 64) cnt[tid] = 0;
        __syncthreads();
        for (uint32_t e = e0 + tid; e < e1; e += HB_NT * U) {
            uint64_t b[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                uint32_t ee = e + (uint32_t)u * HB_NT;
                b[u] = ee < e1 ? mw[ee] : 0ull;
            }
#pragma unroll
            for (int u = 0; u < U; u++)
                while (b[u]) {
                    atomicAdd(&cnt[__ffsll((unsigned long long)b[u]) - 1], 1u);
                    b[u] &= b[u] - 1;
                }
        }
        __syncthreads();
        if (tid < 64) {
            // each of these lanes reads only its own counter, which it alone
            // clears at the start of the next hub
            uint32_t c = cnt[tid];
            hcnt[((uint64_t)h * W + w) * 64 + tid] = c;
            uint32_t incl = wave_incl_scan(c);
            if (tid == 63) {
                bool use = (uint64_t)incl * 4 <= 64ull * (e1 - e0);
                unsigned long long base = 0;
                if (use) {
                    base = atomicAdd(alloc, (unsigned long long)incl);
                    use = base + incl <= cap;
                }
                hbase[(uint64_t)h * W + w] = base;
                if (!use) slot[x] = IM_EMPTY;
            }
        }
    }
}

__global__ __launch_bounds__(HB_NT) void k_hub_fill(const uint32_t *row, const uint32_t *col,
                                                    const uint64_t *mask, uint64_t m, uint32_t W,
                                                    const uint32_t *list, const uint32_t *nhub,
                                                    const uint32_t *slot, const uint32_t *hcnt,
                                                    const unsigned long long *hbase, uint32_t *hoff,
                                                    uint32_t *hadj)
{
    constexpr int U = 8;
    __shared__ uint32_t cur[64];
    const uint32_t w = blockIdx.y, nh = *nhub;
    const int tid = threadIdx.x;
    const uint64_t *mw = mask + (uint64_t)w * m;
    for (uint32_t h = blockIdx.x; h < nh; h += gridDim.x) {
        const uint32_t x = list[h];
        if (slot[x] == IM_EMPTY) continue;   // the same for the whole block
        const uint32_t e0 = row[x], e1 = row[x + 1];
        if (tid < 64) {
            uint32_t c = hcnt[((uint64_t)h * W + w) * 64 + tid];
            uint32_t incl = wave_incl_scan(c);
            uint32_t o = (uint32_t)hbase[(uint64_t)h * W + w] + incl - c;
            cur[tid] = o;
            uint32_t *dst = hoff + ((uint64_t)h * W + w) * 65;
            dst[tid] = o;
            if (tid == 63) dst[64] = o + c;
        }
        __syncthreads();
        for (uint32_t e = e0 + tid; e < e1; e += HB_NT * U) {
            uint64_t b[U];
            uint32_t v[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                uint32_t ee = e + (uint32_t)u * HB_NT;
                b[u] = ee < e1 ? mw[ee] : 0ull;
                v[u] = ee < e1 ? col[ee] : 0u;
            }
#pragma unroll
            for (int u = 0; u < U; u++)
                while (b[u]) {
                    uint32_t pos = atomicAdd(&cur[__ffsll((unsigned long long)b[u]) - 1], 1u);
                    hadj[pos] = v[u];
                    b[u] &= b[u] - 1;
                }
        }
        __syncthreads();   // cur is rewritten for the next hub
    }
}

// Per-snapshot live lists of the nodes below the hub threshold (degree >= 2;
// see SparseLists). A workgroup takes 256 (node, word) pairs at a time and
// spreads the arcs of its eligible pairs evenly over its lanes (node degrees
// are unrelated to node ids, so one row per lane would leave most lanes idle
// behind the longest row); each arc's pair is found by a binary search over
// the pairs' arc offsets, and consecutive lanes read consecutive mask words.
// Every live (arc, snapshot) bit adds one to its pair's counter for that
// snapshot (65 u16 counters per pair in LDS, updated by 32-bit atomics on the
// half that holds them: a count stays below 2^16, so no carry crosses into
// the neighbouring counter). Each lane then turns its pair's row into the 65
// cumulative counts in place, the eligible rows are written out coalesced, one
// atomic per workgroup reserves the heads, and the rows serve as each
// snapshot's cursor while the heads are placed (so the heads of one
// snapshot's list are in no particular order). Pairs of degree >= SP_MAXDEG,
// and pairs whose lists do not fit the capacity, keep base = IM_EMPTY and are
// expanded through the masks; their rows of cum are left unwritten.
constexpr uint32_t SP_MAXDEG = 256;

__device__ __forceinline__ uint32_t sp_bump(uint32_t *cnt32, uint32_t i)
{
    const uint32_t sh = (i & 1u) * 16u;
    return (atomicAdd(&cnt32[i >> 1], 1u << sh) >> sh) & 0xFFFFu;
}

__global__ __launch_bounds__(256) void k_sparse_build(const uint32_t *row, const uint32_t *col,
                                                      const uint64_t *mask, uint64_t m, uint32_t n,
                                                      uint32_t W, uint32_t hub_deg, uint32_t *base,
                                                      uint16_t *cum, uint32_t *adj,
                                                      unsigned long long *alloc, uint64_t cap)
{
    constexpr int U = 4;
    __shared__ uint32_t s_w[256 / 64 + 1];
    __shared__ unsigned long long s_base;
    __shared__ uint32_t s_pre[256], s_e0[256], s_word[256], s_b0[256];
    __shared__ uint8_t s_elig[256];
    __shared__ __attribute__((aligned(16))) uint16_t s_cum[256 * 65];
    uint32_t *cnt32 = (uint32_t *)s_cum;
    const uint64_t P = (uint64_t)W * n;
    const uint32_t t = threadIdx.x;
    for (uint64_t p0 = (uint64_t)blockIdx.x * 256; p0 < P; p0 += (uint64_t)gridDim.x * 256) {
        const uint64_t p = p0 + t;
        uint32_t w = 0, e0 = 0, deg = 0;
        bool elig = false;
        if (p < P) {
            w = (uint32_t)(p / n);
            const uint32_t x = (uint32_t)(p - (uint64_t)w * n);
            e0 = row[x];
            deg = row[x + 1] - e0;
            elig = deg >= 2 && deg < SP_MAXDEG && (hub_deg == 0 || deg < hub_deg);
        }
        for (uint32_t j = t; j < 256 * 65 / 2; j += 256) cnt32[j] = 0u;
        uint32_t T;
        const uint32_t pre = block_excl_scan<256>(elig ? deg : 0u, s_w, &T);
        s_pre[t] = pre;
        s_e0[t] = e0;
        s_word[t] = w;
        s_elig[t] = elig ? 1 : 0;
        __syncthreads();
        // count: the pair's counter b+1 for every live bit b
        for (uint32_t j0 = t; j0 < T; j0 += 256 * U) {
            uint64_t b[U];
            uint32_t q[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const uint32_t j = j0 + (uint32_t)u * 256;
                b[u] = 0ull;
                q[u] = 0;
                if (j < T) {
                    q[u] = (uint32_t)upper_index<256>(s_pre, j);
                    b[u] = mask[(uint64_t)s_word[q[u]] * m + s_e0[q[u]] + (j - s_pre[q[u]])];
                }
            }
#pragma unroll
            for (int u = 0; u < U; u++)
                for (uint64_t v = b[u]; v; v &= v - 1)
                    sp_bump(cnt32, q[u] * 65 + (uint32_t)__ffsll((unsigned long long)v));
        }
        __syncthreads();
        // inclusive prefix over the row: cp[b] = heads live in snapshots before b
        uint16_t *cp = s_cum + t * 65;
        uint32_t total = 0;
        if (elig) {
            for (uint32_t bb = 1; bb < 65; bb++) cp[bb] = (uint16_t)(cp[bb] + cp[bb - 1]);
            total = cp[64];
        }
        uint32_t blk;
        const uint32_t ex = block_excl_scan<256>(total, s_w, &blk);   // syncs: rows complete
        {
            // eligible rows out, as aligned 32-bit words (p0 is a multiple of 256);
            // a word shared by two rows is written when either row is eligible
            const uint64_t npair = min((uint64_t)256, P - p0);
            const uint32_t nu16 = (uint32_t)(npair * 65), nwords = (nu16 + 1) / 2;
            uint32_t *dst = (uint32_t *)(cum + p0 * 65);
            for (uint32_t j = t; j < nwords; j += 256) {
                const uint32_t qa = 2 * j / 65, qb = (2 * j + 1) / 65;
                if (2 * j + 1 < nu16) {
                    if (s_elig[qa] | s_elig[qb]) dst[j] = cnt32[j];
                } else if (s_elig[qa]) {
                    cum[p0 * 65 + 2 * j] = s_cum[2 * j];   // odd tail: one u16
                }
            }
        }
        if (t == 0) s_base = blk ? atomicAdd(alloc, (unsigned long long)blk) : 0ull;
        __syncthreads();
        const unsigned long long b0 = s_base + ex;
        const bool fits = elig && b0 + total <= cap;
        if (p < P) base[p] = fits ? (uint32_t)b0 : IM_EMPTY;
        s_b0[t] = fits ? (uint32_t)b0 : IM_EMPTY;
        __syncthreads();
        // place: the row now serves as each snapshot's cursor
        for (uint32_t j0 = t; j0 < T; j0 += 256 * U) {
            uint64_t b[U];
            uint32_t q[U], e[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const uint32_t j = j0 + (uint32_t)u * 256;
                b[u] = 0ull;
                q[u] = 0;
                e[u] = 0;
                if (j < T) {
                    q[u] = (uint32_t)upper_index<256>(s_pre, j);
                    e[u] = s_e0[q[u]] + (j - s_pre[q[u]]);
                    if (s_b0[q[u]] != IM_EMPTY) b[u] = mask[(uint64_t)s_word[q[u]] * m + e[u]];
                }
            }
#pragma unroll
            for (int u = 0; u < U; u++) {
                if (!b[u]) continue;
                const uint32_t v = col[e[u]], hb = s_b0[q[u]];
                for (uint64_t bits = b[u]; bits; bits &= bits - 1) {
                    const uint32_t bit = (uint32_t)__ffsll((unsigned long long)bits) - 1;
                    adj[hb + sp_bump(cnt32, q[u] * 65 + bit)] = v;
                }
            }
        }
        __syncthreads();   // the LDS arrays and s_base are rewritten by the next chunk
    }
}

// ---------------------------------------------------------------------------
// A4: argmax of (gain, lowest id) over unselected nodes
// ---------------------------------------------------------------------------
// key = (gain << 32) | (0xFFFFFFFF - node): the larger gain wins, then the
// lower id. In a batch every instance gets its own key (keys[i]); instances
// that already have all their seeds (t >= k_i) take no part.
__global__ __launch_bounds__(256) void k_argmax(const uint32_t *gain, const uint8_t *sel,
                                                uint32_t n, unsigned long long *keys, Batch b,
                                                uint32_t t, uint32_t *zero, uint32_t nzero)
{
    __shared__ unsigned long long red[4];
    // also clear this round's reverse-task packing counters
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < nzero; i += gridDim.x * 256u) zero[i] = 0;
    if (b.node_inst) {
        for (uint32_t base = blockIdx.x * 256u; base < n; base += gridDim.x * 256u) {
            const uint32_t u = base + threadIdx.x;
            uint32_t inst = 0xFFFFFFFFu;
            unsigned long long k = 0;
            if (u < n) {
                inst = b.node_inst[u];
                if (t < b.k[inst] && !sel[u])
                    k = ((unsigned long long)gain[u] << 32) | (0xFFFFFFFFu - u);
            }
            // one atomic per wavefront when all its lanes share an instance
            const uint32_t i0 = __shfl(inst, 0, 64);
            const bool same = __all(inst == i0);
            if (same) {
                k = wave_max_u64(k);
                if ((threadIdx.x & 63) == 0 && k && i0 != 0xFFFFFFFFu) atomicMax(&keys[i0], k);
            } else if (k) {
                atomicMax(&keys[inst], k);
            }
        }
        return;
    }
    // a single graph: groups of four nodes (one 16-byte gain load and one
    // 4-byte selection load each; both arrays are allocation-aligned), four
    // groups in flight per lane, then the n % 4 tail nodes one by one
    unsigned long long best = 0;
    const uint32_t ng = n / 4, stride = gridDim.x * 256u;
    const uint4 *g4 = (const uint4 *)gain;
    const uint32_t *s4 = (const uint32_t *)sel;
    for (uint32_t q0 = blockIdx.x * 256u + threadIdx.x; q0 < ng; q0 += 4 * stride) {
        uint4 gv[4];
        uint32_t sv[4];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const uint32_t q = q0 + (uint32_t)i * stride;
            const bool in = q >= q0 && q < ng;   // (q >= q0: no wrap-around)
            gv[i] = in ? g4[q] : make_uint4(0u, 0u, 0u, 0u);
            sv[i] = in ? s4[q] : 0x01010101u;    // out of range: all four taken
        }
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const uint32_t u0 = (q0 + (uint32_t)i * stride) * 4u;
            const uint32_t gg[4] = {gv[i].x, gv[i].y, gv[i].z, gv[i].w};
#pragma unroll
            for (int j = 0; j < 4; j++)
                if (!((sv[i] >> (8 * j)) & 0xFFu)) {
                    const unsigned long long k =
                        ((unsigned long long)gg[j] << 32) | (0xFFFFFFFFu - (u0 + (uint32_t)j));
                    best = k > best ? k : best;
                }
        }
    }
    for (uint32_t u = 4 * ng + blockIdx.x * 256u + threadIdx.x; u < n; u += stride)
        if (!sel[u]) {
            unsigned long long k = ((unsigned long long)gain[u] << 32) | (0xFFFFFFFFu - u);
            best = k > best ? k : best;
        }
    best = wave_max_u64(best);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 4; i++) best = red[i] > best ? red[i] : best;
        if (best) atomicMax(keys, best);
    }
}

// ---------------------------------------------------------------------------
// A5: forward search from the chosen seed, pruned at covered nodes.
// One cooperative grid runs the searches of all W words together, level by
// level: the frontier holds (word, node) entries, every workgroup expands
// tiles of it, and grid-wide barriers separate the levels.
// N[w][x] (newly) collects the newly covered bits; afterwards covered |= N and
// tnodes[w] lists the nodes with N[w][x] != 0 (the reverse tasks).
// ---------------------------------------------------------------------------
// per-round forward counters: 3 frontier counts, the visit count, one visit
// count per word, then the grid barrier's arrival counter and abort flag
constexpr int FWD_CTRS = 4 + 64 + 4;
constexpr int FWD_BAR = 4 + 64;

struct FwdArgs {
    const uint32_t *skip;       // non-zero *skip: the round was committed already (lazy path)
    const uint32_t *row, *col;
    const uint64_t *mask;
    HubLists hub;
    SparseLists sp;
    uint64_t m;
    uint32_t n, R, W;
    uint64_t *covered, *newly, *pend;
    uint64_t *fq0, *fq1;        // frontier entries (word << 32 | node), capacity W*n
    uint32_t *bq0, *bq1;        // per-word frontier queues of the one-workgroup kernel [W][n]
    uint64_t coop_gain;         // rounds whose seed gain reaches this use the cooperative kernel
    uint64_t block_floor;       // ... and k_forward_block takes those in [block_floor, coop_gain)
    uint32_t *cnt;              // [3] frontier counts (ring), [3] visit count, [4..4+W) per-word
                                // visit counts, [FWD_BAR..+2) grid barrier; zero on entry
    uint64_t *vis;              // visited (word << 32 | node), capacity W*n
    uint32_t *tnodes, *tcounts;
    // reverse-task packing counts of the newly covered (word, node) pairs, or
    // bcnt = nullptr for none: per (word, bit) the pairs covered in that one
    // snapshot of the word ([W][64], zero on entry); pairs covered in several
    // snapshots are listed in mlist[w][0 .. mcnt[w])
    uint32_t *bcnt, *mcnt, *mlist;
    const unsigned long long *key;   // keys of this round, one per instance
    uint32_t t;
    Batch b;
    uint32_t *seeds_out;
    uint64_t *gains_out;
    uint8_t *sel;
    unsigned long long *stats;
};

constexpr int FWD_NT = 256, FWD_U = 8;

struct FwdLds {
    uint32_t scan[FWD_NT];
    uint32_t rs[FWD_NT];
    uint32_t wd[FWD_NT];
    uint32_t aux[FWD_NT];   // 0: dense entry, else its sparse plan
    uint64_t del[FWD_NT];
    uint32_t wsum[FWD_NT / 64 + 1];
    unsigned long long red[FWD_NT / 64];
    HubBatch<FWD_NT, 16> H;
    uint32_t bcast;
    uint32_t p0[256];   // level 0: prefix of the seed's per-(word, bit) list lengths
    uint32_t o0[256];   // level 0: start of each (word, bit) list
    uint32_t pk[64 * 64];   // this workgroup's packing counts per (word, bit)
};

__device__ __forceinline__ uint32_t coherent_load(uint32_t *p) { return atomicAdd(p, 0u); }

// one coherent read per workgroup, broadcast through LDS (all threads call)
__device__ __forceinline__ uint32_t group_load(uint32_t *p, uint32_t *slot)
{
    if (threadIdx.x == 0) *slot = coherent_load(p);
    __syncthreads();
    const uint32_t v = *slot;
    __syncthreads();
    return v;
}

// One relaxation (w, v, bits) per lane and unrolled step; bits may be 0.
// Returns whether (w, v) became visited and whether it joins the next frontier.
__device__ __forceinline__ void fwd_relax(const FwdArgs &a, uint32_t w, uint32_t v, uint64_t bits,
                                          bool &first, bool &push)
{
    const uint64_t off = (uint64_t)w * a.n;
    first = false;
    push = false;
    if (!bits) return;
    // covered takes this round's bits as they are reached: the bits it did
    // not hold are new (covered by earlier rounds or reached already this
    // round, they are not), and the newly / pend updates, which depend only
    // on them, go out together
    const uint64_t oc = atomicOr((unsigned long long *)&a.covered[off + v], (unsigned long long)bits);
    const uint64_t nb = bits & ~oc;
    if (!nb) return;
    const uint64_t on = atomicOr((unsigned long long *)&a.newly[off + v], (unsigned long long)nb);
    const uint64_t op = atomicOr((unsigned long long *)&a.pend[off + v], (unsigned long long)nb);
    first = on == 0;
    push = op == 0;
}

// Append up to U entries per lane with one atomic per wavefront: every lane
// of the wavefront must call it with its count and entries.
template <int U>
__device__ __forceinline__ void wave_append_n(uint32_t cnt, const uint64_t *ent, uint32_t *counter,
                                              uint64_t *list)
{
    const uint32_t incl = wave_incl_scan(cnt);
    const uint32_t tot = __shfl(incl, 63, 64);
    if (tot == 0) return;
    uint32_t base = 0;
    if ((threadIdx.x & 63) == 63) base = atomicAdd(counter, tot);
    base = __shfl(base, 63, 64) + incl - cnt;
    for (uint32_t i = 0; i < cnt; i++) list[base + i] = ent[i];
}

// Grid-wide barrier of a cooperative launch. The hardware barrier behind
// cooperative_groups' grid sync costs about 9 us for 64 workgroups on this
// device (and 33 us for 256); this one, about 2 us for 64. bar[0] counts
// arrivals (zero at launch, never reset): the k-th barrier of the launch is
// complete once it reaches k * gridDim.x. Each wavefront first waits for its
// own loads, stores and atomics (a workgroup-scope release does not wait for
// them on this target), so that one agent-scope release by the arriving lane
// publishes the whole workgroup's writes; that lane polls with relaxed loads
// and then acquires for the workgroup (the vector L1 is per compute unit).
// The launch is cooperative, so every workgroup is resident and the poll
// ends; it is bounded all the same (about 10 s of the 100 MHz wall clock).
// A workgroup whose poll times out raises bar[1], counts the failure in
// stats[ST_BARRIER_FAIL] and returns false, as does every later barrier of
// any workgroup: the caller then leaves the kernel, so every workgroup exits.
constexpr int ST_BARRIER_FAIL = 60;
static_assert(ST_BARRIER_FAIL >= ST_MAXLV_BASE + 9 && ST_BARRIER_FAIL < ST_COUNT,
              "barrier failure counter must use a free statistics slot");
constexpr uint64_t BARRIER_TIMEOUT_TICKS = 1000000000ull;

__device__ __forceinline__ bool grid_barrier(uint32_t *bar, uint32_t &k, unsigned long long *stats)
{
    __shared__ uint32_t s_ok;
    k++;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t ok = 1;
        __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t target = k * gridDim.x;
        const uint64_t t0 = wall_clock64();
        uint32_t polls = 0;
        while (__hip_atomic_load(&bar[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if ((++polls & 255u) == 0 &&
                (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                 wall_clock64() - t0 > BARRIER_TIMEOUT_TICKS)) {
                ok = 0;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (ok && __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) ok = 0;
        if (!ok && atomicExch(&bar[1], 1u) == 0) atomicAdd(&stats[ST_BARRIER_FAIL], 1ull);
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

__global__ __launch_bounds__(FWD_NT) void k_forward_coop(FwdArgs a)
{
    __shared__ FwdLds L;
    uint32_t nbar = 0;
    const int tid = threadIdx.x;
    const uint64_t gtid = (uint64_t)blockIdx.x * FWD_NT + tid;
    const bool single = a.b.count == 1;
    const unsigned long long key0 = a.key[0];
    if (a.skip && *a.skip) return;    // uniform over the grid: before any grid barrier
    if (single && key0 == 0) return;  // no unselected node (cannot happen for k <= n)
    if (single && (key0 >> 32) < a.coop_gain) return;  // a small round: k_forward_block runs it
    const uint32_t v = 0xFFFFFFFFu - (uint32_t)(key0 & 0xFFFFFFFFull);
    // a hub seed of a single graph (W <= 4) is expanded by the whole grid at level 0
    const uint32_t hs0 = single ? a.hub.slot[v] : IM_EMPTY;
    const bool split0 = hs0 != IM_EMPTY && a.W <= 4;
    if (blockIdx.x == 0) {
        // commit every instance's argmax and enter its uncovered bits
        for (uint32_t i = tid; i < a.b.count; i += FWD_NT) {
            const unsigned long long key = a.key[i];
            if (key == 0) continue;  // instance already has its k seeds
            const uint32_t sv = 0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull);
            const uint32_t R = single ? a.R : a.b.R[i];
            const uint32_t out = (single ? 0u : a.b.kpre[i]) + a.t;
            a.seeds_out[out] = sv - (single ? 0u : a.b.node_off[i]);
            a.gains_out[out] = key >> 32;
            a.sel[sv] = 1;
            for (uint32_t w = 0; w < a.W; w++) {
                const uint64_t off = (uint64_t)w * a.n;
                uint64_t start = im_valid_bits(R, w) & ~a.covered[off + sv];
                if (!start) continue;
                a.newly[off + sv] = start;
                a.covered[off + sv] |= start;
                a.vis[atomicAdd(&a.cnt[3], 1u)] = ((uint64_t)w << 32) | sv;
                if (!split0) {
                    a.pend[off + sv] = start;
                    a.fq0[atomicAdd(&a.cnt[0], 1u)] = ((uint64_t)w << 32) | sv;
                }
            }
        }
        if (tid == 0) L.H.n = 0;
    } else if (tid == 0) {
        L.H.n = 0;
    }
    uint64_t arcs = 0;
    uint32_t lev0 = 0;
    // the seed's visit entries and counts above must be in place before any
    // workgroup appends to the same lists
    if (!grid_barrier(a.cnt + FWD_BAR, nbar, a.stats)) return;
    if (split0) {
        // every workgroup builds the prefix over (word, bit) of the seed's
        // live-list lengths restricted to its uncovered bits, then takes an
        // interleaved share of the flattened (word, bit, head) range
        const uint32_t w = tid / 64, b = tid % 64;
        uint32_t c = 0, o = 0;
        if (w < a.W) {
            // the seed's start bits as committed (covered holds them already)
            const uint64_t start = a.newly[(uint64_t)w * a.n + v];
            const uint32_t *ho = a.hub.off + ((uint64_t)hs0 * a.W + w) * 65;
            o = ho[b];
            c = ((start >> b) & 1ull) ? ho[b + 1] - o : 0u;
        }
        uint32_t tot;
        const uint32_t ex = block_excl_scan<FWD_NT>(c, L.wsum, &tot);
        L.p0[tid] = ex;
        L.o0[tid] = o;
        __syncthreads();
        uint32_t *ncnt = &a.cnt[1];
        for (uint32_t j0 = blockIdx.x * FWD_NT * FWD_U; j0 < tot; j0 += gridDim.x * FWD_NT * FWD_U) {
            uint64_t vis_e[FWD_U], nxt_e[FWD_U];
            uint32_t nvis = 0, nnxt = 0;
#pragma unroll
            for (int u = 0; u < FWD_U; u++) {
                const uint32_t j = j0 + (uint32_t)u * FWD_NT + tid;
                uint32_t ww = 0, hv = 0;
                uint64_t bits = 0;
                if (j < tot) {
                    const int k = upper_index<FWD_NT>(L.p0, j);
                    ww = (uint32_t)k / 64;
                    hv = a.hub.adj[L.o0[k] + (j - L.p0[k])];
                    bits = 1ull << (k % 64);
                }
                bool first, push;
                fwd_relax(a, ww, hv, bits, first, push);
                const uint64_t ent = ((uint64_t)ww << 32) | hv;
                if (first) vis_e[nvis++] = ent;
                if (push) nxt_e[nnxt++] = ent;
            }
            wave_append_n<FWD_U>(nvis, vis_e, a.cnt + 3, a.vis);
            wave_append_n<FWD_U>(nnxt, nxt_e, ncnt, a.fq1);
        }
        arcs += tot;
        lev0 = 1;
    }
    if (!grid_barrier(a.cnt + FWD_BAR, nbar, a.stats)) return;
    const uint64_t fcap = (uint64_t)a.W * a.n;   // capacity of each frontier queue
    for (uint32_t lev = lev0;; lev++) {
        const uint64_t *cur = (lev & 1) ? a.fq1 : a.fq0;
        uint64_t *nxt = (lev & 1) ? a.fq0 : a.fq1;
        // this workgroup's first frontier entry is loaded while the level's
        // size is read (it is used only if it lies below that size)
        const uint32_t i0 = blockIdx.x * FWD_NT + tid;
        const uint64_t e0 = i0 < fcap ? cur[i0] : 0ull;
        const uint32_t nf = group_load(&a.cnt[lev % 3], &L.bcast);
        if (nf == 0) break;
        uint32_t *ncnt = &a.cnt[(lev + 1) % 3];
        // the ring slot of level lev-1 was last read before the previous barrier
        if (gtid == 0) a.cnt[(lev + 2) % 3] = 0;
        for (uint32_t tile = blockIdx.x * FWD_NT; tile < nf; tile += gridDim.x * FWD_NT) {
            const uint32_t i = tile + tid;
            uint32_t deg = 0, rs = 0, w = 0, aux = 0;
            uint64_t d = 0;
            if (i < nf) {
                const uint64_t e = i == i0 ? e0 : cur[i];
                w = (uint32_t)(e >> 32);
                uint32_t x = (uint32_t)e;
                rs = a.row[x];
                deg = a.row[x + 1] - rs;
                uint32_t hs = deg >= a.hub.min_deg ? a.hub.slot[x] : IM_EMPTY;
                // bits gained since x was last expanded; later ones re-queue x
                d = atomicExch((unsigned long long *)&a.pend[(uint64_t)w * a.n + x], 0ull);
                if (hs != IM_EMPTY) {
                    hub_push(L.H, hs, w, d);
                    deg = 0; d = 0;
                } else {
                    uint32_t work, srs, saux;
                    uint64_t sdel;
                    if (deg >= 2 && sparse_use(sparse_fetch(a.sp, a.n, w, x, d), deg, work, srs, sdel, saux)) {
                        deg = work; rs = srs; d = sdel; aux = saux;
                    }
                }
            }
            uint32_t total;
            uint32_t ex = block_excl_scan<FWD_NT>(deg, L.wsum, &total);
            L.scan[tid] = ex; L.rs[tid] = rs; L.del[tid] = d; L.wd[tid] = w; L.aux[tid] = aux;
            __syncthreads();
            const uint32_t nhub = L.H.n;
            arcs += total;
            for (uint32_t j0 = 0; j0 < total; j0 += FWD_NT * FWD_U) {
                uint32_t kk[FWD_U], ee[FWD_U], vv[FWD_U];
                uint64_t bb[FWD_U];
#pragma unroll
                for (int u = 0; u < FWD_U; u++) {
                    uint32_t j = j0 + (uint32_t)tid + (uint32_t)u * FWD_NT;
                    kk[u] = 0xFFFFFFFFu; ee[u] = 0; bb[u] = 0; vv[u] = 0;
                    if (j < total) {
                        int k = upper_index<FWD_NT>(L.scan, j);
                        kk[u] = (uint32_t)k;
                        ee[u] = j - L.scan[k];   // rank within the entry
                    }
                }
#pragma unroll
                for (int u = 0; u < FWD_U; u++)
                    if (kk[u] != 0xFFFFFFFFu) {
                        const uint32_t k = kk[u], ax = L.aux[k];
                        uint32_t pos = L.rs[k] + ee[u];
                        uint64_t bit = 0;
                        if (ax) sparse_item(L.rs[k], L.del[k], ax, ee[u], pos, bit);
                        const uint32_t *heads = ax ? a.sp.adj : a.col;
                        vv[u] = heads[pos];
                        bb[u] = ax ? bit : (a.mask[(uint64_t)L.wd[k] * a.m + pos] & L.del[k]);
                    }
                uint64_t vis_e[FWD_U], nxt_e[FWD_U];
                uint32_t nvis = 0, nnxt = 0;
#pragma unroll
                for (int u = 0; u < FWD_U; u++) {
                    uint32_t ww = kk[u] != 0xFFFFFFFFu ? L.wd[kk[u]] : 0u;
                    uint64_t bits = kk[u] != 0xFFFFFFFFu ? bb[u] : 0ull;
                    bool first, push;
                    fwd_relax(a, ww, vv[u], bits, first, push);
                    const uint64_t ent = ((uint64_t)ww << 32) | vv[u];
                    if (first) vis_e[nvis++] = ent;
                    if (push) nxt_e[nnxt++] = ent;
                }
                wave_append_n<FWD_U>(nvis, vis_e, a.cnt + 3, a.vis);
                wave_append_n<FWD_U>(nnxt, nxt_e, ncnt, nxt);
            }
            __syncthreads();
            if (nhub) {
                auto word_of = [&](uint32_t own) { return own; };
                uint64_t vis_e[FWD_U], nxt_e[FWD_U];
                uint32_t nvis = 0, nnxt = 0;
                auto relax = [&](uint32_t own, uint32_t hv, uint64_t bits) {
                    bool first, push;
                    fwd_relax(a, own, hv, bits, first, push);
                    const uint64_t ent = ((uint64_t)own << 32) | hv;
                    if (first) vis_e[nvis++] = ent;
                    if (push) nxt_e[nnxt++] = ent;
                };
                auto flush = [&]() {
                    wave_append_n<FWD_U>(nvis, vis_e, a.cnt + 3, a.vis);
                    wave_append_n<FWD_U>(nnxt, nxt_e, ncnt, nxt);
                    nvis = 0;
                    nnxt = 0;
                };
                expand_hubs<FWD_NT, 16, FWD_U>(L.H, nhub, a.hub, a.W, word_of, relax, flush, arcs);
            }
        }
        if (!grid_barrier(a.cnt + FWD_BAR, nbar, a.stats)) return;
    }
    // per-word visit lists (the reverse tasks) are built from the unified
    // list, one atomic per (workgroup, word) and chunk
    uint64_t relax = 0, trav = 0;
    const uint32_t nv = group_load(&a.cnt[3], &L.bcast);
    // reused (W <= 64): per-word visit and multi-bit counts of this chunk, and
    // their global bases
    uint32_t *wcnt = L.scan, *wbase = L.rs, *wmc = L.wd, *wmb = L.aux;
    const bool pack = a.bcnt != nullptr;
    for (uint32_t j = tid; j < a.W * 64; j += FWD_NT) L.pk[j] = 0;
    for (uint32_t base = blockIdx.x * FWD_NT; base < nv; base += gridDim.x * FWD_NT) {
        if (tid < 64) { wcnt[tid] = 0; wmc[tid] = 0; }
        __syncthreads();
        const uint32_t i = base + tid;
        uint32_t w = 0, x = 0, r = 0, rm = 0;
        bool multi = false;
        if (i < nv) {
            uint64_t e = a.vis[i];
            w = (uint32_t)(e >> 32);
            x = (uint32_t)e;
            const uint64_t off = (uint64_t)w * a.n;
            uint64_t b = a.newly[off + x];   // covered took these bits as they were reached
            uint32_t dg = a.row[x + 1] - a.row[x];
            relax += dg;
            trav += (uint64_t)__popcll(b) * dg;
            r = atomicAdd(&wcnt[w], 1u);
            if (pack) {
                multi = __popcll(b) != 1;
                if (multi) rm = atomicAdd(&wmc[w], 1u);
                else atomicAdd(&L.pk[w * 64 + (uint32_t)__ffsll((unsigned long long)b) - 1], 1u);
            }
        }
        __syncthreads();
        if (tid < 64 && tid < (int)a.W) {
            if (wcnt[tid]) wbase[tid] = atomicAdd(&a.cnt[4 + tid], wcnt[tid]);
            if (wmc[tid]) wmb[tid] = atomicAdd(&a.mcnt[tid], wmc[tid]);
        }
        __syncthreads();
        if (i < nv) {
            a.tnodes[(uint64_t)w * a.n + wbase[w] + r] = x;
            if (multi) a.mlist[(uint64_t)w * a.n + wmb[w] + rm] = x;
        }
        __syncthreads();
    }
    if (pack)
        for (uint32_t j = tid; j < a.W * 64; j += FWD_NT)
            if (L.pk[j]) atomicAdd(&a.bcnt[j], L.pk[j]);
    if (!grid_barrier(a.cnt + FWD_BAR, nbar, a.stats)) return;
    if (gtid < a.W) {
        const uint32_t c = coherent_load(&a.cnt[4 + gtid]);
        a.tcounts[gtid] = c;
        atomicAdd(&a.stats[ST_TASKS_REV], (unsigned long long)c);
    }
    relax = group_sum<FWD_NT>(relax, L.red);
    trav = group_sum<FWD_NT>(trav, L.red);
    if (tid == 0) {
        atomicAdd(&a.stats[ST_RELAX_FWD], (unsigned long long)relax);
        atomicAdd(&a.stats[ST_TRAV_FWD], (unsigned long long)trav);
    }
}

// Rounds below the gain threshold: one workgroup per word runs its search
// alone (no grid-wide barriers; per-level latency is what limits small searches).
constexpr int FWB_NT = 1024;

__global__ __launch_bounds__(FWB_NT) void k_forward_block(FwdArgs a)
{
    __shared__ BlockLds<FWB_NT> L;
    const int tid = threadIdx.x;
    const unsigned long long key = a.key[0];
    if (a.skip && *a.skip) return;
    if (key == 0) return;
    if ((key >> 32) >= a.coop_gain) return;  // the cooperative kernel runs this round
    if ((key >> 32) < a.block_floor) return; // an earlier launch ran it
    const uint32_t v = 0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull);
    const uint32_t w = blockIdx.x;
    const uint64_t off = (uint64_t)w * a.n;
    if (w == 0 && tid == 0) {
        a.seeds_out[a.t] = v;
        a.gains_out[a.t] = key >> 32;
        a.sel[v] = 1;
    }
    const uint64_t start = im_valid_bits(a.R, w) & ~a.covered[off + v];
    if (!start) {
        if (tid == 0) a.tcounts[w] = 0;
        return;
    }
    uint64_t arcs = 0;
    const SparseLists no_lists = {nullptr, nullptr, nullptr};
    block_bfs_run<FWB_NT, 8, true, false>(L, v, tid == 0 ? start : 0ull, a.row, a.col, a.mask + (uint64_t)w * a.m, a.hub,
                                   no_lists, a.n, a.W, w, a.covered + off, a.newly + off, a.pend + off, 0u,
                                   a.bq0 + off, a.bq1 + off, a.tnodes + off, arcs);
    const uint32_t nvis = L.nvis;
    uint64_t relax = 0, trav = 0;
    __shared__ uint32_t pk[64];   // packing counts per bit of this word
    const bool pack = a.bcnt != nullptr;
    if (tid < 64) pk[tid] = 0;
    __syncthreads();
    for (uint32_t b0 = 0; b0 < nvis; b0 += FWB_NT) {   // whole wavefronts per step
        const uint32_t i = b0 + tid;
        uint32_t x = 0;
        bool multi = false;
        if (i < nvis) {
            x = a.tnodes[off + i];
            uint64_t b = a.newly[off + x];
            a.covered[off + x] |= b;
            uint32_t dg = a.row[x + 1] - a.row[x];
            relax += dg;
            trav += (uint64_t)__popcll(b) * dg;
            if (pack) {
                multi = __popcll(b) != 1;
                if (!multi) atomicAdd(&pk[__ffsll((unsigned long long)b) - 1], 1u);
            }
        }
        if (pack) {
            const uint32_t p = wave_append(multi, &a.mcnt[w]);
            if (multi) a.mlist[off + p] = x;
        }
    }
    __syncthreads();
    if (pack && tid < 64 && pk[tid]) atomicAdd(&a.bcnt[w * 64 + tid], pk[tid]);
    relax = group_sum<FWB_NT>(relax, L.red);
    trav = group_sum<FWB_NT>(trav, L.red);
    if (tid == 0) {
        a.tcounts[w] = nvis;
        atomicAdd(&a.stats[ST_FWD_LEVELS], (unsigned long long)L.levels);
        atomicAdd(&a.stats[ST_FWD_ENTRIES], (unsigned long long)L.entries);
        atomicAdd(&a.stats[ST_TASKS_REV], (unsigned long long)nvis);
        atomicAdd(&a.stats[ST_RELAX_FWD], (unsigned long long)relax);
        atomicAdd(&a.stats[ST_TRAV_FWD], (unsigned long long)trav);
    }
}

// ---------------------------------------------------------------------------
// Reverse-task packing. Decrements from sources whose start bits are disjoint
// can share one reverse search: a node's bit r can then only come from the
// one source that owns r, so popcount(bits) at that node is the sum of the
// per-source decrements. Sources newly covered in a single snapshot of the
// word are sorted by that snapshot's bit; group g takes the g-th source of
// every bit. Sources covered in several snapshots stay separate tasks.
// ---------------------------------------------------------------------------
constexpr int PK_NT = 256;
constexpr int PK_ZERO = 64 * 64 * 2 + 128;  // bcnt, bcur [W][64]; gcnt, mcnt [64]

// Place the single-bit tasks bit by bit. Every workgroup of word w takes the
// bit offsets as the exclusive prefix of that word's 64 bit counts (counted
// by the forward search as it finished); workgroup 0 of the word also stores
// them, with the largest count, for the reverse pass.
__global__ __launch_bounds__(PK_NT) void k_pack_fill(const uint32_t *tnodes, const uint32_t *tcounts,
                                                     const uint64_t *newly, uint32_t n,
                                                     const uint32_t *bcnt, uint32_t *boff,
                                                     uint32_t *gcnt, uint32_t *bcur, uint32_t *plist,
                                                     uint32_t *mcnt, const unsigned long long *key,
                                                     uint64_t aff_gain)
{
    __shared__ uint32_t cnt[64], base0[64];
    const uint32_t w = blockIdx.y;
    if (aff_gain && (*key >> 32) < aff_gain) {
        // a round updated by the affected-set recompute: no reverse tasks
        if (blockIdx.x == 0 && threadIdx.x == 0) { gcnt[w] = 0; mcnt[w] = 0; }
        return;
    }
    const uint64_t off = (uint64_t)w * n;
    const uint32_t c = tcounts[w];
    if (threadIdx.x < 64) {
        const uint32_t lane = threadIdx.x, k = bcnt[w * 64 + lane];
        const uint32_t ex = wave_incl_scan(k) - k;
        cnt[lane] = 0;
        base0[lane] = ex;
        if (blockIdx.x == 0) {
            boff[w * 64 + lane] = ex;
            uint32_t mx = k;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, d, 64));
            if (lane == 0) gcnt[w] = mx;
        }
    }
    __syncthreads();
    for (uint32_t i = blockIdx.x * PK_NT + threadIdx.x; i < c; i += gridDim.x * PK_NT) {
        const uint64_t b = newly[off + tnodes[off + i]];
        if (__popcll(b) == 1) atomicAdd(&cnt[__ffsll((unsigned long long)b) - 1], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const uint32_t k = cnt[threadIdx.x];
        base0[threadIdx.x] += k ? atomicAdd(&bcur[w * 64 + threadIdx.x], k) : 0u;
        cnt[threadIdx.x] = 0;
    }
    __syncthreads();
    for (uint32_t i = blockIdx.x * PK_NT + threadIdx.x; i < c; i += gridDim.x * PK_NT) {
        const uint32_t x = tnodes[off + i];
        const uint64_t b = newly[off + x];
        if (__popcll(b) != 1) continue;
        const uint32_t r = __ffsll((unsigned long long)b) - 1;
        const uint32_t pos = base0[r] + atomicAdd(&cnt[r], 1u);
        plist[off + pos] = x;
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
// tier 0: 64 lanes, T0_T tasks of up to T0_LIM nodes, degrees <= T0_DMAX
constexpr int T0_T = 8, T0_CS = 32, T0_LIM = 24, T0_U = 4;
constexpr uint32_t T0_DMAX = 1024;
// tier 1: 256 lanes, T1_T tasks of up to T1_LIM nodes, any degree (the
// default shape; two others: 2 tasks x 512 entries, 1 task x 1024 entries)
constexpr int T1_NT = 256, T1_T = 4, T1_CS = 256, T1_LIM = 192, T1_U = 4;
// tier 2: dense global arrays
constexpr int T2_NT = 256, T2_U = 8;
constexpr int T2W_NT = 1024;   // the wide variant: more lanes per task
constexpr int T2S_NT = 64;     // the narrow variant: more tasks at once (long, thin searches)
// per-phase device counters: grab0, n1, grab1, n2, grab2
constexpr int PH_CTRS = 8;

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
struct im_workspace {
    int device = -1;
    int num_cu = 256;
    uint32_t cap_n = 0, cap_W = 0, cap_k = 0, slots = 0;
    uint32_t max_slots = 256, slots_n = 0;  // tier-2: slot limit, length of each slot in use
    uint64_t slots_entries = 0;             // allocated slot entries
    int tier1_shape = 0;     // tier-1 tasks x table entries: 0: 4 x 256, 1: 2 x 512, 2: 1 x 1024
    uint32_t tier2_lanes = T2_NT;   // lanes per tier-2 task: 64, 256 or 1024
    uint64_t cap_m = 0;
    // graph-derived
    uint32_t *row32 = nullptr, *in_row = nullptr, *in_col = nullptr, *in2out = nullptr;
    uint32_t *cnt = nullptr, *scan_sums = nullptr;
    uint64_t *mask_out = nullptr, *mask_in = nullptr;
    // selection state
    uint32_t *gain = nullptr;
    uint8_t *sel = nullptr;
    uint64_t *covered = nullptr, *newly = nullptr, *fpend = nullptr;
    uint64_t *fqa = nullptr, *fqb = nullptr, *fvis = nullptr;
    uint32_t *bqa = nullptr, *bqb = nullptr;
    uint64_t coop_gain = 0;  // every round uses the cooperative forward search
    uint32_t *tnodes = nullptr, *tcounts = nullptr;
    uint32_t *fctr = nullptr;  // [k][FWD_CTRS] forward-search counters
    uint32_t *pk = nullptr;    // packing counters: bcnt, bcur [64][64], gcnt, mcnt [64]
    uint32_t *boff = nullptr;  // [64][64]
    uint32_t *plist = nullptr, *mlist = nullptr;  // [W][n]
    unsigned fwd_grid = 0;      // co-resident workgroups of the cooperative forward search
    unsigned fwd_per_word = 16; // forward-search workgroups per snapshot word
    unsigned long long *keys = nullptr;
    uint64_t cap_keys = 0;
    // batches
    Batch batch = {1, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    uint32_t cap_count = 0;
    uint64_t cap_bn = 0, cap_bm = 0;
    uint32_t *b_node_inst = nullptr, *b_mcol = nullptr;
    float *b_mprob = nullptr;
    uint32_t *b_u32 = nullptr;          // R, k, kpre, node_off per instance
    uint64_t *b_u64 = nullptr;          // arc_off, seed per instance
    InstDesc *b_desc = nullptr;
    void *b_host = nullptr;             // pinned staging of the above
    uint32_t *ovf_q = nullptr, *ovf_q2 = nullptr;
    uint32_t *ctrs = nullptr;
    // hub lists per direction (0: forward arcs, 1: reverse arcs)
    uint32_t hub_deg = 256;
    uint64_t cap_hub = 0, cap_hadj = 0;
    uint32_t *hslot[2] = {}, *hlist[2] = {}, *hcnt[2] = {}, *hoff[2] = {}, *hadj[2] = {};
    unsigned long long *hbase[2] = {};
    uint32_t *hnum = nullptr;            // [2] hub counts
    // per-snapshot live lists of the other nodes, per direction
    int sparse = 1;
    uint64_t sp_nW = 0, sp_cap = 0;
    uint32_t *sp_base[2] = {}, *sp_adj[2] = {};
    uint16_t *sp_cum[2] = {};
    unsigned long long *sp_alloc = nullptr;  // [2]
    unsigned long long *halloc = nullptr;  // [2] allocation counters
    // block engine slots
    uint64_t *b_reach = nullptr;   // tier-2 slots: (reach, pend) per node, interleaved
    uint32_t *b_qa = nullptr, *b_qb = nullptr, *b_vis = nullptr;
    // lazy evaluation (A9)
    uint32_t cap_celf = 0;
    uint64_t cap_sort = 0;
    uint32_t *c_kept = nullptr;  // [2][cap_kept]: visit count and source of each kept search
    uint32_t cap_kept = 0;
    uint32_t *c_bound = nullptr, *c_fresh = nullptr, *c_ev = nullptr, *c_ordB = nullptr,
             *c_ordS = nullptr, *c_E = nullptr, *c_cand = nullptr, *c_ctl = nullptr;
    uint8_t *c_moved = nullptr;
    float *c_score = nullptr, *c_feat = nullptr;
    unsigned long long *c_sort = nullptr;
    int lazy_engine = 2;     // 2: the last tier only (one workgroup per task), 0: the
                             // three tiers, 1: cooperative batched evaluation
    int learned_policy = 2;  // 1: score order among can-win nodes, 2: predicted-gain batches
    uint32_t lazy_batch = 4; // batch of im_select_lazy when it is called with batch = 0
    uint32_t eval_split = 0; // bit groups per kept evaluation search (0: the most of 8, 4, 2 that fit)
    uint32_t rev_split = 1;  // bit groups per last-tier reverse task
    uint32_t rev_first = 0;  // engine tier reverse tasks start on (0 or 1)
    unsigned eval_grid = 0;
    uint64_t cap_eval = 0;
    uint64_t *e_reach = nullptr, *e_pend = nullptr, *e_fq0 = nullptr, *e_fq1 = nullptr,
             *e_vis = nullptr;
    uint32_t *e_cnt = nullptr;
    // spread evaluator: one chunk of snapshot words at a time
    uint32_t cap_sp_n = 0, cap_sp_words = 0;
    uint64_t cap_sp_m = 0;
    uint32_t *v_row32 = nullptr;
    uint64_t *v_mask = nullptr, *v_reach = nullptr, *v_pend = nullptr, *v_cov = nullptr;
    uint32_t *v_qa = nullptr, *v_qb = nullptr, *v_vis = nullptr;
    // linear-threshold snapshots
    int live_edge = 0;                   // 0: independent cascade, 1: linear threshold
    uint64_t *lt_start = nullptr;        // [m] start of each in-arc's draw interval
    uint32_t *lt_task = nullptr;         // [n+1] prefix of the large rows' chunk counts
    uint64_t cap_lt_m = 0;
    uint32_t cap_lt_n = 0;
    // undirected graphs: one coin per pair (directed engines), component method state
    int pair_coins = 0;
    uint32_t *pair = nullptr;
    uint64_t cap_pair = 0;
    UndState *und = nullptr;
    // affected-set recompute (rounds whose gain is below aff_gain; 0: never)
    uint64_t aff_gain = 0;
    uint64_t cap_aff_nW = 0;
    uint32_t cap_aff_n = 0, cap_aff_k = 0;
    uint64_t *a_reach = nullptr, *a_pend = nullptr;
    uint32_t *a_qa = nullptr, *a_qb = nullptr, *a_vis = nullptr;
    uint32_t *a_mark = nullptr, *a_list = nullptr, *a_cnt = nullptr, *a_ctrs = nullptr;
    // misc
    unsigned long long *stats = nullptr;
    uint32_t *err = nullptr;
    uint32_t *host_err = nullptr;
    unsigned long long *host_stats = nullptr;
    hipStream_t last_stream = nullptr;
    // phase timers
    uint32_t prof_mask = 0;
    std::vector<hipEvent_t> ev[IM_PH_COUNT];
    size_t ev_used[IM_PH_COUNT] = {};
    std::vector<float> last_ms[IM_PH_COUNT];  // per-launch durations of the last get
    int open_phase = -1;
};

// bracket a phase's launches with events (only for phases enabled in prof_mask)
struct PhaseTimer {
    im_workspace *ws;
    int ph;
    hipStream_t s;
    bool on;
    PhaseTimer(im_workspace *w, int p, hipStream_t st) : ws(w), ph(p), s(st)
    {
        on = (ws->prof_mask >> ph) & 1u;
        if (on) record();
    }
    ~PhaseTimer()
    {
        if (on) record();
    }
    void record()
    {
        std::vector<hipEvent_t> &v = ws->ev[ph];
        size_t &u = ws->ev_used[ph];
        if (u == v.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) { on = false; return; }
            v.push_back(e);
        }
        (void)hipEventRecord(v[u++], s);
    }
};

// Workspace buffers come from hipMalloc, or, while a call of the entry point
// that allocates nothing is being set up on this thread, from a bump arena
// over that entry point's static device scratch. A measuring arena hands out
// no memory: it only adds up what the buffers would take.
struct Arena {
    char *base;        // device address of the scratch (null while measuring)
    uint64_t cap, used;
    hipStream_t stream;   // the call's stream: buffers are cleared on it
};
static thread_local Arena *t_arena = nullptr;

static int arena_take(Arena *a, void **p, uint64_t bytes)
{
    const uint64_t at = (a->used + 255) & ~255ull;
    a->used = at + bytes;
    if (!a->base) {
        *p = nullptr;
        return IM_OK;
    }
    if (a->used > a->cap) {
        *p = nullptr;
        return im_fail(IM_EINVAL, "the selection needs more than the %llu bytes of static scratch",
                       (unsigned long long)a->cap);
    }
    *p = a->base + at;
    return IM_OK;
}

// hipMemset of a workspace buffer (skipped while an arena only measures)
static int ws_memset(void *p, uint64_t bytes)
{
    if (t_arena) {
        if (t_arena->base) HIPCHK(hipMemsetAsync(p, 0, bytes, t_arena->stream));
        return IM_OK;
    }
    HIPCHK(hipMemset(p, 0, bytes));
    return IM_OK;
}

template <typename Tv>
static int dalloc(Tv **p, uint64_t cnt)
{
    if (cnt == 0) cnt = 1;
    if (t_arena) return arena_take(t_arena, (void **)p, cnt * sizeof(Tv));
    if (*p) { (void)hipFree(*p); *p = nullptr; }
    hipError_t e = hipMalloc((void **)p, cnt * sizeof(Tv));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return im_fail(IM_ENOMEM, "hipMalloc of %llu bytes failed: %s",
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

struct EvalArgs;
__global__ __launch_bounds__(FWD_NT) void k_eval_coop(EvalArgs a);

// device properties and cooperative grid sizes of a new workspace
static int ws_init_device(im_workspace *ws)
{
    HIPCHK(hipGetDevice(&ws->device));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, ws->device));
    ws->num_cu = prop.multiProcessorCount;
    {
        int b = 0;
        HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_forward_coop, FWD_NT, 0));
        if (b < 1) b = 1;
        // 16 workgroups per snapshot word at most: grid barriers stay cheap
        ws->fwd_grid = (unsigned)b * (unsigned)ws->num_cu;
        int be = 0;
        HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&be, k_eval_coop, FWD_NT, 0));
        if (be < 1) be = 1;
        ws->eval_grid = (unsigned)be * (unsigned)ws->num_cu;
    }
    return IM_OK;
}

extern "C" int im_workspace_create(im_workspace **out)
{
    if (!out) return im_fail(IM_EINVAL, "im_workspace_create: null output pointer");
    im_workspace *ws = new im_workspace();
    int rc;
    if ((rc = ws_init_device(ws))) { delete ws; return rc; }
    if ((rc = dalloc(&ws->stats, ST_COUNT * ST_STRIPES))) { delete ws; return rc; }
    if ((rc = dalloc(&ws->err, 1))) { delete ws; return rc; }
    HIPCHK(hipHostMalloc((void **)&ws->host_err, sizeof(uint32_t), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&ws->host_stats, ST_COUNT * ST_STRIPES * sizeof(unsigned long long),
                         hipHostMallocDefault));
    HIPCHK(hipMemset(ws->stats, 0, ST_COUNT * ST_STRIPES * sizeof(unsigned long long)));
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
    dfree(ws->fpend); dfree(ws->fqa); dfree(ws->fqb); dfree(ws->fvis); dfree(ws->bqa); dfree(ws->bqb); dfree(ws->fctr);
    dfree(ws->pk); dfree(ws->boff); dfree(ws->plist); dfree(ws->mlist);
    dfree(ws->tnodes); dfree(ws->tcounts); dfree(ws->keys); dfree(ws->ovf_q); dfree(ws->ovf_q2); dfree(ws->ctrs);
    dfree(ws->b_reach);
    dfree(ws->b_qa); dfree(ws->b_qb); dfree(ws->b_vis);
    for (int d = 0; d < 2; d++) {
        dfree(ws->hslot[d]); dfree(ws->hlist[d]); dfree(ws->hcnt[d]); dfree(ws->hoff[d]);
        dfree(ws->hadj[d]); dfree(ws->hbase[d]);
    }
    dfree(ws->hnum); dfree(ws->halloc);
    for (int d = 0; d < 2; d++) { dfree(ws->sp_base[d]); dfree(ws->sp_cum[d]); dfree(ws->sp_adj[d]); }
    dfree(ws->sp_alloc);
    dfree(ws->b_node_inst); dfree(ws->b_mcol); dfree(ws->b_mprob); dfree(ws->b_u32);
    dfree(ws->b_u64); dfree(ws->b_desc);
    if (ws->b_host) (void)hipHostFree(ws->b_host);
    dfree(ws->c_bound); dfree(ws->c_fresh); dfree(ws->c_ev); dfree(ws->c_ordB); dfree(ws->c_ordS);
    dfree(ws->c_E); dfree(ws->c_cand); dfree(ws->c_ctl); dfree(ws->c_moved); dfree(ws->c_score);
    dfree(ws->c_feat); dfree(ws->c_sort); dfree(ws->c_kept);
    dfree(ws->e_reach); dfree(ws->e_pend); dfree(ws->e_fq0); dfree(ws->e_fq1); dfree(ws->e_vis);
    dfree(ws->e_cnt);
    und_state_free(ws->und);
    ws->und = nullptr;
    dfree(ws->pair);
    dfree(ws->lt_start); dfree(ws->lt_task);
    dfree(ws->a_reach); dfree(ws->a_pend); dfree(ws->a_qa); dfree(ws->a_qb); dfree(ws->a_vis);
    dfree(ws->a_mark); dfree(ws->a_list); dfree(ws->a_cnt); dfree(ws->a_ctrs);
    dfree(ws->v_row32); dfree(ws->v_mask); dfree(ws->v_reach); dfree(ws->v_pend); dfree(ws->v_cov);
    dfree(ws->v_qa); dfree(ws->v_qb); dfree(ws->v_vis);
    dfree(ws->stats); dfree(ws->err);
    if (ws->host_err) (void)hipHostFree(ws->host_err);
    if (ws->host_stats) (void)hipHostFree(ws->host_stats);
    for (int p = 0; p < IM_PH_COUNT; p++)
        for (hipEvent_t e : ws->ev[p]) (void)hipEventDestroy(e);
    delete ws;
    return IM_OK;
}

static uint32_t slots_for(uint32_t n, uint32_t max_slots)
{
    // dense global-engine state: 28 bytes per node per slot, at most 48 GB
    uint64_t per = 28ull * (n ? n : 1);
    uint64_t s = (48ull << 30) / per;
    if (s > max_slots) s = max_slots;
    if (s < 8) s = 8;
    return (uint32_t)s;
}

// tier-2 slot arrays of slot_len nodes each (the largest instance of a
// batch, else the graph); every entry of reach and pend is zero at rest,
// so the arrays may be re-sliced between calls
static int reserve_slots(im_workspace *ws, uint32_t slot_len)
{
    int rc;
    slot_len = std::max<uint32_t>(slot_len, 1);
    const uint32_t slots = slots_for(slot_len, ws->max_slots);
    const uint64_t sn = (uint64_t)slots * slot_len;
    if (sn > ws->slots_entries) {
        if ((rc = dalloc(&ws->b_reach, 2 * sn)) ||
            (rc = dalloc(&ws->b_qa, sn)) || (rc = dalloc(&ws->b_qb, sn)) ||
            (rc = dalloc(&ws->b_vis, sn)))
            return rc;
        if ((rc = ws_memset(ws->b_reach, 2 * sn * sizeof(uint64_t)))) return rc;
        ws->slots_entries = sn;
    }
    ws->slots = slots;
    ws->slots_n = slot_len;
    return IM_OK;
}

// grow the workspace to hold a graph with n nodes, m arcs, W words, k rounds
static int ws_reserve(im_workspace *ws, uint32_t n, uint64_t m, uint32_t W, uint32_t k,
                      uint32_t slot_len)
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
            (rc = dalloc(&ws->fpend, nW)) ||
            (rc = dalloc(&ws->fqa, nW)) || (rc = dalloc(&ws->fqb, nW)) || (rc = dalloc(&ws->fvis, nW)) ||
            (rc = dalloc(&ws->bqa, nW)) || (rc = dalloc(&ws->bqb, nW)) ||
            (rc = dalloc(&ws->plist, nW)) || (rc = dalloc(&ws->mlist, nW)) ||
            (rc = dalloc(&ws->pk, PK_ZERO)) || (rc = dalloc(&ws->boff, 64 * 64)) ||
            (rc = dalloc(&ws->tnodes, nW)) || (rc = dalloc(&ws->tcounts, 64)) ||
            (rc = dalloc(&ws->ovf_q, nW)) || (rc = dalloc(&ws->ovf_q2, nW)))
            return rc;
        for (int d = 0; d < 2; d++)
            if ((rc = dalloc(&ws->hslot[d], cn))) return rc;
        if ((rc = ws_memset(ws->newly, nW * sizeof(uint64_t))) ||
            (rc = ws_memset(ws->fpend, nW * sizeof(uint64_t))))
            return rc;
        ws->cap_n = cn;
    }
    if ((rc = reserve_slots(ws, slot_len))) return rc;
    if (grow_m) {
        if ((rc = dalloc(&ws->in_col, cm)) || (rc = dalloc(&ws->in2out, cm)) ||
            (rc = dalloc(&ws->mask_out, cm * cW)) || (rc = dalloc(&ws->mask_in, cm * cW)))
            return rc;
        uint64_t cap = std::min<uint64_t>(2ull * cm * cW, 0x7FFFFFFFull);
        for (int d = 0; d < 2; d++)
            if ((rc = dalloc(&ws->hadj[d], cap))) return rc;
        if ((rc = dalloc(&ws->hnum, 2)) || (rc = dalloc(&ws->halloc, 2))) return rc;
        ws->cap_hadj = cap;
        ws->cap_hub = 0;
        ws->cap_m = cm;
    }
    ws->cap_W = cW;
    // hub tables: at most m / hub_deg hubs
    const uint64_t maxh = cm / std::max<uint32_t>(ws->hub_deg, 16u) + 1;
    if (grow_m || grow_n || maxh > ws->cap_hub) {
        const uint64_t ch = std::max<uint64_t>(maxh, ws->cap_hub);
        for (int d = 0; d < 2; d++)
            if ((rc = dalloc(&ws->hlist[d], ch)) || (rc = dalloc(&ws->hbase[d], ch * cW)) ||
                (rc = dalloc(&ws->hcnt[d], ch * cW * 64)) || (rc = dalloc(&ws->hoff[d], ch * cW * 65)))
                return rc;
        ws->cap_hub = ch;
    }
    if (ws->sparse) {
        const uint64_t nW = (uint64_t)ws->cap_n * cW;
        if (nW > ws->sp_nW) {
            for (int d = 0; d < 2; d++)
                if ((rc = dalloc(&ws->sp_base[d], nW)) || (rc = dalloc(&ws->sp_cum[d], nW * 65)))
                    return rc;
            if ((rc = dalloc(&ws->sp_alloc, 2))) return rc;
            ws->sp_nW = nW;
        }
        const uint64_t cap = std::min<uint64_t>(16ull * ws->cap_m * cW, 0x7FFFFFFFull);
        if (cap > ws->sp_cap) {
            for (int d = 0; d < 2; d++)
                if ((rc = dalloc(&ws->sp_adj[d], cap))) return rc;
            ws->sp_cap = cap;
        }
    }
    const uint64_t nkeys = (uint64_t)(k + 1) * ws->batch.count;
    if (nkeys > ws->cap_keys) {
        if ((rc = dalloc(&ws->keys, nkeys))) return rc;
        ws->cap_keys = nkeys;
    }
    if (k + 1 > ws->cap_k) {
        uint32_t ck = k + 1;
        if ((rc = dalloc(&ws->ctrs, (uint64_t)(ck + 1) * PH_CTRS)) ||
            (rc = dalloc(&ws->fctr, (uint64_t)ck * FWD_CTRS)))
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
    if (!g) return im_fail(IM_EINVAL, "null graph");
    if (g->m >= (1ull << 32)) return im_fail(IM_EINVAL, "m = %llu must be < 2^32", (unsigned long long)g->m);
    if (!g->row_ptr) return im_fail(IM_EINVAL, "null row_ptr");
    if (g->m && (!g->col || !g->prob)) return im_fail(IM_EINVAL, "null col or prob");
    if (R == 0 || R > IM_R_MAX) return im_fail(IM_EINVAL, "R = %u must be in [1, %u]", R, IM_R_MAX);
    if ((uint64_t)g->n * R >= (1ull << 32))
        return im_fail(IM_EOVERFLOW, "n * R = %llu must be < 2^32", (unsigned long long)g->n * R);
    return IM_OK;
}

static int validate(const im_graph *g, im_workspace *ws, hipStream_t s, uint32_t *row32)
{
    PhaseTimer pt(ws, IM_PH_VALIDATE, s);
    HIPCHK(hipMemsetAsync(ws->err, 0, sizeof(uint32_t), s));
    uint64_t lim = std::max<uint64_t>((uint64_t)g->n + 1, g->m);
    k_validate<<<grid_for(lim, 256), 256, 0, s>>>(g->row_ptr, g->col, g->prob, g->n, g->m,
                                                  ws->err, row32);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(ws->host_err, ws->err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    uint32_t e = *ws->host_err;
    if (e & ERR_ROW0) return im_fail(IM_EINVAL, "row_ptr[0] != 0");
    if (e & ERR_ROWN) return im_fail(IM_EINVAL, "row_ptr[n] != m");
    if (e & (ERR_ROWDEC | ERR_ROWBIG)) return im_fail(IM_EINVAL, "row_ptr is not non-decreasing within [0, m]");
    if (e & ERR_COL) return im_fail(IM_EINVAL, "col entry >= n");
    if (e & ERR_PROB) return im_fail(IM_EINVAL, "prob outside [0, 1] or NaN");
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

// A1: reverse CSR (row32 must already hold the 32-bit offsets). With
// offsets_only, just the in-row offsets (in-degrees) are built: paths
// without reverse searches need no more.
static void build_reverse(const im_graph *g, im_workspace *ws, hipStream_t s, bool offsets_only = false)
{
    uint32_t n = g->n;
    uint64_t m = g->m;
    PhaseTimer pt(ws, IM_PH_TRANSPOSE, s);
    const unsigned tblocks = (unsigned)((m + TR_ARCS - 1) / TR_ARCS);
    fill<uint32_t>(ws->cnt, (uint64_t)n + 1, 0u, s);
    if (m)
        k_transpose<false><<<tblocks, TR_NT, 0, s>>>(ws->row32, g->col, n, m, ws->cnt, nullptr,
                                                     nullptr, nullptr);
    exclusive_scan(ws->cnt, ws->in_row, (uint64_t)n + 1, ws->scan_sums, s);
    if (offsets_only) return;
    fill<uint32_t>(ws->cnt, (uint64_t)n + 1, 0u, s);
    if (m)
        k_transpose<true><<<tblocks, TR_NT, 0, s>>>(ws->row32, g->col, n, m, ws->cnt, ws->in_row,
                                                    ws->in_col, ws->in2out);
}

// ---------------------------------------------------------------------------
// A2, linear-threshold snapshots in live-edge form: per snapshot every node
// keeps at most one of its in-arcs. The in-arcs of v, by increasing arc id,
// own consecutive sub-intervals of [0, 2^32) of lengths t_e = floor(b_e 2^32)
// (b_e = prob[e]; a part past 2^32 is never drawn); the node's draw for
// snapshot r, the top 32 bits of output r+1 of SplitMix64 seeded with output
// v+1 of SplitMix64(seed), keeps the arc whose sub-interval holds it.
// The reverse CSR lists in-arcs in no particular order, so each in-arc's
// interval start is the sum of t over the in-arcs of its row with a smaller
// arc id: one thread per row for rows of up to LT_SMALL in-arcs, one
// workgroup per LT_SMALL-entry chunk (the row streamed through LDS) above.
// ---------------------------------------------------------------------------
constexpr uint32_t LT_SMALL = 256;

__device__ __forceinline__ uint64_t lt_len(const float *prob, uint32_t e)
{
    return (uint64_t)((double)prob[e] * 4294967296.0);
}

__global__ __launch_bounds__(256) void k_lt_start_small(const uint32_t *in_row,
                                                        const uint32_t *in2out, const float *prob,
                                                        uint32_t n, uint64_t *start,
                                                        uint32_t *chunks)
{
    for (uint32_t v = blockIdx.x * 256 + threadIdx.x; v < n; v += gridDim.x * 256) {
        const uint32_t a = in_row[v], b = in_row[v + 1];
        chunks[v] = b - a > LT_SMALL ? (b - a + LT_SMALL - 1) / LT_SMALL : 0u;
        if (b - a > LT_SMALL) continue;
        for (uint32_t j = a; j < b; j++) {
            const uint32_t id = in2out[j];
            uint64_t acc = 0;
            for (uint32_t i = a; i < b; i++) {
                const uint32_t o = in2out[i];
                if (o < id) acc += lt_len(prob, o);
            }
            start[j] = acc;
        }
    }
}

// chunk tasks of the large rows: task t belongs to the row v with
// pre[v] <= t < pre[v+1] (pre: exclusive prefix of the chunk counts, pre[n] = total)
__global__ __launch_bounds__(LT_SMALL) void k_lt_start_large(const uint32_t *in_row,
                                                             const uint32_t *in2out,
                                                             const float *prob, uint32_t n,
                                                             const uint32_t *pre, uint64_t *start)
{
    __shared__ uint32_t s_id[LT_SMALL];
    __shared__ uint64_t s_len[LT_SMALL];
    const uint32_t T = pre[n];
    for (uint32_t t = blockIdx.x; t < T; t += gridDim.x) {
        uint32_t lo = 0, hi = n;   // largest v with pre[v] <= t
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (pre[mid] <= t) lo = mid; else hi = mid;
        }
        const uint32_t v = lo, a = in_row[v], b = in_row[v + 1];
        const uint32_t j = a + (t - pre[v]) * LT_SMALL + threadIdx.x;
        const uint32_t id = j < b ? in2out[j] : 0xFFFFFFFFu;
        uint64_t acc = 0;
        for (uint32_t c = a; c < b; c += LT_SMALL) {
            const uint32_t i = c + threadIdx.x;
            s_id[threadIdx.x] = i < b ? in2out[i] : 0xFFFFFFFFu;
            s_len[threadIdx.x] = i < b ? lt_len(prob, in2out[i]) : 0ull;
            __syncthreads();
            const uint32_t lim = min(LT_SMALL, b - c);
            for (uint32_t q = 0; q < lim; q++)
                if (s_id[q] < id) acc += s_len[q];
            __syncthreads();
        }
        if (j < b) start[j] = acc;
    }
}

// one wavefront per (node, word): lane r draws snapshot 64w + r, then every
// in-arc of the node gets the snapshots whose draw falls in its interval;
// word-major masks for both directions are written directly
__global__ __launch_bounds__(256) void k_lt_masks(const uint32_t *in_row, const uint32_t *in2out,
                                                  const float *prob, const uint64_t *start,
                                                  uint32_t n, uint64_t m, uint32_t R, uint64_t seed,
                                                  uint64_t *mask_out, uint64_t *mask_in)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t waves = (uint64_t)gridDim.x * 4;
    const uint32_t W = (R + 63) / 64;
    for (uint64_t p = blockIdx.x * 4ull + (threadIdx.x >> 6); p < (uint64_t)W * n; p += waves) {
        const uint32_t w = (uint32_t)(p / n), v = (uint32_t)(p - (uint64_t)w * n);
        const uint32_t a = in_row[v], b = in_row[v + 1];
        if (a == b) continue;   // uniform over the wavefront
        const uint32_t r = w * 64 + lane;
        uint64_t d = ~0ull;   // beyond every interval (an interval may pass 2^32)
        if (r < R) {
            const uint64_t key = sm64_finalise(seed + ((uint64_t)v + 1ull) * IM_GOLDEN);
            d = sm64_finalise(key + ((uint64_t)r + 1ull) * IM_GOLDEN) >> 32;
        }
        for (uint32_t base = a; base < b; base += 64) {
            const uint32_t j = base + lane;
            uint64_t lo = 0, len = 0;
            uint32_t e = 0;
            if (j < b) {
                e = in2out[j];
                lo = start[j];
                len = lt_len(prob, e);
            }
            uint64_t bits = 0;
            for (int q = 0; q < 64; q++) {
                const uint64_t dq = __shfl(d, q, 64);
                bits |= (uint64_t)(dq >= lo && dq - lo < len) << q;
            }
            bits &= im_valid_bits(R, w);
            if (j < b) {
                mask_in[(uint64_t)w * m + j] = bits;
                mask_out[(uint64_t)w * m + e] = bits;
            }
        }
    }
}

// A2: masks for both directions
static void build_masks(const im_graph *g, uint32_t R, uint64_t seed, im_workspace *ws,
                        uint64_t *mask_out, bool reverse, hipStream_t s)
{
    uint32_t W = (R + 63) / 64;
    uint64_t m = g->m;
    if (m == 0) return;
    if (ws->live_edge == 1) {
        // linear threshold (the reverse CSR is built): interval starts, then masks
        PhaseTimer pt(ws, IM_PH_MASK_GEN, s);
        const uint32_t n = g->n;
        k_lt_start_small<<<grid_for(n, 256), 256, 0, s>>>(ws->in_row, ws->in2out, g->prob, n,
                                                          ws->lt_start, ws->cnt);
        exclusive_scan(ws->cnt, ws->lt_task, (uint64_t)n + 1, ws->scan_sums, s);
        k_lt_start_large<<<2048, LT_SMALL, 0, s>>>(ws->in_row, ws->in2out, g->prob, n,
                                                   ws->lt_task, ws->lt_start);
        k_lt_masks<<<grid_for((uint64_t)n * W, 4, 16384), 256, 0, s>>>(
            ws->in_row, ws->in2out, g->prob, ws->lt_start, n, m, R, seed, mask_out, ws->mask_in);
        return;
    }
    dim3 grid((unsigned)((m + 255) / 256), W);
    {
        PhaseTimer pt(ws, IM_PH_MASK_GEN, s);
        k_mask_gen<<<grid, 256, 0, s>>>(g->prob, m, R, seed, mask_out, ws->batch, 0u,
                                        ws->pair_coins ? ws->pair : nullptr);
    }
    if (reverse) {
        PhaseTimer pt(ws, IM_PH_MASK_GATHER, s);
        k_mask_gather<<<grid, 256, 0, s>>>(ws->in2out, m, mask_out, ws->mask_in);
    }
}

// A2b: hub lists for one direction (after that direction's masks exist)
static void build_hubs(int d, const uint32_t *row, const uint32_t *col, const uint64_t *mask,
                       uint32_t n, uint64_t m, uint32_t W, im_workspace *ws, hipStream_t s)
{
    if (n == 0) return;
    fill<uint32_t>(ws->hnum + d, 1, 0u, s);
    fill<unsigned long long>(ws->halloc + d, 1, 0ull, s);
    k_hub_mark<<<grid_for(n, 256, 4096), 256, 0, s>>>(row, n, ws->hub_deg, ws->hslot[d],
                                                       ws->hlist[d], ws->hnum + d);
    if (m == 0 || ws->hub_deg == 0) return;
    const unsigned maxh = (unsigned)std::min<uint64_t>(m / ws->hub_deg + 1, ws->cap_hub);
    dim3 grid(std::min(maxh, 1024u), W);
    k_hub_count<<<grid, HB_NT, 0, s>>>(row, mask, m, W, ws->hlist[d], ws->hnum + d, ws->hslot[d],
                                       ws->hcnt[d], ws->hbase[d], ws->halloc + d, ws->cap_hadj);
    k_hub_fill<<<grid, HB_NT, 0, s>>>(row, col, mask, m, W, ws->hlist[d], ws->hnum + d,
                                      ws->hslot[d], ws->hcnt[d], ws->hbase[d], ws->hoff[d],
                                      ws->hadj[d]);
}

// A2c: per-snapshot live lists of the non-hub nodes for one direction
static void build_sparse(int d, const uint32_t *row, const uint32_t *col, const uint64_t *mask,
                         uint32_t n, uint64_t m, uint32_t W, im_workspace *ws, hipStream_t s)
{
    if (!ws->sparse || n == 0) return;
    fill<unsigned long long>(ws->sp_alloc + d, 1, 0ull, s);
    const uint64_t P = (uint64_t)W * n;
    const unsigned grid = (unsigned)std::min<uint64_t>((P + 255) / 256, 8192);
    k_sparse_build<<<grid, 256, 0, s>>>(row, col, mask, m, n, W, ws->hub_deg, ws->sp_base[d],
                                        ws->sp_cum[d], ws->sp_adj[d], ws->sp_alloc + d, ws->sp_cap);
}

static SparseLists sparse_lists(im_workspace *ws, int d)
{
    SparseLists l = {nullptr, nullptr, nullptr};
    if (ws->sparse) {
        l.base = ws->sp_base[d];
        l.cum = ws->sp_cum[d];
        l.adj = ws->sp_adj[d];
    }
    return l;
}

static HubLists hub_lists(im_workspace *ws, int d)
{
    HubLists h;
    h.slot = ws->hslot[d];
    h.off = ws->hoff[d];
    h.adj = ws->hadj[d];
    h.min_deg = ws->hub_deg ? ws->hub_deg : 0xFFFFFFFFu;   // the marking rule of k_hub_mark
    return h;
}

static BfsArgs bfs_args(im_workspace *ws, const uint32_t *row, const uint32_t *col,
                        const uint64_t *mask, uint64_t m, uint32_t n, uint32_t R, uint32_t W)
{
    BfsArgs a;
    memset(&a, 0, sizeof(a));
    a.row = row; a.col = col; a.mask = mask; a.m = m; a.n = n; a.R = R; a.W = W;
    a.bsplit = 1;
    a.node_inst = ws->batch.node_inst; a.inst_R = ws->batch.R; a.inst_off = ws->batch.node_off;
    a.slot_n = ws->slots_n;
    a.gain = ws->gain;
    a.b_reach = ws->b_reach;
    a.b_qa = ws->b_qa; a.b_qb = ws->b_qb; a.b_vis = ws->b_vis;
    a.stats = ws->stats;
    return a;
}

// resident blocks per CU of a kernel (at least 1)
template <typename K>
static unsigned per_cu(K kernel, int nt)
{
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kernel, nt, 0) != hipSuccess || b < 1) b = 1;
    return (unsigned)b;
}

// Run every task of `a` through the three engine tiers. ctr: this phase's
// zeroed counters. ph0: phase-timer id of tier 0 (ph0+1, ph0+2: tiers 1, 2).
template <int MODE, bool PRUNE>
static void run_tiers(BfsArgs a, im_workspace *ws, uint32_t *ctr, int ph0, hipStream_t s)
{
    a.in_q = nullptr; a.in_n = nullptr;
    a.out_q = ws->ovf_q; a.out_n = ctr + 1; a.grab = ctr + 0; a.tier = 0;
    // reverse tasks may start on tier 1, which then takes every task id
    const bool skip0 = MODE == MODE_DEC && ws->rev_first == 1;
    if (!skip0) {
        PhaseTimer pt(ws, ph0, s);
        auto k0 = k_lds_bfs<MODE, 64, T0_T, T0_CS, T0_LIM, T0_DMAX, T0_U, PRUNE>;
        static const unsigned g0 = per_cu(k0, 64);
        k0<<<(unsigned)ws->num_cu * g0, 64, 0, s>>>(a);
        a.in_q = ws->ovf_q; a.in_n = ctr + 1;
    }
    a.out_q = ws->ovf_q2; a.out_n = ctr + 3; a.grab = ctr + 2; a.tier = 1;
    {
        PhaseTimer pt(ws, ph0 + 1, s);
        switch (ws->tier1_shape) {
        case 1: {
            auto k1 = k_lds_bfs<MODE, T1_NT, 2, 512, 384, 0xFFFFFFFFu, T1_U, PRUNE>;
            static const unsigned g1 = per_cu(k1, T1_NT);
            k1<<<(unsigned)ws->num_cu * g1, T1_NT, 0, s>>>(a);
            break;
        }
        case 2: {
            auto k1 = k_lds_bfs<MODE, T1_NT, 1, 1024, 768, 0xFFFFFFFFu, T1_U, PRUNE>;
            static const unsigned g1 = per_cu(k1, T1_NT);
            k1<<<(unsigned)ws->num_cu * g1, T1_NT, 0, s>>>(a);
            break;
        }
        default: {
            auto k1 = k_lds_bfs<MODE, T1_NT, T1_T, T1_CS, T1_LIM, 0xFFFFFFFFu, T1_U, PRUNE>;
            static const unsigned g1 = per_cu(k1, T1_NT);
            k1<<<(unsigned)ws->num_cu * g1, T1_NT, 0, s>>>(a);
        }
        }
    }
    a.in_q = ws->ovf_q2; a.in_n = ctr + 3;
    a.out_q = nullptr; a.out_n = nullptr; a.grab = ctr + 4; a.tier = 2;
    if (MODE == MODE_DEC) a.bsplit = ws->rev_split;
    {
        PhaseTimer pt(ws, ph0 + 2, s);
        if (ws->tier2_lanes == (uint32_t)T2W_NT)
            k_block_bfs<MODE, T2W_NT, T2_U, PRUNE><<<ws->slots, T2W_NT, 0, s>>>(a);
        else if (ws->tier2_lanes == (uint32_t)T2S_NT)
            k_block_bfs<MODE, T2S_NT, T2_U, PRUNE><<<ws->slots, T2S_NT, 0, s>>>(a);
        else
            k_block_bfs<MODE, T2_NT, T2_U, PRUNE><<<ws->slots, T2_NT, 0, s>>>(a);
    }
}

// Every task of `a` on the last tier alone, one workgroup per task: for
// tasks known to be large (the lazy path's candidates are the nodes with the
// largest bounds), which the smaller tiers would only hand on.
// KEEP: one task per slot (ntasks <= slots), the fixpoints stay in the slots.
template <int MODE, bool PRUNE, bool KEEP = false>
static void run_last_tier(BfsArgs a, im_workspace *ws, uint32_t *ctr, int ph, hipStream_t s)
{
    a.in_q = nullptr; a.in_n = nullptr;
    a.out_q = nullptr; a.out_n = nullptr; a.grab = ctr + 4; a.tier = 2;
    if (KEEP) { a.kept_nvis = ws->c_kept; a.kept_src = ws->c_kept + ws->cap_kept; }
    PhaseTimer pt(ws, ph, s);
    const unsigned grid = std::max<unsigned>(1u, std::min<unsigned>(ws->slots, a.ntasks));
    if (ws->tier2_lanes == (uint32_t)T2W_NT)
        k_block_bfs<MODE, T2W_NT, T2_U, PRUNE, KEEP><<<grid, T2W_NT, 0, s>>>(a);
    else if (ws->tier2_lanes == (uint32_t)T2S_NT)
        k_block_bfs<MODE, T2S_NT, T2_U, PRUNE, KEEP><<<grid, T2S_NT, 0, s>>>(a);
    else
        k_block_bfs<MODE, T2_NT, T2_U, PRUNE, KEEP><<<grid, T2_NT, 0, s>>>(a);
}

// A3: initial gains (gain must be zero on entry)
static void initial_gains(const im_graph *g, uint32_t R, im_workspace *ws, uint32_t *ctr,
                          hipStream_t s)
{
    uint32_t n = g->n, W = (R + 63) / 64;
    if (n == 0) return;
    BfsArgs a = bfs_args(ws, ws->row32, g->col, ws->mask_out, g->m, n, R, W);
    a.ntasks = n * W;
    a.hub = hub_lists(ws, 0);
    a.sp = sparse_lists(ws, 0);
    a.pass = PASS_INIT;
    a.st_trav = ST_TRAV_INIT;
    run_tiers<MODE_COUNT, false>(a, ws, ctr, IM_PH_INIT_T0, s);
}

// ---------------------------------------------------------------------------
// A6, the affected-set recompute: the other way to bring the gains up to date
// after a round (identical integers; the autotuner picks the rounds). The
// nodes whose gain changes are exactly those that reach a newly covered node
// in its snapshot (their reach sets lose it): one union search per word over
// the reverse arcs from every newly covered node, carrying its newly covered
// bits, finds them. Each such node's gain is then recomputed from scratch,
// sum over r of |R_r(u) \ covered_r|, by the count engine pruned at covered
// (covered already holds this round's newly covered bits). For a node that
// reaches none, nothing changed.
// ---------------------------------------------------------------------------
constexpr int AFF_NT = 1024;

struct AffArgs {
    const unsigned long long *key;   // the round's key
    uint64_t aff_gain;               // rounds whose gain is below this use the recompute
    const uint32_t *row, *col;       // reverse CSR
    const uint64_t *mask;            // reverse masks [W][m]
    uint64_t m;
    HubLists hub;
    SparseLists sp;
    uint32_t n, W;
    const uint32_t *tnodes, *tcounts;
    const uint64_t *newly;
    uint64_t *reach, *pend;          // [W][n], zero at rest
    uint32_t *qa, *qb, *vis;         // [W][n]
    uint32_t *mark, *list, *cnt;     // affected nodes: mark [n] (zero at rest), list, count
    uint32_t *gain;
};

// one workgroup per word
__global__ __launch_bounds__(AFF_NT) void k_aff_search(AffArgs a)
{
    __shared__ BlockLds<AFF_NT> L;
    const unsigned long long key = *a.key;
    if (key == 0 || (key >> 32) >= a.aff_gain) return;   // a dynamic-update round
    const uint32_t w = blockIdx.x, tid = threadIdx.x;
    const uint64_t off = (uint64_t)w * a.n;
    uint64_t *reach = a.reach + off, *pend = a.pend + off;
    uint32_t *qa = a.qa + off, *qb = a.qb + off, *vis = a.vis + off;
    if (tid == 0) { L.nf = 0; L.nn = 0; L.nvis = 0; L.H.n = 0; L.levels = 0; L.entries = 0; }
    __syncthreads();
    const uint32_t c = a.tcounts[w];
    for (uint32_t i = tid; i < c; i += AFF_NT) {
        const uint32_t x = a.tnodes[off + i];
        global_relax<1>(reach, pend, 0u, vis, qa, &L.nvis, &L.nf, x, a.newly[off + x]);
    }
    __syncthreads();
    uint64_t arcs = 0;
    block_bfs_run<AFF_NT, 8, false, true, 1>(L, 0u, 0ull, a.row, a.col, a.mask + (uint64_t)w * a.m,
                                             a.hub, a.sp, a.n, a.W, w, nullptr, reach, pend, 0u, qa,
                                             qb, vis, arcs, true);
    const uint32_t nv = L.nvis;
    for (uint32_t b0 = 0; b0 < nv; b0 += AFF_NT) {   // whole wavefronts per step
        const uint32_t i = b0 + tid;
        uint32_t x = 0;
        bool first = false;
        if (i < nv) {
            x = vis[i];
            reach[x] = 0;   // pend is zero at the fixpoint
            first = atomicExch(&a.mark[x], 1u) == 0u;
        }
        const uint32_t p = wave_append(first, a.cnt);
        if (first) {
            a.list[p] = x;
            a.gain[x] = 0;   // recomputed from scratch below
        }
    }
}

__global__ void k_aff_clear(uint32_t *mark, const uint32_t *list, const uint32_t *cnt)
{
    const uint32_t c = *cnt;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < c; i += gridDim.x * blockDim.x)
        mark[list[i]] = 0;
}

static void affected_update(const im_graph *g, uint32_t R, uint32_t t, im_workspace *ws,
                            hipStream_t s)
{
    const uint32_t n = g->n, W = (R + 63) / 64;
    {
        AffArgs f;
        f.key = ws->keys + t; f.aff_gain = ws->aff_gain;
        f.row = ws->in_row; f.col = ws->in_col; f.mask = ws->mask_in; f.m = g->m;
        f.hub = hub_lists(ws, 1); f.sp = sparse_lists(ws, 1);
        f.n = n; f.W = W;
        f.tnodes = ws->tnodes; f.tcounts = ws->tcounts; f.newly = ws->newly;
        f.reach = ws->a_reach; f.pend = ws->a_pend;
        f.qa = ws->a_qa; f.qb = ws->a_qb; f.vis = ws->a_vis;
        f.mark = ws->a_mark; f.list = ws->a_list; f.cnt = ws->a_cnt; f.gain = ws->gain;
        PhaseTimer pt(ws, IM_PH_AFFECTED, s);
        k_aff_search<<<W, AFF_NT, 0, s>>>(f);
    }
    BfsArgs a = bfs_args(ws, ws->row32, g->col, ws->mask_out, g->m, n, R, W);
    a.cand = ws->a_list;
    a.ncand_dev = ws->a_cnt;
    a.ntasks = 0;
    a.gain = ws->gain;
    a.prune = ws->covered;
    a.hub = hub_lists(ws, 0);
    a.sp = sparse_lists(ws, 0);
    a.pass = PASS_EVAL;
    a.st_trav = ST_TRAV_EVAL;
    run_tiers<MODE_COUNT, true>(a, ws, ws->a_ctrs + (uint64_t)t * PH_CTRS, IM_PH_EVAL_T0, s);
    {
        PhaseTimer pt(ws, IM_PH_AFFECTED, s);
        k_aff_clear<<<grid_for(n, 256, 1024), 256, 0, s>>>(ws->a_mark, ws->a_list, ws->a_cnt);
        fill<uint32_t>(ws->a_cnt, 1, 0u, s);
    }
}

// The forward search of one round. A single graph's round runs in
// k_forward_block (one workgroup per word) when its seed's gain is below
// coop_gain, else in the cooperative kernel. A cooperative launch can be
// refused while another process on the device holds the hardware's global
// barrier resource; a single graph's round then runs in k_forward_block
// after all (block_floor keeps the first launch's rounds from running twice).
// Batches have no such fallback. During stream capture a refusal is an error:
// the capture would not survive it.
static int launch_forward(FwdArgs f, im_workspace *ws, bool single, hipStream_t s)
{
    f.block_floor = 0;
    // (with a zero threshold every round is cooperative: the one-workgroup
    // kernel would return at once)
    if (single && f.coop_gain > 0) k_forward_block<<<f.W, FWB_NT, 0, s>>>(f);
    // (a gain is a 32-bit count: above that every round is a small one)
    if (single && f.coop_gain > 0xFFFFFFFFull) return IM_OK;
    void *args[] = {&f};
    const unsigned fg = std::min<unsigned>(ws->fwd_grid, ws->fwd_per_word * f.W);
    const hipError_t e = hipLaunchCooperativeKernel((const void *)k_forward_coop, dim3(fg),
                                                    dim3(FWD_NT), args, 0, s);
    if (e == hipSuccess) return IM_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (!single || hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
        return im_fail(IM_EHIP, "cooperative launch of k_forward_coop: %s%s", hipGetErrorString(e),
                       single ? " (during stream capture)"
                              : " (batched selection needs cooperative launches)");
    (void)hipGetLastError();
    f.block_floor = f.coop_gain;
    f.coop_gain = ~0ull;
    k_forward_block<<<f.W, FWB_NT, 0, s>>>(f);
    return IM_OK;
}

// A4-A6: one greedy round
static int greedy_round(const im_graph *g, uint32_t R, uint32_t t, uint32_t *seeds_out,
                        uint64_t *gains_out, im_workspace *ws, uint32_t *ctr, hipStream_t s)
{
    uint32_t n = g->n, W = (R + 63) / 64;
    {
        PhaseTimer pt(ws, IM_PH_ARGMAX, s);
        // a single graph: few workgroups, so that few atomics meet on the key
        k_argmax<<<grid_for(n, 256, ws->batch.count == 1 ? 256 : 2048), 256, 0, s>>>(ws->gain, ws->sel, n,
                                                         ws->keys + (uint64_t)t * ws->batch.count,
                                                         ws->batch, t, ws->pk, (uint32_t)PK_ZERO);
    }

    FwdArgs f;
    f.skip = nullptr;
    f.row = ws->row32; f.col = g->col; f.mask = ws->mask_out; f.m = g->m;
    f.hub = hub_lists(ws, 0);
    f.sp = sparse_lists(ws, 0);
    f.n = n; f.R = R; f.W = W;
    f.covered = ws->covered; f.newly = ws->newly; f.pend = ws->fpend;
    f.fq0 = ws->fqa; f.fq1 = ws->fqb; f.cnt = ws->fctr + (uint64_t)t * FWD_CTRS;
    f.bq0 = ws->bqa; f.bq1 = ws->bqb; f.coop_gain = ws->coop_gain; f.vis = ws->fvis;
    f.tnodes = ws->tnodes; f.tcounts = ws->tcounts;
    uint32_t *bcnt = ws->pk, *bcur = ws->pk + 64 * 64, *gcnt = ws->pk + 2 * 64 * 64,
             *mcnt = gcnt + 64;
    f.bcnt = bcnt; f.mcnt = mcnt; f.mlist = ws->mlist;
    f.key = ws->keys + (uint64_t)t * ws->batch.count; f.t = t; f.b = ws->batch;
    f.seeds_out = seeds_out; f.gains_out = gains_out; f.sel = ws->sel;
    f.stats = ws->stats;
    {
        PhaseTimer pt(ws, IM_PH_FORWARD, s);
        const int rc = launch_forward(f, ws, ws->batch.count == 1, s);
        if (rc) return rc;
    }

    {
        // the forward search counted the single-bit sources per bit and
        // listed the others
        PhaseTimer pt(ws, IM_PH_PACK, s);
        dim3 pg(grid_for(n, PK_NT, 64), W);
        const uint64_t aff = ws->batch.count == 1 ? ws->aff_gain : 0ull;
        k_pack_fill<<<pg, PK_NT, 0, s>>>(ws->tnodes, ws->tcounts, ws->newly, n, bcnt, ws->boff,
                                         gcnt, bcur, ws->plist, mcnt, ws->keys + (uint64_t)t * ws->batch.count,
                                         aff);
    }
    BfsArgs a = bfs_args(ws, ws->in_row, ws->in_col, ws->mask_in, g->m, n, R, W);
    a.gcnt = gcnt; a.mcnt = mcnt; a.bcnt = bcnt; a.boff = ws->boff;
    a.plist = ws->plist; a.mlist = ws->mlist; a.tbits = ws->newly;
    a.hub = hub_lists(ws, 1);
    a.sp = sparse_lists(ws, 1);
    a.pass = PASS_REV;
    a.st_trav = ST_TRAV_REV;
    run_tiers<MODE_DEC, false>(a, ws, ctr, IM_PH_REV_T0, s);
    if (ws->batch.count == 1 && ws->aff_gain) affected_update(g, R, t, ws, s);
    {
        PhaseTimer pt(ws, IM_PH_CLEAR, s);
        k_clear_newly<<<grid_for(n, 256, 1024), 256, 0, s>>>(ws->newly, ws->tnodes, ws->tcounts, n, W);
    }
    return IM_OK;
}

// workspace growth and input validation (synchronous)
static int check_and_reserve(const im_graph *g, uint32_t R, uint32_t k, im_workspace *ws,
                             hipStream_t s)
{
    int rc;
    if ((rc = ws_reserve(ws, g->n, g->m, (R + 63) / 64, k, g->n))) return rc;
    if (ws->aff_gain && ws->batch.count == 1) {
        const uint64_t nW = (uint64_t)g->n * ((R + 63) / 64);
        if (nW > ws->cap_aff_nW || !ws->a_reach) {
            if ((rc = dalloc(&ws->a_reach, nW)) || (rc = dalloc(&ws->a_pend, nW)) ||
                (rc = dalloc(&ws->a_qa, nW)) || (rc = dalloc(&ws->a_qb, nW)) ||
                (rc = dalloc(&ws->a_vis, nW)))
                return rc;
            if ((rc = ws_memset(ws->a_reach, nW * sizeof(uint64_t))) ||
                (rc = ws_memset(ws->a_pend, nW * sizeof(uint64_t))))
                return rc;
            ws->cap_aff_nW = nW;
        }
        if (g->n > ws->cap_aff_n || !ws->a_mark) {
            if ((rc = dalloc(&ws->a_mark, g->n)) || (rc = dalloc(&ws->a_list, g->n)) ||
                (rc = dalloc(&ws->a_cnt, 1)))
                return rc;
            if ((rc = ws_memset(ws->a_mark, (uint64_t)g->n * sizeof(uint32_t))) ||
                (rc = ws_memset(ws->a_cnt, sizeof(uint32_t))))
                return rc;
            ws->cap_aff_n = g->n;
        }
        if (k + 1 > ws->cap_aff_k || !ws->a_ctrs) {
            if ((rc = dalloc(&ws->a_ctrs, (uint64_t)(k + 1) * PH_CTRS))) return rc;
            ws->cap_aff_k = k + 1;
        }
    }
    if ((rc = validate(g, ws, s, ws->row32))) return rc;
    if (ws->live_edge == 1) {
        if (ws->batch.count > 1) return im_fail(IM_EINVAL, "linear-threshold snapshots apply to single graphs only");
        if (ws->pair_coins) return im_fail(IM_EINVAL, "pair coins and linear-threshold snapshots exclude each other");
        if (g->m > ws->cap_lt_m || !ws->lt_start) {
            if ((rc = dalloc(&ws->lt_start, g->m))) return rc;
            ws->cap_lt_m = g->m;
        }
        if (g->n + 1 > ws->cap_lt_n || !ws->lt_task) {
            if ((rc = dalloc(&ws->lt_task, (uint64_t)g->n + 1))) return rc;
            ws->cap_lt_n = g->n + 1;
        }
    }
    if (ws->pair_coins) {
        // the pair of every arc (host-synchronous; before any capture)
        if (ws->batch.count > 1) return im_fail(IM_EINVAL, "pair coins apply to single graphs only");
        if (g->m > ws->cap_pair || !ws->pair) {
            if ((rc = dalloc(&ws->pair, g->m))) return rc;
            ws->cap_pair = g->m;
        }
        if ((rc = und_pair_ids(g, ws->row32, ws->pair, ws, s))) return rc;
    }
    return IM_OK;
}

// What a path reads of the reverse direction: the dynamic update's reverse
// searches need all of it (reverse CSR, reverse-order masks, reverse hub and
// sparse lists); the lazy path and the initial counts alone need none of it,
// or only the in-degrees (the learned policy's node features). Linear
// threshold snapshots are drawn per in-row and always build the reverse CSR.
enum { PREP_FORWARD = 0, PREP_INDEG = 1, PREP_REVERSE = 2 };

// everything after validation up to (and including) the initial gains:
// kernel launches only (no host synchronisation, no memset), so that the
// sequence can be captured into a graph
static int enqueue_prepare(const im_graph *g, uint32_t R, uint64_t seed, uint32_t k,
                           im_workspace *ws, hipStream_t s, int need = PREP_REVERSE)
{
    uint32_t n = g->n, W = (R + 63) / 64;
    fill<unsigned long long>(ws->stats, (uint64_t)ST_COUNT * ST_STRIPES, 0ull, s);
    fill<uint32_t>(ws->ctrs, (uint64_t)(k + 1) * PH_CTRS, 0u, s);
    fill<unsigned long long>(ws->keys, (uint64_t)(k + 1) * ws->batch.count, 0ull, s);
    fill<uint32_t>(ws->fctr, (uint64_t)(k ? k : 1) * FWD_CTRS, 0u, s);
    if (ws->aff_gain && ws->batch.count == 1) fill<uint32_t>(ws->a_ctrs, (uint64_t)(k + 1) * PH_CTRS, 0u, s);
    fill<uint32_t>(ws->gain, n, 0u, s);
    fill<uint8_t>(ws->sel, n, (uint8_t)0, s);
    fill<uint64_t>(ws->covered, (uint64_t)n * W, 0ull, s);
    const bool rev = need == PREP_REVERSE || ws->live_edge == 1;
    if (rev || need == PREP_INDEG) build_reverse(g, ws, s, !rev);
    build_masks(g, R, seed, ws, ws->mask_out, rev, s);
    {
        PhaseTimer pt(ws, IM_PH_HUBS, s);
        build_hubs(0, ws->row32, g->col, ws->mask_out, n, g->m, W, ws, s);
        build_sparse(0, ws->row32, g->col, ws->mask_out, n, g->m, W, ws, s);
        if (rev) {
            build_hubs(1, ws->in_row, ws->in_col, ws->mask_in, n, g->m, W, ws, s);
            build_sparse(1, ws->in_row, ws->in_col, ws->mask_in, n, g->m, W, ws, s);
        }
    }
    initial_gains(g, R, ws, ws->ctrs, s);
    HIPCHK(hipGetLastError());
    ws->last_stream = s;
    return IM_OK;
}

static int prepare(const im_graph *g, uint32_t R, uint64_t seed, uint32_t k, im_workspace *ws,
                   hipStream_t s, int need = PREP_REVERSE)
{
    int rc;
    if ((rc = check_and_reserve(g, R, k, ws, s))) return rc;
    return enqueue_prepare(g, R, seed, k, ws, s, need);
}

// the k greedy rounds (kernel launches only)
static int enqueue_rounds(const im_graph *g, uint32_t R, uint32_t k, uint32_t *seeds_out,
                          uint64_t *gains_out, uint32_t *trace_out, im_workspace *ws, hipStream_t s)
{
    int rc;
    const uint32_t n = g->n;
    for (uint32_t t = 0; t < k; t++) {
        if (trace_out)
            k_copy_u32<<<grid_for(n, 256), 256, 0, s>>>(ws->gain, trace_out + (uint64_t)t * n, n);
        if ((rc = greedy_round(g, R, t, seeds_out, gains_out, ws,
                               ws->ctrs + (uint64_t)(t + 1) * PH_CTRS, s)))
            return rc;
    }
    if (trace_out && n)
        k_copy_u32<<<grid_for(n, 256), 256, 0, s>>>(ws->gain, trace_out + (uint64_t)k * n, n);
    HIPCHK(hipGetLastError());
    return IM_OK;
}

// ---------------------------------------------------------------------------
// A9: lazy evaluation (the StaticGreedyCELF variant of Sec. 5) with an
// optional learned candidate order
// ---------------------------------------------------------------------------
// Every unselected node u keeps a bound b_u: its exact gain when it was last
// evaluated (at first its initial count). Gains only shrink as seeds are
// added (the spread is submodular, Sec. 3.2), so b_u bounds u's current gain.
// A round evaluates candidates exactly, a batch at a time, with the covered
// snapshots pruned (the count engine with prune = covered), until the best
// exact key (gain, lowest id) of the round beats the bound key of every
// unselected node not evaluated in the round. That best is the argmax of
// the exact gains, so the seed and its gain equal the dynamic update's.
//
// Candidate order: bound order (plain), or the network's score among the
// nodes whose bound can still win (learned). An order is kept as the node
// list sorted by the keys the nodes had at the last rebuild (ordB, ordS);
// nodes evaluated since ("moved") sit in a short list E, which every pick
// filters, sorts in LDS and merges with a walk down the sorted list.
constexpr int CP_NT = 1024;
constexpr uint32_t CELF_BMAX = 1024;   // largest batch
constexpr uint32_t CELF_CAPE = 2048;   // moved nodes held before the orders are rebuilt
constexpr uint32_t CELF_CAPW = 2048;   // can-win nodes gathered for a learned pick
constexpr int SORT_TILE = 4096;        // keys sorted per workgroup in LDS
// control words: candidate count, |E|, walk heads of ordB / ordS, then the
// evaluation's tier counters
enum { CC_NCAND = 0, CC_NE = 1, CC_HEADB = 2, CC_HEADS = 3, CC_KEPT = 4, CC_EVCTR = 8,
       CC_COUNT = 8 + PH_CTRS };

__device__ __forceinline__ unsigned long long node_key(uint32_t primary, uint32_t u)
{
    return ((unsigned long long)primary << 32) | (0xFFFFFFFFu - u);
}

__device__ __forceinline__ uint32_t key_node(unsigned long long key)
{
    return 0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull);
}

// order-preserving map of a float score to uint32
__device__ __forceinline__ uint32_t score_bits(float f)
{
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// static inputs of the network (see im_mlp.h), from the out-CSR and the
// reverse CSR's row offsets; one wavefront per node, so that a hub's arcs
// are summed by 64 lanes (fixed lane order: deterministic)
// Nodes of out-degree <= FEAT_SMALL: one thread each, arcs summed in arc order.
constexpr uint32_t FEAT_SMALL = 64;

__device__ __forceinline__ void feat_store(float *feat, uint32_t u, uint32_t indeg, uint32_t deg,
                                           float ps, uint64_t two)
{
    float *f = feat + (uint64_t)u * 4;   // caller memory: 4-byte alignment only
    f[0] = log1pf((float)indeg);
    f[1] = log1pf((float)deg);
    f[2] = log1pf(ps);
    f[3] = log1pf((float)two);
}

__global__ __launch_bounds__(256) void k_features_small(const uint32_t *row, const uint32_t *col,
                                                        const float *prob, const uint32_t *in_row,
                                                        uint32_t n, float *feat)
{
    for (uint32_t u = blockIdx.x * 256u + threadIdx.x; u < n; u += gridDim.x * 256u) {
        const uint32_t rs = row[u], re = row[u + 1];
        if (re - rs > FEAT_SMALL) continue;
        float ps = 0.0f;
        uint64_t two = 0;
#pragma unroll 4
        for (uint32_t e = rs; e < re; e++) {
            ps += prob[e];
            const uint32_t v = col[e];
            two += row[v + 1] - row[v];
        }
        feat_store(feat, u, in_row[u + 1] - in_row[u], re - rs, ps, two);
    }
}

// the other nodes: one 1024-lane workgroup each, so that a hub with 10^5
// arcs is not one wavefront's serial walk; the workgroup scans 1024 nodes'
// degrees in one load and takes their large ones in turn (each node's sums
// in a fixed thread and reduction order: deterministic)
constexpr int FEAT_NT = 1024;

__global__ __launch_bounds__(FEAT_NT) void k_features(const uint32_t *row, const uint32_t *col,
                                                      const float *prob, const uint32_t *in_row,
                                                      uint32_t n, float *feat)
{
    __shared__ uint32_t big[FEAT_NT];
    __shared__ uint32_t nbig;
    __shared__ float fred[FEAT_NT / 64];
    __shared__ unsigned long long ured[FEAT_NT / 64];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (uint32_t b0 = blockIdx.x * FEAT_NT; b0 < n; b0 += gridDim.x * FEAT_NT) {
        if (tid == 0) nbig = 0;
        __syncthreads();
        const uint32_t ul = b0 + tid;
        if (ul < n && row[ul + 1] - row[ul] > FEAT_SMALL) big[atomicAdd(&nbig, 1u)] = ul;
        __syncthreads();
        const uint32_t nb = nbig;
        // (the list order is arbitrary; each node's sums do not depend on it)
        for (uint32_t q = 0; q < nb; q++) {
            const uint32_t u = big[q];
            const uint32_t rs = row[u], re = row[u + 1];
            float ps = 0.0f;
            uint64_t two = 0;
#pragma unroll 4
            for (uint32_t e = rs + tid; e < re; e += FEAT_NT) {
                ps += prob[e];
                const uint32_t v = col[e];
                two += row[v + 1] - row[v];
            }
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) ps += __shfl_xor(ps, d, 64);
            two = wave_sum_u64(two);
            if (lane == 0) { fred[wv] = ps; ured[wv] = two; }
            __syncthreads();
            if (tid == 0) {
                float fs = 0.0f;
                uint64_t us = 0;
                for (int i = 0; i < FEAT_NT / 64; i++) { fs += fred[i]; us += ured[i]; }
                feat_store(feat, u, in_row[u + 1] - in_row[u], re - rs, fs, us);
            }
            __syncthreads();
        }
    }
}

static void launch_features(const uint32_t *row, const uint32_t *col, const float *prob,
                            const uint32_t *in_row, uint32_t n, float *feat, hipStream_t s)
{
    if (n == 0) return;
    k_features_small<<<grid_for(n, 256, 8192), 256, 0, s>>>(row, col, prob, in_row, n, feat);
    k_features<<<grid_for(n, FEAT_NT, 4096), FEAT_NT, 0, s>>>(row, col, prob, in_row, n, feat);
}

// score[u] = network(feat[u], ln(1 + bound[u] / R)) for u in list[0..cnt)
// (list = nullptr: u = 0..cnt-1; cnt_dev != nullptr: count read on the device)
__global__ __launch_bounds__(256) void k_celf_score(const uint16_t *wb, const float *feat,
                                                    const uint32_t *bound, float invR,
                                                    const uint32_t *list, uint32_t cnt,
                                                    const uint32_t *cnt_dev, float *score)
{
    // 16 nodes per wavefront and step on the matrix cores (mlp_tile_mfma)
    MlpFrag f;
    mlp_frag_load(wb, f);
    const uint32_t c = cnt_dev ? *cnt_dev : cnt;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = (blockIdx.x * 256u + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * 256u) >> 6;
    for (uint32_t base = wave * 16u; base < c; base += nwaves * 16u) {
        const uint32_t i = base + (lane & 15u);
        float x[MLP_IN] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        if (i < c) {
            const uint32_t u = list ? list[i] : i;
#pragma unroll
            for (int q = 0; q < 4; q++) x[q] = feat[(uint64_t)u * 4 + q];
            x[4] = log1pf((float)bound[u] * invR);
        }
        float yo[4];
        mlp_tile_mfma(f, x, yo);
        if ((lane & 15u) == 0)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const uint32_t o = base + 4u * (lane >> 4) + (uint32_t)q;
                if (o < c) score[list ? list[o] : o] = yo[q];
            }
    }
}

// sort keys: node_key(primary(u), u) for u < n, 0 for the padding up to len
__global__ void k_order_keys(const uint32_t *bound, const float *score, uint32_t n, uint64_t len,
                             unsigned long long *keys)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < len;
         i += (uint64_t)gridDim.x * blockDim.x) {
        unsigned long long k = 0;
        if (i < n) {
            const uint32_t u = (uint32_t)i;
            k = node_key(score ? score_bits(score[u]) : bound[u], u);
        }
        keys[i] = k;
    }
}

// Bitonic sorting network, descending. Step (kk, j) compares i with i ^ j;
// blocks with (i & kk) == 0 go descending, the others ascending.
__device__ __forceinline__ void bitonic_cx(unsigned long long *a, uint64_t i, uint64_t l,
                                           uint64_t gi, uint64_t kk)
{
    const unsigned long long x = a[i], y = a[l];
    const bool desc = (gi & kk) == 0;
    if (desc ? x < y : x > y) { a[i] = y; a[l] = x; }
}

// all steps with j < SORT_TILE of stages kk in [kk_lo, kk_hi] on one tile
// held in LDS (kk_lo = 2: a full local sort)
__global__ __launch_bounds__(1024) void k_bitonic_tile(unsigned long long *keys, uint64_t kk_lo,
                                                       uint64_t kk_hi)
{
    __shared__ unsigned long long t[SORT_TILE];
    const uint64_t base = (uint64_t)blockIdx.x * SORT_TILE;
    for (int i = threadIdx.x; i < SORT_TILE; i += 1024) t[i] = keys[base + i];
    __syncthreads();
    for (uint64_t kk = kk_lo; kk <= kk_hi; kk <<= 1) {
        for (uint64_t j = std::min<uint64_t>(kk >> 1, SORT_TILE / 2); j >= 1; j >>= 1) {
            for (int p = threadIdx.x; p < SORT_TILE / 2; p += 1024) {
                const uint64_t i = 2 * j * (p / j) + (p % j);
                bitonic_cx(t, i, i + j, base + i, kk);
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < SORT_TILE; i += 1024) keys[base + i] = t[i];
}

__global__ void k_bitonic_step(unsigned long long *keys, uint64_t len, uint64_t kk, uint64_t j)
{
    const uint64_t half = len / 2;
    for (uint64_t p = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; p < half;
         p += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i = 2 * j * (p / j) + (p % j);
        bitonic_cx(keys, i, i + j, i, kk);
    }
}

__global__ void k_order_extract(const unsigned long long *keys, uint32_t n, uint32_t *ord)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        ord[i] = key_node(keys[i]);
}

__global__ void k_celf_reset(uint32_t *ctl)
{
    if (threadIdx.x == 0) { ctl[CC_NE] = 0; ctl[CC_HEADB] = 0; ctl[CC_HEADS] = 0; }
}

struct PickArgs {
    uint32_t n, t, B;
    int learned;               // 0: bound order; 1: score order; 2: predicted-gain batches
    float R;
    const uint32_t *ordB, *ordS;
    const uint32_t *bound;
    const float *score;
    const uint32_t *fresh;
    const uint8_t *sel, *moved;
    const uint32_t *E;
    uint32_t *ctl;
    const unsigned long long *best;
    uint32_t *cand;
    uint32_t *ev;
    unsigned long long *stats;
};

struct PickLds {
    unsigned long long a[CELF_CAPW];                 // walk result, descending
    unsigned long long e[CELF_CAPW + CELF_CAPE];     // moved nodes (and the learned union)
    unsigned long long red[CP_NT / 64];
    uint32_t wsum[CP_NT / 64 + 1];
    uint32_t na, ne, done, full, lead, first;
};

// Walk ord from ctl[head] and collect, in list order, the keys of nodes that
// are neither selected, moved nor evaluated this round and whose key exceeds
// stop, up to cap. Advances ctl[head] past leading entries that can never be
// taken again (selected or moved). Sets L.na; L.full when more may follow.
template <typename KeyOf>
__device__ void pick_walk(const PickArgs &a, const uint32_t *ord, int head, KeyOf key_of,
                          unsigned long long stop, uint32_t cap, PickLds &L)
{
    const int tid = threadIdx.x;
    const uint32_t h0 = a.ctl[head];
    if (tid == 0) { L.na = 0; L.done = 0; L.full = 0; L.lead = 1; }
    __syncthreads();
    for (uint64_t p = h0; p < a.n; p += CP_NT) {
        if (tid == 0) L.first = CP_NT;
        __syncthreads();
        const uint64_t i = p + tid;
        bool take = false, stopped = false;
        unsigned long long key = 0;
        if (i < a.n) {
            const uint32_t u = ord[i];
            const bool gone = a.sel[u] || a.moved[u];
            if (!gone) atomicMin(&L.first, (uint32_t)tid);
            if (!gone && a.fresh[u] != a.t + 1) {
                key = key_of(u);
                take = key > stop;
                stopped = !take;   // keys descend along the list: nothing later passes
            }
        }
        if (__syncthreads_or(stopped) && tid == 0) L.done = 1;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<CP_NT>(take ? 1u : 0u, L.wsum, &tot);
        const uint32_t na = L.na;
        if (take && na + ex < cap) L.a[na + ex] = key;
        __syncthreads();
        if (tid == 0) {
            if (L.lead) {
                if (L.first < CP_NT) { a.ctl[head] = (uint32_t)(p + L.first); L.lead = 0; }
                else a.ctl[head] = (uint32_t)std::min<uint64_t>(p + CP_NT, a.n);
            }
            if (na + tot >= cap) {
                L.full = (na + tot > cap) || (!L.done && p + CP_NT < a.n);
                L.na = cap;
                L.done = 1;
            } else {
                L.na = na + tot;
            }
        }
        __syncthreads();
        if (L.done) break;
    }
    __syncthreads();
}

// sort L.e[0..cnt) descending in LDS (cnt <= CELF_CAPW + CELF_CAPE)
__device__ void lds_sort_desc(unsigned long long *e, uint32_t cnt)
{
    uint32_t len = 1;
    while (len < cnt) len <<= 1;
    for (uint32_t i = cnt + threadIdx.x; i < len; i += CP_NT) e[i] = 0;
    __syncthreads();
    for (uint32_t kk = 2; kk <= len; kk <<= 1)
        for (uint32_t j = kk >> 1; j >= 1; j >>= 1) {
            for (uint32_t p = threadIdx.x; p < len / 2; p += CP_NT) {
                const uint32_t i = 2 * j * (p / j) + (p % j);
                bitonic_cx(e, i, i + j, i, kk);
            }
            __syncthreads();
        }
}

// number of entries of the descending list s[0..cnt) greater than x
__device__ __forceinline__ uint32_t count_greater(const unsigned long long *s, uint32_t cnt,
                                                  unsigned long long x)
{
    uint32_t lo = 0, hi = cnt;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) / 2;
        if (s[mid] > x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// moved nodes passing the pick's filter, keyed by key_of, into L.e (unsorted)
template <typename KeyOf>
__device__ void pick_moved(const PickArgs &a, KeyOf key_of, unsigned long long stop_bound, PickLds &L)
{
    if (threadIdx.x == 0) L.ne = 0;
    __syncthreads();
    const uint32_t ne = min(a.ctl[CC_NE], CELF_CAPE);
    for (uint32_t i = threadIdx.x; i < ne; i += CP_NT) {
        const uint32_t u = a.E[i];
        if (a.sel[u] || a.fresh[u] == a.t + 1) continue;
        if (node_key(a.bound[u], u) <= stop_bound) continue;
        L.e[atomicAdd(&L.ne, 1u)] = key_of(u);
    }
    __syncthreads();
}

// top B of the descending lists L.a[0..na) and L.e[0..ne) -> cand (node ids)
__device__ uint32_t pick_merge(const PickArgs &a, PickLds &L, uint32_t na, uint32_t ne)
{
    for (uint32_t i = threadIdx.x; i < na; i += CP_NT) {
        const uint32_t r = i + count_greater(L.e, ne, L.a[i]);
        if (r < a.B) a.cand[r] = key_node(L.a[i]);
    }
    for (uint32_t j = threadIdx.x; j < ne; j += CP_NT) {
        const uint32_t r = j + count_greater(L.a, na, L.e[j]);
        if (r < a.B) a.cand[r] = key_node(L.e[j]);
    }
    return min(a.B, na + ne);
}

// largest of L.a[0..na) and L.e[0..ne) (0 when both are empty); all threads call
__device__ unsigned long long pick_max(PickLds &L, uint32_t na, uint32_t ne)
{
    unsigned long long m = 0;
    for (uint32_t i = threadIdx.x; i < na; i += CP_NT) m = L.a[i] > m ? L.a[i] : m;
    for (uint32_t i = threadIdx.x; i < ne; i += CP_NT) m = L.e[i] > m ? L.e[i] : m;
    m = wave_max_u64(m);
    if ((threadIdx.x & 63) == 0) L.red[threadIdx.x >> 6] = m;
    __syncthreads();
    m = 0;
    for (int i = 0; i < CP_NT / 64; i++) m = L.red[i] > m ? L.red[i] : m;
    __syncthreads();
    return m;
}

__global__ __launch_bounds__(CP_NT) void k_celf_pick(PickArgs a)
{
    __shared__ PickLds L;
    const unsigned long long best = *a.best;
    auto bkey = [&](uint32_t u) { return node_key(a.bound[u], u); };
    auto skey = [&](uint32_t u) { return node_key(score_bits(a.score[u]), u); };
    uint32_t ncand = 0;
    bool fallback = false;
    if (a.learned == 2 && best == 0) {
        // first batch of the round, sized by the network: its best-scored
        // candidate c and predicted current gain g (the network predicts
        // ln(1 + g/R)); the batch is the top B by bound of the nodes whose
        // bound key reaches (min(g, bound of c), c). When the prediction is
        // right, those are exactly the nodes the round must evaluate.
        pick_walk(a, a.ordS, CC_HEADS, skey, 0ull, 1, L);
        pick_moved(a, skey, 0ull, L);
        const unsigned long long top = pick_max(L, L.na, L.ne);
        unsigned long long thr = 0;
        if (top) {
            const uint32_t c = key_node(top);
            const float g = a.R * expm1f(a.score[c]);
            const uint32_t bc = a.bound[c];
            const uint32_t T = !(g > 0.0f) ? 0u : (g >= (float)bc ? bc : (uint32_t)g);
            thr = node_key(T, c) - 1;
        }
        pick_walk(a, a.ordB, CC_HEADB, bkey, thr, a.B, L);
        pick_moved(a, bkey, thr, L);
        const uint32_t na = L.na, ne = L.ne;
        lds_sort_desc(L.e, ne);
        ncand = pick_merge(a, L, na, ne);
    } else if (a.learned != 1) {
        pick_walk(a, a.ordB, CC_HEADB, bkey, best, a.B, L);
        pick_moved(a, bkey, best, L);
        const uint32_t na = L.na, ne = L.ne;
        lds_sort_desc(L.e, ne);
        ncand = pick_merge(a, L, na, ne);
    } else if (best == 0) {
        // first batch of the round: every unselected node can still win
        pick_walk(a, a.ordS, CC_HEADS, skey, 0ull, a.B, L);
        pick_moved(a, skey, 0ull, L);
        const uint32_t na = L.na, ne = L.ne;
        lds_sort_desc(L.e, ne);
        ncand = pick_merge(a, L, na, ne);
    } else {
        // gather every node whose bound can still win, then order by score
        pick_walk(a, a.ordB, CC_HEADB, bkey, best, CELF_CAPW, L);
        pick_moved(a, bkey, best, L);
        const uint32_t na = L.na, ne = L.ne;
        if (L.full) {
            fallback = true;
            lds_sort_desc(L.e, ne);
            ncand = pick_merge(a, L, na, ne);
        } else {
            // re-key the union by score
            for (uint32_t j = threadIdx.x; j < ne; j += CP_NT) L.e[j] = skey(key_node(L.e[j]));
            for (uint32_t i = threadIdx.x; i < na; i += CP_NT) L.e[ne + i] = skey(key_node(L.a[i]));
            __syncthreads();
            lds_sort_desc(L.e, na + ne);
            ncand = min(a.B, na + ne);
            for (uint32_t i = threadIdx.x; i < ncand; i += CP_NT) a.cand[i] = key_node(L.e[i]);
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < ncand; i += CP_NT) a.ev[a.cand[i]] = 0;
    if (threadIdx.x < PH_CTRS) a.ctl[CC_EVCTR + threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        a.ctl[CC_NCAND] = ncand;
        a.stats[ST_CELF_EVALS] += ncand;
        if (ncand) a.stats[ST_CELF_BATCHES] += 1;
        if (fallback) a.stats[ST_CELF_FALLBACKS] += 1;
    }
}

// record the batch's exact gains: new bounds, fresh marks, the round's best
// key, moved list and (learned) new scores
__global__ __launch_bounds__(256) void k_celf_update(const uint32_t *cand, uint32_t *ctl,
                                                     const uint32_t *ev, uint32_t *bound,
                                                     uint32_t *fresh, uint8_t *moved, uint32_t *E,
                                                     unsigned long long *best, uint32_t t,
                                                     const uint16_t *wb, const float *feat,
                                                     float invR, float *score)
{
    __shared__ float sw[MLP_NP];
    if (wb) mlp_stage(wb, sw);
    const uint32_t ncand = ctl[CC_NCAND];
    for (uint32_t i = threadIdx.x; i < ncand; i += 256) {
        const uint32_t c = cand[i];
        const uint32_t g = ev[c];
        bound[c] = g;
        fresh[c] = t + 1;
        atomicMax(best, node_key(g, c));
        if (!moved[c]) {
            moved[c] = 1;
            const uint32_t q = atomicAdd(&ctl[CC_NE], 1u);
            if (q < CELF_CAPE) E[q] = c;
        }
    }
    if (wb) {
        // new scores: one wavefront per candidate (its input has the new gain)
        for (uint32_t i = threadIdx.x >> 6; i < ncand; i += 4) {
            const uint32_t c = cand[i];
            float x[MLP_IN];
#pragma unroll
            for (int q = 0; q < 4; q++) x[q] = feat[(uint64_t)c * 4 + q];
            x[4] = log1pf((float)ev[c] * invR);
            const float y = mlp_eval_wave(sw, x);
            if ((threadIdx.x & 63) == 0) score[c] = y;
        }
    }
}

// Exact evaluation of a batch of candidates on one cooperative grid. Each
// (candidate slot s, word w) pair is a virtual word vw = s * W + w with its
// own reach map R[vw][x] (dense, [V][n]); the search from candidate s in
// word w starts with the valid bits not covered at s and never enters
// covered bits (Sec. 4: the newly reachable part of the snapshot). All
// V searches advance level by level together; small levels are spread one
// frontier entry per workgroup so that huge nodes do not serialise on one
// workgroup. Afterwards ev[cand[s]] += sum over w, x of popcount(R[vw][x])
// and R is returned to zero.
struct EvalArgs {
    const uint32_t *row, *col;
    const uint64_t *mask;
    HubLists hub;
    SparseLists sp;
    uint64_t m;
    uint32_t n, R, W, V;
    const uint64_t *covered;
    uint64_t *reach, *pend;      // [Vmax][n], zero on entry and on exit
    uint64_t *fq0, *fq1, *vis;   // (vw << 32 | node), capacity V * n each
    uint32_t *cnt;               // [8]: frontier ring [3], visit count, [4..6) grid barrier; zero on entry
    const uint32_t *cand;        // V / W candidates
    uint32_t *ev;
    unsigned long long *stats;
};

__device__ __forceinline__ void eval_relax(const EvalArgs &a, uint32_t vw, uint32_t v, uint64_t bits,
                                           bool &first, bool &push)
{
    first = false;
    push = false;
    if (bits) bits &= ~a.covered[(uint64_t)(vw % a.W) * a.n + v];
    if (!bits) return;
    const uint64_t off = (uint64_t)vw * a.n + v;
    const uint64_t old = atomicOr((unsigned long long *)&a.reach[off], (unsigned long long)bits);
    const uint64_t nb = bits & ~old;
    if (!nb) return;
    first = old == 0;
    const uint64_t op = atomicOr((unsigned long long *)&a.pend[off], (unsigned long long)nb);
    push = op == 0;
}

__global__ __launch_bounds__(FWD_NT) void k_eval_coop(EvalArgs a)
{
    __shared__ FwdLds L;
    uint32_t nbar = 0;
    __shared__ uint32_t slot_sum[256];
    const int tid = threadIdx.x;
    const uint64_t gtid = (uint64_t)blockIdx.x * FWD_NT + tid;
    if (tid == 0) L.H.n = 0;
    // seeds: one virtual word per thread
    if (gtid < a.V) {
        const uint32_t vw = (uint32_t)gtid, s = vw / a.W, w = vw % a.W, c = a.cand[s];
        const uint64_t start = im_valid_bits(a.R, w) & ~a.covered[(uint64_t)w * a.n + c];
        if (start) {
            a.reach[(uint64_t)vw * a.n + c] = start;
            a.pend[(uint64_t)vw * a.n + c] = start;
            a.vis[atomicAdd(&a.cnt[3], 1u)] = ((uint64_t)vw << 32) | c;
            a.fq0[atomicAdd(&a.cnt[0], 1u)] = ((uint64_t)vw << 32) | c;
        }
    }
    if (!grid_barrier(a.cnt + 4, nbar, a.stats)) return;
    uint64_t arcs = 0;
    for (uint32_t lev = 0;; lev++) {
        const uint32_t nf = group_load(&a.cnt[lev % 3], &L.bcast);
        if (nf == 0) break;
        const uint64_t *cur = (lev & 1) ? a.fq1 : a.fq0;
        uint64_t *nxt = (lev & 1) ? a.fq0 : a.fq1;
        uint32_t *ncnt = &a.cnt[(lev + 1) % 3];
        if (gtid == 0) a.cnt[(lev + 2) % 3] = 0;
        // entries per workgroup: a full tile when there is enough work for
        // every workgroup, fewer (down to one) otherwise
        const uint32_t per = std::max<uint32_t>(1u, std::min<uint32_t>(FWD_NT, (nf + gridDim.x - 1) / gridDim.x));
        for (uint64_t tile = (uint64_t)blockIdx.x * per; tile < nf; tile += (uint64_t)gridDim.x * per) {
            const uint64_t i = tile + tid;
            uint32_t deg = 0, rs = 0, vw = 0, aux = 0;
            uint64_t d = 0;
            if ((uint32_t)tid < per && i < nf) {
                const uint64_t e = cur[i];
                vw = (uint32_t)(e >> 32);
                const uint32_t x = (uint32_t)e;
                rs = a.row[x];
                deg = a.row[x + 1] - rs;
                const uint32_t hs = deg >= a.hub.min_deg ? a.hub.slot[x] : IM_EMPTY;
                d = atomicExch((unsigned long long *)&a.pend[(uint64_t)vw * a.n + x], 0ull);
                if (hs != IM_EMPTY) {
                    hub_push(L.H, hs, vw, d);
                    deg = 0; d = 0;
                } else {
                    uint32_t work, srs, saux;
                    uint64_t sdel;
                    if (deg >= 2 && sparse_use(sparse_fetch(a.sp, a.n, vw % a.W, x, d), deg, work, srs, sdel, saux)) {
                        deg = work; rs = srs; d = sdel; aux = saux;
                    }
                }
            }
            uint32_t total;
            const uint32_t ex = block_excl_scan<FWD_NT>(deg, L.wsum, &total);
            L.scan[tid] = ex; L.rs[tid] = rs; L.del[tid] = d; L.wd[tid] = vw; L.aux[tid] = aux;
            __syncthreads();
            const uint32_t nhub = L.H.n;
            arcs += total;
            for (uint32_t j0 = 0; j0 < total; j0 += FWD_NT * FWD_U) {
                uint32_t kk[FWD_U], ee[FWD_U], vv[FWD_U];
                uint64_t bb[FWD_U];
#pragma unroll
                for (int u = 0; u < FWD_U; u++) {
                    const uint32_t j = j0 + (uint32_t)tid + (uint32_t)u * FWD_NT;
                    kk[u] = 0xFFFFFFFFu; ee[u] = 0; bb[u] = 0; vv[u] = 0;
                    if (j < total) {
                        const int k = upper_index<FWD_NT>(L.scan, j);
                        kk[u] = (uint32_t)k;
                        ee[u] = j - L.scan[k];   // rank within the entry
                    }
                }
#pragma unroll
                for (int u = 0; u < FWD_U; u++)
                    if (kk[u] != 0xFFFFFFFFu) {
                        const uint32_t k = kk[u], ax = L.aux[k];
                        uint32_t pos = L.rs[k] + ee[u];
                        uint64_t bit = 0;
                        if (ax) sparse_item(L.rs[k], L.del[k], ax, ee[u], pos, bit);
                        const uint32_t *heads = ax ? a.sp.adj : a.col;
                        vv[u] = heads[pos];
                        bb[u] = ax ? bit : (a.mask[(uint64_t)(L.wd[k] % a.W) * a.m + pos] & L.del[k]);
                    }
                uint64_t vis_e[FWD_U], nxt_e[FWD_U];
                uint32_t nvis = 0, nnxt = 0;
#pragma unroll
                for (int u = 0; u < FWD_U; u++) {
                    const uint32_t ww = kk[u] != 0xFFFFFFFFu ? L.wd[kk[u]] : 0u;
                    const uint64_t bits = kk[u] != 0xFFFFFFFFu ? bb[u] : 0ull;
                    bool first, push;
                    eval_relax(a, ww, vv[u], bits, first, push);
                    const uint64_t ent = ((uint64_t)ww << 32) | vv[u];
                    if (first) vis_e[nvis++] = ent;
                    if (push) nxt_e[nnxt++] = ent;
                }
                wave_append_n<FWD_U>(nvis, vis_e, a.cnt + 3, a.vis);
                wave_append_n<FWD_U>(nnxt, nxt_e, ncnt, nxt);
            }
            __syncthreads();
            if (nhub) {
                const uint32_t W = a.W;
                auto word_of = [W](uint32_t own) { return own % W; };
                uint64_t vis_e[FWD_U], nxt_e[FWD_U];
                uint32_t nvis = 0, nnxt = 0;
                auto relax = [&](uint32_t own, uint32_t hv, uint64_t bits) {
                    bool first, push;
                    eval_relax(a, own, hv, bits, first, push);
                    const uint64_t ent = ((uint64_t)own << 32) | hv;
                    if (first) vis_e[nvis++] = ent;
                    if (push) nxt_e[nnxt++] = ent;
                };
                auto flush = [&]() {
                    wave_append_n<FWD_U>(nvis, vis_e, a.cnt + 3, a.vis);
                    wave_append_n<FWD_U>(nnxt, nxt_e, ncnt, nxt);
                    nvis = 0;
                    nnxt = 0;
                };
                expand_hubs<FWD_NT, 16, FWD_U>(L.H, nhub, a.hub, a.W, word_of, relax, flush, arcs);
            }
        }
        if (!grid_barrier(a.cnt + 4, nbar, a.stats)) return;
    }
    // per-candidate sums of the reached bits; reach returns to zero
    const uint32_t nslot = a.V / a.W;
    for (uint32_t s = tid; s < nslot; s += FWD_NT) slot_sum[s] = 0;
    __syncthreads();
    uint64_t relax = 0, trav = 0;
    const uint32_t nv = group_load(&a.cnt[3], &L.bcast);
    for (uint64_t i = gtid; i < nv; i += (uint64_t)gridDim.x * FWD_NT) {
        const uint64_t e = a.vis[i];
        const uint32_t vw = (uint32_t)(e >> 32), x = (uint32_t)e;
        const uint64_t off = (uint64_t)vw * a.n + x;
        const uint32_t pc = (uint32_t)__popcll(a.reach[off]);
        a.reach[off] = 0;
        const uint32_t dg = a.row[x + 1] - a.row[x];
        relax += dg;
        trav += (uint64_t)pc * dg;
        atomicAdd(&slot_sum[vw / a.W], pc);
    }
    __syncthreads();
    for (uint32_t s = tid; s < nslot; s += FWD_NT)
        if (slot_sum[s]) atomicAdd(&a.ev[a.cand[s]], slot_sum[s]);
    relax = group_sum<FWD_NT>(relax, L.red);
    trav = group_sum<FWD_NT>(trav, L.red);
    if (tid == 0) {
        atomicAdd(&a.stats[st_tier(PASS_EVAL, 2, F_RELAX)], (unsigned long long)relax);
        if (blockIdx.x == 0) atomicAdd(&a.stats[st_tier(PASS_EVAL, 2, F_REACHED)], (unsigned long long)nv);
        atomicAdd(&a.stats[st_tier(PASS_EVAL, 2, F_ARCS)], (unsigned long long)arcs);
        atomicAdd(&a.stats[ST_TRAV_EVAL], (unsigned long long)trav);
    }
}

static int reserve_celf(im_workspace *ws, uint32_t n)
{
    int rc;
    uint64_t len = SORT_TILE;
    while (len < n) len <<= 1;
    if (n > ws->cap_celf || !ws->c_bound) {
        const uint32_t cn = std::max(n, ws->cap_celf);
        if ((rc = dalloc(&ws->c_bound, cn)) || (rc = dalloc(&ws->c_fresh, cn)) ||
            (rc = dalloc(&ws->c_moved, cn)) || (rc = dalloc(&ws->c_ev, cn)) ||
            (rc = dalloc(&ws->c_ordB, cn)) || (rc = dalloc(&ws->c_ordS, cn)) ||
            (rc = dalloc(&ws->c_score, cn)) || (rc = dalloc(&ws->c_feat, 4ull * cn)) ||
            (rc = dalloc(&ws->c_E, CELF_CAPE)) || (rc = dalloc(&ws->c_cand, CELF_BMAX)) ||
            (rc = dalloc(&ws->c_ctl, CC_COUNT)))
            return rc;
        ws->cap_celf = cn;
    }
    if (len > ws->cap_sort) {
        if ((rc = dalloc(&ws->c_sort, len))) return rc;
        ws->cap_sort = len;
    }
    if (ws->slots > ws->cap_kept || !ws->c_kept) {
        if ((rc = dalloc(&ws->c_kept, 2ull * ws->slots))) return rc;
        ws->cap_kept = ws->slots;
    }
    return IM_OK;
}

// virtual words of one cooperative evaluation launch: at most 256 and at
// most EVAL_BUDGET bytes of search state (40 bytes per node and virtual
// word); 0 when not even one candidate fits (the tier engines run then)
constexpr uint64_t EVAL_BUDGET = 8ull << 30;

static uint32_t eval_vmax(uint32_t n, uint32_t W)
{
    uint64_t v = EVAL_BUDGET / (40ull * std::max<uint32_t>(n, 1));
    v = std::min<uint64_t>(v, 256);
    v -= v % W;
    return (uint32_t)v;
}

static int reserve_eval(im_workspace *ws, uint32_t n, uint32_t V)
{
    int rc;
    const uint64_t need = (uint64_t)V * std::max<uint32_t>(n, 1);
    if (need > ws->cap_eval) {
        if ((rc = dalloc(&ws->e_reach, need)) || (rc = dalloc(&ws->e_pend, need)) ||
            (rc = dalloc(&ws->e_fq0, need)) || (rc = dalloc(&ws->e_fq1, need)) ||
            (rc = dalloc(&ws->e_vis, need)) || (rc = dalloc(&ws->e_cnt, 8)))
            return rc;
        HIPCHK(hipMemset(ws->e_reach, 0, need * sizeof(uint64_t)));
        HIPCHK(hipMemset(ws->e_pend, 0, need * sizeof(uint64_t)));
        ws->cap_eval = need;
    }
    return IM_OK;
}

// exact gains of cand[0..ncand) into ev (zeroed by the pick) on cooperative grids
static int eval_coop(const im_graph *g, uint32_t R, uint32_t ncand, uint32_t vmax, im_workspace *ws,
                     hipStream_t s)
{
    const uint32_t n = g->n, W = (R + 63) / 64, per = vmax / W;
    EvalArgs e;
    e.row = ws->row32; e.col = g->col; e.mask = ws->mask_out; e.hub = hub_lists(ws, 0);
    e.sp = sparse_lists(ws, 0);
    e.m = g->m; e.n = n; e.R = R; e.W = W;
    e.covered = ws->covered; e.reach = ws->e_reach; e.pend = ws->e_pend;
    e.fq0 = ws->e_fq0; e.fq1 = ws->e_fq1; e.vis = ws->e_vis; e.cnt = ws->e_cnt;
    e.ev = ws->c_ev; e.stats = ws->stats;
    for (uint32_t c0 = 0; c0 < ncand; c0 += per) {
        const uint32_t nc = std::min(per, ncand - c0);
        e.cand = ws->c_cand + c0;
        e.V = nc * W;
        fill<uint32_t>(ws->e_cnt, 8, 0u, s);   // counters and the grid barrier's pair
        void *args[] = {&e};
        hipError_t err = hipLaunchCooperativeKernel((const void *)k_eval_coop, dim3(ws->eval_grid),
                                                    dim3(FWD_NT), args, 0, s);
        if (err != hipSuccess)
            return im_fail(IM_EHIP, "cooperative launch of k_eval_coop: %s", hipGetErrorString(err));
    }
    return IM_OK;
}

// sort all nodes by (primary desc, id asc): primary = score when given, else bound
static void build_order(im_workspace *ws, uint32_t n, const float *score, uint32_t *ord,
                        hipStream_t s)
{
    uint64_t len = SORT_TILE;
    while (len < n) len <<= 1;
    k_order_keys<<<grid_for(len, 256), 256, 0, s>>>(ws->c_bound, score, n, len, ws->c_sort);
    const unsigned tiles = (unsigned)(len / SORT_TILE);
    k_bitonic_tile<<<tiles, 1024, 0, s>>>(ws->c_sort, 2, SORT_TILE);
    for (uint64_t kk = 2 * SORT_TILE; kk <= len; kk <<= 1) {
        for (uint64_t j = kk >> 1; j >= SORT_TILE; j >>= 1)
            k_bitonic_step<<<grid_for(len / 2, 256), 256, 0, s>>>(ws->c_sort, len, kk, j);
        k_bitonic_tile<<<tiles, 1024, 0, s>>>(ws->c_sort, kk, kk);
    }
    k_order_extract<<<grid_for(n, 256), 256, 0, s>>>(ws->c_sort, n, ord);
}

static void rebuild_orders(im_workspace *ws, uint32_t n, bool learned, hipStream_t s)
{
    PhaseTimer pt(ws, IM_PH_ORDER, s);
    build_order(ws, n, nullptr, ws->c_ordB, s);
    if (learned) build_order(ws, n, ws->c_score, ws->c_ordS, s);
    fill<uint8_t>(ws->c_moved, n, (uint8_t)0, s);
    k_celf_reset<<<1, 64, 0, s>>>(ws->c_ctl);
}

// A5 without A6: commit the round's argmax key keys[t] (forward search,
// covered |= newly covered) and clear the newly-covered words
static int commit_seed(const im_graph *g, uint32_t R, uint32_t t, uint32_t *seeds_out,
                       uint64_t *gains_out, im_workspace *ws, hipStream_t s,
                       const uint32_t *skip = nullptr)
{
    const uint32_t n = g->n, W = (R + 63) / 64;
    FwdArgs f;
    f.skip = skip;
    f.row = ws->row32; f.col = g->col; f.mask = ws->mask_out; f.m = g->m;
    f.hub = hub_lists(ws, 0);
    f.sp = sparse_lists(ws, 0);
    f.n = n; f.R = R; f.W = W;
    f.covered = ws->covered; f.newly = ws->newly; f.pend = ws->fpend;
    f.fq0 = ws->fqa; f.fq1 = ws->fqb; f.cnt = ws->fctr + (uint64_t)t * FWD_CTRS;
    f.bq0 = ws->bqa; f.bq1 = ws->bqb; f.coop_gain = ws->coop_gain; f.vis = ws->fvis;
    f.tnodes = ws->tnodes; f.tcounts = ws->tcounts;
    f.bcnt = nullptr; f.mcnt = nullptr; f.mlist = nullptr;
    f.key = ws->keys + t; f.t = t; f.b = ws->batch;
    f.seeds_out = seeds_out; f.gains_out = gains_out; f.sel = ws->sel;
    f.stats = ws->stats;
    {
        PhaseTimer pt(ws, IM_PH_FORWARD, s);
        const int rc = launch_forward(f, ws, true, s);
        if (rc) return rc;
    }
    {
        PhaseTimer pt(ws, IM_PH_CLEAR, s);
        k_clear_newly<<<grid_for(n, 256, 1024), 256, 0, s>>>(ws->newly, ws->tnodes, ws->tcounts, n, W);
    }
    return IM_OK;
}

// ---------------------------------------------------------------------------
// Committing from a kept evaluation. With the last-tier engine, a batch whose
// (candidate, word) searches fit the slots runs one search per slot and keeps
// its fixpoint there. Every search was pruned at covered, so the reach bits
// of the round's seed v* are exactly its newly covered bits: when v* was in
// the round's last batch, covered |= those bits replaces the forward search
// from v* (which then returns at once).
// ---------------------------------------------------------------------------
struct KeptArgs {
    const unsigned long long *key;   // the round's best key
    uint32_t t, ncand, n, W, slot_n;
    uint32_t split;                  // bit groups per (candidate, word) search
    const uint32_t *nvis, *src;      // per kept search (task = slot)
    const uint64_t *reach;           // slots' (reach, pend) records
    const uint32_t *vis;             // slots' visit lists
    const uint32_t *row;
    uint64_t *covered;
    uint32_t *seeds_out, *tcounts, *flag;
    uint64_t *gains_out;
    uint8_t *sel;
    unsigned long long *stats;
};

// KC_G workgroups per (word, bit group) (grid KC_G x W * split)
constexpr uint32_t KC_G = 64;

__global__ __launch_bounds__(256) void k_kept_commit(KeptArgs a)
{
    __shared__ uint32_t found;
    __shared__ unsigned long long red[4];
    const uint32_t w = blockIdx.y % a.W, grp = blockIdx.y / a.W, part = blockIdx.x, tid = threadIdx.x;
    const unsigned long long key = *a.key;
    if (key == 0) return;
    const uint32_t v = 0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull);
    if (tid == 0) found = 0xFFFFFFFFu;
    __syncthreads();
    for (uint32_t j = tid; j < a.ncand; j += 256)
        if (a.src[j] == v) found = j;   // candidates are distinct: one writer
    __syncthreads();
    const uint32_t j = found;
    if (j == 0xFFFFFFFFu) return;   // evaluated in an earlier batch: the forward search commits
    // the seed's search of word w over bit group grp; groups hold disjoint
    // bits, and a node counts as covered in word w (degree, visit) once: in
    // the first group that reached it
    const uint32_t per = a.ncand * a.W;
    const uint32_t task = grp * per + w * a.ncand + j;
    const uint32_t nv = a.nvis[task];
    const uint32_t *vis = a.vis + (uint64_t)task * a.slot_n;
    const uint64_t *reach = a.reach + (uint64_t)task * a.slot_n * 2;
    uint64_t relax = 0, trav = 0, first_visits = 0;
    for (uint32_t i = part * 256 + tid; i < nv; i += KC_G * 256) {
        const uint32_t x = vis[i];
        const uint64_t b = reach[(uint64_t)x * 2];
        atomicOr((unsigned long long *)&a.covered[(uint64_t)w * a.n + x], (unsigned long long)b);
        const uint32_t dg = a.row[x + 1] - a.row[x];
        bool first = true;
        for (uint32_t g = 0; g < grp; g++)
            first = first && a.reach[((uint64_t)(g * per + w * a.ncand + j) * a.slot_n + x) * 2] == 0;
        if (first) { relax += dg; first_visits += 1; }
        trav += (uint64_t)__popcll(b) * dg;
    }
    relax = group_sum<256>(relax, red);
    trav = group_sum<256>(trav, red);
    first_visits = group_sum<256>(first_visits, red);
    if (tid == 0 && (trav || first_visits)) {
        atomicAdd(&a.stats[ST_RELAX_FWD], (unsigned long long)relax);
        atomicAdd(&a.stats[ST_TRAV_FWD], (unsigned long long)trav);
        atomicAdd(&a.stats[ST_TASKS_REV], (unsigned long long)first_visits);
    }
    if (tid == 0 && part == 0 && grp == 0) {
        a.tcounts[w] = 0;
        if (w == 0) {
            a.seeds_out[a.t] = v;
            a.gains_out[a.t] = key >> 32;
            a.sel[v] = 1;
            *a.flag = 1;
        }
    }
}

// return the kept slots to zero (grid KC_G x slots) and clear the flag
__global__ __launch_bounds__(256) void k_kept_clear(const uint32_t *nvis, const uint32_t *vis,
                                                    uint64_t *reach, uint32_t slot_n, uint32_t *flag)
{
    const uint32_t task = blockIdx.y, part = blockIdx.x;
    const uint32_t nv = nvis[task];
    const uint32_t *vl = vis + (uint64_t)task * slot_n;
    uint64_t *rc = reach + (uint64_t)task * slot_n * 2;
    for (uint32_t i = part * 256 + threadIdx.x; i < nv; i += KC_G * 256) rc[(uint64_t)vl[i] * 2] = 0;
    if (task == 0 && part == 0 && threadIdx.x == 0) *flag = 0;
}

static int select_lazy(const im_graph *g, uint32_t R, uint32_t k, uint32_t B, const im_mlp *model,
                       uint32_t *seeds_out, uint64_t *gains_out, im_workspace *ws, hipStream_t s)
{
    int rc;
    const uint32_t n = g->n, W = (R + 63) / 64;
    const bool learned = model != nullptr;
    const float invR = 1.0f / (float)R;
    if ((rc = reserve_celf(ws, n))) return rc;
    const uint32_t vmax = ws->lazy_engine == 1 ? eval_vmax(n, W) : 0u;
    if (vmax && (rc = reserve_eval(ws, n, vmax))) return rc;
    k_copy_u32<<<grid_for(n, 256), 256, 0, s>>>(ws->gain, ws->c_bound, n);
    fill<uint32_t>(ws->c_fresh, n, 0u, s);
    fill<uint32_t>(ws->c_ctl, CC_COUNT, 0u, s);
    if (learned) {
        PhaseTimer pt(ws, IM_PH_SCORE, s);
        launch_features(ws->row32, g->col, g->prob, ws->in_row, n, ws->c_feat, s);
        k_celf_score<<<grid_for(n, 256, 4096), 256, 0, s>>>(model->wb, ws->c_feat, ws->c_bound, invR,
                                                            nullptr, n, nullptr, ws->c_score);
    }
    rebuild_orders(ws, n, learned, s);
    HIPCHK(hipGetLastError());
    uint64_t moved_bound = 0;  // upper bound of |E| since the last rebuild
    PickArgs pa;
    pa.n = n; pa.B = B; pa.learned = learned ? ws->learned_policy : 0; pa.R = (float)R;
    pa.ordB = ws->c_ordB; pa.ordS = ws->c_ordS; pa.bound = ws->c_bound; pa.score = ws->c_score;
    pa.fresh = ws->c_fresh; pa.sel = ws->sel; pa.moved = ws->c_moved; pa.E = ws->c_E;
    pa.ctl = ws->c_ctl; pa.cand = ws->c_cand; pa.ev = ws->c_ev; pa.stats = ws->stats;
    // round 0: every bound is exact (the initial counts), so the round's
    // argmax needs no evaluation
    {
        PhaseTimer pt(ws, IM_PH_ARGMAX, s);
        // a single graph: few workgroups, so that few atomics meet on the key
        k_argmax<<<grid_for(n, 256, ws->batch.count == 1 ? 256 : 2048), 256, 0, s>>>(ws->gain, ws->sel, n, ws->keys, ws->batch, 0,
                                                         ws->pk, (uint32_t)PK_ZERO);
    }
    if ((rc = commit_seed(g, R, 0, seeds_out, gains_out, ws, s))) return rc;
    // the last batch's searches kept in the slots (last-tier engine): their count
    uint32_t kept_tasks = 0, kept_ncand = 0, kept_split = 1;
    auto clear_kept = [&]() {
        if (!kept_tasks) return;
        PhaseTimer pt(ws, IM_PH_CLEAR, s);
        k_kept_clear<<<dim3(KC_G, kept_tasks), 256, 0, s>>>(ws->c_kept, ws->b_vis, ws->b_reach,
                                                             ws->slots_n, ws->c_ctl + CC_KEPT);
        kept_tasks = 0;
    };
    for (uint32_t t = 1; t < k; t++) {
        pa.t = t;
        pa.best = ws->keys + t;
        for (;;) {
            if (moved_bound + B > CELF_CAPE) {
                rebuild_orders(ws, n, learned, s);
                moved_bound = 0;
            }
            {
                PhaseTimer pt(ws, IM_PH_PICK, s);
                k_celf_pick<<<1, CP_NT, 0, s>>>(pa);
            }
            HIPCHK(hipMemcpyAsync(ws->host_err, ws->c_ctl + CC_NCAND, sizeof(uint32_t),
                                  hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            const uint32_t ncand = *ws->host_err;
            if (ncand == 0) break;
            clear_kept();   // the slots are about to be reused
            if (vmax) {
                PhaseTimer pt(ws, IM_PH_EVAL_T2, s);
                if ((rc = eval_coop(g, R, ncand, vmax, ws, s))) return rc;
            } else {
                BfsArgs a = bfs_args(ws, ws->row32, g->col, ws->mask_out, g->m, n, R, W);
                a.cand = ws->c_cand;
                a.ncand = ncand;
                a.ntasks = ncand * W;
                a.gain = ws->c_ev;
                a.prune = ws->covered;
                a.hub = hub_lists(ws, 0);
                a.sp = sparse_lists(ws, 0);
                a.pass = PASS_EVAL;
                a.st_trav = ST_TRAV_EVAL;
                if (ws->lazy_engine == 2 && ws->batch.count == 1 && ncand * W <= ws->slots) {
                    // the bit groups per search: as many (of 8, 4, 2) as the
                    // slots hold, or the workspace's fixed choice when it fits
                    uint32_t split = ws->eval_split ? ws->eval_split : 8u;
                    while (split > 1 && ncand * W * split > ws->slots) split >>= 1;
                    a.bsplit = split;
                    a.ntasks = ncand * W * split;
                    run_last_tier<MODE_COUNT, true, true>(a, ws, ws->c_ctl + CC_EVCTR, IM_PH_EVAL_T2, s);
                    kept_tasks = ncand * W * split;
                    kept_ncand = ncand;
                    kept_split = split;
                } else if (ws->lazy_engine == 2)
                    run_last_tier<MODE_COUNT, true>(a, ws, ws->c_ctl + CC_EVCTR, IM_PH_EVAL_T2, s);
                else
                    run_tiers<MODE_COUNT, true>(a, ws, ws->c_ctl + CC_EVCTR, IM_PH_EVAL_T0, s);
            }
            {
                PhaseTimer pt(ws, IM_PH_UPDATE, s);
                k_celf_update<<<1, 256, 0, s>>>(ws->c_cand, ws->c_ctl, ws->c_ev, ws->c_bound,
                                                ws->c_fresh, ws->c_moved, ws->c_E, ws->keys + t, t,
                                                learned ? model->wb : nullptr, ws->c_feat, invR,
                                                ws->c_score);
            }
            moved_bound += ncand;
        }
        if (kept_tasks) {
            KeptArgs ka;
            ka.key = ws->keys + t; ka.t = t; ka.ncand = kept_ncand; ka.n = n; ka.W = W;
            ka.split = kept_split;
            ka.slot_n = ws->slots_n; ka.nvis = ws->c_kept; ka.src = ws->c_kept + ws->cap_kept;
            ka.reach = ws->b_reach; ka.vis = ws->b_vis; ka.row = ws->row32; ka.covered = ws->covered;
            ka.seeds_out = seeds_out; ka.gains_out = gains_out; ka.tcounts = ws->tcounts;
            ka.flag = ws->c_ctl + CC_KEPT; ka.sel = ws->sel; ka.stats = ws->stats;
            PhaseTimer pt(ws, IM_PH_FORWARD, s);
            k_kept_commit<<<dim3(KC_G, W * kept_split), 256, 0, s>>>(ka);
        }
        if ((rc = commit_seed(g, R, t, seeds_out, gains_out, ws, s, ws->c_ctl + CC_KEPT))) return rc;
        clear_kept();
    }
    HIPCHK(hipGetLastError());
    return IM_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Spread evaluator: f(T) = sum_r |R_r(T)| (the snapshot estimator of Sec. 3.1,
// times R) for the prefixes of a seed sequence, on snapshots of any seed, so
// a seed set can be scored on snapshots independent of those that chose it
// (the evaluation protocol of Sec. 5.2). One workgroup per snapshot word covers
// the seeds group by group: each group's search is pruned at the nodes the
// earlier groups covered, so its reach count is the group's marginal gain.
// ---------------------------------------------------------------------------
constexpr int SPR_NT = 1024, SPR_U = 8;
constexpr uint64_t SPR_BUDGET = 8ull << 30;   // masks + search state of one chunk
constexpr uint32_t SPR_MAX_WORDS = 256;

struct SpreadArgs {
    const uint32_t *row, *col;
    const uint64_t *mask;          // [chunk words][m]
    uint64_t m;
    uint32_t n, R, W, w0;          // this launch: words w0 .. w0 + gridDim.x - 1
    const uint32_t *S;
    uint32_t nS, group;            // seeds per search
    uint64_t *reach, *pend, *cov;  // [chunk words][n]; reach, pend zero at rest, cov zero on entry
    uint32_t *qa, *qb, *vis;       // [chunk words][n]
    unsigned long long *marg;      // [ceil(nS / group)] (accumulated over words) or nullptr
    uint32_t *per_snapshot;        // [R] or nullptr
};

__global__ __launch_bounds__(SPR_NT) void k_spread(SpreadArgs a)
{
    __shared__ BlockLds<SPR_NT> L;
    __shared__ uint32_t bitcnt[64];
    const int tid = threadIdx.x, lane = tid & 63;
    const uint32_t wl = blockIdx.x, w = a.w0 + wl;
    const uint64_t off = (uint64_t)wl * a.n;
    const uint64_t valid = im_valid_bits(a.R, w);
    uint64_t *reach = a.reach + off, *pend = a.pend + off, *cov = a.cov + off;
    uint32_t *qa = a.qa + off, *qb = a.qb + off, *vis = a.vis + off;
    const uint64_t *mask = a.mask + (uint64_t)wl * a.m;
    const HubLists nohub = {nullptr, nullptr, nullptr};
    const SparseLists nosp = {nullptr, nullptr, nullptr};
    if (tid < 64) bitcnt[tid] = 0;
    __syncthreads();
    uint32_t mine = 0;   // this lane's count of snapshot 64w + lane (per wavefront)
    uint64_t arcs = 0;
    for (uint32_t g0 = 0; g0 < a.nS; g0 += a.group) {
        const uint32_t gn = min(a.group, a.nS - g0);
        uint32_t src = 0;
        uint64_t start = 0;
        if ((uint32_t)tid < gn) {
            src = a.S[g0 + tid];
            start = valid & ~cov[src];
        }
        block_bfs_run<SPR_NT, SPR_U, true, false>(L, src, start, a.row, a.col, mask, nohub, nosp,
                                                  a.n, a.W, w, cov, reach, pend, 0u, qa, qb, vis,
                                                  arcs);
        // fold the group's reach into the cover; wavefront-uniform tiles
        const uint32_t nvis = L.nvis;
        uint64_t cnt = 0;
        for (uint32_t base = (uint32_t)(tid & ~63); base < nvis; base += SPR_NT) {
            const uint32_t j = base + (uint32_t)lane;
            uint64_t b = 0;
            if (j < nvis) {
                const uint32_t x = vis[j];
                b = reach[x];
                cov[x] |= b;
                reach[x] = 0;
            }
            cnt += (uint64_t)__popcll(b);
            if (a.per_snapshot && __ballot(b != 0) != 0ull) {
                for (int t = 0; t < 64; t++) {
                    const uint64_t bal = __ballot((b >> t) & 1ull);
                    if (lane == t) mine += (uint32_t)__popcll(bal);
                }
            }
        }
        cnt = group_sum<SPR_NT>(cnt, L.red);
        if (tid == 0 && a.marg && cnt) atomicAdd(&a.marg[g0 / a.group], (unsigned long long)cnt);
        __syncthreads();
    }
    if (a.per_snapshot) {
        atomicAdd(&bitcnt[lane], mine);
        __syncthreads();
        if (tid < 64 && w * 64u + (uint32_t)tid < a.R) a.per_snapshot[w * 64u + tid] = bitcnt[tid];
    }
}

static int reserve_spread(im_workspace *ws, uint32_t n, uint64_t m, uint32_t words)
{
    int rc;
    if (n > ws->cap_sp_n || m > ws->cap_sp_m || words > ws->cap_sp_words || !ws->v_row32) {
        const uint32_t cn = std::max(n, ws->cap_sp_n), cw = std::max(words, ws->cap_sp_words);
        const uint64_t cm = std::max(m, ws->cap_sp_m), nw = (uint64_t)cn * cw;
        if ((rc = dalloc(&ws->v_row32, (uint64_t)cn + 1)) || (rc = dalloc(&ws->v_mask, cm * cw)) ||
            (rc = dalloc(&ws->v_reach, nw)) || (rc = dalloc(&ws->v_pend, nw)) ||
            (rc = dalloc(&ws->v_cov, nw)) || (rc = dalloc(&ws->v_qa, nw)) ||
            (rc = dalloc(&ws->v_qb, nw)) || (rc = dalloc(&ws->v_vis, nw)))
            return rc;
        HIPCHK(hipMemset(ws->v_reach, 0, nw * sizeof(uint64_t)));
        HIPCHK(hipMemset(ws->v_pend, 0, nw * sizeof(uint64_t)));
        ws->cap_sp_n = cn; ws->cap_sp_m = cm; ws->cap_sp_words = cw;
    }
    return IM_OK;
}

extern "C" int im_spread(const im_graph *g, uint32_t R, uint64_t seed, const uint32_t *S,
                         uint32_t nS, uint64_t *marg_out, uint32_t *per_snapshot_out,
                         im_workspace *ws, void *stream)
{
    int rc;
    if (!g || !ws) return im_fail(IM_EINVAL, "null graph or workspace");
    if ((rc = check_args(g, 1))) return rc;
    if (R == 0 || R > IM_SPREAD_R_MAX)
        return im_fail(IM_EINVAL, "R = %u must be in [1, %u]", R, IM_SPREAD_R_MAX);
    if (nS && !S) return im_fail(IM_EINVAL, "null seed array");
    if (ws->live_edge || ws->pair_coins)
        return im_fail(IM_EINVAL, "the spread evaluator draws one coin per stored arc");
    hipStream_t s = (hipStream_t)stream;
    const uint32_t n = g->n, W = (R + 63) / 64;
    const uint64_t m = g->m;
    // seeds are checked on the host before any output is touched
    std::vector<uint32_t> hs(nS);
    if (nS) {
        HIPCHK(hipMemcpyAsync(hs.data(), S, nS * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (uint32_t i = 0; i < nS; i++)
            if (hs[i] >= n) return im_fail(IM_EINVAL, "S[%u] = %u is not a node (n = %u)", i, hs[i], n);
    }
    const uint64_t per_word = 8 * m + 36ull * n + 1;
    const uint32_t cw = (uint32_t)std::max<uint64_t>(
        1, std::min<uint64_t>({(uint64_t)W, SPR_MAX_WORDS, SPR_BUDGET / per_word}));
    if ((rc = reserve_spread(ws, n, m, cw))) return rc;
    if ((rc = validate(g, ws, s, ws->v_row32))) return rc;
    if (marg_out && nS) fill<unsigned long long>((unsigned long long *)marg_out, nS, 0ull, s);
    if (per_snapshot_out) fill<uint32_t>(per_snapshot_out, R, 0u, s);
    if (nS && n) {
        SpreadArgs a;
        a.row = ws->v_row32; a.col = g->col; a.mask = ws->v_mask; a.m = m;
        a.n = n; a.R = R; a.W = W; a.S = S; a.nS = nS;
        a.group = marg_out ? 1u : (uint32_t)SPR_NT;
        a.reach = ws->v_reach; a.pend = ws->v_pend; a.cov = ws->v_cov;
        a.qa = ws->v_qa; a.qb = ws->v_qb; a.vis = ws->v_vis;
        a.marg = (unsigned long long *)marg_out;
        a.per_snapshot = per_snapshot_out;
        Batch nob = {};
        for (uint32_t w0 = 0; w0 < W; w0 += cw) {
            const uint32_t c = std::min(cw, W - w0);
            if (m) {
                dim3 grid((unsigned)((m + 255) / 256), c);
                k_mask_gen<<<grid, 256, 0, s>>>(g->prob, m, R, seed, ws->v_mask, nob, w0);
            }
            fill<uint64_t>(ws->v_cov, (uint64_t)c * n, 0ull, s);
            a.w0 = w0;
            k_spread<<<c, SPR_NT, 0, s>>>(a);
        }
    }
    HIPCHK(hipGetLastError());
    ws->last_stream = s;
    return IM_OK;
}

// accessors for the other translation units
UndState **im_ws_und(im_workspace *ws) { return &ws->und; }

uint64_t im_scan_sums_len(uint64_t len) { return (len + SCAN_TILE - 1) / SCAN_TILE + 2; }

void im_exclusive_scan(const uint32_t *in, uint32_t *out, uint64_t len, uint32_t *sums,
                       hipStream_t s)
{
    if (len) exclusive_scan(in, out, len, sums, s);
}

int im_ws_validate(const im_graph *g, im_workspace *ws, hipStream_t s, uint32_t *row32)
{
    return validate(g, ws, s, row32);
}

void im_ws_set_last_stream(im_workspace *ws, hipStream_t s) { ws->last_stream = s; }

extern "C" int im_validate(const im_graph *g, uint32_t R, void *stream)
{
    if (!g) return im_fail(IM_EINVAL, "null graph");
    int rc = R ? check_args(g, R) : (g->m >= (1ull << 32) ? im_fail(IM_EINVAL, "m >= 2^32") : IM_OK);
    if (rc) return rc;
    im_workspace *ws;
    if ((rc = im_workspace_create(&ws))) return rc;
    rc = validate(g, ws, (hipStream_t)stream, nullptr);
    im_workspace_destroy(ws);
    return rc;
}

extern "C" int im_stats_get(im_workspace *ws, im_stats *out)
{
    if (!ws || !out) return im_fail(IM_EINVAL, "null argument");
    HIPCHK(hipStreamSynchronize(ws->last_stream));
    HIPCHK(hipMemcpy(ws->host_stats, ws->stats, ST_COUNT * ST_STRIPES * sizeof(unsigned long long),
                     hipMemcpyDeviceToHost));
    // fold the copies into copy 0: sums, maxima for the level counters
    unsigned long long *hs = ws->host_stats;
    for (int c = 1; c < ST_STRIPES; c++)
        for (int i = 0; i < ST_COUNT; i++) {
            const unsigned long long v = hs[c * ST_COUNT + i];
            if (i >= ST_MAXLV_BASE && i < ST_MAXLV_BASE + 9) hs[i] = std::max(hs[i], v);
            else hs[i] += v;
        }
    memset(out, 0, sizeof(*out));
    const unsigned long long *h = ws->host_stats;
    out->trav_init = h[ST_TRAV_INIT];
    out->trav_fwd = h[ST_TRAV_FWD];
    out->trav_rev = h[ST_TRAV_REV];
    out->trav_eval = h[ST_TRAV_EVAL];
    out->relax_fwd = h[ST_RELAX_FWD];
    out->tasks_rev = h[ST_TASKS_REV];
    out->decrements = h[ST_DECREMENTS];
    out->celf_evals = h[ST_CELF_EVALS];
    out->fwd_levels = h[ST_FWD_LEVELS];
    out->fwd_entries = h[ST_FWD_ENTRIES];
    out->celf_batches = h[ST_CELF_BATCHES];
    out->celf_fallbacks = h[ST_CELF_FALLBACKS];
    out->barrier_failures = h[ST_BARRIER_FAIL];
    for (int p = 0; p < 3; p++)
        for (int t = 0; t < 3; t++) {
            out->relax[p][t] = h[st_tier(p, t, F_RELAX)];
            out->reached[p][t] = h[st_tier(p, t, F_REACHED)];
            out->arcs_read[p][t] = h[st_tier(p, t, F_ARCS)];
            out->handed_over[p][t] = h[st_tier(p, t, F_OVF)];
            out->max_levels[p][t] = h[ST_MAXLV_BASE + p * 3 + t];
        }
    return IM_OK;
}

extern "C" int im_snapshot_masks(const im_graph *g, uint32_t R, uint64_t seed, uint64_t *mask_out,
                                 im_workspace *ws, void *stream)
{
    int rc;
    if ((rc = check_args(g, R))) return rc;
    if (!ws || (g->m && !mask_out)) return im_fail(IM_EINVAL, "null workspace or output");
    hipStream_t s = (hipStream_t)stream;
    if ((rc = check_and_reserve(g, R, 0, ws, s))) return rc;
    if (ws->live_edge == 1) build_reverse(g, ws, s);   // linear threshold draws per in-row
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
        return im_fail(IM_EINVAL, "null workspace or output");
    hipStream_t s = (hipStream_t)stream;
    if ((rc = ws_reserve(ws, g->n, g->m, 1, 0, g->n))) return rc;
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
    if (!ws || (g->n && !gain_out)) return im_fail(IM_EINVAL, "null workspace or output");
    hipStream_t s = (hipStream_t)stream;
    if ((rc = prepare(g, R, seed, 0, ws, s, PREP_FORWARD))) return rc;
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
    if (!ws) return im_fail(IM_EINVAL, "null workspace");
    if (k > g->n) return im_fail(IM_EINVAL, "k = %u exceeds n = %u", k, g->n);
    if (k && (!seeds_out || !gains_out)) return im_fail(IM_EINVAL, "null seeds or gains output");
    hipStream_t s = (hipStream_t)stream;
    PhaseTimer pt(ws, IM_PH_CALL, s);
    if ((rc = prepare(g, R, seed, k, ws, s))) return rc;
    return enqueue_rounds(g, R, k, seeds_out, gains_out, trace_out, ws, s);
}

// ---------------------------------------------------------------------------
// Selection that allocates nothing: every workspace buffer is carved from one
// static device array per GPU, laid out afresh by each call
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[IM_NOALLOC_SCRATCH_BYTES];

constexpr int NA_MAX_DEV = 64;
constexpr uint32_t NA_SLOTS = 16;   // last-tier slots (28 bytes per node each)

struct NoAllocDev {
    std::mutex mu;
    char *ptr = nullptr;   // this GPU's copy of `scratch` (from hipGetSymbolAddress)
    int num_cu = 0;
    unsigned fwd_grid = 0, eval_grid = 0;
    im_workspace ws;       // host view of the carved buffers, rebuilt by every call
    uint32_t host_err = 0;
    unsigned long long host_stats[ST_COUNT * ST_STRIPES];
};
static NoAllocDev g_noalloc[NA_MAX_DEV];

// the schedule of the static workspace: no sparse live lists, few slots
static void noalloc_options(im_workspace *ws)
{
    ws->sparse = 0;
    ws->max_slots = NA_SLOTS;
}

// every buffer the selection uses, carved from (or measured against) the arena
static int noalloc_reserve(im_workspace *ws, const im_graph *g, uint32_t R, uint32_t k)
{
    int rc;
    if ((rc = dalloc(&ws->stats, ST_COUNT * ST_STRIPES)) || (rc = dalloc(&ws->err, 1))) return rc;
    return ws_reserve(ws, g->n, g->m, (R + 63) / 64, k, g->n);
}

extern "C" int im_select_noalloc(const im_graph *g, uint32_t R, uint32_t k, uint64_t seed,
                                 uint32_t *seeds_out, uint64_t *gains_out, void *stream)
{
    int rc;
    if ((rc = check_args(g, R))) return rc;
    if (k > g->n) return im_fail(IM_EINVAL, "k = %u exceeds n = %u", k, g->n);
    if (k && (!seeds_out || !gains_out)) return im_fail(IM_EINVAL, "null seeds or gains output");
    {
        // size check before any device work: host arithmetic only
        im_workspace probe;
        noalloc_options(&probe);
        Arena a = {nullptr, IM_NOALLOC_SCRATCH_BYTES, 0, nullptr};
        t_arena = &a;
        rc = noalloc_reserve(&probe, g, R, k);
        t_arena = nullptr;
        if (rc) return rc;
        if (a.used > a.cap)
            return im_fail(IM_EINVAL,
                           "im_select_noalloc: n = %u, m = %llu, R = %u needs %llu bytes of "
                           "scratch, more than the %llu of the static scratch",
                           g->n, (unsigned long long)g->m, R, (unsigned long long)a.used,
                           (unsigned long long)a.cap);
    }
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NA_MAX_DEV) return im_fail(IM_EINVAL, "device %d out of range", dev);
    NoAllocDev &d = g_noalloc[dev];
    std::lock_guard<std::mutex> lock(d.mu);
    if (!d.ptr) {
        // once per device, with that device current: the array's address on it
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return im_fail(IM_EHIP, "hipGetSymbolAddress of the static scratch: %s",
                           hipGetErrorString(e));
        im_workspace tmp;
        if ((rc = ws_init_device(&tmp))) return rc;
        d.num_cu = tmp.num_cu;
        d.fwd_grid = tmp.fwd_grid;
        d.eval_grid = tmp.eval_grid;
        d.ptr = (char *)p;
    }
    hipStream_t s = (hipStream_t)stream;
    // an earlier call on this stream may still be using the scratch
    HIPCHK(hipStreamSynchronize(s));
    d.ws = im_workspace();
    im_workspace *ws = &d.ws;
    ws->device = dev;
    ws->num_cu = d.num_cu;
    ws->fwd_grid = d.fwd_grid;
    ws->eval_grid = d.eval_grid;
    noalloc_options(ws);
    ws->host_err = &d.host_err;
    ws->host_stats = d.host_stats;
    Arena a = {d.ptr, IM_NOALLOC_SCRATCH_BYTES, 0, s};
    t_arena = &a;
    rc = noalloc_reserve(ws, g, R, k);
    t_arena = nullptr;
    if (rc) return rc;
    if ((rc = validate(g, ws, s, ws->row32))) return rc;
    if ((rc = enqueue_prepare(g, R, seed, k, ws, s))) return rc;
    return enqueue_rounds(g, R, k, seeds_out, gains_out, nullptr, ws, s);
}

// ---------------------------------------------------------------------------
// Plans: the whole selection captured once into a HIP graph on a private
// workspace, replayed with one graph launch per selection
// ---------------------------------------------------------------------------
struct im_plan {
    im_workspace *ws = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" int im_plan_destroy(im_plan *p)
{
    if (!p) return IM_OK;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->ws) im_workspace_destroy(p->ws);
    delete p;
    return IM_OK;
}

struct TuneKey;
static int graph_signature(const im_graph *g, uint32_t R, im_workspace *ws, hipStream_t s, TuneKey *key);
static int apply_cached_schedule(const im_graph *g, uint32_t R, im_workspace *ws, hipStream_t s);

extern "C" int im_plan_create(const im_graph *g, uint32_t R, uint32_t k, uint64_t seed,
                              uint32_t *seeds_out, uint64_t *gains_out, void *stream,
                              im_plan **out)
{
    int rc;
    if (!out) return im_fail(IM_EINVAL, "null plan output");
    *out = nullptr;
    if ((rc = check_args(g, R))) return rc;
    if (k > g->n) return im_fail(IM_EINVAL, "k = %u exceeds n = %u", k, g->n);
    if (k && (!seeds_out || !gains_out)) return im_fail(IM_EINVAL, "null seeds or gains output");
    im_plan *p = new im_plan();
    if ((rc = im_workspace_create(&p->ws))) { delete p; return rc; }
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        im_plan_destroy(p);
        return im_fail(IM_EHIP, "hipStreamCreate failed");
    }
    // a schedule chosen by im_autotune for this graph carries over to the plan
    rc = check_and_reserve(g, R, k, p->ws, s);
    if (!rc) rc = apply_cached_schedule(g, R, p->ws, s);
    if (!rc) rc = check_and_reserve(g, R, k, p->ws, s);
    if (!rc) {
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            rc = im_fail(IM_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
        } else {
            // every replay takes the row offsets as they are at that time
            k_row32<<<grid_for((uint64_t)g->n + 1, 256), 256, 0, s>>>(g->row_ptr, g->n, p->ws->row32);
            rc = enqueue_prepare(g, R, seed, k, p->ws, s);
            if (!rc) rc = enqueue_rounds(g, R, k, seeds_out, gains_out, nullptr, p->ws, s);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(s, &graph);
            if (!rc && e != hipSuccess) rc = im_fail(IM_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
            p->graph = graph;
            if (!rc) {
                e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
                if (e != hipSuccess) rc = im_fail(IM_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
            }
        }
    }
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
    if (rc) {
        (void)hipGetLastError();
        im_plan_destroy(p);
        return rc;
    }
    p->ws->last_stream = (hipStream_t)stream;
    *out = p;
    return IM_OK;
}

extern "C" int im_plan_launch(im_plan *p, void *stream)
{
    if (!p || !p->exec) return im_fail(IM_EINVAL, "null plan");
    HIPCHK(hipGraphLaunch(p->exec, (hipStream_t)stream));
    p->ws->last_stream = (hipStream_t)stream;
    return IM_OK;
}

extern "C" int im_plan_stats(im_plan *p, im_stats *out)
{
    if (!p) return im_fail(IM_EINVAL, "null plan");
    return im_stats_get(p->ws, out);
}

extern "C" int im_profile_enable(im_workspace *ws, uint32_t mask)
{
    if (!ws) return im_fail(IM_EINVAL, "null workspace");
    ws->prof_mask = mask;
    for (int p = 0; p < IM_PH_COUNT; p++) ws->ev_used[p] = 0;
    return IM_OK;
}

extern "C" int im_profile_get(im_workspace *ws, im_profile *out)
{
    if (!ws || !out) return im_fail(IM_EINVAL, "null argument");
    memset(out, 0, sizeof(*out));
    HIPCHK(hipStreamSynchronize(ws->last_stream));
    HIPCHK(hipDeviceSynchronize());
    for (int p = 0; p < IM_PH_COUNT; p++) {
        size_t u = ws->ev_used[p] & ~(size_t)1;
        double tot = 0;
        ws->last_ms[p].clear();
        for (size_t i = 0; i < u; i += 2) {
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, ws->ev[p][i], ws->ev[p][i + 1]));
            tot += ms;
            ws->last_ms[p].push_back(ms);
        }
        out->ms[p] = tot;
        out->launches[p] = u / 2;
        ws->ev_used[p] = 0;
    }
    return IM_OK;
}

extern "C" int im_workspace_set(im_workspace *ws, int option, int64_t value)
{
    if (!ws) return im_fail(IM_EINVAL, "null workspace");
    switch (option) {
    case IM_OPT_HUB_DEGREE:
        if (value != 0 && (value < 16 || value > 0x7FFFFFFF))
            return im_fail(IM_EINVAL, "hub degree must be 0 (off) or in [16, 2^31)");
        ws->hub_deg = (uint32_t)value;
        return IM_OK;
    case IM_OPT_COOP_GAIN:
        if (value < 0) return im_fail(IM_EINVAL, "cooperative gain threshold must be >= 0");
        ws->coop_gain = (uint64_t)value;
        return IM_OK;
    case IM_OPT_MAX_SLOTS:
        if (value < 8 || value > 65536) return im_fail(IM_EINVAL, "slots must be in [8, 65536]");
        ws->max_slots = (uint32_t)value;
        return IM_OK;
    case IM_OPT_TIER1_SHAPE:
        if (value < 0 || value > 2) return im_fail(IM_EINVAL, "tier-1 shape must be 0, 1 or 2");
        ws->tier1_shape = (int)value;
        return IM_OK;
    case IM_OPT_TIER2_LANES:
        if (value != T2S_NT && value != T2_NT && value != T2W_NT)
            return im_fail(IM_EINVAL, "tier-2 lanes must be 64, 256 or 1024");
        ws->tier2_lanes = (uint32_t)value;
        return IM_OK;
    case IM_OPT_SPARSE_LISTS:
        if (value != 0 && value != 1) return im_fail(IM_EINVAL, "sparse lists must be 0 or 1");
        ws->sparse = (int)value;
        return IM_OK;
    case IM_OPT_FWD_GROUPS:
        if (value < 1 || value > 1024) return im_fail(IM_EINVAL, "forward workgroups per word must be in [1, 1024]");
        ws->fwd_per_word = (unsigned)value;
        return IM_OK;
    case IM_OPT_LEARNED_POLICY:
        if (value != 1 && value != 2) return im_fail(IM_EINVAL, "learned policy must be 1 or 2");
        ws->learned_policy = (int)value;
        return IM_OK;
    case IM_OPT_AFFECTED_GAIN:
        if (value < 0) return im_fail(IM_EINVAL, "affected-set gain threshold must be >= 0");
        ws->aff_gain = (uint64_t)value;
        return IM_OK;
    case IM_OPT_EVAL_SPLIT:
        if (value != 0 && value != 1 && value != 2 && value != 4 && value != 8)
            return im_fail(IM_EINVAL, "evaluation split must be 0 (automatic), 1, 2, 4 or 8");
        ws->eval_split = (uint32_t)value;
        return IM_OK;
    case IM_OPT_REV_SPLIT:
        if (value != 1 && value != 2 && value != 4)
            return im_fail(IM_EINVAL, "reverse split must be 1, 2 or 4");
        ws->rev_split = (uint32_t)value;
        return IM_OK;
    case IM_OPT_REV_FIRST_TIER:
        if (value != 0 && value != 1) return im_fail(IM_EINVAL, "reverse first tier must be 0 or 1");
        ws->rev_first = (uint32_t)value;
        return IM_OK;
    case IM_OPT_LAZY_BATCH:
        if (value < 1 || value > (int64_t)CELF_BMAX) return im_fail(IM_EINVAL, "lazy batch must be in [1, %u]", CELF_BMAX);
        ws->lazy_batch = (uint32_t)value;
        return IM_OK;
    case IM_OPT_LAZY_ENGINE:
        if (value < 0 || value > 2) return im_fail(IM_EINVAL, "lazy engine must be 0, 1 or 2");
        ws->lazy_engine = (int)value;
        return IM_OK;
    case IM_OPT_PAIR_COINS:
        if (value != 0 && value != 1) return im_fail(IM_EINVAL, "pair coins must be 0 or 1");
        ws->pair_coins = (int)value;
        return IM_OK;
    case IM_OPT_LIVE_EDGE:
        if (value != 0 && value != 1) return im_fail(IM_EINVAL, "live-edge model must be 0 or 1");
        ws->live_edge = (int)value;
        return IM_OK;
    default:
        return im_fail(IM_EINVAL, "unknown option %d", option);
    }
}

extern "C" int im_profile_launches(im_workspace *ws, int phase, float *ms_out, uint32_t max,
                                   uint32_t *count)
{
    if (!ws || !count || phase < 0 || phase >= IM_PH_COUNT) return im_fail(IM_EINVAL, "bad argument");
    const std::vector<float> &v = ws->last_ms[phase];
    *count = (uint32_t)v.size();
    for (uint32_t i = 0; i < max && i < v.size(); i++) ms_out[i] = v[i];
    return IM_OK;
}

// ---------------------------------------------------------------------------
// Batches: many independent instances selected together
// ---------------------------------------------------------------------------
static int reserve_batch(im_workspace *ws, uint32_t count, uint64_t N, uint64_t M)
{
    int rc;
    if (count > ws->cap_count) {
        if ((rc = dalloc(&ws->b_u32, 4ull * (count + 1))) || (rc = dalloc(&ws->b_u64, 2ull * (count + 1))) ||
            (rc = dalloc(&ws->b_desc, count)))
            return rc;
        if (ws->b_host) (void)hipHostFree(ws->b_host);
        ws->b_host = nullptr;
        size_t bytes = (4ull * (count + 1)) * 4 + (2ull * (count + 1)) * 8 + (uint64_t)count * sizeof(InstDesc);
        HIPCHK(hipHostMalloc(&ws->b_host, bytes, hipHostMallocDefault));
        ws->cap_count = count;
    }
    if (N > ws->cap_bn) {
        if ((rc = dalloc(&ws->b_node_inst, N))) return rc;
        ws->cap_bn = N;
    }
    if (M > ws->cap_bm || !ws->b_mcol) {
        if ((rc = dalloc(&ws->b_mcol, M)) || (rc = dalloc(&ws->b_mprob, M))) return rc;
        ws->cap_bm = M;
    }
    return IM_OK;
}

// merge the instances' CSRs into the workspace's block-diagonal graph
// (instance tables already on the device)
static void launch_merge(const im_instance *inst, uint32_t count, im_workspace *ws, hipStream_t s)
{
    uint64_t maxw = 0;
    for (uint32_t i = 0; i < count; i++)
        maxw = std::max<uint64_t>(maxw, std::max<uint64_t>((uint64_t)inst[i].g.n + 1, inst[i].g.m));
    dim3 grid(grid_for(maxw, 256, 256), count);
    k_batch_merge<<<grid, 256, 0, s>>>(ws->b_desc, ws->err, ws->row32, ws->b_mcol, ws->b_mprob,
                                       ws->b_node_inst);
}

// Lay `count` instances out as one block-diagonal graph in the workspace:
// validate them, stage the instance tables, merge the CSRs. On success
// ws->batch describes the batch and *mg the merged graph (the caller resets
// ws->batch afterwards). Synchronous.
static int batch_setup(const im_instance *inst, uint32_t count, bool need_out, im_workspace *ws,
                       hipStream_t s, im_graph *mg, uint32_t *Rmax_out, uint32_t *kmax_out)
{
    int rc;
    uint64_t N = 0, M = 0, K = 0;
    uint32_t Rmax = 0, kmax = 0, nmax = 0;
    if (ws->live_edge || ws->pair_coins)
        return im_fail(IM_EINVAL, "batches draw one coin per stored arc (independent cascade)");
    for (uint32_t i = 0; i < count; i++) {
        if ((rc = check_args(&inst[i].g, inst[i].R)))
            return im_fail(rc, "instance %u: %s", i, g_err.c_str());
        if (inst[i].k > inst[i].g.n) return im_fail(IM_EINVAL, "instance %u: k exceeds n", i);
        nmax = std::max(nmax, inst[i].g.n);
        N += inst[i].g.n;
        M += inst[i].g.m;
        K += inst[i].k;
        Rmax = std::max(Rmax, inst[i].R);
        kmax = std::max(kmax, inst[i].k);
    }
    if (N >= 0xFFFFFFFFull) return im_fail(IM_EINVAL, "batch has %llu nodes; must be < 2^32 - 1", (unsigned long long)N);
    if (M >= (1ull << 32)) return im_fail(IM_EINVAL, "batch has %llu arcs; must be < 2^32", (unsigned long long)M);
    if (K && !need_out) return im_fail(IM_EINVAL, "null seeds or gains output");
    const uint32_t W = (Rmax + 63) / 64;
    ws->batch.count = count;  // sizes the per-round key arrays
    rc = ws_reserve(ws, (uint32_t)N, M, W, kmax, nmax);
    ws->batch.count = 1;
    if (!rc) rc = reserve_batch(ws, count, N, M);
    if (rc) return rc;
    // per-instance tables, staged in pinned memory
    uint32_t *hu = (uint32_t *)ws->b_host;              // R, k, kpre, node_off
    uint64_t *h64 = (uint64_t *)(hu + 4ull * (count + 1));  // arc_off, seed
    InstDesc *hd = (InstDesc *)(h64 + 2ull * (count + 1));
    uint64_t no = 0, ao = 0, kp = 0;
    for (uint32_t i = 0; i < count; i++) {
        if (inst[i].g.m && (!inst[i].g.col || !inst[i].g.prob))
            return im_fail(IM_EINVAL, "instance %u: null col or prob", i);
        if (!inst[i].g.row_ptr) return im_fail(IM_EINVAL, "instance %u: null row_ptr", i);
        hu[i] = inst[i].R;
        hu[(count + 1) + i] = inst[i].k;
        hu[2 * (count + 1) + i] = (uint32_t)kp;
        hu[3 * (count + 1) + i] = (uint32_t)no;
        h64[i] = ao;
        h64[(count + 1) + i] = inst[i].seed;
        hd[i].row_ptr = inst[i].g.row_ptr;
        hd[i].col = inst[i].g.col;
        hd[i].prob = inst[i].g.prob;
        hd[i].m = inst[i].g.m;
        hd[i].arc_off = ao;
        hd[i].n = inst[i].g.n;
        hd[i].node_off = (uint32_t)no;
        no += inst[i].g.n;
        ao += inst[i].g.m;
        kp += inst[i].k;
    }
    hu[3 * (count + 1) + count] = (uint32_t)no;
    h64[count] = ao;
    HIPCHK(hipMemcpyAsync(ws->b_u32, hu, (4ull * (count + 1)) * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ws->b_u64, h64, (2ull * (count + 1)) * 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ws->b_desc, hd, (uint64_t)count * sizeof(InstDesc), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(ws->err, 0, sizeof(uint32_t), s));
    launch_merge(inst, count, ws, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(ws->host_err, ws->err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (*ws->host_err)
        return im_fail(IM_EINVAL, "a batch instance failed validation (flags 0x%x)", *ws->host_err);
    Batch b;
    b.count = count;
    b.node_inst = ws->b_node_inst;
    b.R = ws->b_u32;
    b.k = ws->b_u32 + (count + 1);
    b.kpre = ws->b_u32 + 2 * (count + 1);
    b.node_off = ws->b_u32 + 3 * (count + 1);
    b.arc_off = ws->b_u64;
    b.seed = ws->b_u64 + (count + 1);
    ws->batch = b;
    mg->n = (uint32_t)N;
    mg->m = M;
    mg->row_ptr = nullptr;
    mg->col = ws->b_mcol;
    mg->prob = ws->b_mprob;
    *Rmax_out = Rmax;
    *kmax_out = kmax;
    return IM_OK;
}

static const Batch kSingle = {1, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};

extern "C" int im_select_batch(const im_instance *inst, uint32_t count, uint32_t *seeds_out,
                               uint64_t *gains_out, im_workspace *ws, void *stream)
{
    int rc;
    if (!inst || !ws) return im_fail(IM_EINVAL, "null instances or workspace");
    if (count == 0) return IM_OK;
    if (count == 1)
        return im_select(&inst[0].g, inst[0].R, inst[0].k, inst[0].seed, seeds_out, gains_out,
                         nullptr, ws, stream);
    hipStream_t s = (hipStream_t)stream;
    im_graph mg;
    uint32_t Rmax = 0, kmax = 0;
    rc = batch_setup(inst, count, seeds_out && gains_out, ws, s, &mg, &Rmax, &kmax);
    if (!rc) {
        PhaseTimer pt(ws, IM_PH_CALL, s);
        rc = enqueue_prepare(&mg, Rmax, 0, kmax, ws, s);
        if (!rc) rc = enqueue_rounds(&mg, Rmax, kmax, seeds_out, gains_out, nullptr, ws, s);
    }
    ws->batch = kSingle;
    return rc;
}

extern "C" int im_plan_create_batch(const im_instance *inst, uint32_t count, uint32_t *seeds_out,
                                    uint64_t *gains_out, im_workspace *tuned, void *stream,
                                    im_plan **out)
{
    int rc;
    if (!out) return im_fail(IM_EINVAL, "null plan output");
    *out = nullptr;
    if (!inst || count < 2) return im_fail(IM_EINVAL, "a batch plan needs at least two instances");
    im_plan *p = new im_plan();
    if ((rc = im_workspace_create(&p->ws))) { delete p; return rc; }
    if (tuned) {
        // copy the caller's engine schedule (e.g. set by im_autotune_batch)
        p->ws->hub_deg = tuned->hub_deg;
        p->ws->tier1_shape = tuned->tier1_shape;
        p->ws->tier2_lanes = tuned->tier2_lanes;
        p->ws->max_slots = tuned->max_slots;
        p->ws->coop_gain = tuned->coop_gain;
        p->ws->sparse = tuned->sparse;
        p->ws->fwd_per_word = tuned->fwd_per_word;
        p->ws->rev_split = tuned->rev_split;
        p->ws->rev_first = tuned->rev_first;
    }
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        im_plan_destroy(p);
        return im_fail(IM_EHIP, "hipStreamCreate failed");
    }
    im_graph mg;
    uint32_t Rmax = 0, kmax = 0;
    // validation and the instance tables once, synchronously; the capture
    // merges the instances again, so every replay reads their current arrays
    rc = batch_setup(inst, count, seeds_out && gains_out, p->ws, s, &mg, &Rmax, &kmax);
    if (!rc) {
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            rc = im_fail(IM_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
        } else {
            launch_merge(inst, count, p->ws, s);
            rc = enqueue_prepare(&mg, Rmax, 0, kmax, p->ws, s);
            if (!rc) rc = enqueue_rounds(&mg, Rmax, kmax, seeds_out, gains_out, nullptr, p->ws, s);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(s, &graph);
            if (!rc && e != hipSuccess) rc = im_fail(IM_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
            p->graph = graph;
            if (!rc) {
                e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
                if (e != hipSuccess) rc = im_fail(IM_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
            }
        }
    }
    p->ws->batch = kSingle;
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
    if (rc) {
        (void)hipGetLastError();
        im_plan_destroy(p);
        return rc;
    }
    p->ws->last_stream = (hipStream_t)stream;
    *out = p;
    return IM_OK;
}

// ---------------------------------------------------------------------------
// A8: schedule autotuning. A schedule (hub threshold, tier-1 table, tier-2
// lanes and slots) never changes a result, only where each reachability
// task runs; the best one depends on the reach-size profile of the graph.
// Candidates are timed on a trial -- the initial reach counts and the first
// greedy rounds, which exercise every engine -- and the fastest is kept,
// cached per graph signature.
// ---------------------------------------------------------------------------
struct Schedule {
    int32_t hub_degree, tier1_shape, tier2_lanes, max_slots, coop_forward;
};
static const Schedule kSchedules[] = {
    {256, 0, 256, 256, 1},  {256, 0, 1024, 256, 1}, {256, 0, 256, 2048, 1},
    {256, 0, 256, 1024, 1}, {256, 0, 1024, 1024, 1}, {256, 0, 1024, 256, 0},
    {256, 0, 256, 2048, 0}, {256, 1, 1024, 256, 1}, {256, 0, 64, 8192, 1},
    {256, 0, 64, 8192, 0},
};
constexpr int N_SCHEDULES = sizeof(kSchedules) / sizeof(kSchedules[0]);
constexpr uint32_t TUNE_ROUNDS = 4;   // greedy rounds in a trial

static void apply_schedule(im_workspace *ws, const Schedule &c)
{
    ws->hub_deg = (uint32_t)c.hub_degree;
    ws->tier1_shape = c.tier1_shape;
    ws->tier2_lanes = (uint32_t)c.tier2_lanes;
    ws->max_slots = (uint32_t)c.max_slots;
    ws->coop_gain = c.coop_forward ? 0ull : ~0ull;
}

// signature of a graph: sizes plus a checksum of its arcs (heads and probabilities)
__global__ void k_signature(const uint32_t *col, const float *prob, uint64_t m,
                            unsigned long long *out)
{
    unsigned long long h = 0;
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < m;
         e += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t x = ((uint64_t)col[e] << 32) ^ __float_as_uint(prob[e]) ^ (e * IM_GOLDEN);
        h += sm64_finalise(x);
    }
    h = wave_sum_u64(h);
    if ((threadIdx.x & 63) == 0 && h) atomicAdd(out, h);
}

struct TuneKey {
    uint64_t n, m, R, sum;
    bool operator==(const TuneKey &o) const { return n == o.n && m == o.m && R == o.R && sum == o.sum; }
};
static std::vector<std::pair<TuneKey, im_tuning>> g_tune_cache;
static std::mutex g_tune_mu;   // guards g_tune_cache and the cache file

// The cache file named by IM_TUNE_CACHE (if set): one line per graph
// signature, "im-tune-4 n m R sum hub tier1 lanes slots coop affected fwd split first ms".
// Lines that do not parse are ignored; the last line for a key wins.
static const char *tune_file() { return getenv("IM_TUNE_CACHE"); }

static void tune_file_lookup(const TuneKey &key)
{
    const char *path = tune_file();
    if (!path || !*path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char line[512];
    while (fgets(line, sizeof line, f)) {
        unsigned long long n, m, R, sum, aff;
        int hub, t1, lanes, slots, coop, fwd, split, first;
        float ms;
        if (sscanf(line, "im-tune-4 %llu %llu %llu %llu %d %d %d %d %d %llu %d %d %d %f", &n, &m, &R,
                   &sum, &hub, &t1, &lanes, &slots, &coop, &aff, &fwd, &split, &first, &ms) != 14)
            continue;
        const TuneKey k{n, m, R, sum};
        if (!(k == key)) continue;
        im_tuning t;
        memset(&t, 0, sizeof t);
        t.hub_degree = hub; t.tier1_shape = t1; t.tier2_lanes = lanes; t.max_slots = slots;
        t.coop_forward = coop; t.affected_gain = aff; t.fwd_groups = fwd; t.rev_split = split;
        t.rev_first_tier = first; t.ms = ms; t.tried = 0;
        bool found = false;
        for (auto &kv : g_tune_cache)
            if (kv.first == k) { kv.second = t; found = true; }
        if (!found) g_tune_cache.push_back({k, t});
    }
    fclose(f);
}

static void tune_file_append(const TuneKey &k, const im_tuning &t)
{
    const char *path = tune_file();
    if (!path || !*path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;   // the in-process cache still holds the choice
    fprintf(f, "im-tune-4 %llu %llu %llu %llu %d %d %d %d %d %llu %d %d %d %.4f\n", (unsigned long long)k.n,
            (unsigned long long)k.m, (unsigned long long)k.R, (unsigned long long)k.sum, t.hub_degree,
            t.tier1_shape, t.tier2_lanes, t.max_slots, t.coop_forward,
            (unsigned long long)t.affected_gain, t.fwd_groups, t.rev_split, t.rev_first_tier, t.ms);
    fclose(f);
}

static int graph_signature(const im_graph *g, uint32_t R, im_workspace *ws, hipStream_t s, TuneKey *key)
{
    fill<unsigned long long>(ws->stats, 1, 0ull, s);
    if (g->m)
        k_signature<<<grid_for(g->m, 256, 4096), 256, 0, s>>>(g->col, g->prob, g->m, ws->stats);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(ws->host_stats, ws->stats, sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *key = TuneKey{g->n, g->m, R, ws->host_stats[0]};
    return IM_OK;
}

// time `prepare` (everything up to and including the initial counts) under
// each candidate schedule; keep the fastest on the workspace
template <typename Prep>
static int tune(im_workspace *ws, hipStream_t s, Prep prep, im_tuning *best)
{
    int rc;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const uint32_t saved_mask = ws->prof_mask;
    ws->prof_mask = 0;
    float best_ms = -1.0f;
    int best_i = 0;
    for (int i = 0; i < N_SCHEDULES; i++) {
        apply_schedule(ws, kSchedules[i]);
        float ms_min = -1.0f;
        for (int rep = 0; rep < 2; rep++) {
            if ((rc = prep(true))) break;  // reservation and validation (synchronous)
            HIPCHK(hipEventRecord(e0, s));
            rc = prep(false);
            HIPCHK(hipEventRecord(e1, s));
            HIPCHK(hipEventSynchronize(e1));
            if (rc) break;
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            if (ms_min < 0 || ms < ms_min) ms_min = ms;
        }
        if (rc) break;
        if (best_ms < 0 || ms_min < best_ms) { best_ms = ms_min; best_i = i; }
    }
    ws->prof_mask = saved_mask;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    apply_schedule(ws, kSchedules[best_i]);
    best->hub_degree = kSchedules[best_i].hub_degree;
    best->tier1_shape = kSchedules[best_i].tier1_shape;
    best->tier2_lanes = kSchedules[best_i].tier2_lanes;
    best->max_slots = kSchedules[best_i].max_slots;
    best->coop_forward = kSchedules[best_i].coop_forward;
    best->ms = best_ms;
    best->tried = N_SCHEDULES;
    best->affected_gain = 0;
    best->fwd_groups = (int32_t)ws->fwd_per_word;
    best->rev_split = (int32_t)ws->rev_split;
    best->rev_first_tier = (int32_t)ws->rev_first;
    return IM_OK;
}

// The per-round update strategy under the chosen schedule: reverse decrements
// in every round, or the affected-set recompute below one of three gain
// thresholds. `run(kt)` enqueues a trial of kt rounds (after its reservation).
constexpr uint32_t TUNE_AFF_ROUNDS = 16;

template <typename Run>
static int tune_affected(uint64_t nR, im_workspace *ws, hipStream_t s, Run run, im_tuning *best)
{
    int rc = IM_OK;
    const uint64_t cand[4] = {0ull, nR / 4096, nR / 256, 1ull << 62};
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const uint32_t saved_mask = ws->prof_mask;
    ws->prof_mask = 0;
    float best_ms = -1.0f;
    uint64_t best_t = 0;
    for (int i = 0; i < 4 && !rc; i++) {
        if (i > 0 && cand[i] == cand[i - 1]) continue;
        ws->aff_gain = cand[i];
        float ms_min = -1.0f;
        for (int rep = 0; rep < 2 && !rc; rep++) {
            if ((rc = run(true))) break;
            if (hipEventRecord(e0, s) != hipSuccess) { rc = IM_EHIP; break; }
            rc = run(false);
            if (!rc && hipEventRecord(e1, s) != hipSuccess) rc = IM_EHIP;
            if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = IM_EHIP;
            float ms = 0;
            if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = IM_EHIP;
            if (!rc && (ms_min < 0 || ms < ms_min)) ms_min = ms;
        }
        if (!rc && (best_ms < 0 || ms_min < best_ms)) { best_ms = ms_min; best_t = cand[i]; }
    }
    ws->prof_mask = saved_mask;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ws->aff_gain = best_t;
    if (rc) return rc == IM_EHIP ? im_fail(IM_EHIP, "event timing of an update-strategy trial failed") : rc;
    best->affected_gain = best_t;
    best->ms = best_ms;
    best->tried += 4;
    return IM_OK;
}

// One more knob under the chosen schedule: each value of `cand` is set with
// set(v) and timed on run (two trials, the faster counts); the fastest is
// set and returned in *chosen.
template <typename Run, typename Set>
static int tune_knob(const uint32_t *cand, int ncand, im_workspace *ws, hipStream_t s, Run run, Set set,
                     uint32_t *chosen, im_tuning *best)
{
    int rc = IM_OK;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const uint32_t saved_mask = ws->prof_mask;
    ws->prof_mask = 0;
    float best_ms = -1.0f;
    uint32_t best_v = cand[0];
    for (int i = 0; i < ncand && !rc; i++) {
        set(cand[i]);
        float ms_min = -1.0f;
        for (int rep = 0; rep < 2 && !rc; rep++) {
            if ((rc = run(true))) break;
            if (hipEventRecord(e0, s) != hipSuccess) { rc = IM_EHIP; break; }
            rc = run(false);
            if (!rc && hipEventRecord(e1, s) != hipSuccess) rc = IM_EHIP;
            if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = IM_EHIP;
            float ms = 0;
            if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = IM_EHIP;
            if (!rc && (ms_min < 0 || ms < ms_min)) ms_min = ms;
        }
        if (!rc && (best_ms < 0 || ms_min < best_ms)) { best_ms = ms_min; best_v = cand[i]; }
    }
    ws->prof_mask = saved_mask;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    set(best_v);
    if (rc) return rc == IM_EHIP ? im_fail(IM_EHIP, "event timing of a schedule trial failed") : rc;
    *chosen = best_v;
    best->ms = best_ms;
    best->tried += (uint32_t)ncand;
    return IM_OK;
}

// The width of the cooperative forward search (workgroups per snapshot
// word): wider grids expand large frontiers faster, narrower ones pay less
// per grid barrier. The split of last-tier reverse tasks into bit groups:
// more workgroups per large search, more task starts. The first tier of
// the reverse step: tier 0 finishes small tasks in small tables, tier 1
// saves a launch and the hand-over of the larger tasks.
static const uint32_t kFwdGroups[] = {16, 32};
static const uint32_t kRevSplits[] = {1, 2};
static const uint32_t kRevFirst[] = {0, 1};

template <typename Run>
static int tune_fwd_and_split(im_workspace *ws, hipStream_t s, Run run, im_tuning *best, bool fwd)
{
    int rc;
    uint32_t v;
    if (fwd && ws->coop_gain == 0) {   // (the per-word forward search has no grid)
        if ((rc = tune_knob(kFwdGroups, 2, ws, s, run, [&](uint32_t g) { ws->fwd_per_word = g; }, &v, best)))
            return rc;
        best->fwd_groups = (int32_t)v;
    }
    if ((rc = tune_knob(kRevSplits, 2, ws, s, run, [&](uint32_t g) { ws->rev_split = g; }, &v, best)))
        return rc;
    best->rev_split = (int32_t)v;
    if ((rc = tune_knob(kRevFirst, 2, ws, s, run, [&](uint32_t t) { ws->rev_first = t; }, &v, best)))
        return rc;
    best->rev_first_tier = (int32_t)v;
    return IM_OK;
}

static int tune_cached(const TuneKey &key, im_workspace *ws, im_tuning *out, bool *hit)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    bool mem = false;
    for (auto &kv : g_tune_cache) mem = mem || kv.first == key;
    if (!mem) tune_file_lookup(key);
    for (auto &kv : g_tune_cache)
        if (kv.first == key) {
            const im_tuning &t = kv.second;
            apply_schedule(ws, Schedule{t.hub_degree, t.tier1_shape, t.tier2_lanes, t.max_slots,
                                        t.coop_forward});
            ws->aff_gain = t.affected_gain;
            if (t.fwd_groups > 0) ws->fwd_per_word = (uint32_t)t.fwd_groups;
            if (t.rev_split > 0) ws->rev_split = (uint32_t)t.rev_split;
            if (t.rev_first_tier == 0 || t.rev_first_tier == 1) ws->rev_first = (uint32_t)t.rev_first_tier;
            if (out) { *out = t; out->tried = 0; }
            *hit = true;
            return IM_OK;
        }
    *hit = false;
    return IM_OK;
}

static int apply_cached_schedule(const im_graph *g, uint32_t R, im_workspace *ws, hipStream_t s)
{
    TuneKey key;
    int rc = graph_signature(g, R, ws, s, &key);
    if (rc) return rc;
    bool hit;
    return tune_cached(key, ws, nullptr, &hit);
}

extern "C" int im_autotune(const im_graph *g, uint32_t R, uint64_t seed, im_workspace *ws,
                           void *stream, im_tuning *out)
{
    int rc;
    if ((rc = check_args(g, R))) return rc;
    if (!ws) return im_fail(IM_EINVAL, "null workspace");
    hipStream_t s = (hipStream_t)stream;
    if ((rc = check_and_reserve(g, R, 0, ws, s))) return rc;
    TuneKey key;
    if ((rc = graph_signature(g, R, ws, s, &key))) return rc;
    bool hit;
    tune_cached(key, ws, out, &hit);
    if (hit) return IM_OK;
    im_tuning best;
    // the trial: initial counts and the first few greedy rounds (whose
    // reverse steps are the largest of the selection), under reverse
    // decrements; then the update strategy over a longer trial
    const uint32_t kt = std::min<uint32_t>(TUNE_ROUNDS, g->n);
    const uint32_t ka = std::min<uint32_t>(TUNE_AFF_ROUNDS, g->n);
    uint32_t *sd = nullptr;
    uint64_t *gd = nullptr;
    if ((rc = dalloc(&sd, ka)) || (rc = dalloc(&gd, ka))) { dfree(sd); return rc; }
    ws->aff_gain = 0;
    auto prep = [&](bool reserve) -> int {
        if (reserve) return check_and_reserve(g, R, kt, ws, s);
        int r = enqueue_prepare(g, R, seed, kt, ws, s);
        return r ? r : enqueue_rounds(g, R, kt, sd, gd, nullptr, ws, s);
    };
    rc = tune(ws, s, prep, &best);
    auto run = [&](bool reserve) -> int {
        if (reserve) return check_and_reserve(g, R, ka, ws, s);
        int r = enqueue_prepare(g, R, seed, ka, ws, s);
        return r ? r : enqueue_rounds(g, R, ka, sd, gd, nullptr, ws, s);
    };
    if (!rc) rc = tune_affected((uint64_t)g->n * R, ws, s, run, &best);
    if (!rc) rc = tune_fwd_and_split(ws, s, run, &best, true);
    (void)hipStreamSynchronize(s);
    dfree(sd);
    dfree(gd);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune_cache.push_back({key, best});
        tune_file_append(key, best);
    }
    if (out) *out = best;
    return IM_OK;
}

extern "C" int im_autotune_batch(const im_instance *inst, uint32_t count, im_workspace *ws,
                                 void *stream, im_tuning *out)
{
    int rc;
    if (!inst || !ws || count == 0) return im_fail(IM_EINVAL, "null or empty instances");
    if (count == 1) return im_autotune(&inst[0].g, inst[0].R, inst[0].seed, ws, stream, out);
    hipStream_t s = (hipStream_t)stream;
    im_graph mg;
    uint32_t Rmax = 0, kmax = 0;
    im_tuning best;
    uint64_t K = 0;
    for (uint32_t i = 0; i < count; i++) K += inst[i].k;
    uint32_t *sd = nullptr;
    uint64_t *gd = nullptr;
    if ((rc = dalloc(&sd, K)) || (rc = dalloc(&gd, K))) { dfree(sd); return rc; }
    auto prep = [&](bool reserve) -> int {
        if (reserve) {
            ws->batch = kSingle;
            return batch_setup(inst, count, true, ws, s, &mg, &Rmax, &kmax);
        }
        const uint32_t kt = std::min<uint32_t>(TUNE_ROUNDS, kmax);
        int r = enqueue_prepare(&mg, Rmax, 0, kt, ws, s);
        return r ? r : enqueue_rounds(&mg, Rmax, kt, sd, gd, nullptr, ws, s);
    };
    rc = tune(ws, s, prep, &best);
    if (!rc) rc = tune_fwd_and_split(ws, s, prep, &best, false);
    (void)hipStreamSynchronize(s);
    dfree(sd);
    dfree(gd);
    ws->batch = kSingle;
    if (rc) return rc;
    if (out) *out = best;
    return IM_OK;
}

// Lazy-path tuning: the evaluation engine and the batch size, timed on the
// lazy selection's first rounds. The early rounds hold the largest searches
// and favour small batches, the later ones favour batches that cover a
// round's must-evaluate set at once, so the trial runs the whole selection
// up to 64 rounds.
constexpr uint32_t LAZY_TUNE_ROUNDS = 64;
static const int32_t kLazyEngines[] = {2, 0};
static const uint32_t kLazyBatches[] = {1, 2, 4, 8, 16};

extern "C" int im_autotune_lazy(const im_graph *g, uint32_t R, uint32_t k, uint64_t seed,
                                const im_mlp *model, im_workspace *ws, void *stream,
                                im_lazy_tuning *out)
{
    int rc;
    if ((rc = check_args(g, R))) return rc;
    if (!ws) return im_fail(IM_EINVAL, "null workspace");
    if (k > g->n) return im_fail(IM_EINVAL, "k = %u exceeds n = %u", k, g->n);
    hipStream_t s = (hipStream_t)stream;
    const uint32_t kt = std::min<uint32_t>(std::max<uint32_t>(k, 2u), std::min<uint32_t>(LAZY_TUNE_ROUNDS, g->n));
    if (g->n == 0 || kt < 2) {
        if (out) { out->engine = ws->lazy_engine; out->batch = ws->lazy_batch; out->ms = 0; out->tried = 0; }
        return IM_OK;
    }
    uint32_t *sd = nullptr;
    uint64_t *gd = nullptr;
    if ((rc = dalloc(&sd, kt)) || (rc = dalloc(&gd, kt))) { dfree(sd); return rc; }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        dfree(sd); dfree(gd);
        if (e0) (void)hipEventDestroy(e0);
        return im_fail(IM_EHIP, "hipEventCreate failed");
    }
    const uint32_t saved_mask = ws->prof_mask;
    ws->prof_mask = 0;
    float best_ms = -1.0f;
    int32_t best_e = ws->lazy_engine;
    uint32_t best_b = ws->lazy_batch, tried = 0;
    for (int32_t eng : kLazyEngines) {
        for (uint32_t B : kLazyBatches) {
            ws->lazy_engine = eng;
            float ms_min = -1.0f;
            for (int rep = 0; rep < 2 && !rc; rep++) {
                if ((rc = check_and_reserve(g, R, kt, ws, s))) break;
                if ((rc = (int)(hipEventRecord(e0, s) != hipSuccess ? IM_EHIP : IM_OK))) break;
                rc = enqueue_prepare(g, R, seed, kt, ws, s, model ? PREP_INDEG : PREP_FORWARD);
                if (!rc) rc = select_lazy(g, R, kt, B, model, sd, gd, ws, s);
                if (!rc && hipEventRecord(e1, s) != hipSuccess) rc = IM_EHIP;
                if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = IM_EHIP;
                float ms = 0;
                if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = IM_EHIP;
                if (!rc && (ms_min < 0 || ms < ms_min)) ms_min = ms;
            }
            if (rc) break;
            tried++;
            if (best_ms < 0 || ms_min < best_ms) { best_ms = ms_min; best_e = eng; best_b = B; }
        }
        if (rc) break;
    }
    ws->prof_mask = saved_mask;
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    dfree(sd);
    dfree(gd);
    ws->lazy_engine = best_e;
    ws->lazy_batch = best_b;
    if (rc) return rc == IM_EHIP ? im_fail(IM_EHIP, "event timing of a lazy trial failed") : rc;
    if (out) { out->engine = best_e; out->batch = best_b; out->ms = best_ms; out->tried = tried; }
    return IM_OK;
}

extern "C" int im_select_lazy(const im_graph *g, uint32_t R, uint32_t k, uint64_t seed,
                              uint32_t batch, const im_mlp *model, uint32_t *seeds_out,
                              uint64_t *gains_out, im_workspace *ws, void *stream)
{
    int rc;
    if ((rc = check_args(g, R))) return rc;
    if (!ws) return im_fail(IM_EINVAL, "null workspace");
    if (k > g->n) return im_fail(IM_EINVAL, "k = %u exceeds n = %u", k, g->n);
    if (k && (!seeds_out || !gains_out)) return im_fail(IM_EINVAL, "null seeds or gains output");
    if (batch == 0) batch = ws->lazy_batch;   // the workspace's (tuned) batch
    if (batch > CELF_BMAX)
        return im_fail(IM_EINVAL, "batch = %u must be in [0, %u]", batch, CELF_BMAX);
    if ((uint64_t)batch * ((R + 63) / 64) >= (1ull << 32)) return im_fail(IM_EINVAL, "batch too large");
    hipStream_t s = (hipStream_t)stream;
    PhaseTimer pt(ws, IM_PH_CALL, s);
    if ((rc = prepare(g, R, seed, k, ws, s, model ? PREP_INDEG : PREP_FORWARD))) return rc;
    if (g->n == 0 || k == 0) return IM_OK;
    return select_lazy(g, R, k, batch, model, seeds_out, gains_out, ws, s);
}

extern "C" int im_node_features(const im_graph *g, float *feat_out, im_workspace *ws, void *stream)
{
    int rc;
    if (!g || !ws || (g->n && !feat_out)) return im_fail(IM_EINVAL, "null argument");
    if ((rc = check_args(g, 1))) return rc;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = check_and_reserve(g, 1, 0, ws, s))) return rc;
    if (g->n == 0) return IM_OK;
    build_reverse(g, ws, s);
    launch_features(ws->row32, g->col, g->prob, ws->in_row, g->n, feat_out, s);
    HIPCHK(hipGetLastError());
    ws->last_stream = s;
    return IM_OK;
}
