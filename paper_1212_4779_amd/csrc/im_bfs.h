// im_bfs.h -- word-parallel reachability engines.
//
// One reachability task = one start node and one 64-bit snapshot word w.
// The state of a task is a map x -> reach[x] (bit b set: x is reached in
// snapshot 64w+b). Propagation over arc e = (x -> v) is
//     reach[v] |= delta[x] & mask[w][e]   (& ~prune[w][v] when pruning)
// level by level, where delta[x] holds the bits x gained since it was last
// expanded. The fixpoint is the union over the word's snapshots of the
// reachable sets (Sec. 3.1 snapshot spread), computed for 64 snapshots with
// one 8-byte mask read per arc. Results depend only on the fixpoint, never on
// the order in which lanes apply their atomic ORs.
//
// Three engine tiers share this definition and hand tasks down a chain of
// queues:
//   tier 0  k_lds_bfs with a 64-lane workgroup: T small tasks per
//           wavefront, each in an LDS open-addressing table of CS entries;
//   tier 1  k_lds_bfs with a 256-lane workgroup and larger tables, no degree
//           limit (hub expansions stream through all lanes);
//   tier 2  k_block_bfs: one task per workgroup in dense per-slot global
//           arrays of length n (no size limit).
// A task that fills its table (more than LIM entries) or meets a node of
// degree > DMAX is abandoned whole and queued for the next tier.
#pragma once

#include "im_device.h"

enum { MODE_COUNT = 0, MODE_DEC = 1 };

// statistics slots (uint64 counters in device memory)
enum {
    ST_TRAV_INIT = 0, ST_TRAV_FWD, ST_TRAV_REV, ST_TRAV_EVAL,
    ST_RELAX_FWD, ST_TASKS_REV, ST_DECREMENTS, ST_CELF_EVALS,
    ST_TIER_BASE = 8,   // + pass*12 + tier*4 + field
    ST_FWD_LEVELS = 44, ST_FWD_ENTRIES = 45, ST_CELF_BATCHES = 46, ST_CELF_FALLBACKS = 47,
    ST_MAXLV_BASE = 48,   // + pass*3 + tier: most search levels one workgroup ran in a launch
    ST_COUNT = 64
};
enum { PASS_INIT = 0, PASS_REV = 1, PASS_EVAL = 2 };
enum { F_RELAX = 0, F_REACHED = 1, F_ARCS = 2, F_OVF = 3 };

__host__ __device__ constexpr int st_tier(int pass, int tier, int field)
{
    return ST_TIER_BASE + pass * 12 + tier * 4 + field;
}

// The counters are kept in ST_STRIPES copies of ST_COUNT slots; the engines,
// whose every workgroup adds its totals at the end, spread those atomics over
// the copies by workgroup (the reader sums the copies, or takes their maximum
// for the ST_MAXLV slots). Other kernels add to copy 0.
constexpr int ST_STRIPES = 32;

__device__ __forceinline__ void stat_add(unsigned long long *st, int idx, unsigned long long v)
{
    atomicAdd(&st[(blockIdx.x % ST_STRIPES) * ST_COUNT + idx], v);
}

__device__ __forceinline__ void stat_max(unsigned long long *st, int idx, unsigned long long v)
{
    atomicMax(&st[(blockIdx.x % ST_STRIPES) * ST_COUNT + idx], v);
}

// Per-snapshot adjacency of heavy nodes (degree >= the hub threshold), for
// expanding them with a sparse delta: for hub index h and word w, the heads of
// the arcs live in snapshot 64w+b are adj[off[(h*W+w)*65+b] .. off[(h*W+w)*65+b+1]).
// slot[x] is x's hub index, or IM_EMPTY for nodes expanded through the masks.
struct HubLists {
    const uint32_t *slot;   // [n], nullptr: no hub lists
    const uint32_t *off;    // [nhub][W][65]
    const uint32_t *adj;
    uint32_t min_deg;       // nodes with fewer arcs have no lists (slot[x] is IM_EMPTY)
};

// Per-snapshot live lists of the other nodes (degree >= 2, below the hub
// threshold): for node x and word w (p = w*n + x) the heads live in snapshot
// 64w+b are adj[base[p] + cum[p*65+b] .. base[p] + cum[p*65+b+1]);
// base[p] = IM_EMPTY: x has no lists in word w. A frontier entry whose delta
// has at most SP_BITS bits is expanded through them when they hold no more
// heads than x has arcs: the heads carry their single snapshot bit, so only
// arcs live in the delta's snapshots are read.
struct SparseLists {
    const uint32_t *base;   // [W][n], nullptr: no lists
    const uint16_t *cum;    // [W][n][65]
    const uint32_t *adj;
};
constexpr int SP_BITS = 2;

// Plan the sparse expansion of x with delta d in word w. On success the
// entry's work is the number of listed heads and (rs, del, aux) encode its
// two ranges: rs = start of the first, del = start of the second | len0 << 32
// | len1 << 48, aux = bit0 | bit1 << 8 | 1 << 16 (aux = 0: dense entry).
// The plan is split in two so that its loads can be issued together with the
// entry's row and hub-slot loads: sparse_fetch reads the list base and the
// four cumulative counts that the delta's bits select (in bounds for every
// x < n, w < W; the counts are unused when the base is empty), sparse_use
// decides once the degree is known.
struct SparsePre {
    uint32_t b0, c00, c01, c10, c11, i0, i1;
    bool ok, two;
};

__device__ __forceinline__ SparsePre sparse_fetch(const SparseLists &sp, uint32_t n, uint32_t w,
                                                  uint32_t x, uint64_t d)
{
    SparsePre q;
    q.ok = sp.base && d != 0 && __popcll(d) <= SP_BITS;
    q.b0 = IM_EMPTY; q.c00 = q.c01 = q.c10 = q.c11 = 0; q.i0 = q.i1 = 0; q.two = false;
    if (q.ok) {
        const uint64_t p = (uint64_t)w * n + x;
        const uint64_t d1 = d & (d - 1);
        q.two = d1 != 0;
        q.i0 = (uint32_t)__ffsll((unsigned long long)d) - 1;
        q.i1 = q.two ? (uint32_t)__ffsll((unsigned long long)d1) - 1 : q.i0;
        const uint16_t *c = sp.cum + p * 65;
        q.b0 = sp.base[p];
        q.c00 = c[q.i0]; q.c01 = c[q.i0 + 1]; q.c10 = c[q.i1]; q.c11 = c[q.i1 + 1];
    }
    return q;
}

__device__ __forceinline__ bool sparse_use(const SparsePre &q, uint32_t deg, uint32_t &work,
                                           uint32_t &rs, uint64_t &del, uint32_t &aux)
{
    if (!q.ok || deg < 2 || q.b0 == IM_EMPTY) return false;
    const uint32_t l0 = q.c01 - q.c00, l1 = q.two ? q.c11 - q.c10 : 0u;
    if (l0 + l1 > deg) return false;
    work = l0 + l1;
    rs = q.b0 + q.c00;
    del = (uint64_t)(q.b0 + q.c10) | ((uint64_t)l0 << 32) | ((uint64_t)l1 << 48);
    aux = q.i0 | (q.i1 << 8) | (1u << 16);
    return true;
}

// the r-th listed head of a sparse entry: its position in adj and its bit
__device__ __forceinline__ void sparse_item(uint32_t rs, uint64_t del, uint32_t aux, uint32_t r,
                                            uint32_t &pos, uint64_t &bit)
{
    const uint32_t l0 = (uint32_t)(del >> 32) & 0xFFFFu;
    if (r < l0) { pos = rs + r; bit = 1ull << (aux & 63u); }
    else { pos = (uint32_t)del + (r - l0); bit = 1ull << ((aux >> 8) & 63u); }
}

struct BfsArgs {
    // graph in the direction of this pass
    const uint32_t *row;      // [n+1]
    const uint32_t *col;      // [m]
    const uint64_t *mask;     // [W][m], word-major
    uint64_t m;
    uint32_t n, R, W;
    const uint32_t *node_inst;  // batches: instance of each node (nullptr: one graph)
    const uint32_t *inst_R;     // batches: snapshots per instance
    const uint32_t *inst_off;   // batches: first node of each instance
    uint32_t slot_n;            // length of each global-engine slot array
    // last tier, KEEP launches (one task per workgroup, task = slot): the
    // search state stays in the slot, with its visit count and source here
    uint32_t *kept_nvis, *kept_src;
    HubLists hub;
    SparseLists sp;
    const uint64_t *prune;    // [W][n] or nullptr
    uint32_t *gain;           // [n]
    // task ids: MODE_COUNT: t in [0, n*W) -> word t/n, node t%n (or, when
    // cand != nullptr, t in [0, ncand*W) -> word t/ncand, node cand[t%ncand]);
    // one source with all of the word's bits (minus pruned ones).
    // MODE_DEC, per word w: first gcnt[w] groups of single-snapshot sources
    // (the sources whose only bit is b are plist[w*n + boff[w*64+b] + i],
    // i < bcnt[w*64+b]; group g takes the g-th source of every bit, each with
    // its own bit, so the group's start bits are disjoint), then mcnt[w]
    // multi-snapshot sources mlist[w*n + i] with bits tbits[w*n + node].
    uint32_t ntasks;
    const uint32_t *cand;
    uint32_t ncand;
    // Bit groups (1: none). MODE_COUNT with candidates: every (candidate,
    // word) search is split into bsplit searches over disjoint groups of
    // 64 / bsplit snapshot bits; task t in [0, ncand * W * bsplit) -> group
    // t / (ncand * W). MODE_DEC on the last tier: every queued task runs as
    // bsplit tasks, each with the sources (and bits) of one group.
    uint32_t bsplit;
    const uint32_t *ncand_dev;      // MODE_COUNT: the candidate count in device memory
                                    // (overrides ncand and ntasks = ncand * W), or nullptr
    const uint32_t *gcnt, *mcnt;    // [W]
    const uint32_t *bcnt, *boff;    // [W][64]
    const uint32_t *plist, *mlist;  // [W][n]
    const uint64_t *tbits;          // [W][n]
    // this tier's input queue (nullptr: all task ids) and output queue
    const uint32_t *in_q;
    const uint32_t *in_n;
    uint32_t *out_q;
    uint32_t *out_n;
    uint32_t *grab;           // task counter of this launch (zero before launch)
    // global-engine slots
    uint64_t *b_reach;                     // [slots][slot_n][2]: (reach, pend) of node - base
    uint32_t *b_qa, *b_qb, *b_vis;         // [slots][slot_n], node ids
    unsigned long long *stats;
    int pass, tier;
    int st_trav;
};

// Source `lane` (0..63) of task t: sets the task's word w (every lane) and,
// when the lane has a source, its node and start bits (bits = 0 otherwise).
__device__ __forceinline__ void task_source(const BfsArgs &a, int mode, uint32_t t,
                                            const uint32_t *wpre, uint32_t lane, uint32_t &w,
                                            uint32_t &src, uint64_t &bits)
{
    bits = 0;
    src = 0;
    if (mode == MODE_COUNT) {
        uint64_t group = ~0ull;
        if (a.cand) {
            if (a.bsplit > 1) {
                const uint32_t per = a.ncand * a.W, g = t / per, width = 64u / a.bsplit;
                t -= g * per;
                group = ((1ull << width) - 1ull) << (g * width);
            }
            w = t / a.ncand;
            src = a.cand[t - w * a.ncand];
        } else {
            w = t / a.n;
            src = t - w * a.n;
        }
        if (lane == 0) {
            const uint32_t R = a.node_inst ? a.inst_R[a.node_inst[src]] : a.R;
            bits = im_valid_bits(R, w) & group;
            if (bits && a.prune) bits &= ~a.prune[(uint64_t)w * a.n + src];
        }
        return;
    }
    w = 0;
    while (w + 1 < a.W && wpre[w + 1] <= t) w++;
    const uint32_t tl = t - wpre[w];
    const uint32_t g = a.gcnt[w];
    if (tl < g) {
        const uint32_t c = a.bcnt[w * 64 + lane];
        if (tl < c) {
            src = a.plist[(uint64_t)w * a.n + a.boff[w * 64 + lane] + tl];
            bits = 1ull << lane;
        }
    } else if (lane == 0) {
        src = a.mlist[(uint64_t)w * a.n + (tl - g)];
        bits = a.tbits[(uint64_t)w * a.n + src];
    }
}

// exclusive prefix over words of the task counts (MODE_DEC)
__device__ __forceinline__ void fill_wpre(const BfsArgs &a, uint32_t *wpre)
{
    uint32_t s = 0;
    for (uint32_t w = 0; w < a.W; w++) { wpre[w] = s; s += a.gcnt[w] + a.mcnt[w]; }
    wpre[a.W] = s;
}

template <int NT>
__device__ __forceinline__ uint32_t group_excl_scan(uint32_t v, uint32_t *wsum, uint32_t *total)
{
    if constexpr (NT == 64) {
        uint32_t incl = wave_incl_scan(v);
        *total = __shfl(incl, 63, 64);
        return incl - v;
    } else {
        return block_excl_scan<NT>(v, wsum, total);
    }
}

template <int NT>
__device__ __forceinline__ uint64_t group_sum(uint64_t v, unsigned long long *red)
{
    v = wave_sum_u64(v);
    if constexpr (NT == 64) {
        return v;
    } else {
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        uint64_t s = 0;
#pragma unroll
        for (int i = 0; i < NT / 64; i++) s += red[i];
        __syncthreads();
        return s;
    }
}

// ---------------------------------------------------------------------------
// Hub expansions. Frontier nodes with hub lists are collected per chunk and
// expanded afterwards in batches of HB items, flattened over (item, snapshot
// bit, listed head) so that all lanes share the work of a few huge items as
// well as of many small ones. Each listed head receives its single bit.
// ---------------------------------------------------------------------------
template <int NT, int HB>
struct HubBatch {
    uint32_t hub[NT];       // hub index of item q
    uint32_t own[NT];       // owner of item q (table entry, or unused)
    uint64_t del[NT];       // delta bits of item q
    uint32_t pre[HB][64];   // per batch item: exclusive prefix of per-bit counts
    uint32_t off[HB][64];   // per batch item: start of each bit's list
    uint32_t ipre[HB];      // exclusive prefix of item totals (total past the batch)
    uint32_t tot[HB];
    uint32_t n, total;
};

template <int NT, int HB>
__device__ __forceinline__ void hub_push(HubBatch<NT, HB> &H, uint32_t hs, uint32_t own, uint64_t d)
{
    uint32_t q = atomicAdd(&H.n, 1u);
    H.hub[q] = hs; H.own[q] = own; H.del[q] = d;
}

// word_of(own) -> snapshot word of an item; relax(own, v, bits) applies one relaxation
// nh: number of collected items, read by every thread between the barrier that
// follows their collection and the next collection. relax(own, v, bits) is
// called by every lane for every unrolled step (bits may be 0), flush() once
// per unrolled group of steps.
template <int NT, int HB, int U, typename WordOf, typename Relax, typename Flush>
__device__ void expand_hubs(HubBatch<NT, HB> &H, uint32_t nh, const HubLists &hub, uint32_t W,
                            WordOf word_of, Relax relax, Flush flush, uint64_t &arcs)
{
    static_assert((HB & (HB - 1)) == 0, "HB must be a power of two");
    constexpr int NWAVE = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    for (uint32_t base = 0; base < nh; base += HB) {
        const uint32_t nb = min((uint32_t)HB, nh - base);
        for (uint32_t q = wid; q < nb; q += NWAVE) {
            const uint32_t it = base + q;
            const uint32_t *o = hub.off + ((uint64_t)H.hub[it] * W + word_of(H.own[it])) * 65;
            uint32_t lo = o[lane], hi = o[lane + 1];
            uint32_t c = ((H.del[it] >> lane) & 1ull) ? hi - lo : 0u;
            uint32_t incl = wave_incl_scan(c);
            H.pre[q][lane] = incl - c;
            H.off[q][lane] = lo;
            if (lane == 63) H.tot[q] = incl;
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t acc = 0;
            for (uint32_t q = 0; q < (uint32_t)HB; q++) {
                H.ipre[q] = acc;
                if (q < nb) acc += H.tot[q];
            }
            H.total = acc;
        }
        __syncthreads();
        const uint32_t total = H.total;
        arcs += total;
        // uniform trip count: every lane calls relax() the same number of times
        for (uint32_t j0 = 0; j0 < total; j0 += NT * U) {
            uint32_t vv[U], qq[U];
            uint64_t bb[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                uint32_t j = j0 + (uint32_t)tid + (uint32_t)u * NT;
                bb[u] = 0; vv[u] = 0; qq[u] = 0;
                if (j < total) {
                    int q = upper_index<HB>(H.ipre, j);
                    uint32_t r = j - H.ipre[q];
                    int b = upper_index<64>(H.pre[q], r);
                    vv[u] = hub.adj[H.off[q][b] + (r - H.pre[q][b])];
                    bb[u] = 1ull << b;
                    qq[u] = base + (uint32_t)q;
                }
            }
#pragma unroll
            for (int u = 0; u < U; u++) relax(H.own[qq[u]], vv[u], bb[u]);
            flush();
        }
        __syncthreads();
    }
    if (tid == 0) H.n = 0;
    __syncthreads();
}

// ---------------------------------------------------------------------------
// LDS engine (tiers 0 and 1)
// ---------------------------------------------------------------------------
template <int NT, int T, int CS>
struct LdsState {
    uint32_t keys[T * CS];
    uint64_t reach[T * CS];
    uint64_t pend[T * CS];
    uint32_t deg[T * CS];
    uint32_t fr[2][T * CS];
    uint32_t c_excl[NT];
    uint32_t c_rs[NT];
    uint32_t c_idx[NT];
    uint32_t c_aux[NT];   // 0: dense entry, else the sparse plan's bits
    uint64_t c_del[NT];
    uint32_t wsum[NT / 64 + 1];
    unsigned long long red[NT / 64];
    uint32_t s_task[T], s_src[T], s_word[T], s_cnt[T], s_next[T], s_ovf[T], s_act[T], s_new[T];
    uint32_t s_sum[T];   // MODE_COUNT: reached bits of each finishing slot
    uint32_t wpre[65];
    HubBatch<NT, (NT == 64 ? 2 : 16)> H;
    uint32_t nf, nn, tnext, tend, ntasks, done, chunk, snext;
};

// insert v into slot s's table (if absent) and OR in `bits`; push the entry
// onto frontier list `lst` when its pending bits become non-zero (the next
// frontier during expansion, the current one while seeding a task)
template <int NT, int T, int CS, int LIM>
__device__ __forceinline__ void lds_relax(LdsState<NT, T, CS> &L, uint32_t s, uint32_t v,
                                          uint64_t bits, int nxt, bool seeding = false)
{
    constexpr int LOG_CS = __builtin_ctz(CS);
    if (L.s_ovf[s]) return;  // abandoned: stop touching its full table
    uint32_t h = (v * 0x9E3779B1u) >> (32 - LOG_CS);
    int found = -1;
    for (int p = 0; p < CS; p++) {
        uint32_t pos = s * CS + h;
        uint32_t key = L.keys[pos];
        if (key == v) { found = (int)pos; break; }
        if (key == IM_EMPTY) {
            uint32_t old = atomicCAS(&L.keys[pos], IM_EMPTY, v);
            if (old == IM_EMPTY) {
                uint32_t c = atomicAdd(&L.s_cnt[s], 1u);
                if (c + 1 > (uint32_t)LIM) L.s_ovf[s] = 1;
                found = (int)pos;
                break;
            }
            if (old == v) { found = (int)pos; break; }
        }
        h = (h + 1) & (CS - 1);
    }
    if (found < 0) { L.s_ovf[s] = 1; return; }
    uint64_t old = atomicOr((unsigned long long *)&L.reach[found], (unsigned long long)bits);
    uint64_t nb = bits & ~old;
    if (nb) {
        uint64_t op = atomicOr((unsigned long long *)&L.pend[found], (unsigned long long)nb);
        if (op == 0) {
            if (seeding) {
                L.fr[nxt][atomicAdd(&L.nf, 1u)] = (uint32_t)found;
            } else {
                uint32_t q = atomicAdd(&L.nn, 1u);
                L.fr[nxt][q] = (uint32_t)found;
                atomicAdd(&L.s_next[s], 1u);
            }
        }
    }
}

__device__ __forceinline__ uint32_t slot_hash(uint32_t v) { return v * 0x9E3779B1u; }

// Append from the lanes where pred holds with one atomic per wavefront. Every
// lane of the wavefront must call it. Returns each appending lane's position.
__device__ __forceinline__ uint32_t wave_append(bool pred, uint32_t *counter)
{
    const uint64_t bal = __ballot(pred);
    if (!bal) return 0;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((unsigned long long)bal) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(bal));
    base = __shfl(base, leader, 64);
    return base + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
}

template <int MODE, int NT, int T, int CS, int LIM, uint32_t DMAX, int U, bool PRUNE>
__global__ __launch_bounds__(NT) void k_lds_bfs(BfsArgs a)
{
    static_assert((CS & (CS - 1)) == 0, "CS must be a power of two");
    static_assert(LIM < CS, "LIM must leave free table entries");
    constexpr int LOG_CS = __builtin_ctz(CS);
    constexpr int N = T * CS;
    constexpr uint32_t NONE = 0xFFFFFFFFu;
    __shared__ LdsState<NT, T, CS> L;
    const int tid = threadIdx.x;
    if (MODE == MODE_COUNT && a.ncand_dev) { a.ncand = *a.ncand_dev; a.ntasks = a.ncand * a.W * max(a.bsplit, 1u); }

    for (int i = tid; i < N; i += NT) {
        L.keys[i] = IM_EMPTY; L.reach[i] = 0; L.pend[i] = 0; L.deg[i] = 0;
    }
    if (tid < T) {
        L.s_act[tid] = 0; L.s_cnt[tid] = 0; L.s_next[tid] = 0; L.s_ovf[tid] = 0; L.s_sum[tid] = 0;
    }
    if (MODE == MODE_DEC && tid < 64) {
        // exclusive prefix over words of the task counts, one lane per word
        // (the loads are issued together instead of one after another)
        const uint32_t c = (uint32_t)tid < a.W ? a.gcnt[tid] + a.mcnt[tid] : 0u;
        const uint32_t incl = wave_incl_scan(c);
        if ((uint32_t)tid < a.W) L.wpre[tid] = incl - c;
        if (tid == 63) L.wpre[a.W] = incl;
    }
    __syncthreads();
    if (tid == 0) {
        L.nf = 0; L.nn = 0; L.tnext = 0; L.tend = 0; L.done = 0; L.H.n = 0;
        L.ntasks = a.in_q ? *a.in_n : (MODE == MODE_COUNT ? a.ntasks : L.wpre[a.W]);
        // Task assignment. With up to 64 tasks per slot, each workgroup
        // strides over the task ids (no atomics; the workgroups' task counts
        // differ by at most one, and all of them start at once: chunk = 0).
        // With more, tasks are grabbed from one counter in chunks of at least
        // 8 (the counter, one address for the whole grid, sees few atomics),
        // which balances long runs of tasks better and keeps consecutive
        // task ids, whose sources share cache lines, in one workgroup.
        const uint32_t slots = gridDim.x * (uint32_t)T;
        L.chunk = L.ntasks <= 64u * slots ? 0u : min(256u, max(8u, L.ntasks / slots));
        L.snext = blockIdx.x;
    }
    __syncthreads();

    uint64_t st_relax = 0, st_reached = 0, st_arcs = 0, st_trav = 0, st_ovf = 0, st_dec = 0;
    int cur = 0;
    uint32_t levels = 0;

    for (;;) {
        levels++;
        // ---- refill: thread 0 hands task indices to idle slots
        if (tid == 0) {
            L.nn = 0;
            for (int s = 0; s < T; s++) {
                L.s_next[s] = 0;
                L.s_new[s] = NONE;
                if (L.s_act[s] || L.done) continue;
                if (L.tnext == L.tend) {
                    uint32_t b;
                    if (L.chunk == 0) {   // striding: task blockIdx.x + i * gridDim.x
                        b = L.snext;
                        L.snext += gridDim.x;
                    } else {
                        b = atomicAdd(a.grab, L.chunk);
                    }
                    if (b >= L.ntasks) { L.done = 1; continue; }
                    L.tnext = b;
                    L.tend = min(b + max(L.chunk, 1u), L.ntasks);
                }
                L.s_new[s] = L.tnext++;
                L.s_cnt[s] = 0;
                L.s_ovf[s] = 0;
            }
        }
        __syncthreads();
        // ---- seed the new tasks: lane l of the first wavefront inserts source l.
        // The sources of all new slots are looked up first, so that their
        // dependent load chains overlap instead of running one slot after another.
        if (MODE == MODE_COUNT) {
            // one source per task: lane s seeds slot s. A new slot's table is
            // empty (every finished slot is cleared), so the source takes its
            // hash position without probing, and the seeds join the frontier
            // with one wavefront-wide append.
            if (tid < 64) {
                const uint32_t sn = (uint32_t)tid < (uint32_t)T ? L.s_new[tid] : NONE;
                uint64_t bits = 0;
                uint32_t pos = 0;
                if (sn != NONE) {
                    const uint32_t tq = a.in_q ? a.in_q[sn] : sn;
                    uint32_t w, src;
                    task_source(a, MODE, tq, L.wpre, 0u, w, src, bits);
                    L.s_task[tid] = tq; L.s_src[tid] = src; L.s_word[tid] = w;
                    // a task without start bits leaves the slot idle
                    L.s_act[tid] = bits ? 1u : 0u;
                    if (bits) {
                        pos = (uint32_t)tid * CS + ((src * 0x9E3779B1u) >> (32 - LOG_CS));
                        L.keys[pos] = src; L.reach[pos] = bits; L.pend[pos] = bits;
                        L.s_cnt[tid] = 1;
                    }
                }
                const uint32_t at = wave_append(bits != 0, &L.nf);
                if (bits) L.fr[cur][at] = pos;
            }
        } else if (tid < 64) {
            uint32_t tt[T], ww[T], ss[T];
            uint64_t bb[T];
#pragma unroll
            for (int s = 0; s < T; s++) {
                const uint32_t sn = L.s_new[s];
                tt[s] = NONE; ww[s] = 0; ss[s] = 0; bb[s] = 0;
                if (sn != NONE) tt[s] = a.in_q ? a.in_q[sn] : sn;
            }
#pragma unroll
            for (int s = 0; s < T; s++)
                if (tt[s] != NONE) task_source(a, MODE, tt[s], L.wpre, (uint32_t)tid, ww[s], ss[s], bb[s]);
#pragma unroll
            for (int s = 0; s < T; s++) {
                if (tt[s] == NONE) continue;
                // a task without start bits (e.g. a word beyond an instance's R)
                // leaves the slot idle: an active slot must own frontier entries
                const bool any = __ballot(bb[s] != 0) != 0ull;
                if (tid == 0) {
                    L.s_task[s] = tt[s]; L.s_src[s] = ss[s]; L.s_word[s] = ww[s];
                    L.s_act[s] = any ? 1u : 0u;
                }
                if (bb[s]) lds_relax<NT, T, CS, LIM>(L, s, ss[s], bb[s], cur, true);
            }
        }
        __syncthreads();
        const uint32_t nf = L.nf;
        if (nf == 0) {
            if (L.done) break;
            continue;
        }

        // ---- phase B: expand NT frontier entries per chunk, arcs spread over lanes
        for (uint32_t base = 0; base < nf; base += NT) {
            uint32_t i = base + tid;
            uint32_t deg = 0, rs = 0, idx = 0, aux = 0;
            uint64_t d = 0;
            if (i < nf) {
                idx = L.fr[cur][i];
                uint32_t s = idx >> LOG_CS;
                if (!L.s_ovf[s]) {
                    // take the bits gained since the last expansion; bits that
                    // arrive later re-queue the entry for the next level
                    const uint64_t delta = atomicExch((unsigned long long *)&L.pend[idx], 0ull);
                    uint32_t x = L.keys[idx];
                    // independent loads: hub slot, row bounds, sparse lists
                    uint32_t hs = a.hub.slot ? a.hub.slot[x] : IM_EMPTY;
                    rs = a.row[x];
                    const uint32_t re = a.row[x + 1];
                    const SparsePre sq = sparse_fetch(a.sp, a.n, L.s_word[s], x, delta);
                    deg = re - rs;
                    L.deg[idx] = deg;
                    if (hs != IM_EMPTY) {
                        hub_push(L.H, hs, idx, delta);
                        deg = 0;
                    } else if (deg > DMAX) {
                        L.s_ovf[s] = 1; deg = 0;
                    } else {
                        d = delta;
                        uint32_t work, srs, saux;
                        uint64_t sdel;
                        if (sparse_use(sq, deg, work, srs, sdel, saux)) {
                            deg = work; rs = srs; d = sdel; aux = saux;
                        }
                    }
                }
            }
            uint32_t total;
            uint32_t ex = group_excl_scan<NT>(deg, L.wsum, &total);
            L.c_excl[tid] = ex;
            L.c_rs[tid] = rs;
            L.c_idx[tid] = idx;
            L.c_del[tid] = d;
            L.c_aux[tid] = aux;
            __syncthreads();
            const uint32_t nhub = L.H.n;
            st_arcs += total;
            for (uint32_t j0 = tid; j0 < total; j0 += NT * U) {
                uint32_t kk[U], ee[U], vv[U];
                uint64_t bb[U];
#pragma unroll
                for (int u = 0; u < U; u++) {
                    uint32_t j = j0 + (uint32_t)u * NT;
                    kk[u] = NONE;
                    ee[u] = 0;
                    if (j < total) {
                        int k = upper_index<NT>(L.c_excl, j);
                        kk[u] = (uint32_t)k;
                        ee[u] = j - L.c_excl[k];   // rank within the entry
                    }
                }
                // mask word and head id (or the listed head) are independent
                // loads: issue all of them
#pragma unroll
                for (int u = 0; u < U; u++) {
                    bb[u] = 0;
                    vv[u] = 0;
                    if (kk[u] != NONE && !L.s_ovf[L.c_idx[kk[u]] >> LOG_CS]) {
                        const uint32_t k = kk[u], ax = L.c_aux[k];
                        if (ax) {
                            uint32_t pos;
                            sparse_item(L.c_rs[k], L.c_del[k], ax, ee[u], pos, bb[u]);
                            vv[u] = a.sp.adj[pos];
                        } else {
                            const uint32_t e = L.c_rs[k] + ee[u];
                            uint64_t w = L.s_word[L.c_idx[k] >> LOG_CS];
                            bb[u] = a.mask[w * a.m + e] & L.c_del[k];
                            vv[u] = a.col[e];
                        }
                    } else {
                        kk[u] = NONE;
                    }
                }
                if (PRUNE) {
#pragma unroll
                    for (int u = 0; u < U; u++)
                        if (bb[u]) {
                            uint64_t w = L.s_word[L.c_idx[kk[u]] >> LOG_CS];
                            bb[u] &= ~a.prune[w * a.n + vv[u]];
                        }
                }
#pragma unroll
                for (int u = 0; u < U; u++)
                    if (bb[u]) lds_relax<NT, T, CS, LIM>(L, L.c_idx[kk[u]] >> LOG_CS, vv[u], bb[u], cur ^ 1);
            }
            __syncthreads();
            // hub expansions of this chunk: only the arcs live in the delta's snapshots
            if (nhub) {
                auto word_of = [&](uint32_t own) { return L.s_word[own >> LOG_CS]; };
                auto relax = [&](uint32_t own, uint32_t v, uint64_t bits) {
                    if (!bits) return;
                    const uint32_t s = own >> LOG_CS;
                    if (PRUNE) bits &= ~a.prune[(uint64_t)L.s_word[s] * a.n + v];
                    if (bits) lds_relax<NT, T, CS, LIM>(L, s, v, bits, cur ^ 1);
                };
                expand_hubs<NT, (NT == 64 ? 2 : 16), U>(L.H, nhub, a.hub, a.W, word_of, relax, [] {},
                                                         st_arcs);
            }
        }

        // ---- finish slots whose search ended or overflowed, all in one pass:
        // fin (bit s: slot s finishes) and ovfm (bit s: it is handed over)
        // are the same in every thread (read from LDS after a barrier)
        uint32_t fin = 0, ovfm = 0;
#pragma unroll
        for (int s = 0; s < T; s++) {
            if (!L.s_act[s]) continue;
            const bool ovf = L.s_ovf[s] != 0;
            if (!ovf && L.s_next[s] != 0) continue;
            fin |= 1u << s;
            if (ovf) ovfm |= 1u << s;
        }
        const bool any_ovf_fin = ovfm != 0;
        if (fin) {
            if (tid < 64) {
                // handed-over tasks: one append for the wavefront
                const bool h = (uint32_t)tid < (uint32_t)T && ((ovfm >> tid) & 1u);
                const uint64_t bal = __ballot(h);
                uint32_t q0 = 0;
                if (bal && tid == 0) q0 = atomicAdd(a.out_n, (uint32_t)__popcll(bal));
                q0 = __shfl(q0, 0, 64);
                if (h) a.out_q[q0 + (uint32_t)__popcll(bal & ((1ull << tid) - 1ull))] = L.s_task[tid];
                if (tid == 0) st_ovf += (uint64_t)__popcll(bal);
            }
            // the entries of the finishing slots, slot after slot, spread
            // over all threads
            const uint32_t nfin = (uint32_t)__popc(fin);
            for (uint32_t j = tid; j < nfin * CS; j += NT) {
                uint32_t r = j / CS, f = fin;
                for (uint32_t c = 0; c < r; c++) f &= f - 1u;
                const uint32_t s = (uint32_t)__ffs(f) - 1u;
                const uint32_t i = s * CS + (j % CS);
                const uint32_t key = L.keys[i];
                uint32_t pc = 0;
                if (key != IM_EMPTY && !((ovfm >> s) & 1u)) {
                    pc = (uint32_t)__popcll(L.reach[i]);
                    const uint32_t dg = L.deg[i];
                    st_relax += dg;
                    st_reached += 1;
                    st_trav += (uint64_t)pc * dg;
                    if (MODE == MODE_DEC) { atomicSub(&a.gain[key], pc); st_dec += pc; }
                }
                if (MODE == MODE_COUNT) {
                    // one slot per aligned segment of min(CS, 64) lanes: sum
                    // within the segment, one LDS add per segment
                    constexpr int SEG = CS < 64 ? CS : 64;
#pragma unroll
                    for (int o = SEG / 2; o > 0; o >>= 1) pc += __shfl_xor(pc, o, 64);
                    if ((tid & (SEG - 1)) == 0 && pc) atomicAdd(&L.s_sum[s], pc);
                }
                L.keys[i] = IM_EMPTY; L.reach[i] = 0; L.pend[i] = 0; L.deg[i] = 0;
            }
            __syncthreads();
            if ((uint32_t)tid < (uint32_t)T && ((fin >> tid) & 1u)) {
                if (MODE == MODE_COUNT && !((ovfm >> tid) & 1u))
                    atomicAdd(&a.gain[L.s_src[tid]], L.s_sum[tid]);
                L.s_sum[tid] = 0;
                L.s_act[tid] = 0; L.s_cnt[tid] = 0; L.s_ovf[tid] = 0;
            }
            __syncthreads();
        }

        // ---- drop next-frontier entries that belong to slots just handed over
        uint32_t nn = L.nn;
        if (any_ovf_fin) {
            uint32_t wpos = 0;
            for (uint32_t base = 0; base < nn; base += NT) {
                uint32_t i = base + tid;
                uint32_t idx = i < nn ? L.fr[cur ^ 1][i] : 0;
                uint32_t keep = (i < nn && L.s_act[idx >> LOG_CS]) ? 1u : 0u;
                uint32_t tot;
                uint32_t before = group_excl_scan<NT>(keep, L.wsum, &tot);
                __syncthreads();
                if (keep) L.fr[cur ^ 1][wpos + before] = idx;
                wpos += tot;
                __syncthreads();
            }
            nn = wpos;
        }
        __syncthreads();
        if (tid == 0) L.nf = nn;
        cur ^= 1;
        __syncthreads();
    }

    // ---- statistics: one atomic per counter per workgroup
    st_relax = group_sum<NT>(st_relax, L.red);
    st_reached = group_sum<NT>(st_reached, L.red);
    st_trav = group_sum<NT>(st_trav, L.red);
    st_dec = group_sum<NT>(st_dec, L.red);
    st_ovf = group_sum<NT>(st_ovf, L.red);
    // workgroups that found no task add nothing (no contended atomics)
    if (tid == 0 && st_reached + st_ovf) {
        if (MODE == MODE_DEC) stat_add(a.stats, ST_DECREMENTS, st_dec);
        stat_add(a.stats, st_tier(a.pass, a.tier, F_RELAX), st_relax);
        stat_add(a.stats, st_tier(a.pass, a.tier, F_REACHED), st_reached);
        stat_add(a.stats, st_tier(a.pass, a.tier, F_ARCS), st_arcs);
        stat_add(a.stats, st_tier(a.pass, a.tier, F_OVF), st_ovf);
        stat_add(a.stats, a.st_trav, st_trav);
        stat_max(a.stats, ST_MAXLV_BASE + a.pass * 3 + a.tier, levels);
    }
}

// ---------------------------------------------------------------------------
// Global engine (last tier): one task per workgroup, dense arrays of length n
// per slot. reach and pend are all-zero on entry and are left all-zero.
// ---------------------------------------------------------------------------
template <int NT>
struct BlockLds {
    uint32_t scan[NT];
    uint32_t rs[NT];
    uint32_t aux[NT];
    uint64_t del[NT];
    uint32_t wsum[NT / 64 + 1];
    uint32_t nf, nn, nvis, task, levels, entries;
    unsigned long long red[NT / 64];
    uint32_t gsrc[64];
    uint64_t gbits[64];
    HubBatch<NT, 16> H;
};

// reach and pend are indexed by (v - base) * S (base: the task's instance's
// first node); S = 2 with pend = reach + 1 keeps a node's two words in one
// 16-byte record, so a relaxation touches one cache line
template <int S = 1>
__device__ __forceinline__ void global_relax(uint64_t *reach, uint64_t *pend, uint32_t base,
                                             uint32_t *vis, uint32_t *nxt, uint32_t *nvis,
                                             uint32_t *nn, uint32_t v, uint64_t bits)
{
    const uint64_t i = (uint64_t)(v - base) * S;
    uint64_t old = atomicOr((unsigned long long *)&reach[i], (unsigned long long)bits);
    uint64_t nb = bits & ~old;
    if (!nb) return;
    if (old == 0) vis[atomicAdd(nvis, 1u)] = v;
    uint64_t op = atomicOr((unsigned long long *)&pend[i], (unsigned long long)nb);
    if (op == 0) nxt[atomicAdd(nn, 1u)] = v;
}

// Run one task to its fixpoint; afterwards vis[0..L.nvis) lists every node
// with reach != 0. Each thread passes its own seed (src, start); start = 0
// means none. Every node the task can reach is >= base, and reach / pend
// hold the nodes from base on. All threads of the workgroup must call it.
template <int NT, int U, bool PRUNE, bool SPARSE = true, int S = 1>
__device__ void block_bfs_run(BlockLds<NT> &L, uint32_t src, uint64_t start,
                              const uint32_t *row, const uint32_t *col, const uint64_t *mask,
                              const HubLists &hub, const SparseLists &sp, uint32_t n,
                              uint32_t W, uint32_t w,
                              const uint64_t *prune, uint64_t *reach, uint64_t *pend,
                              uint32_t base, uint32_t *qa, uint32_t *qb, uint32_t *vis,
                              uint64_t &arcs, bool preseeded = false)
{
    constexpr uint32_t NONE = 0xFFFFFFFFu;
    const int tid = threadIdx.x;
    // preseeded: the caller has already entered the seeds with global_relax
    // (after setting L.nf = L.nn = L.nvis = L.H.n = L.levels = L.entries = 0)
    if (!preseeded) {
        if (tid == 0) { L.nf = 0; L.nn = 0; L.nvis = 0; L.H.n = 0; L.levels = 0; L.entries = 0; }
        __syncthreads();
        // seeds: every lane with start bits (lanes 0..63 for multi-source tasks)
        if (start) global_relax<S>(reach, pend, base, vis, qa, &L.nvis, &L.nf, src, start);
        __syncthreads();
    }
    uint32_t *cur = qa, *nxt = qb;
    for (;;) {
        const uint32_t nf = L.nf;
        if (nf == 0) break;
        for (uint32_t tile = 0; tile < nf; tile += NT) {
            uint32_t i = tile + tid;
            uint32_t deg = 0, rs = 0, aux = 0;
            uint64_t d = 0;
            if (i < nf) {
                uint32_t x = cur[i];
                rs = row[x];
                deg = row[x + 1] - rs;
                // only a node with enough arcs can have lists: the others skip
                // the load (one line less per expansion; hubs wait one more load)
                uint32_t hs = (hub.slot && deg >= hub.min_deg) ? hub.slot[x] : IM_EMPTY;
                // bits gained since the last expansion (later ones re-queue x)
                d = atomicExch((unsigned long long *)&pend[(uint64_t)(x - base) * S], 0ull);
                if (hs != IM_EMPTY) {
                    hub_push(L.H, hs, 0u, d);
                    deg = 0; d = 0;
                } else if (SPARSE && deg >= 2) {   // (no lists below 2 arcs: skip their loads)
                    uint32_t work, srs, saux;
                    uint64_t sdel;
                    if (sparse_use(sparse_fetch(sp, n, w, x, d), deg, work, srs, sdel, saux)) {
                        deg = work; rs = srs; d = sdel; aux = saux;
                    }
                }
            }
            uint32_t total;
            uint32_t ex = block_excl_scan<NT>(deg, L.wsum, &total);
            L.scan[tid] = ex;
            L.rs[tid] = rs;
            L.del[tid] = d;
            L.aux[tid] = aux;
            __syncthreads();
            const uint32_t nhub = L.H.n;
            arcs += total;
            for (uint32_t j0 = tid; j0 < total; j0 += NT * U) {
                uint32_t kk[U], ee[U], vv[U];
                uint64_t bb[U];
#pragma unroll
                for (int u = 0; u < U; u++) {
                    uint32_t j = j0 + (uint32_t)u * NT;
                    kk[u] = NONE;
                    ee[u] = 0;
                    if (j < total) {
                        int k = upper_index<NT>(L.scan, j);
                        kk[u] = (uint32_t)k;
                        ee[u] = j - L.scan[k];   // rank within the entry
                    }
                }
#pragma unroll
                for (int u = 0; u < U; u++) {
                    bb[u] = 0;
                    vv[u] = 0;
                    if (kk[u] != NONE) {
                        const uint32_t k = kk[u];
                        const uint32_t ax = SPARSE ? L.aux[k] : 0u;
                        uint32_t pos = L.rs[k] + ee[u];
                        uint64_t bit = 0;
                        if (ax) sparse_item(L.rs[k], L.del[k], ax, ee[u], pos, bit);
                        const uint32_t *heads = ax ? sp.adj : col;
                        vv[u] = heads[pos];
                        bb[u] = ax ? bit : (mask[pos] & L.del[k]);
                    }
                }
                if (PRUNE) {
#pragma unroll
                    for (int u = 0; u < U; u++)
                        if (bb[u]) bb[u] &= ~prune[vv[u]];
                }
#pragma unroll
                for (int u = 0; u < U; u++)
                    if (bb[u]) global_relax<S>(reach, pend, base, vis, nxt, &L.nvis, &L.nn, vv[u], bb[u]);
            }
            __syncthreads();
            // hub expansions of this tile: only the arcs live in the delta's snapshots
            if (nhub) {
                auto word_of = [&](uint32_t) { return w; };
                auto relax = [&](uint32_t, uint32_t v, uint64_t bits) {
                    if (!bits) return;
                    if (PRUNE) bits &= ~prune[v];
                    if (bits) global_relax<S>(reach, pend, base, vis, nxt, &L.nvis, &L.nn, v, bits);
                };
                expand_hubs<NT, 16, U>(L.H, nhub, hub, W, word_of, relax, [] {}, arcs);
            }
        }
        if (tid == 0) { L.levels++; L.entries += nf; L.nf = L.nn; L.nn = 0; }
        uint32_t *t = cur; cur = nxt; nxt = t;
        __syncthreads();
    }
}

template <int MODE, int NT, int U, bool PRUNE, bool KEEP = false>
__global__ __launch_bounds__(NT) void k_block_bfs(BfsArgs a)
{
    // KEEP (MODE_COUNT, single graph, tasks routed here directly): workgroup
    // b runs task b alone and leaves its fixpoint (reach bits, visit list) in
    // slot b for a later kernel, which returns the slot to zero
    __shared__ BlockLds<NT> L;
    __shared__ uint32_t wpre[65];
    const int tid = threadIdx.x;
    const uint64_t slot = blockIdx.x;
    if (MODE == MODE_COUNT && a.ncand_dev) { a.ncand = *a.ncand_dev; a.ntasks = a.ncand * a.W * max(a.bsplit, 1u); }
    // the slot's (reach, pend) records, interleaved
    uint64_t *reach = a.b_reach + slot * a.slot_n * 2;
    uint64_t *pend = reach + 1;
    uint32_t *qa = a.b_qa + slot * a.slot_n;
    uint32_t *qb = a.b_qb + slot * a.slot_n;
    uint32_t *vis = a.b_vis + slot * a.slot_n;
    if (tid == 0 && MODE == MODE_DEC) fill_wpre(a, wpre);
    __syncthreads();
    // in_q = nullptr: every task id below ntasks (tasks routed straight here)
    const uint32_t nq0 = a.in_q ? *a.in_n : a.ntasks;
    // reverse tasks split into bit groups: task q -> group q / nq0 of queued
    // task q % nq0 (the groups' decrements add up to the task's)
    const uint32_t spl = MODE == MODE_DEC ? max(a.bsplit, 1u) : 1u;
    const uint32_t nq = nq0 * spl;
    // In a batch a packed reverse task may hold sources of several instances;
    // its sources are then searched one after the other, each inside its own
    // instance (their bits are disjoint, so the decrements add up to those of
    // the joint search). A single graph searches all sources together.
    const bool split = a.node_inst != nullptr;
    uint64_t arcs = 0, relax = 0, reached = 0, trav = 0, dec = 0, levels = 0;
    bool first = true;
    for (;;) {
        if (tid == 0) L.task = KEEP ? (first ? (uint32_t)blockIdx.x : nq) : atomicAdd(a.grab, 1u);
        first = false;
        __syncthreads();
        const uint32_t q = L.task;
        __syncthreads();
        if (q >= nq) break;
        uint32_t w = 0;
        {
            uint32_t ww, ss;
            uint64_t bb;
            const uint32_t grp = q / nq0, q0 = q - grp * nq0;
            task_source(a, MODE, a.in_q ? a.in_q[q0] : q0, wpre, (uint32_t)(tid & 63), ww, ss, bb);
            if (spl > 1) bb &= ((1ull << (64u / spl)) - 1ull) << (grp * (64u / spl));
            w = ww;
            if (tid < 64) { L.gsrc[tid] = ss; L.gbits[tid] = bb; }
        }
        __syncthreads();
        const uint64_t *mask = a.mask + (uint64_t)w * a.m;
        const uint64_t *prune = PRUNE ? a.prune + (uint64_t)w * a.n : nullptr;
        for (int l = 0; l < (split ? 64 : 1); l++) {
            if (split && L.gbits[l] == 0) continue;   // uniform: read from LDS
            // COUNT tasks have one source, on lane 0
            const uint32_t src0 = L.gsrc[l];
            uint32_t src = 0;
            uint64_t bits = 0;
            if (split) {
                if (tid == 0) { src = src0; bits = L.gbits[l]; }
            } else if (tid < 64) {
                src = L.gsrc[tid]; bits = L.gbits[tid];
            }
            const uint32_t base = split ? a.inst_off[a.node_inst[src0]] : 0u;
                block_bfs_run<NT, U, PRUNE, true, 2>(L, src, bits, a.row, a.col, mask, a.hub, a.sp, a.n, a.W, w, prune,
                                        reach, pend, base, qa, qb, vis, arcs);
            const uint32_t nvis = L.nvis;
            levels += L.levels;
            uint64_t cnt = 0;
            for (uint32_t i = tid; i < nvis; i += NT) {
                uint32_t x = vis[i];
                uint32_t pc = (uint32_t)__popcll(reach[(uint64_t)(x - base) * 2]);
                uint32_t dg = a.row[x + 1] - a.row[x];
                relax += dg;
                reached += 1;
                trav += (uint64_t)pc * dg;
                if (MODE == MODE_COUNT) cnt += pc;
                else { atomicSub(&a.gain[x], pc); dec += pc; }
                if (!KEEP) reach[(uint64_t)(x - base) * 2] = 0;   // pend is zero at the fixpoint
            }
            if (MODE == MODE_COUNT) {
                cnt = group_sum<NT>(cnt, L.red);
                if (tid == 0) atomicAdd(&a.gain[src0], (uint32_t)cnt);
            }
            if (KEEP && tid == 0) {
                a.kept_nvis[q] = nvis;
                a.kept_src[q] = src0;
            }
            __syncthreads();
        }
    }
    relax = group_sum<NT>(relax, L.red);
    reached = group_sum<NT>(reached, L.red);
    trav = group_sum<NT>(trav, L.red);
    dec = group_sum<NT>(dec, L.red);
    if (tid == 0 && reached) {
        if (MODE == MODE_DEC) stat_add(a.stats, ST_DECREMENTS, dec);
        stat_add(a.stats, st_tier(a.pass, a.tier, F_RELAX), relax);
        stat_add(a.stats, st_tier(a.pass, a.tier, F_REACHED), reached);
        stat_add(a.stats, st_tier(a.pass, a.tier, F_ARCS), arcs);
        stat_add(a.stats, a.st_trav, trav);
        stat_max(a.stats, ST_MAXLV_BASE + a.pass * 3 + a.tier, levels);
    }
}
