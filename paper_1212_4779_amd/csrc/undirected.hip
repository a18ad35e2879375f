// undirected.hip -- StaticGreedy on undirected graphs with one coin per
// undirected pair: the component method.
//
// Paper: Cheng et al., CIKM 2013 (arXiv 1212.4779), Sec. 4: in an undirected
// snapshot the nodes a node reaches are the nodes that reach it, so each
// snapshot is described by its connected components. Then
//   s_u = sum_r |C_r(u)|                       (initial gains)
// and adding v* to S covers, in every snapshot where it is still uncovered,
// the whole component C = C_r(v*): every member u loses |C| (Algorithm 2's
// decrements for the |C| newly covered nodes, each reached by every member).
//
// Reading: the caller's CSR stores both directions of every undirected pair
// with the same probability and no parallel arcs; the pair's coin in
// snapshot r is drawn under the index of its canonical arc (the direction
// whose tail is the smaller id) by the same generator rule as directed arcs;
// a self-loop is its own pair and never changes a component.
//
// Pipeline (one stream):
//   U1  pair matching: every arc is inserted into a hash table keyed by its
//       unordered end points; each pair must collect exactly one arc per
//       direction with equal probabilities; the canonical arcs are compacted
//   U2  per (pair, snapshot word): the word's 64 coins, and for every live
//       snapshot a lock-free union of the end points in that snapshot's
//       union-find forest (roots are component minima: a larger root is
//       hooked under a smaller one by compare-and-swap)
//   U3  labels flattened to roots; every non-root member ranked among its
//       root's members (wavefront-aggregated atomics); the member lists of
//       all (snapshot, root) pairs placed by one prefix sum over their
//       counts and filled; s_u = sum_r |C_r(u)|, round-0 key
//   per round: U4 one workgroup per snapshot covers v*'s component if it is
//       still uncovered (its members lose |C|), U5 the next argmax key
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "im.h"
#include "im_device.h"
#include "im_host.h"

namespace {

constexpr uint64_t KEY_EMPTY = ~0ull;
constexpr uint32_t NONE = 0xFFFFFFFFu;
constexpr uint32_t COVERED = 0x80000000u;  // top bit of a root's size: component covered
enum { UE_MISSING = 1, UE_PARALLEL = 2, UE_PROB = 4, UE_BIG = 8 };
constexpr int UN_NT = 256;

template <typename Tv>
int ualloc(Tv **p, uint64_t cnt)
{
    if (*p) { (void)hipFree(*p); *p = nullptr; }
    if (cnt == 0) cnt = 1;
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
void ufree(Tv *&p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

unsigned ugrid(uint64_t work, unsigned nt, unsigned cap = 16384)
{
    uint64_t g = (work + nt - 1) / nt;
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(g, cap));
}

template <typename Tv>
__global__ void k_ufill(Tv *p, uint64_t cnt, Tv v)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < cnt;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename Tv>
void ufill(Tv *p, uint64_t cnt, Tv v, hipStream_t s)
{
    if (cnt) k_ufill<Tv><<<ugrid(cnt, 256), 256, 0, s>>>(p, cnt, v);
}

// ---------------------------------------------------------------------------
// U1: pair matching
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t tail_of(const uint32_t *row, uint32_t n, uint32_t e)
{
    // largest u with row[u] <= e (row non-decreasing, row[0] = 0 <= e < row[n])
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (row[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint64_t slot_hash(uint64_t key)
{
    return sm64_finalise(key + IM_GOLDEN);
}

// insert arc e under its unordered end points; val[dir][slot] = e where
// dir = 1 for the direction whose tail is the larger id
__global__ __launch_bounds__(256) void k_pair_insert(const uint32_t *row, const uint32_t *col,
                                                     uint32_t n, uint64_t m, uint64_t cap,
                                                     unsigned long long *keys, uint32_t *val,
                                                     uint32_t *pair, uint32_t *err)
{
    for (uint64_t e = blockIdx.x * 256ull + threadIdx.x; e < m; e += (uint64_t)gridDim.x * 256) {
        const uint32_t u = tail_of(row, n, (uint32_t)e), v = col[e];
        if (u == v) {
            if (pair) pair[e] = (uint32_t)e;   // a self-loop is its own pair
            continue;
        }
        const uint32_t lo = min(u, v), hi = max(u, v);
        const unsigned long long key = ((unsigned long long)lo << 32) | hi;
        uint64_t h = slot_hash(key) & (cap - 1);
        for (uint64_t probe = 0;; probe++) {
            if (probe == cap) { atomicOr(err, (uint32_t)UE_BIG); return; }
            const unsigned long long prev = atomicCAS(&keys[h], (unsigned long long)KEY_EMPTY, key);
            if (prev == KEY_EMPTY || prev == key) break;
            h = (h + 1) & (cap - 1);
        }
        const uint32_t dir = u > v ? 1u : 0u;
        if (atomicCAS(&val[dir * cap + h], NONE, (uint32_t)e) != NONE)
            atomicOr(err, (uint32_t)UE_PARALLEL);
    }
}

// every used slot: both directions present with equal probabilities; append
// the canonical arc (lo -> hi) to the pair list (one atomic per block and
// chunk of PC_SLOTS slots); pair ids of both arcs
constexpr int PC_PER = 16, PC_SLOTS = 256 * PC_PER;

__device__ __forceinline__ bool pair_ok(const unsigned long long *keys, const uint32_t *val,
                                        uint64_t cap, const float *prob, uint64_t h,
                                        uint32_t *err)
{
    if (h >= cap || keys[h] == KEY_EMPTY) return false;
    const uint32_t c = val[h], r = val[cap + h];
    if (c == NONE || r == NONE) { atomicOr(err, (uint32_t)UE_MISSING); return false; }
    if (__float_as_uint(prob[c]) != __float_as_uint(prob[r])) {
        atomicOr(err, (uint32_t)UE_PROB);
        return false;
    }
    return true;
}

__global__ __launch_bounds__(256) void k_pair_collect(const unsigned long long *keys,
                                                      const uint32_t *val, uint64_t cap,
                                                      const float *prob, uint32_t *pu,
                                                      uint32_t *pv, uint32_t *pe, uint32_t *np,
                                                      uint32_t *pair, uint32_t *err)
{
    __shared__ uint32_t s_w[256 / 64 + 1];
    __shared__ uint32_t s_base;
    for (uint64_t c0 = (uint64_t)blockIdx.x * PC_SLOTS; c0 < cap; c0 += (uint64_t)gridDim.x * PC_SLOTS) {
        uint32_t mine = 0;
        for (int j = 0; j < PC_PER; j++)
            mine += pair_ok(keys, val, cap, prob, c0 + (uint64_t)j * 256 + threadIdx.x, err) ? 1u : 0u;
        uint32_t total;
        const uint32_t ex = block_excl_scan<256>(mine, s_w, &total);
        if (threadIdx.x == 0) s_base = total ? atomicAdd(np, total) : 0u;
        __syncthreads();
        uint32_t q = s_base + ex;
        for (int j = 0; j < PC_PER && mine; j++) {
            const uint64_t h = c0 + (uint64_t)j * 256 + threadIdx.x;
            if (h >= cap || keys[h] == KEY_EMPTY) continue;
            const uint32_t c = val[h], r = val[cap + h];
            if (c == NONE || r == NONE || __float_as_uint(prob[c]) != __float_as_uint(prob[r])) continue;
            const unsigned long long key = keys[h];
            pu[q] = (uint32_t)(key >> 32);
            pv[q] = (uint32_t)key;
            pe[q] = c;
            if (pair) { pair[c] = c; pair[r] = c; }
            q++;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// U2: per-snapshot union-find over the live pairs
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t load_parent(const uint32_t *p)
{
    // device-coherent load: another CU may just have hooked this root
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t uf_root(uint32_t *par, uint32_t x)
{
    for (;;) {
        const uint32_t p = load_parent(&par[x]);
        if (p == x) return x;
        const uint32_t gp = load_parent(&par[p]);
        if (gp != p)   // path halving: gp is still an ancestor of x
            __hip_atomic_store(&par[x], gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = gp;
    }
}

__device__ __forceinline__ void uf_union(uint32_t *par, uint32_t a, uint32_t b)
{
    for (;;) {
        a = uf_root(par, a);
        b = uf_root(par, b);
        if (a == b) return;
        if (a > b) { const uint32_t t = a; a = b; b = t; }
        // hook the larger root under the smaller; fails if b stopped being a root
        if (atomicCAS(&par[b], b, a) == b) return;
    }
}

__global__ __launch_bounds__(256) void k_und_union(const uint32_t *pu, const uint32_t *pv,
                                                   const uint32_t *pe, const uint32_t *np,
                                                   const float *prob, uint32_t n, uint32_t R,
                                                   uint64_t seed, uint32_t *lab)
{
    const uint32_t P = *np;
    const uint32_t w = blockIdx.y;
    const uint32_t r0 = w * 64u;
    const uint32_t cnt = min(64u, R - r0);
    for (uint32_t j = blockIdx.x * 256u + threadIdx.x; j < P; j += gridDim.x * 256u) {
        const uint32_t e = pe[j];
        const uint64_t thr = (uint64_t)((double)prob[e] * 4294967296.0);
        uint64_t word = 0;
        if (thr >= (1ull << 32)) {
            word = im_valid_bits(R, w);
        } else if (thr) {
            const uint64_t key = sm64_finalise(seed + ((uint64_t)e + 1ull) * IM_GOLDEN);
            uint64_t z = key + (uint64_t)(r0 + 1u) * IM_GOLDEN;
            for (uint32_t bt = 0; bt < cnt; bt++) {
                word |= (uint64_t)((sm64_finalise(z) >> 32) < thr) << bt;
                z += IM_GOLDEN;
            }
        }
        const uint32_t a = pu[j], b = pv[j];
        while (word) {
            const uint32_t bt = (uint32_t)__ffsll((unsigned long long)word) - 1;
            word &= word - 1;
            uf_union(lab + (uint64_t)(r0 + bt) * n, a, b);
        }
    }
}

// ---------------------------------------------------------------------------
// U3: roots, sizes, initial gains
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_und_init_labels(uint32_t *lab, uint32_t n, uint64_t total)
{
    for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < total; i += (uint64_t)gridDim.x * 256)
        lab[i] = (uint32_t)(i % n);
}

// Per wavefront, lanes whose keys (a, b) agree form groups; the first lane
// of each group adds the group's size to cnt[idx] atomically and every lane
// gets its rank: returns the value cnt[idx] had plus the lane's rank in its group.
__device__ __forceinline__ uint32_t wave_group_add(bool act, uint64_t idx, uint32_t *cnt)
{
    const uint32_t lane = threadIdx.x & 63;
    uint32_t rank = 0;
    unsigned long long pending = __ballot(act);
    while (pending) {
        const int leader = __ffsll(pending) - 1;
        const uint64_t li = __shfl(idx, leader, 64);
        const unsigned long long same = __ballot(act && idx == li) & pending;
        uint32_t base = 0;
        if ((int)lane == leader) base = atomicAdd(&cnt[li], (uint32_t)__popcll(same));
        base = __shfl(base, leader, 64);
        if ((same >> lane) & 1ull) rank = base + (uint32_t)__popcll(same & ((1ull << lane) - 1ull));
        pending &= ~same;
    }
    return rank;
}

// lab[r][u] = root of u. A non-root member takes a rank among its root's
// other members (cnt[r][root] counts them; roots are component minima, so
// the root itself is the member with the smallest id).
__global__ __launch_bounds__(256) void k_und_flatten(uint32_t *lab, uint32_t *cnt, uint32_t *rk,
                                                     uint32_t n, uint64_t total)
{
    for (uint64_t base = blockIdx.x * 256ull; base < total; base += (uint64_t)gridDim.x * 256) {
        const uint64_t i = base + threadIdx.x;
        uint32_t root = 0, x = 0;
        uint64_t off = 0;
        if (i < total) {
            // the forests are final here: a read-only walk to the root. Other
            // threads replace parents by roots meanwhile; a replaced entry
            // still leads to the same root, and no entry is ever changed to
            // anything but its root (no path compression in this pass).
            x = (uint32_t)(i % n);
            off = i - x;
            const uint32_t *par = lab + off;
            root = x;
            for (uint32_t p = par[root]; p != root; p = par[root]) root = p;
            lab[i] = root;
        }
        const bool member = i < total && root != x;
        const uint32_t r = wave_group_add(member, off + root, cnt);
        if (member) rk[i] = r;
    }
}

// members into the lists: start = exclusive prefix sum of cnt over all
// (snapshot, root) entries, mem[start[r][root] + rank] = u
__global__ __launch_bounds__(256) void k_und_scatter(const uint32_t *lab, const uint32_t *rk,
                                                     const uint32_t *start, uint32_t *mem,
                                                     uint32_t n, uint64_t total)
{
    for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < total; i += (uint64_t)gridDim.x * 256) {
        const uint32_t x = (uint32_t)(i % n);
        const uint64_t off = i - x;
        const uint32_t root = lab[i];
        if (root != x) mem[start[off + root] + rk[i]] = x;
    }
}

__device__ __forceinline__ void block_key_max(unsigned long long best, unsigned long long *red,
                                              unsigned long long *key_out)
{
    best = wave_max_u64(best);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long b = 0;
        for (int i = 0; i < UN_NT / 64; i++) b = red[i] > b ? red[i] : b;
        if (b) atomicMax(key_out, b);
    }
}

// s_u = sum_r |C_r(u)| and the round-0 argmax key (gain << 32 | ~u)
__global__ __launch_bounds__(UN_NT) void k_und_gains(const uint32_t *lab, const uint32_t *cnt,
                                                     uint32_t n, uint32_t R, uint32_t *gain,
                                                     unsigned long long *key_out)
{
    __shared__ unsigned long long s_red[UN_NT / 64];
    unsigned long long best = 0;
    for (uint32_t u = blockIdx.x * UN_NT + threadIdx.x; u < n; u += gridDim.x * UN_NT) {
        uint64_t sum = 0;
        for (uint32_t r = 0; r < R; r++) {
            const uint64_t o = (uint64_t)r * n;
            sum += (cnt[o + lab[o + u]] & ~COVERED) + 1u;
        }
        gain[u] = (uint32_t)sum;
        const unsigned long long k = (sum << 32) | (0xFFFFFFFFu - u);
        best = k > best ? k : best;
    }
    block_key_max(best, s_red, key_out);
}

// U4: one workgroup per snapshot. The picked node v* covers its component C
// if still uncovered: every member (the root and its listed members) loses
// |C|. Workgroup 0 records the pick.
__global__ __launch_bounds__(UN_NT) void k_und_cover(const unsigned long long *key, uint32_t t,
                                                     const uint32_t *lab, uint32_t *cnt,
                                                     const uint32_t *start, const uint32_t *mem,
                                                     uint32_t n, uint8_t *sel, uint32_t *gain,
                                                     uint32_t *seeds_out, uint64_t *gains_out)
{
    const unsigned long long k = *key;
    const uint32_t v = 0xFFFFFFFFu - (uint32_t)(k & 0xFFFFFFFFull);
    const uint32_t r = blockIdx.x;
    if (r == 0 && threadIdx.x == 0) {
        seeds_out[t] = v;
        gains_out[t] = k >> 32;
        sel[v] = 1;
    }
    const uint64_t o = (uint64_t)r * n;
    const uint32_t root = lab[o + v];
    const uint32_t z = cnt[o + root];
    if (z & COVERED) return;   // uniform over the workgroup
    __syncthreads();           // every thread has read z before it is marked
    const uint32_t size = z + 1;
    if (threadIdx.x == 0) {
        cnt[o + root] = z | COVERED;
        atomicSub(&gain[root], size);
    }
    const uint32_t *m = mem + (z ? start[o + root] : 0u);
    for (uint32_t i = threadIdx.x; i < z; i += UN_NT) atomicSub(&gain[m[i]], size);
}

// U5: the next round's key over the unselected nodes
__global__ __launch_bounds__(UN_NT) void k_und_argmax(const uint32_t *gain, const uint8_t *sel,
                                                      uint32_t n, unsigned long long *key_out)
{
    __shared__ unsigned long long s_red[UN_NT / 64];
    unsigned long long best = 0;
    for (uint32_t u = blockIdx.x * UN_NT + threadIdx.x; u < n; u += gridDim.x * UN_NT) {
        if (sel[u]) continue;
        const unsigned long long k = ((unsigned long long)gain[u] << 32) | (0xFFFFFFFFu - u);
        best = k > best ? k : best;
    }
    block_key_max(best, s_red, key_out);
}

__global__ void k_und_copy(const uint32_t *src, uint32_t *dst, uint32_t n)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        dst[i] = src[i];
}

}  // namespace

// ---------------------------------------------------------------------------
// state hung off a workspace
// ---------------------------------------------------------------------------
struct UndState {
    uint32_t cap_n = 0;
    uint64_t cap_m = 0, cap_nR = 0, cap_slots = 0;
    unsigned long long *keys = nullptr;   // [cap_slots] hash keys
    uint32_t *val = nullptr;              // [2][cap_slots]
    uint32_t *pu = nullptr, *pv = nullptr, *pe = nullptr;  // canonical pairs
    uint32_t *np = nullptr, *err = nullptr, *host_err = nullptr;
    uint32_t *row32 = nullptr;
    uint32_t *lab = nullptr, *cnt = nullptr, *rk = nullptr, *start = nullptr,
             *mem = nullptr;                     // [R][n]
    uint32_t *sums = nullptr;                    // scan scratch
    uint64_t cap_sums = 0;
    uint32_t *gain = nullptr;
    uint8_t *sel = nullptr;
    unsigned long long *ukeys = nullptr;         // [k+1] argmax keys
    uint32_t cap_k = 0;
};

void und_state_free(UndState *st)
{
    if (!st) return;
    ufree(st->keys); ufree(st->val); ufree(st->pu); ufree(st->pv); ufree(st->pe);
    ufree(st->np); ufree(st->err); ufree(st->row32); ufree(st->lab); ufree(st->cnt);
    ufree(st->rk); ufree(st->start); ufree(st->mem); ufree(st->sums);
    ufree(st->gain); ufree(st->sel); ufree(st->ukeys);
    if (st->host_err) (void)hipHostFree(st->host_err);
    delete st;
}

static int und_state(im_workspace *ws, UndState **out)
{
    UndState *&st = *im_ws_und(ws);
    if (!st) {
        st = new UndState();
        int rc;
        if ((rc = ualloc(&st->np, 1)) || (rc = ualloc(&st->err, 1))) return rc;
        HIPCHK(hipHostMalloc((void **)&st->host_err, sizeof(uint32_t), hipHostMallocDefault));
    }
    *out = st;
    return IM_OK;
}

static int reserve_pairs(UndState *st, uint32_t n, uint64_t m)
{
    int rc;
    uint64_t slots = 1024;
    while (slots < m + 1) slots <<= 1;   // load factor <= 1/2 (m/2 pairs)
    if (slots > st->cap_slots) {
        if ((rc = ualloc(&st->keys, slots)) || (rc = ualloc(&st->val, 2 * slots))) return rc;
        st->cap_slots = slots;
    }
    if (m > st->cap_m || !st->pu) {
        const uint64_t cm = std::max<uint64_t>(m, st->cap_m);
        if ((rc = ualloc(&st->pu, cm / 2 + 1)) || (rc = ualloc(&st->pv, cm / 2 + 1)) ||
            (rc = ualloc(&st->pe, cm / 2 + 1)))
            return rc;
        st->cap_m = cm;
    }
    if (n > st->cap_n || !st->row32) {
        const uint32_t cn = std::max(n, st->cap_n);
        if ((rc = ualloc(&st->row32, (uint64_t)cn + 1)) || (rc = ualloc(&st->gain, cn)) ||
            (rc = ualloc(&st->sel, cn)))
            return rc;
        st->cap_n = cn;
    }
    return IM_OK;
}

// U1 on a validated graph (st->row32 filled): the canonical pair list, and
// pair ids of every arc if `pair` is non-null
static int match_pairs(const im_graph *g, UndState *st, uint32_t *pair, hipStream_t s)
{
    const uint64_t m = g->m, cap = st->cap_slots;
    ufill<uint32_t>(st->np, 1, 0u, s);
    ufill<uint32_t>(st->err, 1, 0u, s);
    if (m) {
        ufill<unsigned long long>(st->keys, cap, (unsigned long long)KEY_EMPTY, s);
        ufill<uint32_t>(st->val, 2 * cap, NONE, s);
        k_pair_insert<<<ugrid(m, 256), 256, 0, s>>>(st->row32, g->col, g->n, m, cap, st->keys,
                                                    st->val, pair, st->err);
        k_pair_collect<<<ugrid(cap, 256), 256, 0, s>>>(st->keys, st->val, cap, g->prob, st->pu,
                                                       st->pv, st->pe, st->np, pair, st->err);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(st->host_err, st->err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const uint32_t e = *st->host_err;
    if (e & UE_PARALLEL) return im_fail(IM_EINVAL, "undirected graph: a pair is stored twice in one direction");
    if (e & UE_MISSING) return im_fail(IM_EINVAL, "undirected graph: an arc's reverse is not stored");
    if (e & UE_PROB) return im_fail(IM_EINVAL, "undirected graph: the two directions of a pair differ in probability");
    if (e & UE_BIG) return im_fail(IM_EINVAL, "pair table full");
    return IM_OK;
}

int und_pair_ids(const im_graph *g, const uint32_t *row32, uint32_t *pair, im_workspace *ws,
                 hipStream_t s)
{
    UndState *st;
    int rc;
    if ((rc = und_state(ws, &st)) || (rc = reserve_pairs(st, g->n, g->m))) return rc;
    if (g->n)
        HIPCHK(hipMemcpyAsync(st->row32, row32, ((uint64_t)g->n + 1) * sizeof(uint32_t),
                              hipMemcpyDeviceToDevice, s));
    return match_pairs(g, st, pair, s);
}

extern "C" int im_pair_ids(const im_graph *g, uint32_t *pair_out, im_workspace *ws, void *stream)
{
    int rc;
    if (!g || !ws) return im_fail(IM_EINVAL, "null graph or workspace");
    if (g->m && !pair_out) return im_fail(IM_EINVAL, "null output");
    if (g->m >= (1ull << 32)) return im_fail(IM_EINVAL, "m must be < 2^32");
    hipStream_t s = (hipStream_t)stream;
    UndState *st;
    if ((rc = und_state(ws, &st)) || (rc = reserve_pairs(st, g->n, g->m))) return rc;
    if ((rc = im_ws_validate(g, ws, s, st->row32))) return rc;
    if ((rc = match_pairs(g, st, pair_out, s))) return rc;
    im_ws_set_last_stream(ws, s);
    return IM_OK;
}

extern "C" int im_select_undirected(const im_graph *g, uint32_t R, uint32_t k, uint64_t seed,
                                    uint32_t *seeds_out, uint64_t *gains_out, uint32_t *trace_out,
                                    im_workspace *ws, void *stream)
{
    int rc;
    if (!g || !ws) return im_fail(IM_EINVAL, "null graph or workspace");
    if (g->m >= (1ull << 32)) return im_fail(IM_EINVAL, "m must be < 2^32");
    if (!g->row_ptr || (g->m && (!g->col || !g->prob))) return im_fail(IM_EINVAL, "null graph array");
    if (R == 0 || R > IM_R_MAX) return im_fail(IM_EINVAL, "R = %u must be in [1, %u]", R, IM_R_MAX);
    const uint32_t n = g->n;
    if ((uint64_t)n * R >= (1ull << 32))
        return im_fail(IM_EOVERFLOW, "n * R = %llu must be < 2^32", (unsigned long long)n * R);
    if (k > n) return im_fail(IM_EINVAL, "k = %u exceeds n = %u", k, n);
    if (k && (!seeds_out || !gains_out)) return im_fail(IM_EINVAL, "null seeds or gains output");
    hipStream_t s = (hipStream_t)stream;
    UndState *st;
    if ((rc = und_state(ws, &st)) || (rc = reserve_pairs(st, n, g->m))) return rc;
    const uint64_t nR = (uint64_t)n * R;
    if (nR > st->cap_nR || !st->lab) {
        if ((rc = ualloc(&st->lab, nR)) || (rc = ualloc(&st->cnt, nR)) || (rc = ualloc(&st->rk, nR)) ||
            (rc = ualloc(&st->start, nR)) || (rc = ualloc(&st->mem, nR)))
            return rc;
        st->cap_nR = nR;
    }
    if (im_scan_sums_len(nR) > st->cap_sums || !st->sums) {
        if ((rc = ualloc(&st->sums, im_scan_sums_len(nR)))) return rc;
        st->cap_sums = im_scan_sums_len(nR);
    }
    if (k + 1 > st->cap_k || !st->ukeys) {
        if ((rc = ualloc(&st->ukeys, (uint64_t)k + 1))) return rc;
        st->cap_k = k + 1;
    }
    if ((rc = im_ws_validate(g, ws, s, st->row32))) return rc;
    if ((rc = match_pairs(g, st, nullptr, s))) return rc;
    if (n == 0) { im_ws_set_last_stream(ws, s); return IM_OK; }

    // U2: forests of all snapshots
    k_und_init_labels<<<ugrid(nR, 256), 256, 0, s>>>(st->lab, n, nR);
    ufill<uint32_t>(st->cnt, nR, 0u, s);
    const uint32_t W = (R + 63) / 64;
    if (g->m) {
        dim3 grid(ugrid(g->m / 2 + 1, 256, 8192), W);
        k_und_union<<<grid, 256, 0, s>>>(st->pu, st->pv, st->pe, st->np, g->prob, n, R, seed,
                                         st->lab);
    }
    // U3: roots, member lists, initial gains and the round-0 key
    k_und_flatten<<<ugrid(nR, 256), 256, 0, s>>>(st->lab, st->cnt, st->rk, n, nR);
    im_exclusive_scan(st->cnt, st->start, nR, st->sums, s);
    k_und_scatter<<<ugrid(nR, 256), 256, 0, s>>>(st->lab, st->rk, st->start, st->mem, n, nR);
    ufill<uint8_t>(st->sel, n, (uint8_t)0, s);
    ufill<unsigned long long>(st->ukeys, (uint64_t)k + 1, 0ull, s);
    const unsigned ug = ugrid(n, UN_NT, 4096);
    k_und_gains<<<ug, UN_NT, 0, s>>>(st->lab, st->cnt, n, R, st->gain, st->ukeys);
    for (uint32_t t = 0; t < k; t++) {
        if (trace_out)
            k_und_copy<<<ugrid(n, 256), 256, 0, s>>>(st->gain, trace_out + (uint64_t)t * n, n);
        k_und_cover<<<R, UN_NT, 0, s>>>(st->ukeys + t, t, st->lab, st->cnt, st->start, st->mem, n,
                                        st->sel, st->gain, seeds_out, gains_out);
        k_und_argmax<<<ugrid(n, UN_NT, 256), UN_NT, 0, s>>>(st->gain, st->sel, n, st->ukeys + t + 1);
    }
    if (trace_out)
        k_und_copy<<<ugrid(n, 256), 256, 0, s>>>(st->gain, trace_out + (uint64_t)k * n, n);
    HIPCHK(hipGetLastError());
    im_ws_set_last_stream(ws, s);
    return IM_OK;
}
