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
// Two engines share this definition:
//   * the wavefront engine keeps T tasks per wavefront, each in an
//     LDS-resident open-addressing table of CS entries; a task whose table
//     fills, or which meets a node with degree > DMAX, is handed over whole
//     to the overflow queue;
//   * the block engine keeps one task per workgroup in dense per-slot global
//     arrays of length n (reach, pending bits, frontier queues, visit list).
#pragma once

#include "im_device.h"

enum { MODE_COUNT = 0, MODE_DEC = 1 };

// statistics slots (uint64 counters in device memory)
enum {
    ST_TRAV_INIT = 0, ST_TRAV_FWD, ST_TRAV_REV,
    ST_RELAX_INIT, ST_REACHED_INIT, ST_RELAX_REV, ST_REACHED_REV, ST_RELAX_FWD,
    ST_ARCS_INIT, ST_ARCS_REV, ST_OVF_INIT, ST_OVF_REV, ST_TASKS_REV, ST_DECREMENTS,
    ST_CELF_EVALS, ST_COUNT = 32
};

struct BfsArgs {
    // graph in the direction of this pass
    const uint32_t *row;      // [n+1]
    const uint32_t *col;      // [m]
    const uint64_t *mask;     // [W][m], word-major
    uint64_t m;
    uint32_t n, R, W;
    const uint64_t *prune;    // [W][n] or nullptr
    uint32_t *gain;           // [n]
    // task source
    uint32_t ntasks;          // MODE_COUNT: n*W (task t -> word t/n, node t%n)
    const uint32_t *tnodes;   // MODE_DEC: per-word node lists [W][n]
    const uint32_t *tcounts;  // MODE_DEC: [W] list lengths
    const uint64_t *tbits;    // MODE_DEC: start bits [W][n]
    // scheduling counters (zero before launch)
    uint32_t *grab;           // wavefront engine task counter
    uint32_t *ovf_q;          // overflow queue of task ids
    uint32_t *ovf_n;          // its length
    uint32_t *bgrab;          // block engine task counter
    // block engine slots
    uint64_t *b_reach, *b_pend, *b_fdel;   // [slots][n]
    uint32_t *b_qa, *b_qb, *b_vis;         // [slots][n]
    unsigned long long *stats;
    int st_trav, st_relax, st_reached, st_arcs, st_ovf;
};


// Decode a task id into (start node, word, start bits). Returns false when
// the task has nothing to propagate.
__device__ __forceinline__ bool decode_task(const BfsArgs &a, int mode, uint32_t t,
                                            const uint32_t *wpre, uint32_t &src,
                                            uint32_t &w, uint64_t &bits)
{
    if (mode == MODE_COUNT) {
        w = t / a.n;
        src = t - w * a.n;
        bits = im_valid_bits(a.R, w);
        if (a.prune) bits &= ~a.prune[(uint64_t)w * a.n + src];
    } else {
        w = 0;
        while (w + 1 < a.W && wpre[w + 1] <= t) w++;
        src = a.tnodes[(uint64_t)w * a.n + (t - wpre[w])];
        bits = a.tbits[(uint64_t)w * a.n + src];
    }
    return bits != 0;
}

// ---------------------------------------------------------------------------
// Wavefront engine
// ---------------------------------------------------------------------------
template <int T, int CS>
struct WaveLds {
    uint32_t keys[T * CS];
    uint64_t reach[T * CS];
    uint64_t pend[T * CS];
    uint64_t fdel[T * CS];
    uint32_t deg[T * CS];
    uint32_t fr[2][T * CS];
    uint32_t c_excl[64];
    uint32_t c_rs[64];
    uint32_t c_idx[64];
    uint64_t c_del[64];
    uint32_t s_task[T], s_src[T], s_word[T], s_cnt[T], s_next[T], s_ovf[T], s_act[T];
    uint32_t wpre[65];
    uint32_t nf, nn, tnext, tend, ntasks, done;
};

__device__ __forceinline__ uint32_t slot_hash(uint32_t v) { return v * 0x9E3779B1u; }

template <int MODE, int T, int CS, int LIM, int DMAX, bool PRUNE>
__global__ __launch_bounds__(64) void k_wave_bfs(BfsArgs a)
{
    static_assert((CS & (CS - 1)) == 0, "CS must be a power of two");
    constexpr int LOG_CS = __builtin_ctz(CS);
    constexpr int N = T * CS;
    constexpr uint32_t CHUNK = 16;
    __shared__ WaveLds<T, CS> L;
    const int lane = threadIdx.x;

    for (int i = lane; i < N; i += 64) {
        L.keys[i] = IM_EMPTY; L.reach[i] = 0; L.pend[i] = 0; L.deg[i] = 0;
    }
    if (lane < T) {
        L.s_act[lane] = 0; L.s_cnt[lane] = 0; L.s_next[lane] = 0; L.s_ovf[lane] = 0;
    }
    if (lane == 0) {
        L.nf = 0; L.nn = 0; L.tnext = 0; L.tend = 0; L.done = 0;
        if (MODE == MODE_COUNT) {
            L.ntasks = a.ntasks;
        } else {
            uint32_t s = 0;
            for (uint32_t w = 0; w < a.W; w++) { L.wpre[w] = s; s += a.tcounts[w]; }
            L.wpre[a.W] = s;
            L.ntasks = s;
        }
    }
    __syncthreads();

    uint64_t st_relax = 0, st_reached = 0, st_arcs = 0, st_trav = 0, st_ovf = 0, st_dec = 0;
    int cur = 0;

    for (;;) {
        // ---- refill idle slots with new tasks (lane 0 grabs, all lanes wait)
        if (lane == 0 && !L.done) {
            for (int s = 0; s < T; s++) {
                if (L.s_act[s]) continue;
                for (;;) {
                    if (L.tnext == L.tend) {
                        uint32_t b = atomicAdd(a.grab, CHUNK);
                        if (b >= L.ntasks) { L.done = 1; break; }
                        L.tnext = b;
                        L.tend = min(b + CHUNK, L.ntasks);
                    }
                    uint32_t t = L.tnext++;
                    uint32_t src, w;
                    uint64_t bits;
                    if (!decode_task(a, MODE, t, L.wpre, src, w, bits)) continue;
                    uint32_t idx = s * CS + (slot_hash(src) >> (32 - LOG_CS));
                    L.keys[idx] = src;
                    L.reach[idx] = bits;
                    L.pend[idx] = bits;
                    L.s_task[s] = t; L.s_src[s] = src; L.s_word[s] = w;
                    L.s_cnt[s] = 1; L.s_ovf[s] = 0; L.s_next[s] = 0; L.s_act[s] = 1;
                    L.fr[cur][L.nf++] = idx;
                    break;
                }
                if (L.done) break;
            }
        }
        __syncthreads();
        const uint32_t nf = L.nf;
        if (nf == 0) break;

        // ---- phase A: take the pending bits of every frontier entry
        for (uint32_t i = lane; i < nf; i += 64) {
            uint32_t idx = L.fr[cur][i];
            L.fdel[i] = L.pend[idx];
            L.pend[idx] = 0;
        }
        if (lane < T) L.s_next[lane] = 0;
        if (lane == 0) L.nn = 0;
        __syncthreads();

        // ---- phase B: expand, 64 frontier entries per chunk, arcs spread over lanes
        for (uint32_t base = 0; base < nf; base += 64) {
            uint32_t i = base + lane;
            uint32_t deg = 0, rs = 0, idx = 0;
            uint64_t d = 0;
            if (i < nf) {
                idx = L.fr[cur][i];
                uint32_t s = idx >> LOG_CS;
                if (!L.s_ovf[s]) {
                    uint32_t x = L.keys[idx];
                    rs = a.row[x];
                    deg = a.row[x + 1] - rs;
                    if (deg > (uint32_t)DMAX) { L.s_ovf[s] = 1; deg = 0; }
                    else { L.deg[idx] = deg; d = L.fdel[i]; }
                }
            }
            uint32_t incl = wave_incl_scan(deg);
            uint32_t total = __shfl(incl, 63, 64);
            L.c_excl[lane] = incl - deg;
            L.c_rs[lane] = rs;
            L.c_idx[lane] = idx;
            L.c_del[lane] = d;
            __syncthreads();
            st_arcs += total;
            for (uint32_t j = lane; j < total; j += 64) {
                int k = upper_index<64>(L.c_excl, j);
                uint32_t e = L.c_rs[k] + (j - L.c_excl[k]);
                uint32_t cidx = L.c_idx[k];
                uint32_t s = cidx >> LOG_CS;
                uint64_t w = L.s_word[s];
                uint64_t bits = L.c_del[k] & a.mask[w * a.m + e];
                if (!bits) continue;
                uint32_t v = a.col[e];
                if (PRUNE) {
                    bits &= ~a.prune[w * a.n + v];
                    if (!bits) continue;
                }
                // find or insert v in slot s
                uint32_t h = slot_hash(v) >> (32 - LOG_CS);
                int found = -1;
                for (int p = 0; p < CS; p++) {
                    uint32_t pos = s * CS + h;
                    uint32_t kk = L.keys[pos];
                    if (kk == v) { found = (int)pos; break; }
                    if (kk == IM_EMPTY) {
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
                if (found < 0) { L.s_ovf[s] = 1; continue; }
                uint64_t old = atomicOr((unsigned long long *)&L.reach[found], (unsigned long long)bits);
                uint64_t nb = bits & ~old;
                if (nb) {
                    uint64_t op = atomicOr((unsigned long long *)&L.pend[found], (unsigned long long)nb);
                    if (op == 0) {
                        uint32_t q = atomicAdd(&L.nn, 1u);
                        L.fr[cur ^ 1][q] = (uint32_t)found;
                        atomicAdd(&L.s_next[s], 1u);
                    }
                }
            }
            __syncthreads();
        }

        // ---- finish slots whose search ended or overflowed
        bool any_ovf_fin = false;
        for (int s = 0; s < T; s++) {
            if (!L.s_act[s]) continue;
            bool ovf = L.s_ovf[s] != 0;
            if (!ovf && L.s_next[s] != 0) continue;
            uint32_t base = s * CS;
            if (ovf) {
                any_ovf_fin = true;
                if (lane == 0) {
                    uint32_t q = atomicAdd(a.ovf_n, 1u);
                    a.ovf_q[q] = L.s_task[s];
                }
                st_ovf += (lane == 0);
            } else {
                uint64_t cnt = 0;
                for (int i = lane; i < CS; i += 64) {
                    uint32_t key = L.keys[base + i];
                    if (key == IM_EMPTY) continue;
                    uint32_t pc = (uint32_t)__popcll(L.reach[base + i]);
                    uint32_t dg = L.deg[base + i];
                    st_relax += dg;
                    st_reached += 1;
                    st_trav += (uint64_t)pc * dg;
                    if (MODE == MODE_COUNT) cnt += pc;
                    else { atomicSub(&a.gain[key], pc); st_dec += pc; }
                }
                if (MODE == MODE_COUNT) {
                    cnt = wave_sum_u64(cnt);
                    if (lane == 0) atomicAdd(&a.gain[L.s_src[s]], (uint32_t)cnt);
                }
            }
            for (int i = lane; i < CS; i += 64) {
                L.keys[base + i] = IM_EMPTY; L.reach[base + i] = 0;
                L.pend[base + i] = 0; L.deg[base + i] = 0;
            }
            __syncthreads();
            if (lane == 0) { L.s_act[s] = 0; L.s_cnt[s] = 0; L.s_ovf[s] = 0; }
            __syncthreads();
        }

        // ---- drop next-frontier entries that belong to slots just handed over
        uint32_t nn = L.nn;
        if (any_ovf_fin) {
            uint32_t w = 0;
            for (uint32_t base = 0; base < nn; base += 64) {
                uint32_t i = base + lane;
                uint32_t idx = i < nn ? L.fr[cur ^ 1][i] : 0;
                bool keep = i < nn && L.s_act[idx >> LOG_CS];
                uint64_t bal = __ballot(keep);
                uint32_t before = (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
                __syncthreads();
                if (keep) L.fr[cur ^ 1][w + before] = idx;
                w += (uint32_t)__popcll(bal);
                __syncthreads();
            }
            nn = w;
        }
        __syncthreads();
        if (lane == 0) L.nf = nn;
        cur ^= 1;
        __syncthreads();
    }

    // ---- per-wavefront statistics
    st_relax = wave_sum_u64(st_relax);
    st_reached = wave_sum_u64(st_reached);
    st_trav = wave_sum_u64(st_trav);
    st_dec = wave_sum_u64(st_dec);
    if (lane == 0) {
        if (MODE == MODE_DEC) atomicAdd(&a.stats[ST_DECREMENTS], (unsigned long long)st_dec);
        atomicAdd(&a.stats[a.st_relax], (unsigned long long)st_relax);
        atomicAdd(&a.stats[a.st_reached], (unsigned long long)st_reached);
        atomicAdd(&a.stats[a.st_trav], (unsigned long long)st_trav);
        atomicAdd(&a.stats[a.st_arcs], (unsigned long long)st_arcs);
        atomicAdd(&a.stats[a.st_ovf], (unsigned long long)st_ovf);
    }
}

// ---------------------------------------------------------------------------
// Block engine: one task per workgroup, dense arrays of length n per slot.
// reach and pend are all-zero on entry and are left all-zero on exit.
// ---------------------------------------------------------------------------
template <int NT>
struct BlockLds {
    uint32_t scan[NT];
    uint32_t rs[NT];
    uint64_t del[NT];
    uint32_t wsum[NT / 64 + 1];
    uint32_t nf, nn, nvis, task;
    unsigned long long red[NT / 64];
};

// Run one task to its fixpoint; afterwards vis[0..L.nvis) lists every node
// with reach != 0.
template <int NT, bool PRUNE>
__device__ void block_bfs_run(BlockLds<NT> &L, uint32_t src, uint64_t start,
                              const uint32_t *row, const uint32_t *col, const uint64_t *mask,
                              const uint64_t *prune, uint64_t *reach, uint64_t *pend,
                              uint64_t *fdel, uint32_t *qa, uint32_t *qb, uint32_t *vis,
                              uint64_t &arcs)
{
    const int tid = threadIdx.x;
    if (tid == 0) {
        reach[src] = start;
        fdel[0] = start;
        qa[0] = src;
        vis[0] = src;
        L.nf = 1; L.nn = 0; L.nvis = 1;
    }
    __syncthreads();
    uint32_t *cur = qa, *nxt = qb;
    bool first = true;
    for (;;) {
        const uint32_t nf = L.nf;
        if (nf == 0) break;
        if (!first) {
            for (uint32_t i = tid; i < nf; i += NT) {
                uint32_t x = cur[i];
                fdel[i] = pend[x];
                pend[x] = 0;
            }
        }
        first = false;
        __syncthreads();
        for (uint32_t tile = 0; tile < nf; tile += NT) {
            uint32_t i = tile + tid;
            uint32_t deg = 0, rs = 0;
            uint64_t d = 0;
            if (i < nf) {
                uint32_t x = cur[i];
                rs = row[x];
                deg = row[x + 1] - rs;
                d = fdel[i];
            }
            uint32_t total;
            uint32_t ex = block_excl_scan<NT>(deg, L.wsum, &total);
            L.scan[tid] = ex;
            L.rs[tid] = rs;
            L.del[tid] = d;
            __syncthreads();
            arcs += total;
            for (uint32_t j = tid; j < total; j += NT) {
                int k = upper_index<NT>(L.scan, j);
                uint32_t e = L.rs[k] + (j - L.scan[k]);
                uint64_t bits = L.del[k] & mask[e];
                if (!bits) continue;
                uint32_t v = col[e];
                if (PRUNE) {
                    bits &= ~prune[v];
                    if (!bits) continue;
                }
                uint64_t old = atomicOr((unsigned long long *)&reach[v], (unsigned long long)bits);
                uint64_t nb = bits & ~old;
                if (!nb) continue;
                if (old == 0) vis[atomicAdd(&L.nvis, 1u)] = v;
                uint64_t op = atomicOr((unsigned long long *)&pend[v], (unsigned long long)nb);
                if (op == 0) nxt[atomicAdd(&L.nn, 1u)] = v;
            }
            __syncthreads();
        }
        if (tid == 0) { L.nf = L.nn; L.nn = 0; }
        uint32_t *t = cur; cur = nxt; nxt = t;
        __syncthreads();
    }
}

template <int MODE, int NT, bool PRUNE>
__global__ __launch_bounds__(NT) void k_block_bfs(BfsArgs a)
{
    __shared__ BlockLds<NT> L;
    __shared__ uint32_t wpre[65];
    const int tid = threadIdx.x;
    const uint64_t slot = blockIdx.x;
    uint64_t *reach = a.b_reach + slot * a.n;
    uint64_t *pend = a.b_pend + slot * a.n;
    uint64_t *fdel = a.b_fdel + slot * a.n;
    uint32_t *qa = a.b_qa + slot * a.n;
    uint32_t *qb = a.b_qb + slot * a.n;
    uint32_t *vis = a.b_vis + slot * a.n;
    if (tid == 0 && MODE == MODE_DEC) {
        uint32_t s = 0;
        for (uint32_t w = 0; w < a.W; w++) { wpre[w] = s; s += a.tcounts[w]; }
        wpre[a.W] = s;
    }
    __syncthreads();
    const uint32_t nq = *a.ovf_n;
    uint64_t arcs = 0, relax = 0, reached = 0, trav = 0, dec = 0;
    for (;;) {
        if (tid == 0) L.task = atomicAdd(a.bgrab, 1u);
        __syncthreads();
        const uint32_t q = L.task;
        __syncthreads();
        if (q >= nq) break;
        uint32_t src, w;
        uint64_t bits;
        if (!decode_task(a, MODE, a.ovf_q[q], wpre, src, w, bits)) continue;
        const uint64_t *mask = a.mask + (uint64_t)w * a.m;
        const uint64_t *prune = PRUNE ? a.prune + (uint64_t)w * a.n : nullptr;
        block_bfs_run<NT, PRUNE>(L, src, bits, a.row, a.col, mask, prune, reach, pend, fdel,
                                 qa, qb, vis, arcs);
        const uint32_t nvis = L.nvis;
        uint64_t cnt = 0;
        for (uint32_t i = tid; i < nvis; i += NT) {
            uint32_t x = vis[i];
            uint32_t pc = (uint32_t)__popcll(reach[x]);
            uint32_t dg = a.row[x + 1] - a.row[x];
            relax += dg;
            reached += 1;
            trav += (uint64_t)pc * dg;
            if (MODE == MODE_COUNT) cnt += pc;
            else { atomicSub(&a.gain[x], pc); dec += pc; }
            reach[x] = 0;
        }
        if (MODE == MODE_COUNT) {
            cnt = wave_sum_u64(cnt);
            if ((tid & 63) == 0) L.red[tid >> 6] = cnt;
            __syncthreads();
            if (tid == 0) {
                uint64_t s = 0;
                for (int i = 0; i < NT / 64; i++) s += L.red[i];
                atomicAdd(&a.gain[src], (uint32_t)s);
            }
        }
        __syncthreads();
    }
    arcs = (tid == 0) ? arcs : 0;  // arcs is uniform across the block
    relax = wave_sum_u64(relax);
    reached = wave_sum_u64(reached);
    trav = wave_sum_u64(trav);
    dec = wave_sum_u64(dec);
    if ((tid & 63) == 0) {
        if (MODE == MODE_DEC) atomicAdd(&a.stats[ST_DECREMENTS], (unsigned long long)dec);
        atomicAdd(&a.stats[a.st_relax], (unsigned long long)relax);
        atomicAdd(&a.stats[a.st_reached], (unsigned long long)reached);
        atomicAdd(&a.stats[a.st_trav], (unsigned long long)trav);
        if (tid == 0) atomicAdd(&a.stats[a.st_arcs], (unsigned long long)arcs);
    }
}
