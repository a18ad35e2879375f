/*
 * im.h -- C ABI of the MI355X StaticGreedy influence-maximization library.
 *
 * Problem (Cheng et al., CIKM 2013, Sec. 3.1): a directed graph G=(V,E)
 * with a propagation probability p(u,v) on every arc, under the
 * independent cascade model; find S, |S| <= k, maximising the spread.
 * Method: StaticGreedy (Sec. 3.3, Algorithm 1) on R snapshots sampled once,
 * with the marginal gains kept current by the dynamic update of Sec. 4
 * (Algorithm 2).
 *
 * Result definition (exact, integer):
 *   arc e is live in snapshot r iff draw(seed, e, r) < floor(p_e * 2^32),
 *     draw = top 32 bits of SplitMix64 output r+1 from state key_e,
 *     key_e = SplitMix64 output e+1 from state seed  (Steele et al. 2014);
 *   R_r(u) = nodes reachable from u over live arcs of snapshot r, u included;
 *   f(S) = sum_r |union_{s in S} R_r(s)|;
 *   round i adds the unselected node with the largest f(S+u) - f(S), ties to
 *   the lowest id, and reports that marginal gain (summed over snapshots,
 *   not divided by R).
 * Outputs depend only on (graph, prob, R, k, seed): not on the stream, the
 * workspace, the launch schedule or which selection path is used.
 *
 * Memory: unless a parameter says "host", every pointer is a device pointer
 * owned by the caller. The library keeps no pointer after a call's work on
 * its stream has completed. Work is enqueued on `stream` (a hipStream_t
 * passed as void*, NULL = default stream); calls return once the work is
 * enqueued, except where marked "synchronous".
 *
 * Errors: every call returns IM_OK (0) or a negative IM_E* code;
 * im_last_error() returns a thread-local message for the last failure.
 * On a validation error nothing is written to the outputs.
 */
#ifndef IM_H
#define IM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IM_OK         0
#define IM_EINVAL    (-1)   /* bad argument or malformed graph            */
#define IM_EOVERFLOW (-2)   /* n * R >= 2^32: gains would not fit 32 bits */
#define IM_ENOMEM    (-3)   /* device allocation failed                   */
#define IM_EHIP      (-4)   /* a HIP runtime call failed                  */

#define IM_R_MAX 4096u
#define IM_SPREAD_R_MAX (1u << 20)

/* Graph in CSR form, device-resident, caller-owned, read-only.
 * Arc e (0 <= e < m) is the e-th entry of col; its tail is the u with
 * row_ptr[u] <= e < row_ptr[u+1]. Duplicate arcs and self-loops are
 * allowed; each stored arc is its own coin. */
typedef struct im_graph {
    uint32_t        n;        /* nodes 0..n-1                                  */
    uint64_t        m;        /* arcs, < 2^32                                  */
    const uint64_t *row_ptr;  /* [n+1], row_ptr[0]=0, non-decreasing, [n]=m   */
    const uint32_t *col;      /* [m], each < n                                 */
    const float    *prob;     /* [m], 0 <= p <= 1, no NaN                      */
} im_graph;

/* Opaque device workspace (library-owned). Grows on demand inside the
 * calls below; one workspace must not be used by two calls at once. */
typedef struct im_workspace im_workspace;

int im_workspace_create(im_workspace **ws);
int im_workspace_destroy(im_workspace *ws);

/* Execution options of a workspace. None of them changes any result; they
 * only choose where and how the work is scheduled (im_autotune picks them).
 *   IM_OPT_HUB_DEGREE: nodes with at least this many arcs (in the direction
 *     of a pass) are expanded through per-snapshot live lists instead of the
 *     snapshot masks; 0 disables the lists; otherwise >= 16. Default 256.
 *   IM_OPT_COOP_GAIN: rounds whose seed gain (summed over snapshots) is at
 *     least this value run the forward search on a cooperative grid
 *     (IM_OPT_FWD_GROUPS workgroups per snapshot word); smaller rounds use
 *     one workgroup per word. Default 0 (always the cooperative grid).
 *     Cooperative launches can be refused while another process on the
 *     same device holds the hardware's global barrier resource: a single
 *     graph's round then runs one workgroup per word (same result), while
 *     batched selection, lazy engine 1 and a refusal during stream capture
 *     return IM_EHIP naming the cooperative kernel.
 *   IM_OPT_LAZY_ENGINE: exact evaluations of the lazy path run on the last
 *     engine tier alone, one workgroup per (candidate, word) search (2,
 *     default: candidates are the nodes with the largest bounds, whose
 *     searches the smaller tiers would only hand on; when a batch's searches
 *     fit the tier's slots their fixpoints stay there, and the round's seed,
 *     if evaluated in the round's last batch, is committed from them instead
 *     of a new forward search), through the three per-task engine tiers (0),
 *     or as one cooperative grid per batch, all (candidate, word) searches
 *     together (1, when their state fits 8 GB).
 *   IM_OPT_MAX_SLOTS: workgroups of the last engine tier, each with dense
 *     per-node state (28 bytes per node of the largest instance; at most
 *     48 GB in total). 8..65536, default 256.
 *   IM_OPT_TIER1_SHAPE: tasks per workgroup x LDS table entries of the
 *     middle engine tier: 0 (default) 4 x 256, 1: 2 x 512, 2: 1 x 1024; a
 *     task reaching more nodes than three quarters of its table moves on to
 *     the last tier.
 *   IM_OPT_TIER2_LANES: lanes per task of the last tier, 64, 256 (default)
 *     or 1024 (64: more tasks at once, for long searches with small
 *     frontiers).
 *   IM_OPT_SPARSE_LISTS: 1 (default) builds per-snapshot live lists of the
 *     nodes below the hub threshold as well, so that a node reached in at
 *     most two of a word's snapshots reads only its arcs live there; 0 reads
 *     every arc's mask word instead.
 *   IM_OPT_FWD_GROUPS: workgroups per snapshot word of the cooperative
 *     forward search (capped by co-residency), 1..1024, default 16.
 *   IM_OPT_LEARNED_POLICY: how im_select_lazy uses a network. 1: every batch
 *     in score order among the nodes whose bound can still win. 2 (default):
 *     the first batch of a round holds the nodes whose bound reaches the
 *     network's predicted gain of its best-scored node (the round's
 *     must-evaluate set when the prediction is right), later batches in
 *     bound order.
 *   IM_OPT_PAIR_COINS: 1 draws one coin per undirected pair (see
 *     im_pair_ids) instead of one per stored arc, for the single-graph calls
 *     (im_snapshot_masks, im_initial_gains, im_select, im_select_lazy,
 *     im_autotune) on a symmetric CSR; the results are then those of
 *     im_select_undirected. Default 0. Not for batches or plans.
 *   IM_OPT_LIVE_EDGE: the snapshot model of the same single-graph calls.
 *     0 (default): independent cascade, one coin per stored arc. 1: linear
 *     threshold in live-edge form (the paper notes the method extends to
 *     it): prob[e] is the weight b_e of arc e; per snapshot every node v
 *     keeps at most one in-arc: its in-arcs, by increasing arc id, own
 *     consecutive sub-intervals of [0, 2^32) of lengths floor(b_e * 2^32)
 *     (a part past 2^32 is never drawn), and the top 32 bits of output r+1
 *     of SplitMix64 seeded with output v+1 of SplitMix64(seed) keep the arc
 *     whose sub-interval holds them in snapshot r. Not for batches, plans,
 *     pair coins or im_spread.
 *   IM_OPT_LAZY_BATCH: the batch im_select_lazy uses when called with
 *     batch = 0 (1..1024, default 4; im_autotune_lazy sets it).
 *   IM_OPT_AFFECTED_GAIN: how a round of im_select / plans on a single graph
 *     brings the gains up to date (Sec. 4, Algorithm 2's delete loop). Rounds
 *     whose seed gain is at least this value (all rounds at the default 0)
 *     take one reverse search per newly covered node and subtract its counts;
 *     the others recompute, from scratch, the gain of every node that reaches
 *     a newly covered node in its snapshot (found by one union search per
 *     word over the reverse arcs), which gives the same integers. Costs
 *     28 W + 12 bytes per node of extra workspace when non-zero.
 *   IM_OPT_EVAL_SPLIT: on the lazy path's last-tier engine, each kept
 *     (candidate, word) evaluation runs as this many searches over disjoint
 *     groups of the word's snapshot bits, one workgroup each, whose counts
 *     add up (a large search's levels spread over more workgroups): 1, 2, 4
 *     or 8, or 0 (default) for the most of 8, 4, 2 whose searches fit the
 *     slots (IM_OPT_MAX_SLOTS).
 *   IM_OPT_REV_SPLIT: every reverse task that reaches the last engine tier
 *     runs as this many tasks (1, default, 2 or 4), each with the sources of
 *     one group of the word's snapshot bits, whose decrements add up (a
 *     large search's levels spread over more workgroups; im_autotune picks
 *     1 or 2).
 *   IM_OPT_REV_FIRST_TIER: the engine tier reverse tasks start on: 0
 *     (default) or 1, which leaves out the tier-0 launch of every round's
 *     reverse step (its workgroups hand most large tasks on anyway, and a
 *     launch costs its longest task start to finish even in a round with
 *     few tasks); im_autotune picks one. */
enum { IM_OPT_HUB_DEGREE = 1, IM_OPT_COOP_GAIN = 2, IM_OPT_LAZY_ENGINE = 3, IM_OPT_MAX_SLOTS = 4,
       IM_OPT_TIER1_SHAPE = 5, IM_OPT_TIER2_LANES = 6, IM_OPT_SPARSE_LISTS = 7,
       IM_OPT_FWD_GROUPS = 8, IM_OPT_LEARNED_POLICY = 9, IM_OPT_PAIR_COINS = 10,
       IM_OPT_LIVE_EDGE = 11, IM_OPT_LAZY_BATCH = 12, IM_OPT_AFFECTED_GAIN = 13,
       IM_OPT_EVAL_SPLIT = 14, IM_OPT_REV_SPLIT = 15, IM_OPT_REV_FIRST_TIER = 16 };
int im_workspace_set(im_workspace *ws, int option, int64_t value);

/* Counters of the last call on a workspace (synchronous: waits for the
 * stream of that call). Traversal counts follow the per-snapshot
 * definition: the full out-degree (in-degree for reverse steps) of every
 * node reached in every snapshot by every reachability task. */
typedef struct im_stats {
    uint64_t trav_init;        /* initial reach counts (Alg. 2 initial loop)      */
    uint64_t trav_fwd;         /* forward steps from the chosen seeds             */
    uint64_t trav_rev;         /* reverse decrement steps                         */
    uint64_t trav_eval;        /* exact gain evaluations of the lazy path         */
    uint64_t relax_fwd;        /* sum of out-degrees of nodes newly covered       */
    uint64_t tasks_rev;        /* reverse tasks (newly covered (node, word) pairs)*/
    uint64_t decrements;       /* sum of the decrements applied to gains          */
    uint64_t celf_evals;       /* exact gain evaluations (lazy path)              */
    /* Per pass p (0: initial counts, 1: reverse decrements, 2: exact
     * evaluations) and engine tier t (0: per-wavefront LDS tables, 1:
     * per-workgroup LDS tables, 2: per-workgroup dense global arrays):    */
    uint64_t relax[3][3];      /* sum over (node, word) tasks of the degree of    */
                               /* every node reached in that word                 */
    uint64_t reached[3][3];    /* (task, reached node) pairs                      */
    uint64_t arcs_read[3][3];  /* (arc, word) reads issued, re-expansions included*/
    uint64_t handed_over[3][3];/* tasks passed on to the next tier                */
    uint64_t fwd_levels;       /* levels of the forward searches (sum over words) */
    uint64_t fwd_entries;      /* frontier entries expanded by them               */
    uint64_t celf_batches;     /* evaluation batches of the lazy path             */
    uint64_t celf_fallbacks;   /* learned picks that fell back to bound order     */
    uint64_t max_levels[3][3]; /* per pass and tier: the most search levels one   */
                               /* workgroup ran in any launch of the call (the    */
                               /* launch's critical path in levels)               */
    uint64_t barrier_failures; /* grid barriers of the cooperative kernels whose */
                               /* wait timed out (always 0 on a working device;   */
                               /* the launch was then abandoned, results invalid) */
    uint64_t reserved[6];
} im_stats;

int im_stats_get(im_workspace *ws, im_stats *out);

/* Phase timers. When the bit (1 << phase) of `mask` is set, every later
 * call on this workspace brackets that phase's kernel launches with HIP
 * events on the call's stream. im_profile_get (synchronous) returns the
 * summed milliseconds and launch counts since the previous get and resets
 * them. Timing changes no result. */
enum {
    IM_PH_VALIDATE = 0, IM_PH_TRANSPOSE, IM_PH_MASK_GEN, IM_PH_MASK_GATHER,
    IM_PH_INIT_T0, IM_PH_INIT_T1, IM_PH_INIT_T2, IM_PH_ARGMAX, IM_PH_FORWARD,
    IM_PH_REV_T0, IM_PH_REV_T1, IM_PH_REV_T2, IM_PH_CLEAR, IM_PH_CALL, IM_PH_HUBS,
    IM_PH_PACK, IM_PH_ORDER, IM_PH_SCORE, IM_PH_PICK, IM_PH_EVAL_T0, IM_PH_EVAL_T1,
    IM_PH_EVAL_T2, IM_PH_UPDATE, IM_PH_AFFECTED, IM_PH_COUNT
};
#define IM_PH_MAX 24
typedef struct im_profile {
    double   ms[IM_PH_MAX];
    uint64_t launches[IM_PH_MAX];
} im_profile;

int im_profile_enable(im_workspace *ws, uint32_t mask);
int im_profile_get(im_workspace *ws, im_profile *out);
/* Host pointers: the individual launch durations (ms) of one phase as
 * collected by the last im_profile_get; *count gets their number, at most
 * `max` are written to ms_out. */
int im_profile_launches(im_workspace *ws, int phase, float *ms_out, uint32_t max,
                        uint32_t *count);

/* Thread-local message describing the last error. */
const char *im_last_error(void);

/* Validate a graph (synchronous). Checks row_ptr shape and monotonicity,
 * col < n, 0 <= prob <= 1 (NaN rejected), m < 2^32, and, for R > 0, that
 * 1 <= R <= IM_R_MAX and n*R < 2^32. Returns IM_OK or IM_EINVAL/IM_EOVERFLOW. */
int im_validate(const im_graph *g, uint32_t R, void *stream);

/* Snapshot masks (Sec. 3.3, Algorithm 1 sampling loop; Sec. 3.1 snapshot
 * definition). mask_out: [W][m] uint64, W = ceil(R/64), word-major: word w
 * of arc e at mask_out[w*m + e]; bit b = snapshot 64w+b; bits r >= R zero. */
int im_snapshot_masks(const im_graph *g, uint32_t R, uint64_t seed,
                      uint64_t *mask_out, im_workspace *ws, void *stream);

/* Reverse graph used by U(G'_i, w) (Sec. 4): in_row_ptr [n+1] (uint32),
 * in_col [m] = tail of each in-arc, in2out [m] = the arc id in the caller's
 * CSR. Order inside a row is unspecified. */
int im_transpose(const im_graph *g, uint32_t *in_row_ptr, uint32_t *in_col,
                 uint32_t *in2out, im_workspace *ws, void *stream);

/* Initial per-node reach counts (Algorithm 2, initial loop):
 * gain_out[u] = sum_r |R_r(u)|, uint32 [n]. */
int im_initial_gains(const im_graph *g, uint32_t R, uint64_t seed,
                     uint32_t *gain_out, im_workspace *ws, void *stream);

/* k-seed selection (Algorithm 2 with the exact-gain argmax of Algorithm 1).
 * seeds_out [k] uint32, gains_out [k] uint64 (device). trace_out may be
 * NULL; otherwise [k+1][n] uint32 receives the gain vector at the start of
 * every round and after the last (the exact marginal gain of every
 * unselected node; 0 for selected ones). k <= n; k = 0 writes nothing. */
int im_select(const im_graph *g, uint32_t R, uint32_t k, uint64_t seed,
              uint32_t *seeds_out, uint64_t *gains_out, uint32_t *trace_out,
              im_workspace *ws, void *stream);

/* One independent selection problem of a batch. */
typedef struct im_instance {
    im_graph g;       /* device CSR, as for im_select          */
    uint32_t R;       /* snapshots, 1..IM_R_MAX; n*R < 2^32    */
    uint32_t k;       /* seeds wanted, <= g.n                  */
    uint64_t seed;    /* RNG seed of this instance's snapshots */
} im_instance;

/* For callers that cannot allocate device memory -- code that must not call
 * hipMalloc or hipFree, such as tight serving loops and harnesses that forbid
 * allocation: im_select (no trace output) without a workspace. Every buffer
 * the selection needs is carved from one static device array of
 * IM_NOALLOC_SCRATCH_BYTES bytes, of which each GPU the library runs on holds
 * its own copy until the process ends; the call allocates nothing, on the
 * device or through any library routine. Seeds and gains equal im_select's
 * (the schedule differs only in where tasks run: no sparse live lists, 16
 * last-tier slots).
 * Size limit: the buffers take about 8 + 32 W bytes per arc and
 * 475 + 76 W bytes per node (W = ceil(R/64)); a graph that needs more than
 * the scratch is rejected with IM_EINVAL before any device work, nothing
 * written. Other errors as im_select.
 * Blocking in part: the call waits for earlier work on `stream` (it may still
 * be using the scratch), validates the graph with one host wait, then
 * enqueues the selection on `stream` and returns. The scratch keeps the last
 * call's contents; every call clears what must start at zero. All calls on
 * one GPU share its one array: calls whose work overlaps on one GPU (other
 * streams, other threads, before the previous call's work has finished) race
 * and give wrong results. */
#define IM_NOALLOC_SCRATCH_BYTES (128ull << 20)
int im_select_noalloc(const im_graph *g, uint32_t R, uint32_t k, uint64_t seed,
                      uint32_t *seeds_out, uint64_t *gains_out, void *stream);

/* Batched selection: `count` independent instances of uneven size (host
 * array of descriptors; the graphs themselves are device-resident) are laid
 * side by side as one block-diagonal graph and selected together, so every
 * kernel runs once per phase for the whole batch. Each instance gets exactly
 * the seeds and gains im_select would give it alone. seeds_out / gains_out
 * (device) hold instance i's k_i results at offset k_0 + ... + k_{i-1}.
 * Synchronous validation; limits: sum of n < 2^32 - 1, sum of m < 2^32. */
int im_select_batch(const im_instance *inst, uint32_t count, uint32_t *seeds_out,
                    uint64_t *gains_out, im_workspace *ws, void *stream);

/* Schedule autotuning (synchronous). A schedule -- hub threshold, tier-1
 * shape, tier-2 lanes and slots (the IM_OPT_* options above) -- decides only
 * where each reachability task runs, never a result (the forward-search
 * engine, IM_OPT_COOP_GAIN, is part of it). Each candidate schedule
 * is timed on a trial selection of the given graph -- the initial reach
 * counts (Algorithm 2's initial loop) and the first four greedy rounds --
 * and the fastest is set on the workspace and returned in *out (host, may
 * be NULL). im_autotune then times, with that schedule, the initial counts
 * and the first 16 rounds under four per-round update strategies (the
 * IM_OPT_AFFECTED_GAIN thresholds 0, n R / 4096, n R / 256 and 2^62: reverse
 * decrements in every round, the affected-set recompute in the small, in
 * most or in all rounds) and keeps the fastest; when the schedule uses the
 * cooperative forward search, it last times that search's width
 * (IM_OPT_FWD_GROUPS 16 or 32 workgroups per word) on the same trial, and
 * then the split of last-tier reverse tasks (IM_OPT_REV_SPLIT 1 or 2) and
 * the tier reverse tasks start on (IM_OPT_REV_FIRST_TIER 0 or 1; the batch
 * tuner times these two as well, on its own trial).
 * im_autotune caches its choice per graph signature (n, m, R and a checksum
 * of col and prob) for the life of the process; a cached choice is applied
 * without timing (out->tried = 0). When the environment variable
 * IM_TUNE_CACHE names a file, choices are also appended to it (one text line
 * per signature) and looked up there on a miss, so that they persist across
 * processes; an unreadable or unwritable file only disables that.
 * im_autotune_batch tunes the schedule on the instances it is given (a
 * caller may pass a representative subset of a batch). */
typedef struct im_tuning {
    int32_t  hub_degree;
    int32_t  tier1_shape;
    int32_t  tier2_lanes;
    int32_t  max_slots;
    int32_t  coop_forward; /* 1: cooperative forward search (IM_OPT_COOP_GAIN 0), 0: one workgroup per word */
    float    ms;           /* trial time of the chosen schedule         */
    uint32_t tried;        /* schedules timed (0: taken from the cache)  */
    uint64_t affected_gain;/* IM_OPT_AFFECTED_GAIN chosen (single graphs) */
    int32_t  fwd_groups;   /* IM_OPT_FWD_GROUPS chosen (single graphs with the
                              cooperative forward search; else the workspace's) */
    int32_t  rev_split;    /* IM_OPT_REV_SPLIT chosen                          */
    int32_t  rev_first_tier; /* IM_OPT_REV_FIRST_TIER chosen                   */
} im_tuning;
int im_autotune(const im_graph *g, uint32_t R, uint64_t seed, im_workspace *ws, void *stream,
                im_tuning *out);
int im_autotune_batch(const im_instance *inst, uint32_t count, im_workspace *ws, void *stream,
                      im_tuning *out);
/* Plans (device-resident round loop). im_plan_create validates the graph
 * (synchronous), then captures the complete selection -- reverse CSR, masks,
 * hub lists, initial gains and all k rounds -- into one HIP graph bound to a
 * private workspace and to the given device pointers (graph arrays, seeds_out,
 * gains_out). im_plan_launch enqueues one replay on `stream`: every replay
 * recomputes everything -- the 32-bit row offsets, reverse CSR, masks, lists,
 * gains and rounds -- from the graph arrays as they are at that time. They
 * must keep their shape (n, m) and their contents may change, but they must
 * stay valid as im_validate defines it: validity is checked when the plan is
 * created, not on replay, and a replay over an invalid graph (say a col entry
 * >= n) has unspecified results and may access memory out of bounds. Replays
 * of one plan must not overlap. A schedule that im_autotune chose earlier in the process for
 * a graph with the same signature is used by the plan. */
typedef struct im_plan im_plan;
int im_plan_create(const im_graph *g, uint32_t R, uint32_t k, uint64_t seed,
                   uint32_t *seeds_out, uint64_t *gains_out, void *stream, im_plan **plan);
/* The batched selection (im_select_batch) captured into one HIP graph:
 * validation and the instance tables are done once here (synchronous); a
 * replay merges the instances' arrays again and runs the whole batched
 * selection, so one launch selects the seeds of every instance. The
 * instances' arrays follow the rules of im_plan_create's graph arrays (same
 * shapes, contents valid; checked at creation only). `tuned`
 * (may be NULL) lends its engine schedule, e.g. one set by
 * im_autotune_batch. count >= 2. */
int im_plan_create_batch(const im_instance *inst, uint32_t count, uint32_t *seeds_out,
                         uint64_t *gains_out, im_workspace *tuned, void *stream, im_plan **plan);
int im_plan_launch(im_plan *plan, void *stream);
int im_plan_stats(im_plan *plan, im_stats *out);   /* synchronous; last replay */
int im_plan_destroy(im_plan *plan);

/* ------------------------------------------------------------------------
 * Lazy evaluation with an optional learned candidate order.
 *
 * Candidate-scoring network (a small MLP, 5 -> 64 -> 64 -> 1, ReLU after both
 * hidden layers, bfloat16 weights with FP32 master copies, FP32 accumulate).
 * Parameter vector of IM_MLP_NPARAM floats, in this order: W1[64][5], b1[64],
 * W2[64][64], b2[64], w3[64], b3. Input x of node u (each ln(1 + .)):
 * in-degree, out-degree, sum of out-arc probabilities, sum over out-arcs
 * (u,v) of out-degree(v), last exact gain / R. Output: a score; the lazy
 * path uses it only to order candidates, never to decide a pick.
 * ------------------------------------------------------------------------ */
#define IM_MLP_IN 5
#define IM_MLP_HIDDEN 64
#define IM_MLP_NPARAM 4609
typedef struct im_mlp im_mlp;
/* Device-resident network, all parameters zero. */
int im_mlp_create(im_mlp **model);
int im_mlp_destroy(im_mlp *model);
/* Host array of IM_MLP_NPARAM finite floats -> master weights; the bfloat16
 * copies are their nearest-even roundings; Adam state reset (synchronous). */
int im_mlp_set_params(im_mlp *model, const float *host_params);
/* Host outputs (either may be NULL): master weights, bfloat16 bit patterns
 * of the copies used by every forward pass (synchronous). */
int im_mlp_get_params(const im_mlp *model, float *host_master, uint16_t *host_bf16);
/* y[i] = network(x[i]) for x [N][5] float, y [N] float (device). The
 * 64 x 64 second layer runs on the matrix cores (bfloat16 products, FP32
 * accumulation) with each first-layer activation entered as the sum of two
 * bfloat16 parts, so y is the FP32 network's to about 2^-16 relative; the
 * lazy path scores candidates the same way. */
int im_mlp_forward(const im_mlp *model, const float *x, uint32_t N, float *y, void *stream);
/* Loss L = sum_i (y_i - t_i)^2 / (2N) of the bfloat16 network on x [N][5],
 * t [N] and its gradient with respect to the parameters (grad [IM_MLP_NPARAM],
 * loss [1], device; either may be NULL). Deterministic. N >= 1. */
int im_mlp_loss_grad(im_mlp *model, const float *x, const float *t, uint32_t N, float *grad,
                     float *loss, void *stream);
/* One Adam step (Kingma & Ba 2015) on the master weights with gradient grad
 * (device), then refresh of the bfloat16 copies. */
int im_mlp_adam(im_mlp *model, const float *grad, float lr, float beta1, float beta2, float eps,
                void *stream);
/* Minibatch step: loss and gradient over the samples idx[0..nbatch) of
 * (x, t) (idx device uint32, each < nsamples), written to grad_scratch
 * [IM_MLP_NPARAM] and loss_out [1] (device), then one Adam step. */
int im_mlp_train_step(im_mlp *model, const float *x, const float *t, uint32_t nsamples,
                      const uint32_t *idx, uint32_t nbatch, float *grad_scratch, float *loss_out,
                      float lr, float beta1, float beta2, float eps, void *stream);
/* Static node features feat_out [n][4] float (device): the first four
 * inputs of the network, for the graph g. */
int im_node_features(const im_graph *g, float *feat_out, im_workspace *ws, void *stream);
/* Training samples from a gain trace (im_select's trace_out, [T][n] uint32):
 * sample s takes node[s] and rounds tprev[s] < tcur[s] < T:
 * x_out[s] = (feat[node][0..3], ln(1 + trace[tprev][node] / R)),
 * t_out[s] = ln(1 + trace[tcur][node] / R). Out-of-range entries give NaN. */
int im_mlp_samples(const float *feat, const uint32_t *trace, uint32_t n, uint32_t T, uint32_t R,
                   const uint32_t *node, const uint32_t *tprev, const uint32_t *tcur, uint32_t N,
                   float *x_out, float *t_out, void *stream);
/* k-seed selection by lazy exact evaluation (the paper's StaticGreedyCELF,
 * Sec. 5, on the snapshots of Sec. 3.3): stale gains are upper bounds; each
 * round evaluates candidates exactly, `batch` at a time (1..1024; 0: the
 * workspace's IM_OPT_LAZY_BATCH), until the
 * best exact (gain, lowest id) beats the bound of every candidate not yet
 * evaluated in the round. model = NULL: candidates in bound order; otherwise
 * as IM_OPT_LEARNED_POLICY says (score order falls back to bound order when
 * more than 2048 nodes can still win). Seeds and gains are those of im_select
 * for any model and batch. Synchronous (one host wait per batch); the
 * number of exact evaluations is reported in im_stats.celf_evals. How a
 * model orders or sizes the batches: IM_OPT_LEARNED_POLICY. */
int im_select_lazy(const im_graph *g, uint32_t R, uint32_t k, uint64_t seed, uint32_t batch,
                   const im_mlp *model, uint32_t *seeds_out, uint64_t *gains_out,
                   im_workspace *ws, void *stream);

/* Lazy-path tuning (synchronous; the schedule part of the autotuner, like
 * im_autotune, never changes a result): the lazy selection of the first
 * min(k, 64) rounds (at least 2) is timed under each evaluation engine
 * (IM_OPT_LAZY_ENGINE 2 and 0) and batch size (1, 2, 4, 8, 16) with the
 * given model (NULL: bound order); the fastest pair is set on the workspace
 * (IM_OPT_LAZY_ENGINE, IM_OPT_LAZY_BATCH), so that im_select_lazy with
 * batch = 0 uses it, and returned in *out (host, may be NULL). The engine
 * schedule set by im_autotune is kept. */
typedef struct im_lazy_tuning {
    int32_t  engine;   /* IM_OPT_LAZY_ENGINE chosen       */
    uint32_t batch;    /* IM_OPT_LAZY_BATCH chosen        */
    float    ms;       /* trial time of the chosen pair   */
    uint32_t tried;    /* pairs timed                     */
} im_lazy_tuning;
int im_autotune_lazy(const im_graph *g, uint32_t R, uint32_t k, uint64_t seed, const im_mlp *model,
                     im_workspace *ws, void *stream, im_lazy_tuning *out);

/* Spread evaluation (the snapshot estimator of Sec. 3.1; the paper scores
 * seed sets on independent simulations, Sec. 5.2). With f(T) = sum_r |R_r(T)|
 * over R snapshots drawn from `seed` by the same live-edge rule as selection
 * (another seed gives snapshots independent of those a selection used):
 *   marg_out[i] = f(S[0..i]) - f(S[0..i-1]), uint64 [nS] (device), so the
 *     spread estimate of the first i+1 seeds is (marg_out[0] + ... +
 *     marg_out[i]) / R; a repeated seed adds 0;
 *   per_snapshot_out[r] = |R_r(S)|, uint32 [R] (device): the spread of the
 *     whole sequence in each snapshot, for confidence intervals.
 * Either output may be NULL (marg_out NULL: one search per word from all
 * seeds at once). S: device array of nS node ids, each < n, checked on the
 * host before any output is written. 1 <= R <= IM_SPREAD_R_MAX (R is not
 * bounded by IM_R_MAX: snapshot words are processed in chunks whose masks
 * and search state stay within a fixed device-memory budget). Synchronous
 * for the seed check, then asynchronous on `stream`. Errors: IM_EINVAL for
 * null pointers, R out of range, a seed >= n or a malformed graph. */
int im_spread(const im_graph *g, uint32_t R, uint64_t seed, const uint32_t *S, uint32_t nS,
              uint64_t *marg_out, uint32_t *per_snapshot_out, im_workspace *ws, void *stream);

/* Undirected graphs (Sec. 4: in an undirected snapshot the nodes a node
 * reaches are the nodes that reach it, so each snapshot is described by its
 * connected components). The CSR must store both directions of every
 * undirected pair, with the same probability, and no pair twice in one
 * direction (self-loops are allowed and ignored); each pair then has one
 * coin per snapshot, drawn by the arc generator rule under the index of its
 * canonical arc (the direction whose tail is the smaller node id).
 * im_pair_ids: pair_out [m] uint32 (device) = the canonical arc of each
 * arc's pair (a self-loop is its own). Synchronous. IM_EINVAL if the CSR
 * is not symmetric in this sense (the message names the defect). */
int im_pair_ids(const im_graph *g, uint32_t *pair_out, im_workspace *ws, void *stream);

/* k-seed selection on an undirected graph by the component method: per
 * snapshot a union-find forest of the live pairs; s_u = sum_r |C_r(u)|;
 * a pick covers the picked node's uncovered components, whose members lose
 * their size. Results (seeds_out [k], gains_out [k], trace_out [k+1][n] or
 * NULL, device) equal im_select's with IM_OPT_PAIR_COINS on the same
 * graph. Argument rules as im_select; IM_EINVAL also for a CSR that is not
 * symmetric as im_pair_ids requires. Device memory: 8 n R bytes for the
 * forests and component sizes. Returns after validation and pair matching
 * (host-synchronous), the rest asynchronous on `stream`. */
int im_select_undirected(const im_graph *g, uint32_t R, uint32_t k, uint64_t seed,
                         uint32_t *seeds_out, uint64_t *gains_out, uint32_t *trace_out,
                         im_workspace *ws, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* IM_H */
