"""Python binding of the C ABI (include/im.h).

torch supplies device memory and the current HIP stream; every step of the
selection runs in libim's kernels. Tensors passed in must already live on
the GPU; nothing here computes on the host.
"""
import atexit
import ctypes
import weakref

import numpy as np
import torch

from . import _native as N

# every open workspace, plan and network: released by _release_all before
# the interpreter exits
_live = weakref.WeakSet()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else ctypes.c_void_p(0)


def _u32(t):
    """int32 tensor holding uint32 bit patterns -> int64 values."""
    return t.to(torch.int64) & 0xFFFFFFFF


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Graph:
    """Device-resident CSR graph with one IC probability per stored arc.

    row_ptr: int64 [n+1]; col: int32 or uint32 [m] (node ids < n);
    prob: float32 [m]. Arc e is position e of col.
    """

    def __init__(self, row_ptr, col, prob):
        if not (row_ptr.is_cuda and col.is_cuda and prob.is_cuda):
            raise ValueError("graph tensors must be on the GPU")
        if row_ptr.dtype not in (torch.int64, torch.uint64):
            raise ValueError("row_ptr must be int64")
        if col.dtype not in (torch.int32, torch.uint32):
            raise ValueError("col must be int32 or uint32")
        if prob.dtype != torch.float32:
            raise ValueError("prob must be float32")
        self.row_ptr = row_ptr.contiguous()
        self.col = col.contiguous()
        self.prob = prob.contiguous()
        self.n = int(row_ptr.numel()) - 1
        self.m = int(col.numel())
        self.device = row_ptr.device

    @classmethod
    def from_numpy(cls, row_ptr, col, prob, device="cuda"):
        rp = torch.from_numpy(np.ascontiguousarray(row_ptr, dtype=np.uint64).view(np.int64))
        c = torch.from_numpy(np.ascontiguousarray(col, dtype=np.uint32).view(np.int32))
        p = torch.from_numpy(np.ascontiguousarray(prob, dtype=np.float32))
        return cls(rp.to(device), c.to(device), p.to(device))

    def c_struct(self):
        return N.ImGraph(self.n, self.m, self.row_ptr.data_ptr(),
                         self.col.data_ptr() if self.m else 0,
                         self.prob.data_ptr() if self.m else 0)


class Workspace:
    """Library-owned device workspace; grows on demand, reused across calls."""

    def __init__(self):
        h = ctypes.c_void_p()
        N.check(N.lib().im_workspace_create(ctypes.byref(h)))
        self.handle = h
        _live.add(self)

    def close(self):
        if self.handle:
            N.lib().im_workspace_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_hub_degree(self, deg):
        """Heavy-node threshold for per-snapshot live lists (0: off). No result changes."""
        N.check(N.lib().im_workspace_set(self.handle, N.IM_OPT_HUB_DEGREE, int(deg)))

    def set_coop_gain(self, gain):
        """Rounds with seed gain >= gain use the grid-wide forward search. No result changes."""
        N.check(N.lib().im_workspace_set(self.handle, N.IM_OPT_COOP_GAIN, int(gain)))

    def set_lazy_engine(self, engine):
        """Exact evaluations of the lazy path: 2 the last tier alone, one
        workgroup per candidate and word (default), 0 the three per-task engine
        tiers, 1 one cooperative grid per batch. No result changes."""
        N.check(N.lib().im_workspace_set(self.handle, N.IM_OPT_LAZY_ENGINE, int(engine)))

    def set_max_slots(self, slots):
        """Workgroups of the last engine tier (8..65536). No result changes."""
        N.check(N.lib().im_workspace_set(self.handle, N.IM_OPT_MAX_SLOTS, int(slots)))

    def set_tier1_shape(self, shape):
        """Middle-tier tasks x table entries: 0: 4 x 256, 1: 2 x 512, 2: 1 x 1024. No result changes."""
        N.check(N.lib().im_workspace_set(self.handle, N.IM_OPT_TIER1_SHAPE, int(shape)))

    def set_tier2_lanes(self, lanes):
        """Lanes per task of the last engine tier (64, 256 or 1024). No result changes."""
        N.check(N.lib().im_workspace_set(self.handle, N.IM_OPT_TIER2_LANES, int(lanes)))

    def set_sparse_lists(self, on):
        """Per-snapshot live lists for low-degree nodes (1) or masks only (0). No result changes."""
        N.check(N.lib().im_workspace_set(self.handle, N.IM_OPT_SPARSE_LISTS, int(on)))

    def set_forward_groups(self, per_word):
        """Workgroups per snapshot word of the grid-wide forward search. No result changes."""
        N.check(N.lib().im_workspace_set(self.handle, N.IM_OPT_FWD_GROUPS, int(per_word)))

    def set_lazy_batch(self, batch):
        """Batch of select_lazy(batch=0) (1..1024)."""
        N.check(N.lib().im_workspace_set(self.handle, N.IM_OPT_LAZY_BATCH, int(batch)))

    def set_eval_split(self, groups):
        """Bit groups per kept lazy evaluation search (0: automatic, 1, 2, 4, 8). No result changes."""
        N.check(N.lib().im_workspace_set(self.handle, N.IM_OPT_EVAL_SPLIT, int(groups)))

    def set_rev_split(self, groups):
        """Bit groups per last-tier reverse task (1, 2 or 4). No result changes."""
        N.check(N.lib().im_workspace_set(self.handle, N.IM_OPT_REV_SPLIT, int(groups)))

    def set_rev_first_tier(self, tier):
        """Engine tier the reverse tasks start on (0 or 1). No result changes."""
        N.check(N.lib().im_workspace_set(self.handle, N.IM_OPT_REV_FIRST_TIER, int(tier)))

    def set_affected_gain(self, gain):
        """Rounds whose seed gain is below `gain` update the gains by the
        affected-set recompute instead of reverse decrements (0: never)."""
        N.check(N.lib().im_workspace_set(self.handle, N.IM_OPT_AFFECTED_GAIN, int(gain)))

    def set_learned_policy(self, policy):
        """1: score order among can-win nodes; 2: first batch sized by the predicted gain."""
        N.check(N.lib().im_workspace_set(self.handle, N.IM_OPT_LEARNED_POLICY, int(policy)))

    def set_pair_coins(self, on):
        """One coin per undirected pair (symmetric CSR) for single-graph calls."""
        N.check(N.lib().im_workspace_set(self.handle, N.IM_OPT_PAIR_COINS, int(bool(on))))

    def set_live_edge(self, model):
        """Snapshot model of single-graph calls: 0 independent cascade, 1 linear
        threshold (prob = in-arc weights)."""
        N.check(N.lib().im_workspace_set(self.handle, N.IM_OPT_LIVE_EDGE, int(model)))

    def profile_enable(self, phases=None):
        """Time the named phases (None: all) with HIP events from now on."""
        names = N.PHASES if phases is None else phases
        mask = 0
        for nm in names:
            mask |= 1 << N.PHASES.index(nm)
        N.check(N.lib().im_profile_enable(self.handle, mask))

    def profile(self):
        """{phase: (total_ms, launches)} since the previous call (synchronous)."""
        pr = N.ImProfile()
        N.check(N.lib().im_profile_get(self.handle, ctypes.byref(pr)))
        return {nm: (float(pr.ms[i]), int(pr.launches[i])) for i, nm in enumerate(N.PHASES)}

    def launches(self, phase):
        """Per-launch milliseconds of `phase` from the last profile() call."""
        cnt = ctypes.c_uint32(0)
        N.check(N.lib().im_profile_launches(self.handle, N.PHASES.index(phase), None, 0,
                                            ctypes.byref(cnt)))
        buf = (ctypes.c_float * max(1, cnt.value))()
        N.check(N.lib().im_profile_launches(self.handle, N.PHASES.index(phase), buf, cnt.value,
                                            ctypes.byref(cnt)))
        return [float(buf[i]) for i in range(cnt.value)]

    def stats(self):
        st = N.ImStats()
        N.check(N.lib().im_stats_get(self.handle, ctypes.byref(st)))
        return st.as_dict()


_default_ws = {}


def _ws(ws, device):
    if ws is not None:
        return ws
    key = torch.device(device).index or 0
    if key not in _default_ws:
        with torch.cuda.device(key):
            _default_ws[key] = Workspace()
    return _default_ws[key]


def validate(graph, R=0):
    g = graph.c_struct()
    N.check(N.lib().im_validate(ctypes.byref(g), R, _stream(graph.device)))


def snapshot_masks(graph, R, seed, ws=None):
    """uint64 masks, word-major [W, m] (returned as int64 bit patterns)."""
    W = (R + 63) // 64
    out = torch.empty((W, graph.m), dtype=torch.int64, device=graph.device)
    g = graph.c_struct()
    ws = _ws(ws, graph.device)
    N.check(N.lib().im_snapshot_masks(ctypes.byref(g), R, seed, _ptr(out), ws.handle,
                                      _stream(graph.device)))
    return out


def transpose(graph, ws=None):
    """Reverse CSR: (in_row_ptr [n+1], in_col [m], in2out [m]) as int32 tensors."""
    dev = graph.device
    in_row = torch.empty(graph.n + 1, dtype=torch.int32, device=dev)
    in_col = torch.empty(graph.m, dtype=torch.int32, device=dev)
    in2out = torch.empty(graph.m, dtype=torch.int32, device=dev)
    g = graph.c_struct()
    ws = _ws(ws, dev)
    N.check(N.lib().im_transpose(ctypes.byref(g), _ptr(in_row), _ptr(in_col), _ptr(in2out),
                                 ws.handle, _stream(dev)))
    return in_row, in_col, in2out


def initial_gains(graph, R, seed, ws=None):
    """s_u = sum_r |R_r(u)| as an int64 tensor [n]."""
    out = torch.empty(graph.n, dtype=torch.int32, device=graph.device)
    g = graph.c_struct()
    ws = _ws(ws, graph.device)
    N.check(N.lib().im_initial_gains(ctypes.byref(g), R, seed, _ptr(out), ws.handle,
                                     _stream(graph.device)))
    return _u32(out)


def select(graph, R, k, seed, ws=None, trace=False):
    """k seeds and their marginal gains (summed over the R snapshots).

    Returns (seeds int64 [k], gains int64 [k], trace int64 [k+1, n] or None).
    """
    dev = graph.device
    seeds = torch.empty(k, dtype=torch.int32, device=dev)
    gains = torch.empty(k, dtype=torch.int64, device=dev)
    tr = torch.empty((k + 1, graph.n), dtype=torch.int32, device=dev) if trace else None
    g = graph.c_struct()
    ws = _ws(ws, dev)
    N.check(N.lib().im_select(ctypes.byref(g), R, k, seed, _ptr(seeds), _ptr(gains),
                              _ptr(tr) if trace else ctypes.c_void_p(0), ws.handle,
                              _stream(dev)))
    return _u32(seeds), gains, (_u32(tr) if trace else None)


def select_noalloc(graph, R, k, seed, seeds=None, gains=None):
    """im_select without a workspace: the library allocates nothing, every
    buffer comes from its static device scratch. The caller passes the
    output tensors (int32 [k], int64 [k]) or gets new ones.
    Returns (seeds int64 [k], gains int64 [k])."""
    dev = graph.device
    if seeds is None:
        seeds = torch.empty(k, dtype=torch.int32, device=dev)
    if gains is None:
        gains = torch.empty(k, dtype=torch.int64, device=dev)
    g = graph.c_struct()
    N.check(N.lib().im_select_noalloc(ctypes.byref(g), R, k, seed, _ptr(seeds), _ptr(gains),
                                      _stream(dev)))
    return _u32(seeds), gains


def autotune(graph, R, seed, ws=None):
    """Pick the fastest engine schedule for this graph (set on `ws`); returns it as a dict."""
    g = graph.c_struct()
    ws = _ws(ws, graph.device)
    t = N.ImTuning()
    N.check(N.lib().im_autotune(ctypes.byref(g), R, seed, ws.handle, _stream(graph.device),
                                ctypes.byref(t)))
    return t.as_dict()


def _instances(instances):
    arr = (N.ImInstance * len(instances))()
    keep = []
    for i, (g, R, k, seed) in enumerate(instances):
        cg = g.c_struct()
        keep.append(cg)
        arr[i].g = cg
        arr[i].R = R
        arr[i].k = k
        arr[i].seed = seed
    return arr, keep


def autotune_batch(instances, ws=None):
    """Pick the fastest engine schedule for a batch (or a sample of it); set on `ws`."""
    dev = instances[0][0].device
    arr, _keep = _instances(instances)
    ws = _ws(ws, dev)
    t = N.ImTuning()
    N.check(N.lib().im_autotune_batch(arr, len(instances), ws.handle, _stream(dev), ctypes.byref(t)))
    return t.as_dict()


def select_batch(instances, ws=None):
    """Select seeds for several independent instances in one batched pass.

    instances: list of (Graph, R, k, seed), all graphs on one GPU.
    Returns a list of (seeds int64 [k_i], gains int64 [k_i]), one per instance,
    each identical to what select() gives that instance alone.
    """
    if not instances:
        return []
    dev = instances[0][0].device
    arr, _keep = _instances(instances)
    K = sum(int(x[2]) for x in instances)
    seeds = torch.empty(K, dtype=torch.int32, device=dev)
    gains = torch.empty(K, dtype=torch.int64, device=dev)
    ws = _ws(ws, dev)
    N.check(N.lib().im_select_batch(arr, len(instances), _ptr(seeds), _ptr(gains), ws.handle,
                                    _stream(dev)))
    s64 = _u32(seeds)
    out, off = [], 0
    for (_, _, k, _) in instances:
        out.append((s64[off:off + k], gains[off:off + k]))
        off += k
    return out


class Plan:
    """The whole selection captured into one HIP graph (device-resident loop).

    Bound to `graph`'s device arrays and to its own output tensors; each
    launch() recomputes the k seeds from the current contents of the arrays.
    """

    def __init__(self, graph, R, k, seed):
        dev = graph.device
        self.graph = graph
        self.seeds_raw = torch.empty(k, dtype=torch.int32, device=dev)
        self.gains = torch.empty(k, dtype=torch.int64, device=dev)
        self._g = graph.c_struct()
        h = ctypes.c_void_p()
        N.check(N.lib().im_plan_create(ctypes.byref(self._g), R, k, seed, _ptr(self.seeds_raw),
                                       _ptr(self.gains), _stream(dev), ctypes.byref(h)))
        self.handle = h
        _live.add(self)

    def launch(self):
        N.check(N.lib().im_plan_launch(self.handle, _stream(self.graph.device)))

    @property
    def seeds(self):
        return _u32(self.seeds_raw)

    def stats(self):
        st = N.ImStats()
        N.check(N.lib().im_plan_stats(self.handle, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if self.handle:
            N.lib().im_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# lazy evaluation and the candidate-scoring network
# ---------------------------------------------------------------------------
MLP_NPARAM = N.IM_MLP_NPARAM
MLP_IN = 5


class Mlp:
    """Device-resident candidate-scoring network (bfloat16 weights, FP32 masters)."""

    def __init__(self, params=None):
        h = ctypes.c_void_p()
        N.check(N.lib().im_mlp_create(ctypes.byref(h)))
        self.handle = h
        _live.add(self)
        if params is not None:
            self.set_params(params)

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.shape != (MLP_NPARAM,):
            raise ValueError(f"expected {MLP_NPARAM} parameters")
        N.check(N.lib().im_mlp_set_params(self.handle, p.ctypes.data_as(ctypes.c_void_p)))

    def params(self):
        """(master float32 [P], bfloat16 copies as uint16 bit patterns [P])."""
        m = np.zeros(MLP_NPARAM, np.float32)
        b = np.zeros(MLP_NPARAM, np.uint16)
        N.check(N.lib().im_mlp_get_params(self.handle, m.ctypes.data_as(ctypes.c_void_p),
                                          b.ctypes.data_as(ctypes.c_void_p)))
        return m, b

    def forward(self, x):
        """x: float32 [N, 5] on the GPU -> float32 [N]."""
        x = x.contiguous()
        y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        N.check(N.lib().im_mlp_forward(self.handle, _ptr(x), x.shape[0], _ptr(y), _stream(x.device)))
        return y

    def loss_grad(self, x, t):
        """(loss float32 [1], grad float32 [P]) of sum (y - t)^2 / (2N)."""
        x, t = x.contiguous(), t.contiguous()
        g = torch.empty(MLP_NPARAM, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        N.check(N.lib().im_mlp_loss_grad(self.handle, _ptr(x), _ptr(t), x.shape[0], _ptr(g),
                                         _ptr(loss), _stream(x.device)))
        return loss, g

    def adam(self, grad, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        N.check(N.lib().im_mlp_adam(self.handle, _ptr(grad.contiguous()), lr, beta1, beta2, eps,
                                    _stream(grad.device)))

    def train_step(self, x, t, idx, grad_scratch, loss_out, lr=1e-3, beta1=0.9, beta2=0.999,
                   eps=1e-8):
        """One minibatch (rows idx of x, t) gradient + Adam step, all on the GPU."""
        N.check(N.lib().im_mlp_train_step(self.handle, _ptr(x), _ptr(t), x.shape[0], _ptr(idx),
                                          idx.shape[0], _ptr(grad_scratch), _ptr(loss_out), lr,
                                          beta1, beta2, eps, _stream(x.device)))

    def close(self):
        if self.handle:
            N.lib().im_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def node_features(graph, ws=None):
    """Static network inputs float32 [n, 4]."""
    out = torch.empty((graph.n, 4), dtype=torch.float32, device=graph.device)
    g = graph.c_struct()
    ws = _ws(ws, graph.device)
    N.check(N.lib().im_node_features(ctypes.byref(g), _ptr(out), ws.handle, _stream(graph.device)))
    return out


def mlp_samples(feat, trace, R, node, tprev, tcur):
    """Training inputs/targets gathered from a gain trace (int32 tensors on the GPU)."""
    T, n = trace.shape
    Ns = node.shape[0]
    x = torch.empty((Ns, MLP_IN), dtype=torch.float32, device=feat.device)
    t = torch.empty(Ns, dtype=torch.float32, device=feat.device)
    N.check(N.lib().im_mlp_samples(_ptr(feat.contiguous()), _ptr(trace.contiguous()), n, T, R,
                                   _ptr(node.contiguous()), _ptr(tprev.contiguous()),
                                   _ptr(tcur.contiguous()), Ns, _ptr(x), _ptr(t),
                                   _stream(feat.device)))
    return x, t


def select_lazy(graph, R, k, seed, batch=64, model=None, ws=None):
    """Lazy exact evaluation (bound order, or `model`'s score order); batch 0
    takes the workspace's batch (set by autotune_lazy).

    Returns (seeds int64 [k], gains int64 [k]) -- always those of select().
    """
    dev = graph.device
    seeds = torch.empty(k, dtype=torch.int32, device=dev)
    gains = torch.empty(k, dtype=torch.int64, device=dev)
    g = graph.c_struct()
    ws = _ws(ws, dev)
    N.check(N.lib().im_select_lazy(ctypes.byref(g), R, k, seed, batch,
                                   model.handle if model is not None else ctypes.c_void_p(0),
                                   _ptr(seeds), _ptr(gains), ws.handle, _stream(dev)))
    return _u32(seeds), gains


def autotune_lazy(graph, R, k, seed, model=None, ws=None):
    """Pick the lazy path's evaluation engine and batch size (set on `ws`,
    used by select_lazy(batch=0)); returns them as a dict."""
    dev = graph.device
    g = graph.c_struct()
    ws = _ws(ws, dev)
    t = N.ImLazyTuning()
    N.check(N.lib().im_autotune_lazy(ctypes.byref(g), R, k, seed,
                                     model.handle if model is not None else ctypes.c_void_p(0),
                                     ws.handle, _stream(dev), ctypes.byref(t)))
    return t.as_dict()


def pair_ids(graph, ws=None):
    """Canonical arc of every arc's undirected pair (int64 [m]); ImError
    unless the CSR is symmetric (both directions, equal probabilities, no
    pair twice in one direction)."""
    dev = graph.device
    out = torch.empty(graph.m, dtype=torch.int32, device=dev)
    g = graph.c_struct()
    ws = _ws(ws, dev)
    N.check(N.lib().im_pair_ids(ctypes.byref(g), _ptr(out), ws.handle, _stream(dev)))
    return _u32(out)


def select_undirected(graph, R, k, seed, ws=None, trace=False):
    """k seeds on an undirected graph by the component method (one coin per
    pair). Returns (seeds int64 [k], gains int64 [k], trace int64 [k+1, n] or None),
    the results of select() with pair coins."""
    dev = graph.device
    seeds = torch.empty(k, dtype=torch.int32, device=dev)
    gains = torch.empty(k, dtype=torch.int64, device=dev)
    tr = torch.empty((k + 1, graph.n), dtype=torch.int32, device=dev) if trace else None
    g = graph.c_struct()
    ws = _ws(ws, dev)
    N.check(N.lib().im_select_undirected(ctypes.byref(g), R, k, seed, _ptr(seeds), _ptr(gains),
                                         _ptr(tr) if trace else ctypes.c_void_p(0), ws.handle,
                                         _stream(dev)))
    return _u32(seeds), gains, (_u32(tr) if trace else None)


def spread(graph, R, seed, seeds, ws=None, marginals=True, per_snapshot=False):
    """Snapshot spread of a seed sequence on R snapshots drawn from `seed`.

    Returns (marg int64 [len(seeds)] or None, per_snapshot int64 [R] or None):
    marg[i] = f(S[:i+1]) - f(S[:i]) with f(T) = sum_r |R_r(T)|, so
    marg.cumsum() / R are the spread estimates of the prefixes;
    per_snapshot[r] = |R_r(S)|.
    """
    dev = graph.device
    S = torch.as_tensor(seeds, dtype=torch.int64).to(torch.int32).to(dev).contiguous()
    nS = S.numel()
    marg = torch.empty(nS, dtype=torch.int64, device=dev) if marginals else None
    per = torch.empty(R, dtype=torch.int32, device=dev) if per_snapshot else None
    g = graph.c_struct()
    ws = _ws(ws, dev)
    N.check(N.lib().im_spread(ctypes.byref(g), R, seed, _ptr(S) if nS else ctypes.c_void_p(0), nS,
                              _ptr(marg) if marginals else ctypes.c_void_p(0),
                              _ptr(per) if per_snapshot else ctypes.c_void_p(0), ws.handle,
                              _stream(dev)))
    return marg, (_u32(per) if per_snapshot else None)


class BatchPlan:
    """A batched selection captured into one HIP graph (one launch per replay).

    instances: list of (Graph, R, k, seed). `tuned` lends a Workspace's engine
    schedule (e.g. after autotune_batch). Results per instance as select_batch.
    """

    def __init__(self, instances, tuned=None):
        dev = instances[0][0].device
        self.device = dev
        self.instances = instances
        self._arr, self._keep = _instances(instances)
        K = sum(int(x[2]) for x in instances)
        self.seeds_raw = torch.empty(K, dtype=torch.int32, device=dev)
        self.gains = torch.empty(K, dtype=torch.int64, device=dev)
        h = ctypes.c_void_p()
        N.check(N.lib().im_plan_create_batch(self._arr, len(instances), _ptr(self.seeds_raw),
                                             _ptr(self.gains),
                                             tuned.handle if tuned is not None else ctypes.c_void_p(0),
                                             _stream(dev), ctypes.byref(h)))
        self.handle = h
        _live.add(self)

    def launch(self):
        N.check(N.lib().im_plan_launch(self.handle, _stream(self.device)))

    def results(self):
        s64 = _u32(self.seeds_raw)
        out, off = [], 0
        for (_, _, k, _) in self.instances:
            out.append((s64[off:off + k], self.gains[off:off + k]))
            off += k
        return out

    def stats(self):
        st = N.ImStats()
        N.check(N.lib().im_plan_stats(self.handle, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if self.handle:
            N.lib().im_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _release_all():
    """Destroy every workspace, plan and network still open once the device
    work has finished. Runs before the interpreter shuts down, so that no HIP
    object is released from a finalizer after the runtime (or a profiler
    attached to it) has begun its own shutdown."""
    try:
        if torch.cuda.is_initialized():
            torch.cuda.synchronize()
    except Exception:
        pass
    for obj in list(_live):
        try:
            obj.close()
        except Exception:
            pass
    _default_ws.clear()


atexit.register(_release_all)
