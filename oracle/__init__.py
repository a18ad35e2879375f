"""Plain CPU StaticGreedy oracle (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU product path never imports it
and shares no code with it. The arithmetic lives in ``oracle.c`` (plain C,
single-threaded) and ``mlp.c`` (FP64 reference of the candidate-scoring
network); this module only compiles them with gcc and marshals numpy arrays
through ctypes.

Paper: Cheng et al., "StaticGreedy: Solving the Scalability-Accuracy Dilemma
in Influence Maximization", CIKM 2013 (arXiv 1212.4779): Sec. 3.1 (IC model,
snapshots), Algorithm 1 (StaticGreedy), Algorithm 2 (StaticGreedyDU), Sec. 5
(StaticGreedyCELF).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "mlp.c")]
_LIB = os.path.join(_HERE, "liboracle.so")

NSTATS = 8
STAT_NAMES = ("trav_init", "trav_fwd", "trav_rev", "celf_evals", "live_pairs",
              "word_reach_deg", "word_reach_nodes", "decrements")


class OracleError(RuntimeError):
    pass


def build():
    """Compile oracle.c and mlp.c with gcc into liboracle.so (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                           "-Wextra", "-o", tmp, *_SRC, "-lm"])
    os.replace(tmp, _LIB)


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        u32, u64, p = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p
        lib.oracle_splitmix64_output.restype = u64
        lib.oracle_splitmix64_output.argtypes = [u64, u64]
        lib.oracle_live_bits.argtypes = [u64, p, u32, u64, p]
        graph = [u32, u64, p, p, p, u32]
        lib.oracle_initial_gains.argtypes = graph + [u64, p, p]
        lib.oracle_select_du.argtypes = graph + [u32, u64, p, p, p, p]
        lib.oracle_select_alg1.argtypes = graph + [u32, u64, p, p]
        lib.oracle_select_celf.argtypes = graph + [u32, u64, p, p, p]
        lib.oracle_spread.argtypes = graph + [u64, p, u32, p]
        lib.oracle_spread_prefix.argtypes = graph + [u64, p, u32, p, p]
        lib.oracle_live_bits_keyed.argtypes = [u64, p, u32, u64, p, p]
        lib.oracle_pair_ids.argtypes = [u32, u64, p, p, p, p]
        lib.oracle_select_du_pairs.argtypes = graph + [u32, u64, p, p, p, p]
        lib.oracle_select_components.argtypes = graph + [u32, u64, p, p, p]
        lib.oracle_live_bits_lt.argtypes = [u32, u64, p, p, p, u32, u64, p]
        lib.oracle_select_du_lt.argtypes = graph + [u32, u64, p, p, p, p]
        lib.oracle_mlp_nparams.restype = ctypes.c_int
        lib.oracle_bf16_round.argtypes = [u64, p, p]
        lib.oracle_node_features.argtypes = [u32, u64, p, p, p, p]
        lib.oracle_mlp_forward.argtypes = [p, u64, p, p]
        lib.oracle_mlp_loss_grad.argtypes = [p, u64, p, p, p]
        lib.oracle_mlp_loss_grad.restype = ctypes.c_double
        d = ctypes.c_double
        lib.oracle_adam_step.argtypes = [u64, p, p, p, p, d, d, d, d, u32]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _graph(row_ptr, col, prob):
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.uint64)
    col = np.ascontiguousarray(col, dtype=np.uint32)
    prob = np.ascontiguousarray(prob, dtype=np.float32)
    n = len(row_ptr) - 1
    return n, len(col), row_ptr, col, prob


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


def splitmix64_output(state, i):
    """i-th output (i >= 1) of a SplitMix64 generator with initial state `state`."""
    return int(_load().oracle_splitmix64_output(state, i))


def live_bits(prob, R, seed, key_of=None):
    """Arc-major live bits: uint64[m, W]; bit b of word w = snapshot 64w+b.
    key_of[e]: the index arc e's coins are drawn under (default e)."""
    prob = np.ascontiguousarray(prob, dtype=np.float32)
    W = (R + 63) // 64
    out = np.zeros((len(prob), W), dtype=np.uint64)
    if key_of is None:
        _check(_load().oracle_live_bits(len(prob), _ptr(prob), R, seed, _ptr(out)), "live_bits")
    else:
        key_of = np.ascontiguousarray(key_of, dtype=np.uint32)
        _check(_load().oracle_live_bits_keyed(len(prob), _ptr(prob), R, seed, _ptr(key_of),
                                              _ptr(out)), "live_bits")
    return out


def initial_gains(row_ptr, col, prob, R, seed):
    """s_u = sum_r |R_r(u)| (Algorithm 2, initial loop). Returns (gains, stats)."""
    n, m, row_ptr, col, prob = _graph(row_ptr, col, prob)
    gains = np.zeros(n, dtype=np.uint32)
    stats = np.zeros(NSTATS, dtype=np.uint64)
    _check(_load().oracle_initial_gains(n, m, _ptr(row_ptr), _ptr(col), _ptr(prob), R, seed,
                                        _ptr(gains), _ptr(stats)), "initial_gains")
    return gains, dict(zip(STAT_NAMES, (int(x) for x in stats)))


def select_du(row_ptr, col, prob, R, k, seed, trace=False):
    """StaticGreedyDU (Algorithm 2). Returns (seeds, gains, trace_or_None, stats)."""
    n, m, row_ptr, col, prob = _graph(row_ptr, col, prob)
    seeds = np.zeros(k, dtype=np.uint32)
    gains = np.zeros(k, dtype=np.uint64)
    tr = np.zeros((k + 1, n), dtype=np.uint32) if trace else None
    stats = np.zeros(NSTATS, dtype=np.uint64)
    _check(_load().oracle_select_du(n, m, _ptr(row_ptr), _ptr(col), _ptr(prob), R, k, seed,
                                    _ptr(seeds), _ptr(gains),
                                    _ptr(tr) if trace else None, _ptr(stats)), "select_du")
    return seeds, gains, tr, dict(zip(STAT_NAMES, (int(x) for x in stats)))


def select_alg1(row_ptr, col, prob, R, k, seed):
    """StaticGreedy exactly as Algorithm 1 (slow). Returns (seeds, gains)."""
    n, m, row_ptr, col, prob = _graph(row_ptr, col, prob)
    seeds = np.zeros(k, dtype=np.uint32)
    gains = np.zeros(k, dtype=np.uint64)
    _check(_load().oracle_select_alg1(n, m, _ptr(row_ptr), _ptr(col), _ptr(prob), R, k, seed,
                                      _ptr(seeds), _ptr(gains)), "select_alg1")
    return seeds, gains


def select_celf(row_ptr, col, prob, R, k, seed):
    """StaticGreedyCELF (lazy exact re-evaluation). Returns (seeds, gains, stats)."""
    n, m, row_ptr, col, prob = _graph(row_ptr, col, prob)
    seeds = np.zeros(k, dtype=np.uint32)
    gains = np.zeros(k, dtype=np.uint64)
    stats = np.zeros(NSTATS, dtype=np.uint64)
    _check(_load().oracle_select_celf(n, m, _ptr(row_ptr), _ptr(col), _ptr(prob), R, k, seed,
                                      _ptr(seeds), _ptr(gains), _ptr(stats)), "select_celf")
    return seeds, gains, dict(zip(STAT_NAMES, (int(x) for x in stats)))


def spread(row_ptr, col, prob, R, seed, S):
    """f(S) = sum_r |R_r(S)|, the snapshot estimate of I(S) times R."""
    n, m, row_ptr, col, prob = _graph(row_ptr, col, prob)
    S = np.ascontiguousarray(S, dtype=np.uint32)
    out = ctypes.c_uint64(0)
    _check(_load().oracle_spread(n, m, _ptr(row_ptr), _ptr(col), _ptr(prob), R, seed,
                                 _ptr(S), len(S), ctypes.byref(out)), "spread")
    return int(out.value)


def live_bits_lt(row_ptr, col, prob, R, seed):
    """Linear-threshold live bits, arc-major uint64[m, W] (prob = the weights):
    per snapshot each node keeps at most one in-arc."""
    n, m, row_ptr, col, prob = _graph(row_ptr, col, prob)
    W = (R + 63) // 64
    out = np.zeros((m, W), dtype=np.uint64)
    _check(_load().oracle_live_bits_lt(n, m, _ptr(row_ptr), _ptr(col), _ptr(prob), R, seed,
                                       _ptr(out)), "live_bits_lt")
    return out


def select_du_lt(row_ptr, col, prob, R, k, seed, trace=False):
    """Algorithm 2 on linear-threshold snapshots. Returns (seeds, gains, trace_or_None)."""
    n, m, row_ptr, col, prob = _graph(row_ptr, col, prob)
    seeds = np.zeros(k, dtype=np.uint32)
    gains = np.zeros(k, dtype=np.uint64)
    tr = np.zeros((k + 1, n), dtype=np.uint32) if trace else None
    stats = np.zeros(NSTATS, dtype=np.uint64)
    _check(_load().oracle_select_du_lt(n, m, _ptr(row_ptr), _ptr(col), _ptr(prob), R, k, seed,
                                       _ptr(seeds), _ptr(gains), _ptr(tr) if trace else None,
                                       _ptr(stats)), "select_du_lt")
    return seeds, gains, tr


def pair_ids(row_ptr, col, prob):
    """Canonical arc (the direction with the smaller tail) of every arc's
    undirected pair; raises unless the CSR is symmetric as the undirected
    reading requires."""
    n, m, row_ptr, col, prob = _graph(row_ptr, col, prob)
    out = np.zeros(m, dtype=np.uint32)
    _check(_load().oracle_pair_ids(n, m, _ptr(row_ptr), _ptr(col), _ptr(prob), _ptr(out)),
           "pair_ids")
    return out


def select_du_pairs(row_ptr, col, prob, R, k, seed, trace=False):
    """Algorithm 2 on pair-coin snapshots of a symmetric CSR."""
    n, m, row_ptr, col, prob = _graph(row_ptr, col, prob)
    seeds = np.zeros(k, dtype=np.uint32)
    gains = np.zeros(k, dtype=np.uint64)
    tr = np.zeros((k + 1, n), dtype=np.uint32) if trace else None
    stats = np.zeros(NSTATS, dtype=np.uint64)
    _check(_load().oracle_select_du_pairs(n, m, _ptr(row_ptr), _ptr(col), _ptr(prob), R, k, seed,
                                          _ptr(seeds), _ptr(gains),
                                          _ptr(tr) if trace else None, _ptr(stats)),
           "select_du_pairs")
    return seeds, gains, tr


def select_components(row_ptr, col, prob, R, k, seed, trace=False):
    """The undirected component method (Sec. 4) on pair-coin snapshots."""
    n, m, row_ptr, col, prob = _graph(row_ptr, col, prob)
    seeds = np.zeros(k, dtype=np.uint32)
    gains = np.zeros(k, dtype=np.uint64)
    tr = np.zeros((k + 1, n), dtype=np.uint32) if trace else None
    _check(_load().oracle_select_components(n, m, _ptr(row_ptr), _ptr(col), _ptr(prob), R, k,
                                            seed, _ptr(seeds), _ptr(gains),
                                            _ptr(tr) if trace else None), "select_components")
    return seeds, gains, tr


def spread_prefix(row_ptr, col, prob, R, seed, S):
    """(marg uint64 [len(S)], per uint32 [R]): marg[i] = f(S[:i+1]) - f(S[:i]),
    per[r] = |R_r(S)| (Sec. 3.1 estimator; every prefix searched from scratch)."""
    n, m, row_ptr, col, prob = _graph(row_ptr, col, prob)
    S = np.ascontiguousarray(S, dtype=np.uint32)
    marg = np.zeros(len(S), dtype=np.uint64)
    per = np.zeros(R, dtype=np.uint32)
    _check(_load().oracle_spread_prefix(n, m, _ptr(row_ptr), _ptr(col), _ptr(prob), R, seed,
                                        _ptr(S), len(S), _ptr(marg), _ptr(per)), "spread_prefix")
    return marg, per


# ---------------------------------------------------------------------------
# candidate-scoring network (mlp.c)
# ---------------------------------------------------------------------------
MLP_IN, MLP_H = 5, 64


def mlp_nparams():
    return int(_load().oracle_mlp_nparams())


def bf16_round(a):
    """Round float32 values to bfloat16 precision (nearest, ties to even)."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    out = np.empty_like(a)
    _load().oracle_bf16_round(a.size, _ptr(a), _ptr(out))
    return out


def node_features(row_ptr, col, prob):
    """Static node features float64 [n, 4] (ln(1+x) of in/out degree, out-probability
    sum, two-hop out-degree sum)."""
    n, m, row_ptr, col, prob = _graph(row_ptr, col, prob)
    out = np.zeros((n, 4), dtype=np.float64)
    _check(_load().oracle_node_features(n, m, _ptr(row_ptr), _ptr(col), _ptr(prob), _ptr(out)),
           "node_features")
    return out


def mlp_forward(params, x):
    params = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, MLP_IN)
    y = np.zeros(len(x), dtype=np.float64)
    _load().oracle_mlp_forward(_ptr(params), len(x), _ptr(x), _ptr(y))
    return y


def mlp_loss_grad(params, x, t):
    """(L, dL/dparams) for L = sum (y - t)^2 / (2N), in float64."""
    params = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, MLP_IN)
    t = np.ascontiguousarray(t, dtype=np.float64)
    g = np.zeros(mlp_nparams(), dtype=np.float64)
    loss = _load().oracle_mlp_loss_grad(_ptr(params), len(x), _ptr(x), _ptr(t), _ptr(g))
    return float(loss), g


def adam_step(theta, m, v, g, lr, b1, b2, eps, t):
    """One Adam step in place on float64 arrays theta, m, v."""
    for a in (theta, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = np.ascontiguousarray(g, dtype=np.float64)
    _load().oracle_adam_step(len(theta), _ptr(theta), _ptr(m), _ptr(v), _ptr(g), lr, b1, b2, eps, t)
