"""Plain CPU StaticGreedy oracle (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU product path never imports it
and shares no code with it. The arithmetic lives in ``oracle.c`` (plain C,
single-threaded); this module only compiles it with gcc and marshals numpy
arrays through ctypes.

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
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

NSTATS = 8
STAT_NAMES = ("trav_init", "trav_fwd", "trav_rev", "celf_evals", "live_pairs",
              "word_reach_deg", "word_reach_nodes", "decrements")


class OracleError(RuntimeError):
    pass


def build():
    """Compile oracle.c with gcc into liboracle.so (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                           "-Wextra", "-o", tmp, _SRC, "-lm"])
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


def live_bits(prob, R, seed):
    """Arc-major live bits: uint64[m, W]; bit b of word w = snapshot 64w+b."""
    prob = np.ascontiguousarray(prob, dtype=np.float32)
    W = (R + 63) // 64
    out = np.zeros((len(prob), W), dtype=np.uint64)
    _check(_load().oracle_live_bits(len(prob), _ptr(prob), R, seed, _ptr(out)), "live_bits")
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
