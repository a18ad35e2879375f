"""Seeded synthetic influence graphs (input generation only).

This module produces the inputs that both the GPU path and the CPU oracle
consume: a CSR graph with one IC probability per stored arc. It holds none of
the selection method's arithmetic (no snapshot sampling, no reachability).

The paper's datasets (NetHEPT, NetPHY, DBLP, Epinions, Slashdot, Douban;
Sec. 5, Table 2) are not available, so power-law Chung-Lu graphs of matching
shape stand in for them. Probabilities follow the two models of Sec. 3.4.1 /
Sec. 5: uniform IC (one p for every arc) and weighted cascade, where
p(u,v) = 1/d_v with d_v the in-degree of v.

Generator ("fast Chung-Lu"): node weights w_i = (i+1)^(-1/(gamma-1)), handed
to nodes through seeded permutations (independent ones for out- and
in-weights on directed graphs, one for undirected graphs). Endpoints are drawn
in proportion to the weights; self-loops are dropped and repeated pairs keep
their first occurrence, until exactly the requested number of arcs (directed)
or pairs (undirected, both directions stored) exists. Arcs are stored sorted by
(tail, head); the arc id is the CSR position.
"""
from dataclasses import dataclass

import numpy as np


@dataclass
class Graph:
    n: int
    row_ptr: np.ndarray  # uint64[n+1]
    col: np.ndarray      # uint32[m]
    prob: np.ndarray     # float32[m]

    @property
    def m(self):
        return int(len(self.col))

    def out_degree(self):
        return np.diff(self.row_ptr.astype(np.int64))

    def in_degree(self):
        return np.bincount(self.col.astype(np.int64), minlength=self.n)


def _weights(n, gamma):
    return (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (gamma - 1.0))


def _sample(cdf, u):
    idx = np.searchsorted(cdf, u, side="right")
    return np.minimum(idx, len(cdf) - 1)


def chung_lu_arcs(n, target, gamma, seed, directed=True):
    """Return (src, dst) of `target` distinct arcs (directed) or pairs (undirected)."""
    if n < 2 or target == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    max_pairs = n * (n - 1) if directed else n * (n - 1) // 2
    if target > max_pairs // 4:
        raise ValueError("graph too dense for this generator")
    rng = np.random.default_rng(seed)
    base = _weights(n, gamma)
    w_out = base[rng.permutation(n)]
    w_in = base[rng.permutation(n)] if directed else w_out
    cdf_out = np.cumsum(w_out)
    cdf_out /= cdf_out[-1]
    cdf_in = np.cumsum(w_in)
    cdf_in /= cdf_in[-1]
    keys = np.zeros(0, np.int64)
    have = 0
    rounds = 0
    while have < target:
        rounds += 1
        if rounds > 200:
            raise RuntimeError("Chung-Lu sampling did not reach the target arc count")
        b = int((target - have) * 1.25) + 1024
        a = _sample(cdf_out, rng.random(b))
        c = _sample(cdf_in, rng.random(b))
        keep = a != c
        a, c = a[keep], c[keep]
        if not directed:
            a, c = np.minimum(a, c), np.maximum(a, c)
        keys = np.concatenate([keys, a.astype(np.int64) * n + c])
        _, first = np.unique(keys, return_index=True)
        first.sort()
        keys = keys[first]
        have = len(keys)
    keys = keys[:target]
    return keys // n, keys % n


def to_csr(n, src, dst):
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    row_ptr = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(np.bincount(src, minlength=n), out=row_ptr[1:])
    return row_ptr, dst.astype(np.uint32)


def uniform_prob(m, p):
    return np.full(m, p, dtype=np.float32)


def weighted_cascade_prob(n, col):
    """p(u,v) = 1/indeg(v), computed in IEEE single precision."""
    indeg = np.bincount(col.astype(np.int64), minlength=n).astype(np.float32)
    return (np.float32(1.0) / indeg[col.astype(np.int64)]).astype(np.float32)


def chung_lu_graph(n, m, gamma, seed, directed=True, p=None):
    """Chung-Lu graph with `m` stored arcs; p=None means weighted cascade."""
    if directed:
        s, d = chung_lu_arcs(n, m, gamma, seed, True)
    else:
        s0, d0 = chung_lu_arcs(n, m // 2, gamma, seed, False)
        s, d = np.concatenate([s0, d0]), np.concatenate([d0, s0])
    row_ptr, col = to_csr(n, s, d)
    prob = weighted_cascade_prob(n, col) if p is None else uniform_prob(len(col), p)
    return Graph(n, row_ptr, col, prob)


# Workloads, named by what they are. Each entry: graph recipe + (R, k, seed).
WORKLOADS = {
    # directed power law 2.5, 2,000 nodes, 20,000 arcs, uniform IC p=0.05, R=64, k=10
    "tiny_uic": dict(n=2000, m=20000, gamma=2.5, graph_seed=1, directed=True, p=0.05,
                     R=64, k=10, seed=1),
    # undirected (both directions stored) 15,000 nodes, 59,000 arcs, weighted cascade,
    # R=100, k=50: the shape of the paper's NetHEPT setting
    "nethept_wc": dict(n=15000, m=59000, gamma=2.5, graph_seed=2, directed=False, p=None,
                       R=100, k=50, seed=1),
    # directed power law 2.1, 1,000,000 nodes, 10,000,000 arcs, uniform IC p=0.01,
    # R=256, k=50
    "million_uic": dict(n=1000000, m=10000000, gamma=2.1, graph_seed=3, directed=True,
                        p=0.01, R=256, k=50, seed=1),
    # the NetHEPT-shaped undirected graph under uniform IC p=0.01 with one coin
    # per undirected pair, R=100, k=50
    "nethept_uic": dict(n=15000, m=59000, gamma=2.5, graph_seed=2, directed=False, p=0.01,
                        R=100, k=50, seed=1),
    # undirected power law 2.1, 1,000,000 nodes, 5,000,000 pairs (10,000,000 stored
    # arcs), uniform IC p=0.01 with one coin per pair, R=256, k=50: a DBLP-like
    # scale, large enough that every snapshot has a giant component
    "million_undirected_uic": dict(n=1000000, m=10000000, gamma=2.1, graph_seed=5,
                                   directed=False, p=0.01, R=256, k=50, seed=1),
    # linear threshold with weighted-cascade weights b(u,v) = 1/indeg(v) (every
    # node's in-weights sum to 1): the NetHEPT-shaped graph, R=100, k=50 ...
    "nethept_lt": dict(n=15000, m=59000, gamma=2.5, graph_seed=2, directed=False, p=None,
                       R=100, k=50, seed=1, model="lt"),
    # ... and the million-node directed graph, R=256, k=50
    "million_lt": dict(n=1000000, m=10000000, gamma=2.1, graph_seed=3, directed=True, p=None,
                       R=256, k=50, seed=1, model="lt"),
}


def workload_graph(name):
    w = WORKLOADS[name]
    return chung_lu_graph(w["n"], w["m"], w["gamma"], w["graph_seed"], w["directed"], w["p"])


BATCH_WORKLOAD = dict(count=512, master_seed=4)


def batch_instances(count=512, master_seed=4):
    """Recipe of the batched workload: `count` uneven instances.

    Per instance i: n log-uniform in [1e3, 2e5], mean degree uniform in [4, 16],
    directed Chung-Lu with exponent 2.5 (graph seed 1000+i); even i uniform IC with
    p alternating 0.01 / 0.05, odd i weighted cascade; R uniform over {64,128,256};
    k = 20; selection seed 1.
    """
    rng = np.random.default_rng(master_seed)
    out = []
    for i in range(count):
        n = int(round(np.exp(rng.uniform(np.log(1e3), np.log(2e5)))))
        deg = rng.uniform(4.0, 16.0)
        R = int(rng.choice([64, 128, 256]))
        if i % 2 == 0:
            p = 0.01 if (i // 2) % 2 == 0 else 0.05
        else:
            p = None
        out.append(dict(n=n, m=int(round(n * deg)), gamma=2.5, graph_seed=1000 + i,
                        directed=True, p=p, R=R, k=20, seed=1))
    return out


TRAINING_WORKLOAD = dict(count=200, master_seed=5, first_graph_seed=5000)


def training_recipes(count=200, master_seed=5, first_graph_seed=5000):
    """Graphs whose selection traces train the candidate-scoring network.

    Per graph i: n log-uniform in [1e5, 1e6], exponent uniform in [2.1, 2.5],
    mean degree uniform in [4, 16], directed Chung-Lu (graph seed 5000+i);
    even i uniform IC with p alternating 0.01 / 0.05, odd i weighted cascade;
    R = 256, k = 50, selection seed 1. The last tenth is held out for
    validation.
    """
    rng = np.random.default_rng(master_seed)
    out = []
    for i in range(count):
        n = int(round(np.exp(rng.uniform(np.log(1e5), np.log(1e6)))))
        gamma = float(rng.uniform(2.1, 2.5))
        deg = float(rng.uniform(4.0, 16.0))
        if i % 2 == 0:
            p = 0.01 if (i // 2) % 2 == 0 else 0.05
        else:
            p = None
        out.append(dict(n=n, m=int(round(n * deg)), gamma=gamma, graph_seed=first_graph_seed + i,
                        directed=True, p=p, R=256, k=50, seed=1, validation=i >= count * 9 // 10))
    return out


def graph_from_recipe(w):
    return chung_lu_graph(w["n"], w["m"], w["gamma"], w["graph_seed"], w["directed"], w["p"])


def graphs_from_recipes(recipes, workers=8):
    """Generate many graphs in worker processes (same output as one by one)."""
    if workers <= 1 or len(recipes) < 2:
        return [graph_from_recipe(w) for w in recipes]
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        return pool.map(graph_from_recipe, recipes, chunksize=1)


def graph_digest(g):
    """SHA-256 over the CSR arrays (detects generator drift between machines)."""
    import hashlib
    h = hashlib.sha256()
    for a in (np.asarray(g.row_ptr, np.uint64), np.asarray(g.col, np.uint32),
              np.asarray(g.prob, np.float32)):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()
