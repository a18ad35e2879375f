"""Write the stored expected values of the undirected (pair-coin) parity tests.

Calls only the CPU oracle (``oracle/``) and the seeded input generator. For
each undirected workload: a digest of the generated graph, the component
method's seeds and gains (Sec. 4, undirected snapshots), digests of every
round's full gain vector, and the pair ids' digest. Where Algorithm 2 on the
same pair-coin snapshots is affordable it must agree round by round.

Usage: python tests/golden/make_golden_undirected.py [workload ...]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1212_4779_amd import graphgen as gg  # noqa: E402

NAMES = ["nethept_uic", "million_undirected_uic"]
CROSS_CHECK = {"nethept_uic"}   # Algorithm 2 is affordable here


def vec_digest(v):
    return hashlib.sha256(np.ascontiguousarray(v, dtype="<u4").tobytes()).hexdigest()


def make(name):
    w = gg.WORKLOADS[name]
    t0 = time.time()
    g = gg.workload_graph(name)
    R, k, seed = w["R"], w["k"], w["seed"]
    pair = oracle.pair_ids(g.row_ptr, g.col, g.prob)
    seeds, gains, tr = oracle.select_components(g.row_ptr, g.col, g.prob, R, k, seed, trace=True)
    if name in CROSS_CHECK:
        s2, g2, tr2 = oracle.select_du_pairs(g.row_ptr, g.col, g.prob, R, k, seed, trace=True)
        assert (s2 == seeds).all() and (g2 == gains).all() and (tr2 == tr).all()
    out = dict(
        workload=name, recipe=w, n=g.n, m=g.m, graph_sha256=gg.graph_digest(g),
        pair_sha256=vec_digest(pair),
        seeds=[int(x) for x in seeds], gains=[int(x) for x in gains],
        round_gain_sha256=[vec_digest(tr[t]) for t in range(k + 1)],
        init_gain_sum=int(tr[0].astype(np.uint64).sum()),
    )
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"{name}: {time.time() - t0:.1f}s seeds[:5]={out['seeds'][:5]} gains[:5]={out['gains'][:5]}")


if __name__ == "__main__":
    for name in sys.argv[1:] or NAMES:
        make(name)
