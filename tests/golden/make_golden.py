"""Write the stored expected values for the GPU parity tests.

Calls only the CPU oracle (``oracle/``) and the seeded input generator. For
each named workload it stores: a digest of the generated graph (so a run on
another machine can tell the generator drifted), the oracle's seeds and
gains, its work counters, a digest of the initial gain vector and one digest
per round of the full gain vector (StaticGreedyDU trace, Algorithm 2).

Usage: python tests/golden/make_golden.py [workload ...]
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


def vec_digest(v):
    return hashlib.sha256(np.ascontiguousarray(v, dtype="<u4").tobytes()).hexdigest()


def make(name):
    w = gg.WORKLOADS[name]
    t0 = time.time()
    g = gg.workload_graph(name)
    R, k, seed = w["R"], w["k"], w["seed"]
    seeds, gains, tr, st = oracle.select_du(g.row_ptr, g.col, g.prob, R, k, seed, trace=True)
    init, st0 = oracle.initial_gains(g.row_ptr, g.col, g.prob, R, seed)
    assert (init == tr[0]).all()
    out = dict(
        workload=name, recipe=w, n=g.n, m=g.m,
        graph_sha256=gg.graph_digest(g),
        seeds=[int(x) for x in seeds], gains=[int(x) for x in gains],
        stats=st, init_stats=st0,
        init_gain_sha256=vec_digest(tr[0]),
        round_gain_sha256=[vec_digest(tr[t]) for t in range(k + 1)],
        init_gain_sum=int(init.astype(np.uint64).sum()),
        max_out_degree=int(g.out_degree().max()), max_in_degree=int(g.in_degree().max()),
    )
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"{name}: {time.time() - t0:.1f}s seeds[:5]={out['seeds'][:5]}")


if __name__ == "__main__":
    names = sys.argv[1:] or list(gg.WORKLOADS)
    for nm in names:
        make(nm)
