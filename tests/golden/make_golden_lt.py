"""Write the stored expected values of the linear-threshold parity tests.

Calls only the CPU oracle (``oracle/``) and the seeded input generator: for
each linear-threshold workload a digest of the graph, of the live bits, the
seeds and gains of Algorithm 2 on the linear-threshold snapshots and the
digest of every round's full gain vector.

Usage: python tests/golden/make_golden_lt.py [workload ...]
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

NAMES = ["nethept_lt", "million_lt"]


def digest(v, dt):
    return hashlib.sha256(np.ascontiguousarray(v, dtype=dt).tobytes()).hexdigest()


def make(name):
    w = gg.WORKLOADS[name]
    t0 = time.time()
    g = gg.workload_graph(name)
    R, k, seed = w["R"], w["k"], w["seed"]
    bits = oracle.live_bits_lt(g.row_ptr, g.col, g.prob, R, seed)
    seeds, gains, tr = oracle.select_du_lt(g.row_ptr, g.col, g.prob, R, k, seed, trace=True)
    out = dict(
        workload=name, recipe=w, n=g.n, m=g.m, graph_sha256=gg.graph_digest(g),
        mask_sha256=digest(bits.T, "<u8"),   # word-major, as the library lays it out
        seeds=[int(x) for x in seeds], gains=[int(x) for x in gains],
        round_gain_sha256=[digest(tr[t], "<u4") for t in range(k + 1)],
    )
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"{name}: {time.time() - t0:.1f}s seeds[:5]={out['seeds'][:5]} gains[:5]={out['gains'][:5]}")


if __name__ == "__main__":
    for name in sys.argv[1:] or NAMES:
        make(name)
