"""Write the stored expected values of the spread-evaluation parity tests.

Calls only the CPU oracle (``oracle/``) and the seeded input generator. For
each workload it scores the oracle's own greedy seeds (from the stored
selection golden file) on snapshots of an independent seed (the paper's
protocol scores seed sets on fresh simulations, Sec. 5.2): the prefix
increments of f and the per-snapshot reach sizes of the whole set.

Usage: python tests/golden/make_golden_spread.py [workload ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1212_4779_amd import graphgen as gg  # noqa: E402

EVAL = {"nethept_wc": {"R": 1000, "seed": 1001}, "million_uic": {"R": 256, "seed": 1001}}


def make(name):
    t0 = time.time()
    with open(os.path.join(HERE, f"{name}.json")) as f:
        sel = json.load(f)
    g = gg.workload_graph(name)
    assert gg.graph_digest(g) == sel["graph_sha256"]
    ev = EVAL[name]
    marg, per = oracle.spread_prefix(g.row_ptr, g.col, g.prob, ev["R"], ev["seed"], sel["seeds"])
    out = dict(workload=name, graph_sha256=sel["graph_sha256"], seeds=sel["seeds"],
               eval_R=ev["R"], eval_seed=ev["seed"],
               marg=[int(x) for x in marg], per_snapshot=[int(x) for x in per])
    with open(os.path.join(HERE, f"{name}_spread.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"{name}: {time.time() - t0:.1f}s f(S) = {int(marg.sum())} over R = {ev['R']}")


if __name__ == "__main__":
    for name in sys.argv[1:] or list(EVAL):
        make(name)
