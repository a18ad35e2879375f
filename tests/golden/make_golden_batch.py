"""Write the stored expected values of the 512-instance batched workload.

Calls only the CPU oracle (``oracle/``) and the seeded input generator. Every
one of the 512 instances is stored: a digest of the generated graph and the
oracle's StaticGreedyDU seeds, gains and traversal count. The
weighted-cascade instances are near-critical (the largest one alone costs the
single-threaded oracle minutes), so the instances run in worker processes,
largest first.

Usage: python tests/golden/make_golden_batch.py [workers]
"""
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1212_4779_amd import graphgen as gg  # noqa: E402


def one(i_w):
    i, w = i_w
    g = gg.graph_from_recipe(w)
    seeds, gains, _, st = oracle.select_du(g.row_ptr, g.col, g.prob, w["R"], w["k"], w["seed"])
    return dict(i=i, n=g.n, m=g.m, graph_sha256=gg.graph_digest(g), seeds=[int(x) for x in seeds],
                gains=[int(x) for x in gains],
                trav=st["trav_init"] + st["trav_fwd"] + st["trav_rev"])


if __name__ == "__main__":
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 6
    oracle._load()
    rec = gg.batch_instances(**gg.BATCH_WORKLOAD)
    t0 = time.time()
    # largest first, so that no long instance starts last
    todo = sorted(enumerate(rec), key=lambda iw: -iw[1]["n"] * iw[1]["R"])
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(one, todo, chunksize=1)
    res.sort(key=lambda r: r["i"])
    out = dict(workload="batch512", recipe=gg.BATCH_WORKLOAD, instances=res)
    with open(os.path.join(HERE, "batch512.json"), "w") as f:
        json.dump(out, f)
    print(f"batch512: {time.time() - t0:.1f}s")
