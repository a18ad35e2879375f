"""Accuracy of StaticGreedy against the number of snapshots R (Sec. 3.4).

For each R the selection runs `runs` times with different snapshot seeds (all
runs of one R as one batched call); every solution is scored on one common
set of independent snapshots (the spread evaluator, R_eval of them). The
paper's measures:

  d_{R,k} = (I(S*_k) - I(S_{R,k})) / I(S*_k), averaged over the runs, where
            S*_k is the reference solution (the paper takes CELFGreedy with
            20,000 simulations; here one StaticGreedy run with R_ref
            snapshots, the comparison system being out of scope);
  R_min   = the smallest R of the sweep with mean d_{R,k} <= 0.005;
  H_{R,k} = -sum_S p(S) log p(S) over the distinct solutions (as sets) of
            the runs, p(S) their frequency (natural logarithm).

Every selection and evaluation runs in the library's kernels; this module
only arranges the calls and computes the summary numbers.

Usage: python -m paper_1212_4779_amd.accuracy [--workload nethept_uic] [--runs 100]
"""
import argparse
import json
import math
import sys
import time
from collections import Counter


def entropy(solutions):
    """H = -sum p log p over the distinct solutions (order-free sets)."""
    counts = Counter(frozenset(s) for s in solutions)
    total = sum(counts.values())
    h = -sum(c / total * math.log(c / total) for c in counts.values())
    return h if h > 0.0 else 0.0


def relative_differences(ref_spread, spreads):
    """(I(S*) - I(S)) / I(S*) for every solution's spread."""
    return [(ref_spread - x) / ref_spread for x in spreads]


def r_min(sweep, tol=0.005):
    """Smallest R whose mean relative difference is within tol (None if none)."""
    ok = [row["R"] for row in sweep if row["d_mean"] <= tol]
    return min(ok) if ok else None


def _score(api, graph, S, R_eval, eval_seed, ws):
    _, per = api.spread(graph, R_eval, eval_seed, S, ws=ws, marginals=False, per_snapshot=True)
    return int(per.sum().item()) / R_eval


def study(graph, Rs, k, runs, R_eval, eval_seed, R_ref=4096, k_entropy=5, log=print,
          keep_runs=False):
    """The sweep on one device graph; returns a dict with one row per R (with
    keep_runs, each row also lists every run's seeds and scored spread, and
    the result the reference seeds)."""
    from . import api

    ws = api.Workspace()
    t0 = time.perf_counter()
    ref_seeds, _, _ = api.select(graph, R_ref, k, 999, ws=ws)
    sols = {}
    for R in Rs:
        out = api.select_batch([(graph, R, k, 1000 + r) for r in range(runs)], ws=ws)
        sols[R] = [s.cpu().tolist() for s, _ in out]
    t_sel = time.perf_counter() - t0
    # one common set of independent snapshots scores every solution
    t1 = time.perf_counter()
    ref = _score(api, graph, ref_seeds.cpu().tolist(), R_eval, eval_seed, ws)
    rows = []
    for R in Rs:
        spreads = [_score(api, graph, S, R_eval, eval_seed, ws) for S in sols[R]]
        d = relative_differences(ref, spreads)
        rows.append({"R": R, "spread_mean": sum(spreads) / runs, "d_mean": sum(d) / runs,
                     "H_k": entropy([S[:k_entropy] for S in sols[R]]),
                     "distinct_solutions": len({frozenset(S) for S in sols[R]})})
        if keep_runs:
            rows[-1]["runs"] = [{"seed": 1000 + r, "seeds": sols[R][r], "spread": spreads[r]}
                                for r in range(runs)]
        log(f"R={R}: spread {rows[-1]['spread_mean']:.2f}, d {rows[-1]['d_mean']:.5f}, "
            f"H_{k_entropy} {rows[-1]['H_k']:.3f}")
    out = {"rows": rows, "reference_R": R_ref, "reference_spread": ref, "R_min": r_min(rows),
            "runs": runs, "k": k, "k_entropy": k_entropy, "R_eval": R_eval,
            "eval_seed": eval_seed, "selection_s": round(t_sel, 3),
            "evaluation_s": round(time.perf_counter() - t1, 3)}
    if keep_runs:
        out["reference_seeds"] = ref_seeds.cpu().tolist()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workload", default="nethept_uic")
    ap.add_argument("--runs", type=int, default=100)
    ap.add_argument("--k", type=int, default=50)
    ap.add_argument("--R", default="1,5,10,25,50,100,200,500,1000")
    ap.add_argument("--R-ref", type=int, default=4096)
    ap.add_argument("--R-eval", type=int, default=20000)
    ap.add_argument("--eval-seed", type=int, default=777)
    args = ap.parse_args()
    from . import api
    from . import graphgen as gg
    g = gg.workload_graph(args.workload)
    d = api.Graph.from_numpy(g.row_ptr, g.col, g.prob)
    res = study(d, [int(x) for x in args.R.split(",")], args.k, args.runs, args.R_eval,
                args.eval_seed, R_ref=args.R_ref,
                log=lambda msg: print(msg, file=sys.stderr, flush=True))
    res["workload"] = args.workload
    print(json.dumps(res))


if __name__ == "__main__":
    main()
