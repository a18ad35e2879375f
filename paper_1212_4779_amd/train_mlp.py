"""Train the candidate-scoring network on exact gains from selection traces.

Labels come from the method itself: im_select's trace holds the exact gain
of every node at the start of every round. A sample is a node u and two
rounds t' < t (u unselected at t): input = static features of u and its
exact gain at t', target = its exact gain at t (both as ln(1 + g / R)).
This is what the lazy path knows about a node whose last evaluation was in
round t' when it scores it in round t. Everything (traces, features, sample
gather, forward, backward, Adam) runs in libim's kernels; numpy only draws
the random sample indices and the initial weights.

Usage:
    python -m paper_1212_4779_amd.train_mlp [--graphs 180] [--val 20] [--budget-s 0]
        [--steps 4000] [--out FILE]
"""
import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import api
from . import graphgen as gg

DEFAULT_OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "celf_mlp.json")


def init_params(seed):
    """He-normal initial weights, zero biases."""
    rng = np.random.default_rng(seed)
    H, IN = 64, 5
    parts = [rng.normal(0, np.sqrt(2.0 / IN), H * IN), np.zeros(H),
             rng.normal(0, np.sqrt(2.0 / H), H * H), np.zeros(H),
             rng.normal(0, np.sqrt(1.0 / H), H), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def draw_pairs(rng, gains0, seeds, k, n_top, n_rand, pairs_per_node):
    """(node, t', t) triples: the n_top nodes with the largest initial gain plus
    n_rand uniform ones; t' = 0 half of the time (never re-evaluated), else
    uniform; t uniform in (t', k); pairs where u was selected before t dropped."""
    n = len(gains0)
    top = np.argsort(-gains0.astype(np.int64), kind="stable")[:min(n_top, n)]
    rnd = rng.integers(0, n, n_rand)
    nodes = np.repeat(np.concatenate([top, rnd]), pairs_per_node)
    tp = np.where(rng.random(len(nodes)) < 0.5, 0, rng.integers(0, k - 1, len(nodes)))
    tc = tp + 1 + (rng.random(len(nodes)) * (k - 1 - tp)).astype(np.int64)
    sel_round = np.full(n, k + 1, np.int64)
    sel_round[seeds] = np.arange(len(seeds))
    keep = (tc < k) & (sel_round[nodes] >= tc)
    return nodes[keep].astype(np.uint32), tp[keep].astype(np.uint32), tc[keep].astype(np.uint32)


def samples_from_graph(w, g, rng, ws, n_top=4096, n_rand=4096, pairs=4):
    d = api.Graph.from_numpy(g.row_ptr, g.col, g.prob)
    seeds, _, trace = api.select(d, w["R"], w["k"], w["seed"], ws=ws, trace=True)
    feat = api.node_features(d, ws=ws)
    gains0 = trace[0].cpu().numpy()
    node, tp, tc = draw_pairs(rng, gains0, seeds.cpu().numpy(), w["k"], n_top, n_rand, pairs)
    to = lambda a: torch.from_numpy(a.view(np.int32)).cuda()
    x, t = api.mlp_samples(feat, trace.to(torch.int32), w["R"], to(node), to(tp), to(tc))
    return x, t


def train(x, t, xv, tv, params, steps, batch, lr, seed, log=print):
    rng = np.random.default_rng(seed)
    model = api.Mlp(params)
    grad = torch.empty(api.MLP_NPARAM, dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    hist = []
    for step in range(1, steps + 1):
        idx = torch.from_numpy(rng.integers(0, x.shape[0], batch).astype(np.int32)).cuda()
        model.train_step(x, t, idx, grad, loss, lr=lr)
        if step % 500 == 0 or step == steps:
            tr = model.loss_grad(x, t)[0].item()
            va = model.loss_grad(xv, tv)[0].item()
            hist.append((step, tr, va))
            log(f"step {step}: train {tr:.5f} val {va:.5f}")
    return model, hist


def _order(recipes):
    """Smallest graphs first, the two probability models interleaved, so that
    a time budget cut keeps a balanced subset."""
    uic = sorted((r for r in recipes if r["p"] is not None), key=lambda r: r["n"])
    wc = sorted((r for r in recipes if r["p"] is None), key=lambda r: r["n"])
    out = []
    for i in range(max(len(uic), len(wc))):
        out += [x[i] for x in (uic, wc) if i < len(x)]
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--graphs", type=int, default=180, help="training graphs used (at most)")
    ap.add_argument("--val", type=int, default=20, help="held-out validation graphs used")
    ap.add_argument("--models", default="both", choices=("both", "uic"),
                    help="probability models of the graphs: uniform IC and weighted cascade, or uniform IC only")
    ap.add_argument("--budget-s", type=float, default=0.0,
                    help="stop adding graphs once the traces took this long (0: no limit)")
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--out", default=DEFAULT_OUT)
    a = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)
    rec = gg.training_recipes(**{k: v for k, v in gg.TRAINING_WORKLOAD.items()})
    if a.models == "uic":
        rec = [r for r in rec if r["p"] is not None]
    train_rec = [r for r in rec if not r["validation"]][:a.graphs]
    val_rec = [r for r in rec if r["validation"]][:a.val]
    rng = np.random.default_rng(a.seed)
    xs, ts = {"train": [], "val": []}, {"train": [], "val": []}
    used = {"train": [], "val": []}
    t0 = time.time()
    trace_s = 0.0
    import multiprocessing as mp
    # smallest graphs first, both models and both splits interleaved, so that
    # a budget cut keeps a balanced subset
    jobs = [("val" if r["validation"] else "train", r) for r in _order(val_rec + train_rec)]
    # the generator workers are forked before this process touches the GPU
    pool = mp.get_context("fork").Pool(a.workers)
    try:
        graphs = pool.imap(gg.graph_from_recipe, [r for _, r in jobs])
        ws = api.Workspace()
        for (split, r), g in zip(jobs, graphs):
            if a.budget_s and trace_s > a.budget_s:
                log(f"trace budget of {a.budget_s:.0f}s reached: {len(used['train'])} training, "
                    f"{len(used['val'])} validation graphs")
                break
            torch.cuda.synchronize()
            t1 = time.time()
            x, t = samples_from_graph(r, g, rng, ws)
            torch.cuda.synchronize()
            dt = time.time() - t1
            trace_s += dt
            xs[split].append(x)
            ts[split].append(t)
            used[split].append(dict(graph_seed=r["graph_seed"], n=g.n, m=g.m, p=r["p"],
                                    trace_s=round(dt, 3)))
            log(f"{split} graph seed {r['graph_seed']}: n={g.n} m={g.m} p={r['p']} "
                f"samples={x.shape[0]} trace {dt:.2f}s ({time.time() - t0:.1f}s)")
            del g
    finally:
        pool.terminate()
    x, t = torch.cat(xs["train"]), torch.cat(ts["train"])
    xv, tv = torch.cat(xs["val"]), torch.cat(ts["val"])
    log(f"samples: train {x.shape[0]}, val {xv.shape[0]}")
    model, hist = train(x, t, xv, tv, init_params(a.seed), a.steps, a.batch, a.lr, a.seed, log)
    master, _ = model.params()
    out = dict(params=[float(v) for v in master], layout="W1[64][5] b1 W2[64][64] b2 w3 b3",
               features="ln1p(indeg, outdeg, sum p_out, sum outdeg(out-nbrs), gain/R)",
               training=dict(graphs=used["train"], validation=used["val"],
                             trace_seconds=round(trace_s, 1), budget_s=a.budget_s,
                             recipes_available=dict(train=len(train_rec), val=len(val_rec)),
                             samples=int(x.shape[0]), steps=a.steps, batch=a.batch, lr=a.lr,
                             seed=a.seed, history=hist))
    with open(a.out, "w") as f:
        json.dump(out, f)
    log(f"wrote {a.out} ({time.time() - t0:.1f}s)")
    return 0


def load(path=DEFAULT_OUT):
    """The trained network as an api.Mlp (raises if the file is missing)."""
    with open(path) as f:
        d = json.load(f)
    return api.Mlp(np.array(d["params"], np.float32))


if __name__ == "__main__":
    sys.exit(main())
