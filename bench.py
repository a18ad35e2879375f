#!/usr/bin/env python3
"""Benchmark: StaticGreedy k-seed selection on one MI355X.

One step = one full im_select call on a device-resident graph: validation,
reverse CSR, snapshot masks, initial reach counts, and k greedy rounds of
argmax + forward search + reverse decrements. The graph is uploaded before the
timed region. The same selection is also timed on the lazy path
(im_select_lazy) in bound order ("plain") and with the trained network
("learned": first batch of each round sized by its predicted gain;
"learned_score_order": batches in its score order), with their
exact-evaluation counts; all paths must return the same seeds and gains.

Prints ONE JSON line. `value` is snapshot-edge traversals per second: the
per-snapshot work the method defines (the full out-degree of every node
reached in every snapshot by every reachability task, in-degree for the
reverse steps), the same numerator the CPU oracle counts, divided by the
selection wall time. `roofline` reports the dominant propagation kernel's
algorithmic bytes per launch over its event-timed average duration, against
the 8 TB/s HBM peak. `cpu_baseline` times the plain single-threaded CPU oracle
on the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = ("k-seed selection wall time + snapshot-edge traversals/s (% HBM peak), "
          "learned vs plain")
# algorithmic bytes: per (task, reached node) the two row offsets (8 B); per
# (arc, word) relaxation the head id (4 B) and the snapshot word (8 B); per
# reached node of a reverse task the gain read-modify-write (8 B); per node of
# the forward search the covered word read-modify-write (16 B)
B_NODE, B_RELAX, B_DEC, B_COVER = 8, 12, 8, 16
PROPAGATION = ("init_t0", "init_t1", "init_t2", "forward", "rev_t0", "rev_t1", "rev_t2")


def kernel_bytes(st, n, W):
    """Algorithmic bytes of each propagation phase over one call."""
    out = {}
    for t in range(3):
        out[f"init_t{t}"] = (B_RELAX * st[f"relax_init_t{t}"] + B_NODE * st[f"reached_init_t{t}"]
                             + (4 * n * W if t == 0 else 0))
        out[f"rev_t{t}"] = B_RELAX * st[f"relax_rev_t{t}"] + (B_NODE + B_DEC) * st[f"reached_rev_t{t}"]
    out["forward"] = B_RELAX * st["relax_fwd"] + (B_NODE + B_COVER) * st["tasks_rev"]
    return out


KERNEL_NAMES = {
    "init_t0": "k_lds_bfs<COUNT,64,...>", "init_t1": "k_lds_bfs<COUNT,256,...>",
    "init_t2": "k_block_bfs<COUNT,...>", "forward": "k_forward",
    "rev_t0": "k_lds_bfs<DEC,64,...>", "rev_t1": "k_lds_bfs<DEC,256,...>",
    "rev_t2": "k_block_bfs<DEC,...>",
}


def source_digest(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1212_4779_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


T1_SHAPES = {0: "256, 4, 256, 192,", 1: "256, 2, 512, 384,", 2: "256, 1, 1024, 768,"}


def kernel_signature(phase, schedule):
    """The part of the launched kernel's name that the schedule decides (the
    tier-1 shape and tier-2 lanes are template arguments)."""
    mode = "0" if phase.startswith("init") else "1"
    if phase == "forward":
        return "k_forward_coop"
    if phase.endswith("_t0"):
        return f"k_lds_bfs<{mode}, 64, 8, 32, 24,"
    if phase.endswith("_t1"):
        return f"k_lds_bfs<{mode}, " + T1_SHAPES[int(schedule.get("tier1_shape", 0))]
    return f"k_block_bfs<{mode}, {int(schedule.get('tier2_lanes', 256))}, 8,"


# options that change how much work a kernel instance does per launch (not
# which instance runs): the last tier runs what tier 1 hands on, which its
# table size (the tier-1 shape) decides; tier 1 takes every reverse task when
# the reverse tasks start there; the split multiplies the last tier's tasks
WORK_OPTIONS = {"init_t2": (("tier1_shape", 0),),
                "rev_t1": (("rev_first_tier", 0),),
                "rev_t2": (("tier1_shape", 0), ("rev_first_tier", 0), ("rev_split", 1))}


def load_traffic(phase, workload, schedule):
    """HBM bytes per launch of `phase` from the committed rocprofv3 counter
    summary (profiles/traffic.json), if it was taken on this workload, on the
    current source of that kernel, on the kernel this schedule launches and
    with the same share of the work; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    t = t.get("workloads", {}).get(workload, {})
    k = t.get("kernels", {}).get(phase)
    if not k:
        return None
    if k.get("source_digest") != source_digest(k.get("sources", [])):
        return None
    if kernel_signature(phase, schedule) not in k.get("kernel", ""):
        return None
    for key, default in WORK_OPTIONS.get(phase, ()):
        if int(schedule.get(key, default)) != int(t.get("schedule", {}).get(key, default)):
            return None
    return k.get("hbm_bytes_per_launch")


def cpu_baseline(g, w, log):
    import oracle
    oracle._load()
    t0 = time.perf_counter()
    seeds, gains, _, st = oracle.select_du(g.row_ptr, g.col, g.prob, w["R"], w["k"], w["seed"])
    dt = time.perf_counter() - t0
    trav = st["trav_init"] + st["trav_fwd"] + st["trav_rev"]
    log(f"cpu oracle: {dt:.2f}s, {trav:.3e} traversals")
    return {"value": trav / dt, "unit": "snapshot-edge traversals/s", "cores": 1, "kind": "oracle",
            "sample": f"whole workload (R={w['R']}, k={w['k']}), StaticGreedyDU oracle, one thread",
            "seconds": round(dt, 3)}, seeds, gains


def spread_leg(im, dg, R, seed, seeds, gains, stream, log):
    """Score the selected seeds: on the selection's own snapshots (the prefix
    increments must equal the gains) and on independent snapshots, R of them
    and 20,000 (the paper's simulation count), with the time of each."""
    import torch
    out = {}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ws = im.Workspace()
    for label, r, sd in (("same_snapshots", R, seed), ("independent", R, seed + 1000),
                         ("independent_20000", 20000, seed + 1000)):
        marg, per = im.spread(dg, r, sd, seeds, ws=ws, per_snapshot=True)   # warm-up, allocation
        torch.cuda.synchronize()
        ev0.record(stream)
        marg, per = im.spread(dg, r, sd, seeds, ws=ws, per_snapshot=True)
        ev1.record(stream)
        torch.cuda.synchronize()
        f = int(marg.sum().item())
        p = per.double()
        est, half = f / r, 1.96 * float(p.std()) / r ** 0.5 if r > 1 else 0.0
        out[label] = {"R": r, "seed": sd, "ms": round(ev0.elapsed_time(ev1), 3), "f": f,
                      "spread": round(est, 2), "ci95_half_width": round(half, 2)}
        log(f"spread {label}: R={r} {out[label]['ms']:.2f} ms, spread {est:.1f} +- {half:.1f}")
    out["same_snapshots"]["equals_gains"] = bool(
        im.spread(dg, R, seed, seeds, ws=ws)[0].cpu().tolist() == gains.cpu().tolist())
    ws.close()
    return out


def lazy_paths(im, dg, w, seeds, gains, ws, stream, steps, log):
    """Lazy exact evaluation, plain (bound order) vs learned (network order).
    For each, the lazy tuner first picks the evaluation engine and batch size
    (on the first rounds); then the whole selection is timed at that batch
    and at batches 1, 2, 4 and 16 (same engine)."""
    import torch
    from paper_1212_4779_amd.train_mlp import DEFAULT_OUT, load
    model = load(DEFAULT_OUT) if os.path.exists(DEFAULT_OUT) else None
    out = {"dynamic_update_ms": None, "plain": [], "learned": [], "learned_score_order": [],
           "tuned": {}}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for label, m, policy in (("plain", None, 2), ("learned", model, 2),
                             ("learned_score_order", model, 1)):
        if m is None and label != "plain":
            continue
        ws.set_learned_policy(policy)
        t = im.autotune_lazy(dg, w["R"], w["k"], w["seed"], model=m, ws=ws)
        out["tuned"][label] = t
        log(f"lazy tuner {label}: {t}")
        for B in (0, 1, 2, 4, 16):
            s, g = im.select_lazy(dg, w["R"], w["k"], w["seed"], batch=B, model=m, ws=ws)
            torch.cuda.synchronize()
            ev0.record(stream)
            for _ in range(steps):
                s, g = im.select_lazy(dg, w["R"], w["k"], w["seed"], batch=B, model=m, ws=ws)
            ev1.record(stream)
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1) / steps
            st = ws.stats()
            same = s.cpu().tolist() == seeds.cpu().tolist() and g.cpu().tolist() == gains.cpu().tolist()
            out[label].append({"batch": B if B else t["batch"], "tuned": B == 0, "engine": t["engine"],
                               "ms": round(ms, 3), "exact_evaluations": st["celf_evals"],
                               "batches": st["celf_batches"], "fallbacks": st["celf_fallbacks"],
                               "traversals": st["trav_init"] + st["trav_fwd"] + st["trav_eval"],
                               "same_output": same})
            log(f"lazy {label} B={B if B else t['batch']}{' (tuned)' if B == 0 else ''}: {ms:.2f} ms, "
                f"{st['celf_evals']} evaluations, same={same}")
    ws.set_learned_policy(2)
    for label in ("plain", "learned", "learned_score_order"):
        if out[label]:
            best = min(out[label], key=lambda r: r["ms"])
            out[f"{label}_best_ms"] = best["ms"]
            out[f"{label}_best_batch"] = best["batch"]
    return out


def run_batch(args, log):
    """512 uneven instances selected together (one block-diagonal graph)."""
    import numpy as np
    import torch

    import oracle
    import paper_1212_4779_amd as im
    from paper_1212_4779_amd import graphgen as gg

    rec = gg.batch_instances(**gg.BATCH_WORKLOAD)
    t0 = time.perf_counter()
    graphs = gg.graphs_from_recipes(rec, workers=min(16, os.cpu_count() or 1))
    log(f"batch: {len(graphs)} instances, n={sum(g.n for g in graphs)} "
        f"m={sum(g.m for g in graphs)} ({time.perf_counter() - t0:.1f}s)")
    dev = torch.device("cuda:0")
    insts = [(im.Graph.from_numpy(g.row_ptr, g.col, g.prob, device=dev), w["R"], w["k"], w["seed"])
             for g, w in zip(graphs, rec)]
    ws = im.Workspace()
    if args.once:
        # counter profiling: the autotuner's schedule for this batch, one
        # selection, then the calibration stream
        ws.set_tier2_lanes(64)
        ws.set_max_slots(8192)
        im.select_batch(insts, ws=ws)
        torch.cuda.synchronize()
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = src.mul(1.0)
        torch.cuda.synchronize()
        log(f"once: batched selection and a {4 * dst.numel()} B read+write stream done")
        return None
    # schedule: tuned on the largest instances of each probability model
    order = sorted(range(len(rec)), key=lambda i: -graphs[i].n)
    wc = [i for i in order if rec[i]["p"] is None][:6]
    uic = [i for i in order if rec[i]["p"] is not None][:6]
    t1 = time.perf_counter()
    tuning = im.autotune_batch([insts[i] for i in wc + uic], ws=ws)
    log(f"autotune on {len(wc + uic)} instances: {tuning} ({time.perf_counter() - t1:.1f}s)")
    for i in range(args.warmup):
        t1 = time.perf_counter()
        im.select_batch(insts, ws=ws)
        torch.cuda.synchronize()
        log(f"warmup {i}: {time.perf_counter() - t1:.2f}s")
    ws.profile_enable()
    res = im.select_batch(insts, ws=ws)
    prof = ws.profile()
    st = ws.stats()
    W = 4
    n_tot = sum(g.n for g in graphs)
    kb = kernel_bytes(st, n_tot, W)
    dom = max(PROPAGATION, key=lambda p: prof[p][0])
    log("phases (ms, launches): " + ", ".join(f"{p}={prof[p][0]:.3f}/{prof[p][1]}" for p in prof))
    ws.profile_enable([dom])
    stream = torch.cuda.current_stream(dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        res = im.select_batch(insts, ws=ws)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    dprof = ws.profile()[dom]
    st = ws.stats()
    trav = st["trav_init"] + st["trav_fwd"] + st["trav_rev"]
    launches = max(1, dprof[1] // args.steps)
    avg_ms = dprof[0] / max(1, dprof[1])
    bpl = kb[dom] / launches
    ach = bpl / (avg_ms / 1e3) / 1e9
    gold_path = os.path.join(ROOT, "tests", "golden", "batch512.json")
    parity, parity_n = None, 0
    if os.path.exists(gold_path):
        with open(gold_path) as f:
            gold = json.load(f)["instances"]
        parity = all(res[gi["i"]][0].cpu().tolist() == gi["seeds"] and
                     res[gi["i"]][1].cpu().tolist() == gi["gains"] for gi in gold)
        parity_n = len(gold)
    cpu = cpu_all = None
    if not args.no_cpu_baseline:
        # a sample stratified by size: every 16th instance in order of n
        by_n = sorted(range(len(rec)), key=lambda i: graphs[i].n)
        sample = by_n[8::16]
        oracle._load()
        t0 = time.perf_counter()
        tr, used = 0, []
        for i in sample:   # one thread, smallest first, about 20 s
            _, _, _, ost = oracle.select_du(graphs[i].row_ptr, graphs[i].col, graphs[i].prob,
                                            rec[i]["R"], rec[i]["k"], rec[i]["seed"])
            tr += ost["trav_init"] + ost["trav_fwd"] + ost["trav_rev"]
            used.append(i)
            if time.perf_counter() - t0 > 20:
                break
        dt = time.perf_counter() - t0
        cpu = {"value": tr / dt, "unit": "snapshot-edge traversals/s", "cores": 1, "kind": "oracle",
               "sample": f"{len(used)} instances (n {graphs[used[0]].n}..{graphs[used[-1]].n}) of a "
                         f"size-stratified sample (every 16th instance in order of n), "
                         f"StaticGreedyDU oracle, one thread",
               "seconds": round(dt, 3)}
        log(f"cpu oracle, one thread: {dt:.1f}s, {len(used)} instances")
        # all host cores: the 32 sampled instances in worker processes (fresh
        # interpreters; each regenerates its graph, untimed, and times the oracle)
        import multiprocessing as mp
        workers = min(16, os.cpu_count() or 1)
        t0 = time.perf_counter()
        with mp.get_context("forkserver").Pool(workers) as pool:
            res_cpu = pool.map(_oracle_on_recipe, [rec[i] for i in sample], chunksize=1)
        wall = time.perf_counter() - t0
        tr_all = sum(r[0] for r in res_cpu)
        busy = sum(r[1] for r in res_cpu)
        cpu_all = {"value": tr_all / wall, "unit": "snapshot-edge traversals/s", "cores": workers,
                   "kind": "oracle",
                   "sample": f"the {len(sample)} size-stratified instances, StaticGreedyDU oracle, "
                             f"one process per core ({workers}); wall time includes each worker's "
                             f"graph generation",
                   "seconds": round(wall, 3), "oracle_busy_seconds": round(busy, 3)}
        log(f"cpu oracle, {workers} processes: {wall:.1f}s wall, {busy:.1f}s busy")
    return {
        "metric": METRIC,
        "value": trav / (ms / 1e3), "unit": "snapshot-edge traversals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "batch512", "instances": len(graphs), "n_total": n_tot,
                   "m_total": sum(g.m for g in graphs), "R": "64/128/256", "k": 20,
                   "path": "dynamic update, batched"},
        "selection_ms": ms, "traversals_per_step": trav,
        "phase_ms": {p: round(prof[p][0], 4) for p in prof},
        "roofline": {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": load_traffic(dom, "batch512", tuning),
                     "kernel": KERNEL_NAMES[dom], "phase": dom,
                     "algorithmic_bytes_per_launch": int(bpl), "avg_launch_ms": round(avg_ms, 4)},
        "schedule": tuning,
        "cpu_baseline": cpu, "cpu_baseline_all_cores": cpu_all, "parity_vs_oracle_golden": parity,
        "parity_instances": parity_n,
    }


def _oracle_on_recipe(w):
    """(traversals, oracle seconds) of one batch instance (worker process)."""
    import oracle
    from paper_1212_4779_amd import graphgen as gg
    g = gg.graph_from_recipe(w)
    t0 = time.perf_counter()
    _, _, _, st = oracle.select_du(g.row_ptr, g.col, g.prob, w["R"], w["k"], w["seed"])
    return st["trav_init"] + st["trav_fwd"] + st["trav_rev"], time.perf_counter() - t0


UNDIRECTED = ("nethept_uic", "million_undirected_uic")
LINEAR_THRESHOLD = ("nethept_lt", "million_lt")


def run_lt(args, log):
    """Linear-threshold workload (live-edge snapshots): the dynamic update."""
    import numpy as np
    import torch

    import paper_1212_4779_amd as im
    from paper_1212_4779_amd import graphgen as gg

    w = gg.WORKLOADS[args.workload]
    g = gg.workload_graph(args.workload)
    dev = torch.device("cuda:0")
    dg = im.Graph.from_numpy(g.row_ptr, g.col, g.prob, device=dev)
    R, k, seed = w["R"], w["k"], w["seed"]
    W = (R + 63) // 64
    ws = im.Workspace()
    ws.set_live_edge(1)
    tuning = im.autotune(dg, R, seed, ws=ws)
    log(f"schedule: {tuning}")
    for _ in range(args.warmup):
        im.select(dg, R, k, seed, ws=ws)
    ws.profile_enable()
    seeds, gains, _ = im.select(dg, R, k, seed, ws=ws)
    prof = ws.profile()
    st = ws.stats()
    kb = kernel_bytes(st, g.n, W)
    dom = max(PROPAGATION, key=lambda p: prof[p][0])
    ws.profile_enable([dom])
    stream = torch.cuda.current_stream(dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        seeds, gains, _ = im.select(dg, R, k, seed, ws=ws)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    dprof = ws.profile()[dom]
    st = ws.stats()
    trav = st["trav_init"] + st["trav_fwd"] + st["trav_rev"]
    avg_ms = dprof[0] / max(1, dprof[1])
    bpl = kb[dom] / max(1, dprof[1] // args.steps)
    ach = bpl / (avg_ms / 1e3) / 1e9
    log(f"linear threshold: {ms:.2f} ms per selection")
    gold_path = os.path.join(ROOT, "tests", "golden", f"{args.workload}.json")
    parity = None
    if os.path.exists(gold_path):
        with open(gold_path) as f:
            gold = json.load(f)
        parity = (seeds.cpu().tolist() == gold["seeds"] and gains.cpu().tolist() == gold["gains"])
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle._load()
        t0 = time.perf_counter()
        cs, cg, _ = oracle.select_du_lt(g.row_ptr, g.col, g.prob, R, k, seed)
        dt = time.perf_counter() - t0
        cpu = {"value": 1.0 / dt, "unit": "selections/s", "cores": 1, "kind": "oracle",
               "sample": f"whole workload (R={R}, k={k}), linear-threshold StaticGreedyDU oracle, one thread",
               "seconds": round(dt, 3),
               "same_seeds_as_gpu": bool(np.array_equal(cs.astype(np.int64), seeds.cpu().numpy()))}
        log(f"cpu oracle: {dt:.2f}s")
    return {
        "metric": "k-seed selection wall time + snapshot-edge traversals/s, linear threshold",
        "value": trav / (ms / 1e3), "unit": "snapshot-edge traversals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": args.workload, "n": g.n, "m": g.m, "R": R, "k": k,
                   "weights": "1/indeg(v)", "model": "linear threshold (live-edge)",
                   "path": "dynamic update"},
        "selection_ms": ms, "traversals_per_step": trav,
        "phase_ms": {p: round(prof[p][0], 4) for p in prof},
        "roofline": {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": KERNEL_NAMES[dom], "phase": dom,
                     "algorithmic_bytes_per_launch": int(bpl), "avg_launch_ms": round(avg_ms, 4)},
        "schedule": tuning, "cpu_baseline": cpu, "parity_vs_oracle_golden": parity,
    }


def run_undirected(args, log):
    """Undirected workload, one coin per pair: the component method."""
    import numpy as np
    import torch

    import paper_1212_4779_amd as im
    from paper_1212_4779_amd import graphgen as gg

    w = gg.WORKLOADS[args.workload]
    g = gg.workload_graph(args.workload)
    dev = torch.device("cuda:0")
    dg = im.Graph.from_numpy(g.row_ptr, g.col, g.prob, device=dev)
    R, k, seed = w["R"], w["k"], w["seed"]
    ws = im.Workspace()
    for _ in range(args.warmup):
        im.select_undirected(dg, R, k, seed, ws=ws)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        seeds, gains, _ = im.select_undirected(dg, R, k, seed, ws=ws)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    log(f"component method: {ms:.2f} ms per selection")
    # the directed engines on the same pair-coin snapshots (small graphs only)
    directed_ms = None
    if g.n <= 100000:
        ws2 = im.Workspace()
        ws2.set_pair_coins(True)
        s2, g2, _ = im.select(dg, R, k, seed, ws=ws2)
        torch.cuda.synchronize()
        ev0.record(stream)
        s2, g2, _ = im.select(dg, R, k, seed, ws=ws2)
        ev1.record(stream)
        torch.cuda.synchronize()
        directed_ms = round(ev0.elapsed_time(ev1), 3)
        assert s2.cpu().tolist() == seeds.cpu().tolist()
        log(f"directed engines, pair coins: {directed_ms:.2f} ms")
    gold_path = os.path.join(ROOT, "tests", "golden", f"{args.workload}.json")
    parity = None
    if os.path.exists(gold_path):
        with open(gold_path) as f:
            gold = json.load(f)
        parity = (seeds.cpu().tolist() == gold["seeds"] and gains.cpu().tolist() == gold["gains"])
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle._load()
        t0 = time.perf_counter()
        cs, cg, _ = oracle.select_components(g.row_ptr, g.col, g.prob, R, k, seed)
        dt = time.perf_counter() - t0
        cpu = {"value": 1.0 / dt, "unit": "selections/s", "cores": 1, "kind": "oracle",
               "sample": f"whole workload (R={R}, k={k}), component-method oracle, one thread",
               "seconds": round(dt, 3),
               "same_seeds_as_gpu": bool(np.array_equal(cs.astype(np.int64), seeds.cpu().numpy()))}
        log(f"cpu oracle: {dt:.2f}s")
    return {
        "metric": "k-seed selection wall time, undirected graph, component method",
        "value": 1e3 / ms, "unit": "selections/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": args.workload, "n": g.n, "m": g.m, "R": R, "k": k, "p": w["p"],
                   "gamma": w["gamma"], "directed": False, "coins": "one per undirected pair",
                   "path": "component method"},
        "directed_engines_pair_coins_ms": directed_ms,
        "cpu_baseline": cpu, "parity_vs_oracle_golden": parity,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="million_uic")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--schedule", default=None,
                    help="hub,tier1,lanes,slots,coop[,fwd_groups[,rev_split[,rev_first_tier]]]: use this "
                         "engine schedule instead of autotuning")
    ap.add_argument("--once", action="store_true",
                    help="one selection and one 1 GiB read + 1 GiB write stream (counter profiling)")
    args = ap.parse_args()

    def log(msg):
        if not args.quiet:
            print(msg, file=sys.stderr, flush=True)

    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(snapshot words would shard over GPUs with one gain reduction per round; not implemented)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch512":
        res = run_batch(args, log)
        if res is not None:
            print(json.dumps(res), flush=True)
        return
    if args.workload in UNDIRECTED:
        print(json.dumps(run_undirected(args, log)), flush=True)
        return
    if args.workload in LINEAR_THRESHOLD:
        print(json.dumps(run_lt(args, log)), flush=True)
        return

    import numpy as np
    import torch

    import paper_1212_4779_amd as im
    from paper_1212_4779_amd import graphgen as gg

    w = gg.WORKLOADS[args.workload]
    t0 = time.perf_counter()
    g = gg.workload_graph(args.workload)
    log(f"graph {args.workload}: n={g.n} m={g.m} ({time.perf_counter() - t0:.1f}s)")
    dev = torch.device("cuda:0")
    dg = im.Graph.from_numpy(g.row_ptr, g.col, g.prob, device=dev)
    R, k, seed = w["R"], w["k"], w["seed"]
    W = (R + 63) // 64
    ws = im.Workspace()
    if args.schedule:
        vals = [int(x) for x in args.schedule.split(",")]
        hub, t1, lanes, slots, coop = vals[:5]
        fwd = vals[5] if len(vals) > 5 else 16
        rev = vals[6] if len(vals) > 6 else 1
        first = vals[7] if len(vals) > 7 else 0
        ws.set_forward_groups(fwd)
        ws.set_rev_split(rev)
        ws.set_rev_first_tier(first)
        ws.set_hub_degree(hub)
        ws.set_tier1_shape(t1)
        ws.set_tier2_lanes(lanes)
        ws.set_max_slots(slots)
        ws.set_coop_gain(0 if coop else (1 << 62))
        tuning = {"hub_degree": hub, "tier1_shape": t1, "tier2_lanes": lanes, "max_slots": slots,
                  "coop_forward": coop, "fwd_groups": fwd, "rev_split": rev, "rev_first_tier": first,
                  "tried": 0}
    else:
        tuning = im.autotune(dg, R, seed, ws=ws)
    log(f"schedule: {tuning}")
    if args.once:
        im.select(dg, R, k, seed, ws=ws)
        torch.cuda.synchronize()
        # calibration for the HBM byte counters: a streaming kernel that reads
        # 1 GiB and writes 1 GiB (elementwise multiply of 2^28 floats)
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = src.mul(1.0)
        torch.cuda.synchronize()
        log(f"once: selection and a {4 * dst.numel()} B read+write stream done")
        return

    for _ in range(args.warmup):
        im.select(dg, R, k, seed, ws=ws)
    torch.cuda.synchronize()

    # one profiled call (all phases) to find the dominant propagation kernel
    ws.profile_enable()
    seeds, gains, _ = im.select(dg, R, k, seed, ws=ws)
    prof = ws.profile()
    st = ws.stats()
    kb = kernel_bytes(st, g.n, W)
    dom = max(PROPAGATION, key=lambda p: prof[p][0])
    log("phases (ms, launches): " + ", ".join(f"{p}={prof[p][0]:.3f}/{prof[p][1]}" for p in prof))

    # timed region: only the dominant kernel is bracketed by events
    ws.profile_enable([dom])
    stream = torch.cuda.current_stream(dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        seeds, gains, _ = im.select(dg, R, k, seed, ws=ws)
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    ms_per_step = total_ms / args.steps
    log(f"dynamic update: {ms_per_step:.2f} ms per selection")
    dprof = ws.profile()[dom]
    st = ws.stats()
    trav = st["trav_init"] + st["trav_fwd"] + st["trav_rev"]
    value = trav / (ms_per_step / 1e3)
    launches_per_step = max(1, dprof[1] // args.steps)
    avg_launch_ms = dprof[0] / max(1, dprof[1])
    bytes_per_launch = kb[dom] / launches_per_step
    achieved = bytes_per_launch / (avg_launch_ms / 1e3) / 1e9
    # every propagation phase of the profiled call against the same peak
    per_kernel = {}
    for ph in PROPAGATION:
        tms, nl = prof[ph]
        if nl == 0 or tms <= 0:
            continue
        a_gbs = kb[ph] / (tms / 1e3) / 1e9
        per_kernel[ph] = {"kernel": KERNEL_NAMES[ph], "launches": nl, "ms": round(tms, 4),
                          "algorithmic_bytes_per_launch": int(kb[ph] / nl),
                          "achieved": round(a_gbs, 2), "frac": round(a_gbs / HBM_PEAK_GBS, 5),
                          "traffic": load_traffic(ph, args.workload, tuning)}
    traffic = load_traffic(dom, args.workload, tuning)
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": KERNEL_NAMES[dom], "phase": dom,
                "algorithmic_bytes_per_launch": int(bytes_per_launch),
                "avg_launch_ms": round(avg_launch_ms, 4)}

    # the same selection captured into one HIP graph (device-resident round loop)
    plan = im.Plan(dg, R, k, seed)
    plan.launch()
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        plan.launch()
    ev1.record(stream)
    torch.cuda.synchronize()
    graph_ms = ev0.elapsed_time(ev1) / args.steps
    graph_same = (plan.seeds.cpu().tolist() == seeds.cpu().tolist() and
                  plan.gains.cpu().tolist() == gains.cpu().tolist())
    plan.close()

    lazy = lazy_paths(im, dg, w, seeds, gains, ws, stream, max(1, min(args.steps, 3)), log)
    lazy["dynamic_update_ms"] = round(ms_per_step, 3)
    if "learned_best_ms" in lazy:
        lazy["learned_faster_than_dynamic_update"] = lazy["learned_best_ms"] < lazy["dynamic_update_ms"]
        lazy["learned_faster_than_plain_lazy"] = lazy["learned_best_ms"] < lazy["plain_best_ms"]
        lazy["all_same_output"] = all(r["same_output"] for lab in ("plain", "learned", "learned_score_order")
                                      for r in lazy[lab])
    spread_eval = spread_leg(im, dg, R, seed, seeds, gains, stream, log)

    gold_path = os.path.join(ROOT, "tests", "golden", f"{args.workload}.json")
    parity = None
    if os.path.exists(gold_path):
        with open(gold_path) as f:
            gold = json.load(f)
        parity = (seeds.cpu().tolist() == gold["seeds"] and gains.cpu().tolist() == gold["gains"])

    cpu = None
    if not args.no_cpu_baseline:
        cpu, cs, cgains = cpu_baseline(g, w, log)
        ok = np.array_equal(cs.astype(np.int64), seeds.cpu().numpy())
        cpu["same_seeds_as_gpu"] = bool(ok)

    out = {
        "metric": METRIC,
        "value": value, "unit": "snapshot-edge traversals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": g.n, "m": g.m, "R": R, "k": k,
                   "p": w["p"] if w["p"] is not None else "weighted cascade",
                   "gamma": w["gamma"], "directed": w["directed"], "path": "dynamic update"},
        "selection_ms": ms_per_step,
        "graph_replay_ms": graph_ms,
        "graph_replay_same_output": graph_same,
        "traversals_per_step": trav,
        "phase_ms": {p: round(prof[p][0], 4) for p in prof},
        "counters": st,
        "schedule": tuning,
        "roofline": roofline,
        "roofline_kernels": per_kernel,
        "learned_vs_plain": lazy,
        "spread_eval": spread_eval,
        "cpu_baseline": cpu,
        "parity_vs_oracle_golden": parity,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
