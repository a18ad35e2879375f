"""Schedules never change results: every engine option combination and the
autotuner's choice give the oracle's full per-round gain trace."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1212_4779_amd import graphgen as gg

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

SCHEDULES = [  # (hub degree, tier-1 shape, tier-2 lanes, tier-2 slots)
    (256, 0, 256, 256), (256, 1, 1024, 256), (256, 2, 256, 2048),
    (1024, 0, 256, 8), (0, 1, 1024, 8), (16, 2, 1024, 64),
    (256, 0, 64, 8192), (16, 1, 64, 8),
]


@pytest.fixture(scope="module")
def im():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1212_4779_amd as im
    return im


def _dev(im, g):
    return im.Graph.from_numpy(g.row_ptr, g.col, g.prob, device="cuda:0")


def _cases():
    return [
        ("nethept_wc", gg.workload_graph("nethept_wc"), 100, 50, 1),
        ("dense_p30", gg.chung_lu_graph(3000, 24000, 2.3, 7, True, 0.3), 130, 12, 5),
        ("wc_directed", gg.chung_lu_graph(20000, 160000, 2.3, 11, True, None), 256, 10, 2),
    ]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_every_schedule_gives_the_oracle_trace(im, case):
    _, g, R, k, seed = case
    s_ref, g_ref, tr_ref, _ = oracle.select_du(g.row_ptr, g.col, g.prob, R, k, seed, trace=True)
    d = _dev(im, g)
    for hub, t1, lanes, slots in SCHEDULES:
        ws = im.Workspace()
        ws.set_hub_degree(hub)
        ws.set_tier1_shape(t1)
        ws.set_tier2_lanes(lanes)
        ws.set_max_slots(slots)
        seeds, gains, tr = im.select(d, R, k, seed, ws=ws, trace=True)
        assert seeds.cpu().tolist() == s_ref.tolist(), (hub, t1, lanes, slots)
        assert gains.cpu().tolist() == g_ref.tolist()
        assert np.array_equal(tr.cpu().numpy().astype(np.uint32), tr_ref)


def test_autotune_choice_and_cache(im):
    with open(os.path.join(GOLDEN, "nethept_wc.json")) as f:
        gold = json.load(f)
    w = gg.WORKLOADS["nethept_wc"]
    g = gg.workload_graph("nethept_wc")
    d = _dev(im, g)
    ws = im.Workspace()
    t = im.autotune(d, w["R"], w["seed"], ws=ws)
    assert t["tried"] >= 2 and t["ms"] > 0
    assert t["tier1_shape"] in (0, 1, 2) and t["tier2_lanes"] in (64, 256, 1024)
    seeds, gains, _ = im.select(d, w["R"], w["k"], w["seed"], ws=ws)
    assert seeds.cpu().tolist() == gold["seeds"]
    assert gains.cpu().tolist() == gold["gains"]
    ws2 = im.Workspace()
    t2 = im.autotune(d, w["R"], w["seed"], ws=ws2)
    assert t2["tried"] == 0
    keys = ("hub_degree", "tier1_shape", "tier2_lanes", "max_slots", "coop_forward")
    assert {k: t2[k] for k in keys} == {k: t[k] for k in keys}


def test_autotune_batch_then_select_batch(im):
    rng = np.random.default_rng(3)
    graphs, insts, refs = [], [], []
    for i in range(6):
        n = int(rng.integers(300, 3000))
        g = gg.chung_lu_graph(n, n * 6, 2.5, 100 + i, True, None if i % 2 else 0.05)
        R, k = int(rng.choice([64, 100, 256])), 5
        graphs.append(g)
        insts.append((_dev(im, g), R, k, 1 + i))
        s, gn, _, _ = oracle.select_du(g.row_ptr, g.col, g.prob, R, k, 1 + i)
        refs.append((s.tolist(), gn.tolist()))
    ws = im.Workspace()
    t = im.autotune_batch(insts, ws=ws)
    assert t["tried"] >= 2
    out = im.select_batch(insts, ws=ws)
    for (s, gn), (rs, rg) in zip(out, refs):
        assert s.cpu().tolist() == rs and gn.cpu().tolist() == rg


def test_batch_plan_replays(im):
    # the batched selection captured into one HIP graph: every replay, with
    # eager work and synchronisations in between, equals the oracle
    import torch
    rng = np.random.default_rng(5)
    insts, refs = [], []
    for i in range(5):
        n = int(rng.integers(200, 2500))
        g = gg.chung_lu_graph(n, n * 5, 2.5, 200 + i, True, None if i % 2 else 0.05)
        R, k = int(rng.choice([64, 100, 200])), 4 + i
        insts.append((_dev(im, g), R, k, 7 + i))
        s, gn, _, _ = oracle.select_du(g.row_ptr, g.col, g.prob, R, k, 7 + i)
        refs.append((s.tolist(), gn.tolist()))
    ws = im.Workspace()
    im.autotune_batch(insts, ws=ws)
    plan = im.BatchPlan(insts, tuned=ws)
    for rep in range(3):
        plan.launch()
        torch.cuda.synchronize()
        for (s, gn), (rs, rg) in zip(plan.results(), refs):
            assert s.cpu().tolist() == rs and gn.cpu().tolist() == rg, rep
        im.select_batch(insts, ws=ws)   # eager work between replays
        torch.cuda.synchronize()
    assert plan.stats()["trav_init"] > 0
    plan.close()


@pytest.mark.parametrize("name", ["tiny_uic", "nethept_wc"])
def test_lazy_autotune_then_select(im, name):
    # the lazy tuner's engine and batch size, and every pair it tries, give
    # the oracle's seeds and gains
    from paper_1212_4779_amd.train_mlp import load
    with open(os.path.join(GOLDEN, f"{name}.json")) as f:
        gold = json.load(f)
    w = gg.WORKLOADS[name]
    d = _dev(im, gg.workload_graph(name))
    for model in (None, load()):
        ws = im.Workspace()
        t = im.autotune_lazy(d, w["R"], w["k"], w["seed"], model=model, ws=ws)
        assert t["tried"] == 10 and t["ms"] > 0
        assert t["engine"] in (0, 2) and t["batch"] in (1, 2, 4, 8, 16)
        seeds, gains = im.select_lazy(d, w["R"], w["k"], w["seed"], batch=0, model=model, ws=ws)
        assert seeds.cpu().tolist() == gold["seeds"] and gains.cpu().tolist() == gold["gains"]
        st = ws.stats()
        assert st["celf_batches"] >= w["k"] - 1
        for engine in (0, 2):
            for batch in (1, 2, 4, 8, 16):
                ws.set_lazy_engine(engine)
                ws.set_lazy_batch(batch)
                seeds, gains = im.select_lazy(d, w["R"], w["k"], w["seed"], batch=0, model=model,
                                              ws=ws)
                assert seeds.cpu().tolist() == gold["seeds"], (engine, batch)
                assert gains.cpu().tolist() == gold["gains"], (engine, batch)


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_affected_set_recompute_gives_the_oracle_trace(im, case):
    # the other per-round update (recompute the gains of the nodes that reach
    # a newly covered node) in every round, and from a middle gain on (mixed
    # rounds), gives the same gain vector as reverse decrements in every round
    _, g, R, k, seed = case
    s_ref, g_ref, tr_ref, _ = oracle.select_du(g.row_ptr, g.col, g.prob, R, k, seed, trace=True)
    d = _dev(im, g)
    mid = int(g_ref[len(g_ref) // 2]) + 1
    for thr in (1 << 62, mid):
        for hub, t1, lanes, slots in (SCHEDULES[0], SCHEDULES[5], SCHEDULES[6]):
            ws = im.Workspace()
            ws.set_hub_degree(hub)
            ws.set_tier1_shape(t1)
            ws.set_tier2_lanes(lanes)
            ws.set_max_slots(slots)
            ws.set_affected_gain(thr)
            seeds, gains, tr = im.select(d, R, k, seed, ws=ws, trace=True)
            assert seeds.cpu().tolist() == s_ref.tolist(), (thr, hub, t1, lanes, slots)
            assert gains.cpu().tolist() == g_ref.tolist()
            assert np.array_equal(tr.cpu().numpy().astype(np.uint32), tr_ref), (thr, hub)
            st = ws.stats()
            if thr == 1 << 62:
                assert st["trav_rev"] == 0 and st["trav_eval"] > 0


def test_affected_set_recompute_in_a_plan_and_the_tuner(im):
    import torch
    with open(os.path.join(GOLDEN, "nethept_wc.json")) as f:
        gold = json.load(f)
    w = gg.WORKLOADS["nethept_wc"]
    d = _dev(im, gg.workload_graph("nethept_wc"))
    t = im.autotune(d, w["R"], w["seed"], ws=im.Workspace())
    assert t["affected_gain"] in (0, d.n * w["R"] // 4096, d.n * w["R"] // 256, 1 << 62)
    ws = im.Workspace()
    ws.set_affected_gain(1 << 62)
    seeds, gains, _ = im.select(d, w["R"], w["k"], w["seed"], ws=ws)
    assert seeds.cpu().tolist() == gold["seeds"] and gains.cpu().tolist() == gold["gains"]
    # a plan captured after the tuner chose a strategy for this graph uses it
    plan = im.Plan(d, w["R"], w["k"], w["seed"])
    for _ in range(2):
        plan.launch()
        torch.cuda.synchronize()
        assert plan.seeds.cpu().tolist() == gold["seeds"]
        assert plan.gains.cpu().tolist() == gold["gains"]
    plan.close()


def test_autotune_choice_persists_in_the_cache_file(im, tmp_path):
    # IM_TUNE_CACHE: the first process tunes and appends its choice; a second
    # process finds it in the file and applies it without timing
    import subprocess
    import sys
    cache = tmp_path / "tune.txt"
    env = dict(os.environ, IM_TUNE_CACHE=str(cache))
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import json, sys; sys.path.insert(0, %r)\n"
            "import paper_1212_4779_amd as im\n"
            "from paper_1212_4779_amd import graphgen as gg\n"
            "g = gg.workload_graph('tiny_uic')\n"
            "d = im.Graph.from_numpy(g.row_ptr, g.col, g.prob, device='cuda:0')\n"
            "t = im.autotune(d, 64, 1)\n"
            "s, gn, _ = im.select(d, 64, 10, 1)\n"
            "print(json.dumps([t, s.cpu().tolist()]))\n" % root)
    outs = []
    for _ in range(2):
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           timeout=240)
        assert r.returncode == 0, r.stderr[-2000:]
        outs.append(json.loads(r.stdout.strip().splitlines()[-1]))
    (t1, s1), (t2, s2) = outs
    assert t1["tried"] > 0 and t2["tried"] == 0
    keys = ("hub_degree", "tier1_shape", "tier2_lanes", "max_slots", "coop_forward", "affected_gain",
            "fwd_groups", "rev_split", "rev_first_tier")
    assert {k: t1[k] for k in keys} == {k: t2[k] for k in keys}
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("im-tune-4 2000 20000 64 ")
    with open(os.path.join(GOLDEN, "tiny_uic.json")) as f:
        assert s1 == s2 == json.load(f)["seeds"]


def test_second_process_selects_with_every_round_cooperative(im, tmp_path):
    # a process started while this one holds the device: when its cooperative
    # launches are refused, a single graph's rounds run in the per-word
    # workgroups instead and the seeds are unchanged; a batch either runs or
    # reports an error that names the cooperative launch
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import json, sys; sys.path.insert(0, %r)\n"
            "import paper_1212_4779_amd as im\n"
            "from paper_1212_4779_amd import graphgen as gg\n"
            "g = gg.workload_graph('tiny_uic')\n"
            "d = im.Graph.from_numpy(g.row_ptr, g.col, g.prob, device='cuda:0')\n"
            "out = {}\n"
            "for gain in (0, 64, 2**63 - 1):\n"
            "    ws = im.Workspace()\n"
            "    ws.set_coop_gain(gain)\n"
            "    s, gn, _ = im.select(d, 64, 10, 1, ws=ws)\n"
            "    out[str(gain)] = [s.cpu().tolist(), gn.cpu().tolist()]\n"
            "try:\n"
            "    b = im.select_batch([(d, 64, 10, 1), (d, 64, 10, 1)])\n"
            "    out['batch'] = [[s.cpu().tolist(), gn.cpu().tolist()] for s, gn in b]\n"
            "except im.ImError as e:\n"
            "    out['batch_error'] = str(e)\n"
            "print(json.dumps(out))\n" % root)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    out = json.loads(r.stdout.strip().splitlines()[-1])
    with open(os.path.join(GOLDEN, "tiny_uic.json")) as f:
        gold = json.load(f)
    for gain in ("0", "64", str(2**63 - 1)):
        assert out[gain] == [gold["seeds"], gold["gains"]], gain
    if "batch" in out:
        assert out["batch"] == [[gold["seeds"], gold["gains"]]] * 2
    else:
        assert "k_forward_coop" in out["batch_error"]
