"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

All integer results must be bit-identical: snapshot masks, the reverse CSR
(up to the order inside a row, which the ABI leaves unspecified), initial
gains, every round's full gain vector, seeds, gains and the work counters.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from paper_1212_4779_amd import graphgen as gg

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def im():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1212_4779_amd as im
    return im


def _dev(im, g):
    return im.Graph.from_numpy(g.row_ptr, g.col, g.prob, device="cuda:0")


def _csr(n, arcs, p):
    arcs = sorted(arcs)
    row_ptr = np.zeros(n + 1, np.uint64)
    for u, _ in arcs:
        row_ptr[u + 1] += 1
    row_ptr = np.cumsum(row_ptr).astype(np.uint64)
    col = np.array([v for _, v in arcs], np.uint32)
    prob = np.array(p if np.ndim(p) else [p] * len(arcs), np.float32)
    return gg.Graph(n, row_ptr, col, prob)


def _cases():
    """(name, graph, R, k, seed): small cases spanning several tiles and ragged tails."""
    out = []
    out.append(("tiny_uic", gg.workload_graph("tiny_uic"), 64, 10, 1))
    out.append(("nethept_wc", gg.workload_graph("nethept_wc"), 100, 50, 1))
    # denser and supercritical graphs: large reach sets exercise the block engine
    out.append(("dense_p30", gg.chung_lu_graph(3000, 24000, 2.3, 7, True, 0.3), 130, 12, 5))
    out.append(("undirected_wc_R300", gg.chung_lu_graph(5000, 30000, 2.2, 8, False, None), 300, 20, 9))
    out.append(("directed_wc_R1", gg.chung_lu_graph(4000, 40000, 2.1, 9, True, None), 1, 15, 3))
    out.append(("p1_chain", _csr(300, [(i, i + 1) for i in range(299)], 1.0), 65, 4, 2))
    out.append(("hub_star", _csr(3000, [(0, i) for i in range(1, 3000)] +
                                 [(i, (i * 7) % 2999 + 1) for i in range(1, 3000)
                                  if (i * 7) % 2999 + 1 != i], 0.2), 70, 6, 4))
    return out


CASES = _cases()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_masks_bit_exact(im, case):
    _, g, R, _, seed = case
    d = _dev(im, g)
    got = im.snapshot_masks(d, R, seed).cpu().numpy().view(np.uint64)
    ref = oracle.live_bits(g.prob, R, seed)              # arc-major [m, W]
    assert got.shape == (ref.shape[1], ref.shape[0])
    assert np.array_equal(got.T, ref)


@pytest.mark.parametrize("case", CASES[:4], ids=[c[0] for c in CASES[:4]])
def test_transpose(im, case):
    _, g, _, _, _ = case
    d = _dev(im, g)
    in_row, in_col, in2out = (t.cpu().numpy().view(np.uint32) for t in im.transpose(d))
    n, m = g.n, g.m
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.row_ptr.astype(np.int64)))
    expect_row = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(g.col.astype(np.int64), minlength=n), out=expect_row[1:])
    assert np.array_equal(in_row.astype(np.int64), expect_row)
    # as multisets per row: (tail, arc id) pairs
    assert np.array_equal(g.col[in2out.astype(np.int64)], np.repeat(np.arange(n), np.diff(expect_row)))
    assert np.array_equal(src[in2out.astype(np.int64)], in_col.astype(np.int64))
    assert np.array_equal(np.sort(in2out), np.arange(m, dtype=np.uint32))


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_initial_gains_and_counters(im, case):
    _, g, R, _, seed = case
    d = _dev(im, g)
    ws = im.Workspace()
    got = im.initial_gains(d, R, seed, ws=ws).cpu().numpy()
    ref, st = oracle.initial_gains(g.row_ptr, g.col, g.prob, R, seed)
    assert np.array_equal(got, ref.astype(np.int64))
    gs = ws.stats()
    assert gs["trav_init"] == st["trav_init"]
    assert gs["relax_init"] == st["word_reach_deg"]
    assert gs["reached_init"] == st["word_reach_nodes"]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_select_full_trace(im, case):
    _, g, R, k, seed = case
    d = _dev(im, g)
    ws = im.Workspace()
    seeds, gains, tr = im.select(d, R, k, seed, ws=ws, trace=True)
    s_ref, g_ref, tr_ref, st = oracle.select_du(g.row_ptr, g.col, g.prob, R, k, seed, trace=True)
    tr = tr.cpu().numpy()
    for t in range(k + 1):
        assert np.array_equal(tr[t], tr_ref[t].astype(np.int64)), f"gain vector differs in round {t}"
    assert np.array_equal(seeds.cpu().numpy(), s_ref.astype(np.int64))
    assert np.array_equal(gains.cpu().numpy(), g_ref.astype(np.int64))
    gs = ws.stats()
    for a, b in (("trav_init", "trav_init"), ("trav_fwd", "trav_fwd"), ("trav_rev", "trav_rev"),
                 ("decrements", "decrements")):
        assert gs[a] == st[b], a
    assert gs["barrier_failures"] == 0


@pytest.mark.parametrize("case", [CASES[0], CASES[2], CASES[6]], ids=["tiny_uic", "dense_p30", "hub_star"])
def test_schedule_invariance_hub_lists(im, case):
    # the heavy-node threshold only changes how nodes are expanded, never results
    _, g, R, k, seed = case
    d = _dev(im, g)
    ref = None
    for deg in (0, 16, 64, 256, 1 << 20):
        ws = im.Workspace()
        ws.set_hub_degree(deg)
        seeds, gains, tr = im.select(d, R, k, seed, ws=ws, trace=True)
        got = (seeds.cpu().numpy(), gains.cpu().numpy(), tr.cpu().numpy(), ws.stats())
        if ref is None:
            ref = got
            s_ref, g_ref, _, _ = oracle.select_du(g.row_ptr, g.col, g.prob, R, k, seed)
            assert np.array_equal(got[0], s_ref.astype(np.int64))
            continue
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
        assert np.array_equal(got[2], ref[2])
        # relax_rev counts word-level work of packed task groups: schedule dependent
        for key in ("trav_init", "trav_fwd", "trav_rev", "decrements", "relax_init"):
            assert got[3][key] == ref[3][key], (deg, key)


@pytest.mark.parametrize("case", [CASES[1], CASES[2], CASES[6]], ids=["nethept_wc", "dense_p30", "hub_star"])
def test_schedule_invariance_forward(im, case):
    # grid-wide or per-word forward search: identical results
    _, g, R, k, seed = case
    d = _dev(im, g)
    outs = []
    for gain in (0, 1 << 62, 2000):
        ws = im.Workspace()
        ws.set_coop_gain(gain)
        seeds, gains, tr = im.select(d, R, k, seed, ws=ws, trace=True)
        outs.append((seeds.cpu().numpy(), gains.cpu().numpy(), tr.cpu().numpy(), ws.stats()))
    s_ref, g_ref, _, st = oracle.select_du(g.row_ptr, g.col, g.prob, R, k, seed)
    for o in outs:
        assert np.array_equal(o[0], s_ref.astype(np.int64))
        assert np.array_equal(o[1], g_ref.astype(np.int64))
        assert np.array_equal(o[2], outs[0][2])
        assert o[3]["trav_fwd"] == st["trav_fwd"]
        assert o[3]["barrier_failures"] == 0


@pytest.mark.parametrize("case", [CASES[1], CASES[2], CASES[6]], ids=["nethept_wc", "dense_p30", "hub_star"])
def test_schedule_invariance_reverse_split(im, case):
    # last-tier reverse tasks split into 1, 2 or 4 bit groups: identical
    # gain vectors in every round
    _, g, R, k, seed = case
    d = _dev(im, g)
    s_ref, g_ref, tr_ref, st = oracle.select_du(g.row_ptr, g.col, g.prob, R, k, seed, trace=True)
    for split in (1, 2, 4):
        ws = im.Workspace()
        ws.set_rev_split(split)
        ws.set_tier2_lanes(64)
        seeds, gains, tr = im.select(d, R, k, seed, ws=ws, trace=True)
        assert np.array_equal(seeds.cpu().numpy(), s_ref.astype(np.int64)), split
        assert np.array_equal(gains.cpu().numpy(), g_ref.astype(np.int64)), split
        tr = tr.cpu().numpy()
        for t in range(k + 1):
            assert np.array_equal(tr[t], tr_ref[t].astype(np.int64)), (split, t)
        gs = ws.stats()
        assert gs["trav_rev"] == st["trav_rev"] and gs["decrements"] == st["decrements"], split
        reached_t2 = gs["reached_rev_t2"]
        ws.close()
    if case[0] == "dense_p30":
        assert reached_t2 > 0   # the last tier did run reverse tasks
    with pytest.raises(im.ImError):
        im.Workspace().set_rev_split(3)


@pytest.mark.parametrize("case", [CASES[1], CASES[2], CASES[6]], ids=["nethept_wc", "dense_p30", "hub_star"])
def test_schedule_invariance_reverse_first_tier(im, case):
    # reverse tasks starting on tier 0 or on tier 1 (no tier-0 launch):
    # identical gain vectors in every round, and the same decrements
    _, g, R, k, seed = case
    d = _dev(im, g)
    s_ref, g_ref, tr_ref, st = oracle.select_du(g.row_ptr, g.col, g.prob, R, k, seed, trace=True)
    for first in (0, 1):
        ws = im.Workspace()
        ws.set_rev_first_tier(first)
        ws.profile_enable(["rev_t0", "rev_t1"])
        seeds, gains, tr = im.select(d, R, k, seed, ws=ws, trace=True)
        assert np.array_equal(seeds.cpu().numpy(), s_ref.astype(np.int64)), first
        assert np.array_equal(gains.cpu().numpy(), g_ref.astype(np.int64)), first
        tr = tr.cpu().numpy()
        for t in range(k + 1):
            assert np.array_equal(tr[t], tr_ref[t].astype(np.int64)), (first, t)
        gs = ws.stats()
        assert gs["trav_rev"] == st["trav_rev"] and gs["decrements"] == st["decrements"], first
        prof = ws.profile()
        if first == 1:
            assert prof["rev_t0"][1] == 0 and gs["reached_rev_t0"] == 0   # no tier-0 launch
            assert prof["rev_t1"][1] > 0
        ws.close()
    with pytest.raises(im.ImError):
        im.Workspace().set_rev_first_tier(2)


def test_repeat_and_workspace_reuse(im):
    g1 = gg.workload_graph("nethept_wc")
    g2 = gg.workload_graph("tiny_uic")
    ws = im.Workspace()
    d1, d2 = _dev(im, g1), _dev(im, g2)
    a = im.select(d1, 100, 50, 1, ws=ws)
    b = im.select(d2, 64, 10, 1, ws=ws)
    c = im.select(d1, 100, 50, 1, ws=ws)
    assert np.array_equal(a[0].cpu().numpy(), c[0].cpu().numpy())
    assert np.array_equal(a[1].cpu().numpy(), c[1].cpu().numpy())
    s_ref, g_ref, _, _ = oracle.select_du(g2.row_ptr, g2.col, g2.prob, 64, 10, 1)
    assert np.array_equal(b[0].cpu().numpy(), s_ref.astype(np.int64))


def test_edge_cases(im):
    # no arcs: every gain is R, seeds 0..k-1
    g = _csr(7, [], 0.5)
    s, gn, _ = im.select(_dev(im, g), 100, 7, 1)
    assert s.cpu().tolist() == list(range(7)) and gn.cpu().tolist() == [100] * 7
    # one node, k = 1
    g = _csr(1, [], 0.5)
    s, gn, _ = im.select(_dev(im, g), 3, 1, 1)
    assert s.cpu().tolist() == [0] and gn.cpu().tolist() == [3]
    # k = 0 writes nothing
    g = gg.workload_graph("tiny_uic")
    s, gn, _ = im.select(_dev(im, g), 64, 0, 1)
    assert s.numel() == 0
    # self loops and duplicated arcs are separate coins
    g = _csr(4, [(0, 0), (0, 1), (0, 1), (1, 2), (2, 3), (3, 1)], 0.5)
    s, gn, tr = im.select(_dev(im, g), 200, 4, 11, trace=True)
    s_ref, g_ref, tr_ref, _ = oracle.select_du(g.row_ptr, g.col, g.prob, 200, 4, 11, trace=True)
    assert np.array_equal(tr.cpu().numpy(), tr_ref.astype(np.int64))
    assert s.cpu().tolist() == s_ref.tolist()
    # k = n on a small random graph: every node gets picked
    g = gg.chung_lu_graph(300, 1500, 2.5, 3, True, 0.2)
    s, gn, _ = im.select(_dev(im, g), 64, 300, 2)
    s_ref, g_ref, _, _ = oracle.select_du(g.row_ptr, g.col, g.prob, 64, 300, 2)
    assert s.cpu().tolist() == s_ref.tolist() and gn.cpu().tolist() == g_ref.tolist()
    # the argmax reads nodes in groups of four plus the n % 4 last ones: the
    # best node among the last, and k = n with n % 4 = 3
    g = _csr(11, [(10, i) for i in range(10)] + [(3, 4)], 0.6)
    s, gn, _ = im.select(_dev(im, g), 70, 4, 5)
    s_ref, g_ref, _, _ = oracle.select_du(g.row_ptr, g.col, g.prob, 70, 4, 5)
    assert s.cpu().tolist()[0] == 10
    assert s.cpu().tolist() == s_ref.tolist() and gn.cpu().tolist() == g_ref.tolist()
    g = gg.chung_lu_graph(303, 1500, 2.5, 6, True, 0.2)
    s, gn, _ = im.select(_dev(im, g), 64, 303, 2)
    s_ref, g_ref, _, _ = oracle.select_du(g.row_ptr, g.col, g.prob, 64, 303, 2)
    assert s.cpu().tolist() == s_ref.tolist() and gn.cpu().tolist() == g_ref.tolist()


def test_errors(im):
    import torch
    from paper_1212_4779_amd import _native as N
    g = _csr(3, [(0, 1), (1, 2)], 0.5)
    d = _dev(im, g)
    with pytest.raises(N.ImError) as e:
        im.select(d, 0, 1, 1)
    assert e.value.code == N.IM_EINVAL
    with pytest.raises(N.ImError) as e:
        im.select(d, 4097, 1, 1)
    assert e.value.code == N.IM_EINVAL
    with pytest.raises(N.ImError) as e:
        im.select(d, 64, 4, 1)
    assert e.value.code == N.IM_EINVAL
    bad = _csr(3, [(0, 1), (1, 2)], 0.5)
    bad.prob[0] = np.nan
    with pytest.raises(N.ImError) as e:
        im.select(_dev(im, bad), 64, 1, 1)
    assert e.value.code == N.IM_EINVAL
    bad = _csr(3, [(0, 1), (1, 2)], 0.5)
    bad.col[1] = 3
    with pytest.raises(N.ImError) as e:
        im.select(_dev(im, bad), 64, 1, 1)
    assert e.value.code == N.IM_EINVAL
    bad = _csr(3, [(0, 1), (1, 2)], 0.5)
    bad.prob[1] = 1.5
    with pytest.raises(N.ImError) as e:
        im.select(_dev(im, bad), 64, 1, 1)
    assert e.value.code == N.IM_EINVAL
    bad = _csr(3, [(0, 1), (1, 2)], 0.5)
    bad.row_ptr[1], bad.row_ptr[2] = 2, 1
    with pytest.raises(N.ImError) as e:
        im.select(_dev(im, bad), 64, 1, 1)
    assert e.value.code == N.IM_EINVAL
    # n * R >= 2^32
    big = im.Graph(torch.zeros(2 ** 22 + 1, dtype=torch.int64, device="cuda:0"),
                   torch.zeros(0, dtype=torch.int32, device="cuda:0"),
                   torch.zeros(0, dtype=torch.float32, device="cuda:0"))
    with pytest.raises(N.ImError) as e:
        im.select(big, 1024, 1, 1)
    assert e.value.code == N.IM_EOVERFLOW
    # outputs untouched after a validation error
    seeds = torch.full((1,), 7, dtype=torch.int32, device="cuda:0")
    gains = torch.full((1,), 9, dtype=torch.int64, device="cuda:0")
    import ctypes
    bad = _csr(3, [(0, 1), (1, 2)], 0.5)
    bad.col[1] = 3
    db = _dev(im, bad)
    cg = db.c_struct()
    ws = im.Workspace()
    rc = N.lib().im_select(ctypes.byref(cg), 64, 1, 1, ctypes.c_void_p(seeds.data_ptr()),
                           ctypes.c_void_p(gains.data_ptr()), ctypes.c_void_p(0), ws.handle,
                           ctypes.c_void_p(0))
    assert rc == N.IM_EINVAL
    torch.cuda.synchronize()
    assert seeds.item() == 7 and gains.item() == 9


def _digest(v):
    return hashlib.sha256(np.ascontiguousarray(v, dtype="<u4").tobytes()).hexdigest()


@pytest.mark.parametrize("name", ["tiny_uic", "nethept_wc", "million_uic"])
def test_golden_workloads(im, name):
    with open(os.path.join(GOLDEN, f"{name}.json")) as f:
        gold = json.load(f)
    g = gg.workload_graph(name)
    assert gg.graph_digest(g) == gold["graph_sha256"], "input generator drifted"
    w = gg.WORKLOADS[name]
    d = _dev(im, g)
    ws = im.Workspace()
    seeds, gains, tr = im.select(d, w["R"], w["k"], w["seed"], ws=ws, trace=True)
    assert seeds.cpu().tolist() == gold["seeds"]
    assert gains.cpu().tolist() == gold["gains"]
    tr = tr.cpu().numpy().astype(np.uint32)
    for t, dg in enumerate(gold["round_gain_sha256"]):
        assert _digest(tr[t]) == dg, f"round {t}"
    gs = ws.stats()
    st = gold["stats"]
    assert gs["trav_init"] == st["trav_init"]
    assert gs["trav_fwd"] == st["trav_fwd"]
    assert gs["trav_rev"] == st["trav_rev"]
    assert gs["decrements"] == st["decrements"]
    assert gs["relax_init"] == st["word_reach_deg"]


@pytest.mark.parametrize("name", ["tiny_uic", "nethept_wc"])
def test_plan_graph_replays(im, name):
    # the selection captured into one HIP graph: every replay, with eager work
    # and synchronisations in between, equals the eager call and the oracle
    import torch
    w = gg.WORKLOADS[name]
    g = gg.workload_graph(name)
    d = _dev(im, g)
    s_ref, g_ref, _, _ = oracle.select_du(g.row_ptr, g.col, g.prob, w["R"], w["k"], w["seed"])
    eager = im.select(d, w["R"], w["k"], w["seed"])
    plan = im.Plan(d, w["R"], w["k"], w["seed"])
    for rep in range(4):
        plan.seeds_raw.fill_(-1)
        plan.gains.fill_(-1)
        plan.launch()
        torch.cuda.synchronize()
        assert plan.seeds.cpu().tolist() == s_ref.tolist(), rep
        assert plan.gains.cpu().tolist() == g_ref.tolist(), rep
        # unrelated eager work between replays
        other = im.select(_dev(im, gg.workload_graph("tiny_uic")), 64, 3, 7)
        torch.cuda.synchronize()
    assert eager[0].cpu().tolist() == s_ref.tolist()
    st = plan.stats()
    assert st["trav_init"] > 0
    plan.close()


def test_plan_replay_after_the_graph_changed(im):
    # a replay recomputes everything from the arrays as they are then: new
    # probabilities and a different (valid, same-shape) row_ptr and col
    import torch
    R, k, seed = 64, 8, 5
    ga = gg.chung_lu_graph(2000, 20000, 2.5, 1, True, 0.05)
    gb = gg.chung_lu_graph(2000, 20000, 2.5, 2, True, 0.05)
    assert ga.m == gb.m and ga.n == gb.n
    gb.prob[:] = np.float32(0.08)
    gb.prob[::7] = np.float32(0.01)
    d = _dev(im, ga)
    plan = im.Plan(d, R, k, seed)
    for g in (ga, gb, ga):
        src = _dev(im, g)
        d.row_ptr.copy_(src.row_ptr)
        d.col.copy_(src.col)
        d.prob.copy_(src.prob)
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        s_ref, g_ref, _, _ = oracle.select_du(g.row_ptr, g.col, g.prob, R, k, seed)
        assert plan.seeds.cpu().tolist() == s_ref.tolist()
        assert plan.gains.cpu().tolist() == g_ref.tolist()
    plan.close()


def _batch_instances():
    out = []
    recipes = gg.batch_instances(24, master_seed=11)
    for i, w in enumerate(recipes):
        # keep the CPU oracle fast: shrink the sampled sizes, keep the mix
        n = max(200, w["n"] // 40)
        w = dict(w, n=n, m=int(n * w["m"] / w["n"]), k=min(w["k"], 12))
        out.append((gg.graph_from_recipe(w), w["R"], w["k"], 100 + i))
    # degenerate members: no arcs, k = 0, k = n
    out.append((_csr(30, [], 0.5), 64, 5, 3))
    out.append((gg.chung_lu_graph(200, 900, 2.5, 4, True, 0.1), 128, 0, 4))
    out.append((gg.chung_lu_graph(40, 150, 2.5, 5, True, 0.3), 100, 40, 5))
    return out


def test_batch_matches_oracle_and_single_runs(im):
    insts = _batch_instances()
    dev = [(_dev(im, g), R, k, seed) for (g, R, k, seed) in insts]
    res = im.select_batch(dev)
    for (g, R, k, seed), (d, _, _, _), (s_b, g_b) in zip(insts, dev, res):
        s_ref, g_ref, _, _ = oracle.select_du(g.row_ptr, g.col, g.prob, R, k, seed)
        assert s_b.cpu().tolist() == s_ref.tolist()
        assert g_b.cpu().tolist() == g_ref.tolist()
        alone = im.select(d, R, k, seed)
        assert alone[0].cpu().tolist() == s_b.cpu().tolist()


def test_batch_rejects_bad_instance(im):
    from paper_1212_4779_amd import _native as N
    good = _dev(im, gg.workload_graph("tiny_uic"))
    bad = _csr(3, [(0, 1), (1, 2)], 0.5)
    bad.col[1] = 3
    with pytest.raises(N.ImError) as e:
        im.select_batch([(good, 64, 3, 1), (_dev(im, bad), 64, 1, 1)])
    assert e.value.code == N.IM_EINVAL
    with pytest.raises(N.ImError):
        im.select_batch([(good, 64, 3, 1), (good, 0, 1, 1)])


@pytest.mark.parametrize("R", [4096, 4033])
def test_maximum_snapshot_count(im, R):
    # R = IM_R_MAX (64 snapshot words) and a ragged last word: every round's
    # gain vector, through the cooperative and the one-workgroup forward search
    g = gg.chung_lu_graph(300, 1500, 2.5, 17, True, 0.1)
    s_ref, g_ref, tr_ref, _ = oracle.select_du(g.row_ptr, g.col, g.prob, R, 6, 3, trace=True)
    d = _dev(im, g)
    for gain in (0, 1 << 62):
        ws = im.Workspace()
        ws.set_coop_gain(gain)
        s, gn, tr = im.select(d, R, 6, 3, ws=ws, trace=True)
        assert s.cpu().tolist() == s_ref.tolist() and gn.cpu().tolist() == g_ref.tolist(), gain
        assert np.array_equal(tr.cpu().numpy(), tr_ref.astype(np.int64)), gain


def test_maximum_snapshot_count_weighted_cascade(im):
    # a supercritical weighted-cascade graph at R = IM_R_MAX: large reach sets
    # in all 64 words (tier 2 and hub lists)
    g = gg.chung_lu_graph(2000, 12000, 2.3, 18, True, None)
    s_ref, g_ref, tr_ref, _ = oracle.select_du(g.row_ptr, g.col, g.prob, 4096, 4, 5, trace=True)
    s, gn, tr = im.select(_dev(im, g), 4096, 4, 5, trace=True)
    assert s.cpu().tolist() == s_ref.tolist() and gn.cpu().tolist() == g_ref.tolist()
    assert np.array_equal(tr.cpu().numpy(), tr_ref.astype(np.int64))
