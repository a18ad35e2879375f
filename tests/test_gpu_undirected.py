"""GPU parity of the undirected path (one coin per undirected pair) through
the C ABI: pair matching, the component method and the directed engines run
with pair coins, all against the CPU oracle, bit-exact, every round's gain
vector included."""
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


def _sym(n, pairs, p, loops=()):
    ps = list(p) if np.ndim(p) else [p] * len(pairs)
    arcs = {}
    for (u, v), q in zip(pairs, ps):
        arcs[(u, v)] = q
        arcs[(v, u)] = q
    for u in loops:
        arcs[(u, u)] = 0.5
    keys = sorted(arcs)
    row_ptr = np.zeros(n + 1, np.uint64)
    for u, _ in keys:
        row_ptr[u + 1] += 1
    row_ptr = np.cumsum(row_ptr).astype(np.uint64)
    col = np.array([v for _, v in keys], np.uint32)
    prob = np.array([arcs[k] for k in keys], np.float32)
    return gg.Graph(n, row_ptr, col, prob)


def _shuffled_rows(g, seed):
    # the same graph with every row's arcs in a random order (arc ids change)
    rng = np.random.default_rng(seed)
    col, prob = g.col.copy(), g.prob.copy()
    for u in range(g.n):
        a, b = int(g.row_ptr[u]), int(g.row_ptr[u + 1])
        perm = rng.permutation(b - a) + a
        col[a:b], prob[a:b] = g.col[perm], g.prob[perm]
    return gg.Graph(g.n, g.row_ptr, col, prob)


def vec_digest(v):
    return hashlib.sha256(np.ascontiguousarray(v, dtype="<u4").tobytes()).hexdigest()


def _cases():
    rng = np.random.default_rng(9)
    big = gg.chung_lu_graph(6000, 40000, 2.2, 31, False, 0.05)
    return [
        ("nethept_uic", gg.workload_graph("nethept_uic"), 100, 50, 1),
        ("supercritical_R64", big, 64, 20, 3),
        ("supercritical_R300", big, 300, 10, 4),
        ("shuffled_rows_R65", _shuffled_rows(gg.chung_lu_graph(3000, 12000, 2.4, 32, False, 0.2), 5),
         65, 15, 6),
        ("mixed_p_R1", _sym(500, [(i, (i * 7 + 1) % 500) for i in range(499) if (i * 7 + 1) % 500 != i],
                            rng.uniform(0, 1, 499).astype(np.float32), loops=(3, 77)), 1, 30, 2),
        ("p1_two_paths", _sym(12, [(0, 1), (1, 2), (5, 6), (6, 7), (7, 8)], 1.0), 70, 12, 1),
        ("max_R", gg.chung_lu_graph(400, 1600, 2.3, 33, False, 0.1), 4096, 6, 7),
    ]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_components_match_oracle(im, case):
    _, g, R, k, seed = case
    s_ref, g_ref, tr_ref = oracle.select_components(g.row_ptr, g.col, g.prob, R, k, seed, trace=True)
    d = _dev(im, g)
    assert im.pair_ids(d).cpu().tolist() == oracle.pair_ids(g.row_ptr, g.col, g.prob).tolist()
    seeds, gains, tr = im.select_undirected(d, R, k, seed, trace=True)
    assert seeds.cpu().tolist() == s_ref.tolist()
    assert gains.cpu().tolist() == g_ref.tolist()
    assert np.array_equal(tr.cpu().numpy().astype(np.uint32), tr_ref)


@pytest.mark.parametrize("case", _cases()[:4], ids=lambda c: c[0])
def test_directed_engines_with_pair_coins(im, case):
    # the reachability engines of the directed path on the same pair-coin
    # snapshots give the component method's results
    _, g, R, k, seed = case
    if case[0].startswith("supercritical"):
        k = 4   # giant components make every reverse search large
    s_ref, g_ref, tr_ref = oracle.select_components(g.row_ptr, g.col, g.prob, R, k, seed, trace=True)
    d = _dev(im, g)
    ws = im.Workspace()
    ws.set_pair_coins(True)
    seeds, gains, tr = im.select(d, R, k, seed, ws=ws, trace=True)
    assert seeds.cpu().tolist() == s_ref.tolist() and gains.cpu().tolist() == g_ref.tolist()
    assert np.array_equal(tr.cpu().numpy().astype(np.uint32), tr_ref)
    ls, lg = im.select_lazy(d, R, k, seed, batch=4, ws=ws)
    assert ls.cpu().tolist() == s_ref.tolist() and lg.cpu().tolist() == g_ref.tolist()


@pytest.mark.parametrize("name", ["nethept_uic", "million_undirected_uic"])
def test_undirected_workload_golden(im, name):
    with open(os.path.join(GOLDEN, f"{name}.json")) as f:
        gold = json.load(f)
    w = gg.WORKLOADS[name]
    g = gg.workload_graph(name)
    assert gg.graph_digest(g) == gold["graph_sha256"]
    d = _dev(im, g)
    assert vec_digest(im.pair_ids(d).cpu().numpy().astype(np.uint32)) == gold["pair_sha256"]
    seeds, gains, tr = im.select_undirected(d, w["R"], w["k"], w["seed"], trace=True)
    assert seeds.cpu().tolist() == gold["seeds"]
    assert gains.cpu().tolist() == gold["gains"]
    trn = tr.cpu().numpy().astype(np.uint32)
    assert [vec_digest(trn[t]) for t in range(w["k"] + 1)] == gold["round_gain_sha256"]


def test_undirected_edge_cases(im):
    # no arcs: every node alone; k = n picks every node once
    e = gg.Graph(7, np.zeros(8, np.uint64), np.zeros(0, np.uint32), np.zeros(0, np.float32))
    seeds, gains, _ = im.select_undirected(_dev(im, e), 10, 7, 1)
    assert seeds.cpu().tolist() == list(range(7)) and gains.cpu().tolist() == [10] * 7
    g = _sym(6, [(0, 1), (2, 3)], 0.3)
    d = _dev(im, g)
    seeds, gains, _ = im.select_undirected(d, 64, 0, 1)
    assert seeds.numel() == 0
    # asymmetric, unequal probabilities, a pair stored twice: rejected
    asym = gg.Graph(3, np.array([0, 1, 2, 2], np.uint64), np.array([1, 2], np.uint32),
                    np.array([0.5, 0.5], np.float32))
    with pytest.raises(im.ImError):
        im.select_undirected(_dev(im, asym), 64, 1, 1)
    bad_p = _sym(4, [(0, 1)], 0.5)
    bad_p.prob[0] = 0.25
    with pytest.raises(im.ImError):
        im.pair_ids(_dev(im, bad_p))
    twice = gg.Graph(2, np.array([0, 2, 4], np.uint64), np.array([1, 1, 0, 0], np.uint32),
                     np.full(4, 0.5, np.float32))
    with pytest.raises(im.ImError):
        im.pair_ids(_dev(im, twice))
    with pytest.raises(im.ImError):
        im.select_undirected(d, 0, 1, 1)
