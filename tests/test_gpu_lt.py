"""GPU parity of the linear-threshold snapshots (live-edge form) through the
C ABI: masks, every round's gain vector, seeds and gains of the dynamic
update and of the lazy path, bit-exact against the CPU oracle."""
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


def _lt_ws(im):
    ws = im.Workspace()
    ws.set_live_edge(1)
    return ws


def _random_weights(g, rng, hi=1.1):
    # per head a random split of a total in [0.2, hi] (a total over 1 is cut)
    prob = np.zeros(g.m, np.float32)
    heads = g.col.astype(np.int64)
    order = np.argsort(heads, kind="stable")
    bounds = np.searchsorted(heads[order], np.arange(g.n + 1))
    for v in range(g.n):
        idx = order[bounds[v]:bounds[v + 1]]
        if len(idx):
            w = rng.dirichlet(np.ones(len(idx))) * rng.uniform(0.2, hi)
            prob[idx] = np.minimum(w, 1.0).astype(np.float32)
    return gg.Graph(g.n, g.row_ptr, g.col, prob)


def _star_in(n):
    # every node points at node 0 (an in-row far above the per-thread size)
    # and along a chain; weighted-cascade weights
    arcs = sorted({(i, 0) for i in range(1, n)} | {(i, i + 1) for i in range(1, n - 1)})
    row_ptr = np.zeros(n + 1, np.uint64)
    for u, _ in arcs:
        row_ptr[u + 1] += 1
    row_ptr = np.cumsum(row_ptr).astype(np.uint64)
    col = np.array([v for _, v in arcs], np.uint32)
    return gg.Graph(n, row_ptr, col, gg.weighted_cascade_prob(n, col))


def _cases():
    rng = np.random.default_rng(21)
    return [
        ("nethept_lt", gg.workload_graph("nethept_lt"), 100, 20, 1),
        ("random_weights_R65", _random_weights(gg.chung_lu_graph(3000, 20000, 2.2, 12, True, None), rng),
         65, 10, 3),
        ("heavy_rows_R130", _random_weights(gg.chung_lu_graph(20000, 200000, 2.05, 13, True, None), rng, 1.0),
         130, 8, 4),
        ("in_star_R1", _star_in(3000), 1, 5, 2),
        ("in_star_R256", _star_in(600), 256, 5, 9),
        ("max_R", _random_weights(gg.chung_lu_graph(300, 1500, 2.5, 14, True, None), rng), 4096, 5, 7),
    ]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_lt_masks_match_oracle(im, case):
    _, g, R, _, seed = case
    ref = oracle.live_bits_lt(g.row_ptr, g.col, g.prob, R, seed).T   # word-major
    got = im.snapshot_masks(_dev(im, g), R, seed, ws=_lt_ws(im)).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_lt_selection_matches_oracle(im, case):
    _, g, R, k, seed = case
    s_ref, g_ref, tr_ref = oracle.select_du_lt(g.row_ptr, g.col, g.prob, R, k, seed, trace=True)
    d = _dev(im, g)
    ws = _lt_ws(im)
    seeds, gains, tr = im.select(d, R, k, seed, ws=ws, trace=True)
    assert seeds.cpu().tolist() == s_ref.tolist() and gains.cpu().tolist() == g_ref.tolist()
    assert np.array_equal(tr.cpu().numpy().astype(np.uint32), tr_ref)
    ls, lg = im.select_lazy(d, R, k, seed, batch=4, ws=ws)
    assert ls.cpu().tolist() == s_ref.tolist() and lg.cpu().tolist() == g_ref.tolist()


@pytest.mark.parametrize("name", ["nethept_lt", "million_lt"])
def test_lt_workload_golden(im, name):
    path = os.path.join(GOLDEN, f"{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"no stored oracle values for {name}")
    with open(path) as f:
        gold = json.load(f)
    w = gg.WORKLOADS[name]
    g = gg.workload_graph(name)
    assert gg.graph_digest(g) == gold["graph_sha256"]
    d = _dev(im, g)
    ws = _lt_ws(im)
    masks = im.snapshot_masks(d, w["R"], w["seed"], ws=ws).cpu().numpy().view(np.uint64)
    assert hashlib.sha256(np.ascontiguousarray(masks, dtype="<u8").tobytes()).hexdigest() == gold["mask_sha256"]
    seeds, gains, tr = im.select(d, w["R"], w["k"], w["seed"], ws=ws, trace=True)
    assert seeds.cpu().tolist() == gold["seeds"] and gains.cpu().tolist() == gold["gains"]
    trn = tr.cpu().numpy().astype(np.uint32)
    digests = [hashlib.sha256(np.ascontiguousarray(trn[t], dtype="<u4").tobytes()).hexdigest()
               for t in range(w["k"] + 1)]
    assert digests == gold["round_gain_sha256"]


def test_lt_rejected_where_unsupported(im):
    g = gg.chung_lu_graph(500, 3000, 2.5, 3, True, None)
    d = _dev(im, g)
    ws = _lt_ws(im)
    with pytest.raises(im.ImError):
        im.select_batch([(d, 64, 3, 1), (d, 64, 3, 2)], ws=ws)
    with pytest.raises(im.ImError):
        im.spread(d, 64, 1, [0, 1], ws=ws)
