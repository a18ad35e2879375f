"""GPU parity of the spread evaluator (through the C ABI) against the oracle.

Prefix increments of f and per-snapshot reach sizes must be bit-identical to
the oracle's on the same snapshots: small graphs across tiles, snapshot
counts with ragged last words, repeated seeds, more snapshots than a
selection allows (several chunks of words), and the full-size workloads
against stored oracle values.
"""
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


def _cases():
    rng = np.random.default_rng(12)
    return [
        ("tiny_uic", gg.workload_graph("tiny_uic"), 64, 3, list(rng.integers(0, 2000, 12))),
        ("nethept_wc_R100", gg.workload_graph("nethept_wc"), 100, 7, list(rng.integers(0, 15000, 30))),
        ("dense_p30_R1", gg.chung_lu_graph(3000, 24000, 2.3, 7, True, 0.3), 1, 5, [5, 9, 5, 2999]),
        ("dense_p30_R130", gg.chung_lu_graph(3000, 24000, 2.3, 7, True, 0.3), 130, 2,
         list(rng.integers(0, 3000, 9))),
        ("undirected_wc_R300", gg.chung_lu_graph(5000, 30000, 2.2, 8, False, None), 300, 4,
         list(rng.integers(0, 5000, 20))),
        # more than 256 words: the evaluator runs several chunks of words
        ("small_uic_R20000", gg.chung_lu_graph(300, 1500, 2.5, 3, True, 0.08), 20000, 6,
         [1, 7, 7, 250, 0]),
        # the evaluator's maximum R = 2^20 (16,384 words)
        ("tiny_R2p20", gg.chung_lu_graph(60, 240, 2.5, 19, True, 0.15), 1 << 20, 3, [5, 0, 5, 17]),
    ]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_spread_matches_oracle(im, case):
    _, g, R, seed, S = case
    S = [int(x) for x in S]
    marg_ref, per_ref = oracle.spread_prefix(g.row_ptr, g.col, g.prob, R, seed, S)
    d = _dev(im, g)
    marg, per = im.spread(d, R, seed, S, per_snapshot=True)
    assert marg.cpu().tolist() == marg_ref.tolist()
    assert per.cpu().tolist() == per_ref.tolist()
    # the whole set at once (no prefix increments) gives the same snapshots
    none, per2 = im.spread(d, R, seed, S, marginals=False, per_snapshot=True)
    assert none is None and per2.cpu().tolist() == per_ref.tolist()


def test_spread_of_greedy_seeds_is_their_gain_sequence(im):
    # scored on the snapshots that chose them, the seeds' prefix increments
    # are the selection's gains (full-size workload, oracle-stored values)
    with open(os.path.join(GOLDEN, "million_uic.json")) as f:
        gold = json.load(f)
    w = gg.WORKLOADS["million_uic"]
    d = _dev(im, gg.workload_graph("million_uic"))
    marg, _ = im.spread(d, w["R"], w["seed"], gold["seeds"])
    assert marg.cpu().tolist() == gold["gains"]


@pytest.mark.parametrize("name", ["nethept_wc", "million_uic"])
def test_spread_on_independent_snapshots_golden(im, name):
    with open(os.path.join(GOLDEN, f"{name}_spread.json")) as f:
        gold = json.load(f)
    g = gg.workload_graph(name)
    assert gg.graph_digest(g) == gold["graph_sha256"]
    d = _dev(im, g)
    marg, per = im.spread(d, gold["eval_R"], gold["eval_seed"], gold["seeds"], per_snapshot=True)
    assert marg.cpu().tolist() == gold["marg"]
    assert per.cpu().tolist() == gold["per_snapshot"]


def test_spread_edge_cases(im):
    g = gg.chung_lu_graph(500, 2500, 2.5, 4, True, 0.05)
    d = _dev(im, g)
    marg, per = im.spread(d, 64, 1, [], per_snapshot=True)
    assert marg.numel() == 0 and per.cpu().tolist() == [0] * 64
    marg, per = im.spread(d, 65, 2, [3, 3, 3], per_snapshot=True)
    ref, pref = oracle.spread_prefix(g.row_ptr, g.col, g.prob, 65, 2, [3, 3, 3])
    assert marg.cpu().tolist() == ref.tolist() and marg.cpu().tolist()[1:] == [0, 0]
    assert per.cpu().tolist() == pref.tolist()
    with pytest.raises(im.ImError):
        im.spread(d, 64, 1, [0, 500])
    with pytest.raises(im.ImError):
        im.spread(d, 0, 1, [0])
    with pytest.raises(im.ImError):
        im.spread(d, (1 << 20) + 1, 1, [0])
    # a graph without arcs: every seed reaches only itself
    e = gg.Graph(10, np.zeros(11, np.uint64), np.zeros(0, np.uint32), np.zeros(0, np.float32))
    marg, per = im.spread(_dev(im, e), 100, 1, [4, 9, 4], per_snapshot=True)
    assert marg.cpu().tolist() == [100, 100, 0] and per.cpu().tolist() == [2] * 100
