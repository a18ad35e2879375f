"""The selection entry point that allocates nothing (im_select_noalloc),
through the C ABI, against im_select with a workspace and against the
oracle's stored values: two calls in a row, the second on a smaller graph,
so that the second reuses the static scratch the first left behind.
Collected last (pytest -x stops at the first failure)."""
import ctypes
import json
import os

import numpy as np
import pytest

from paper_1212_4779_amd import _native as N
from paper_1212_4779_amd import graphgen as gg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLDEN, f"{name}.json")) as f:
        return json.load(f)


def test_noalloc_rejects_a_graph_larger_than_the_scratch():
    # host arithmetic only: rejected before any device work (runs on the CPU)
    lib = N.lib()
    n, m = 1_000_000, 10_000_000
    g = N.ImGraph(n, m, 8, 8, 8)   # never dereferenced: the size check comes first
    rc = lib.im_select_noalloc(ctypes.byref(g), 256, 50, 1, ctypes.c_void_p(8),
                               ctypes.c_void_p(8), ctypes.c_void_p(0))
    assert rc == N.IM_EINVAL
    msg = lib.im_last_error().decode()
    assert "scratch" in msg and str(N.IM_NOALLOC_SCRATCH_BYTES) in msg, msg


@pytest.mark.gpu
def test_noalloc_equals_select_twice_second_smaller():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1212_4779_amd as im
    for name in ("nethept_wc", "tiny_uic"):   # the second call is the smaller graph
        w = gg.WORKLOADS[name]
        g = gg.workload_graph(name)
        d = im.Graph.from_numpy(g.row_ptr, g.col, g.prob, device="cuda:0")
        print(f"noalloc: {name} n={g.n} m={g.m} R={w['R']} k={w['k']}", flush=True)
        ref_s, ref_g, _ = im.select(d, w["R"], w["k"], w["seed"])
        s, gn = im.select_noalloc(d, w["R"], w["k"], w["seed"])
        torch.cuda.synchronize()
        assert s.cpu().tolist() == ref_s.cpu().tolist()
        assert gn.cpu().tolist() == ref_g.cpu().tolist()
        gold = _gold(name)
        assert s.cpu().tolist() == gold["seeds"]
        assert gn.cpu().tolist() == gold["gains"]
    # and once more on the larger graph after the smaller one
    w = gg.WORKLOADS["nethept_wc"]
    g = gg.workload_graph("nethept_wc")
    d = im.Graph.from_numpy(g.row_ptr, g.col, g.prob, device="cuda:0")
    s, gn = im.select_noalloc(d, w["R"], w["k"], w["seed"])
    gold = _gold("nethept_wc")
    assert s.cpu().tolist() == gold["seeds"] and gn.cpu().tolist() == gold["gains"]
