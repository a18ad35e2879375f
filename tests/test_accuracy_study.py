"""The accuracy study's summary measures (Sec. 3.4) on hand-made inputs (CPU),
and one small sweep on the GPU whose numbers must be consistent."""
import math

import pytest

from paper_1212_4779_amd import accuracy, graphgen as gg


def test_entropy_of_solution_sets():
    assert accuracy.entropy([[1, 2, 3]] * 10) == 0.0
    # order inside a solution does not matter
    assert accuracy.entropy([[1, 2], [2, 1]]) == 0.0
    assert math.isclose(accuracy.entropy([[1], [2]]), math.log(2))
    assert math.isclose(accuracy.entropy([[1], [2], [3], [3]]),
                        -(2 * 0.25 * math.log(0.25) + 0.5 * math.log(0.5)))


def test_relative_difference_and_r_min():
    assert accuracy.relative_differences(200.0, [200.0, 190.0, 210.0]) == [0.0, 0.05, -0.05]
    rows = [{"R": 1, "d_mean": 0.2}, {"R": 10, "d_mean": 0.004}, {"R": 100, "d_mean": 0.001}]
    assert accuracy.r_min(rows) == 10
    assert accuracy.r_min([{"R": 5, "d_mean": 0.1}]) is None


@pytest.mark.gpu
def test_small_sweep_is_consistent():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1212_4779_amd as im
    g = gg.chung_lu_graph(3000, 12000, 2.4, 41, False, 0.05)
    d = im.Graph.from_numpy(g.row_ptr, g.col, g.prob)
    res = accuracy.study(d, [1, 16, 256], 5, 8, 2048, 99, R_ref=256, k_entropy=3,
                         log=lambda *_: None)
    rows = {r["R"]: r for r in res["rows"]}
    assert res["reference_R"] == 256 and res["reference_spread"] > 0
    for r in rows.values():
        assert 0.0 <= r["H_k"] <= math.log(8) + 1e-12
        assert 1 <= r["distinct_solutions"] <= 8
    # a single snapshot is a poorer estimate than 256 of them
    assert rows[1]["spread_mean"] <= rows[256]["spread_mean"] * 1.001
    # the spreads are those of the evaluator, the entropy that of the solutions
    S = im.select(d, 16, 5, 1000)[0].cpu().tolist()
    _, per = im.spread(d, 2048, 99, S, marginals=False, per_snapshot=True)
    assert per.sum().item() > 0


@pytest.mark.gpu
def test_sweep_runs_equal_the_oracle():
    # every run of a small sweep against the oracle: its seeds are the
    # oracle's StaticGreedyDU seeds on the run's snapshots, its spread the
    # oracle's f(S) / R_eval on the common evaluation snapshots, and the
    # summary measures (Sec. 3.4: d_{R,k}, H_{R,k}) follow from those
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import numpy as np
    import oracle
    import paper_1212_4779_amd as im
    g = gg.chung_lu_graph(400, 1600, 2.4, 43, True, 0.08)
    d = im.Graph.from_numpy(g.row_ptr, g.col, g.prob)
    Rs, k, runs, R_eval, eval_seed, R_ref = [1, 8, 64], 5, 4, 512, 99, 128
    res = accuracy.study(d, Rs, k, runs, R_eval, eval_seed, R_ref=R_ref, k_entropy=3,
                         log=lambda *_: None, keep_runs=True)

    def f(S):
        marg, _ = oracle.spread_prefix(g.row_ptr, g.col, g.prob, R_eval, eval_seed, S)
        return int(marg.sum()) / R_eval

    ref_seeds, _, _, _ = oracle.select_du(g.row_ptr, g.col, g.prob, R_ref, k, 999)
    assert res["reference_seeds"] == ref_seeds.tolist()
    ref = f(ref_seeds)
    assert res["reference_spread"] == ref
    for row, R in zip(res["rows"], Rs):
        sols, spreads = [], []
        for run in row["runs"]:
            s_ref, _, _, _ = oracle.select_du(g.row_ptr, g.col, g.prob, R, k, run["seed"])
            assert run["seeds"] == s_ref.tolist(), (R, run["seed"])
            assert run["spread"] == f(s_ref), (R, run["seed"])
            sols.append(s_ref.tolist())
            spreads.append(f(s_ref))
        assert row["d_mean"] == pytest.approx(float(np.mean([(ref - x) / ref for x in spreads])),
                                              rel=0, abs=1e-12)
        assert row["H_k"] == accuracy.entropy([S[:3] for S in sols])
