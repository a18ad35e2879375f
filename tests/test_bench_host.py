"""Host logic of bench.py (CPU): which committed counter figure the roofline
line may carry.

profiles/traffic.json holds, per workload and phase, the HBM bytes per launch
that rocprofv3's FETCH_SIZE + WRITE_SIZE counters gave for one kernel
instance. The tier-1 shape and the tier-2 lane count are template arguments,
so a different schedule launches a different kernel: the figure may be
attached only when the schedule of the run selects the profiled instance
and gives it the same share of the work: the last tier runs what tier 1
hands on (its table size is the tier-1 shape), reverse tier 1 takes every
reverse task when they start there, and last-tier reverse tasks may be split
into bit groups.
"""
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")
PHASES = ["init_t0", "init_t1", "init_t2", "forward", "rev_t0", "rev_t1", "rev_t2"]
SCHEDULES = [{"tier1_shape": s, "tier2_lanes": l, "rev_split": p, "rev_first_tier": f}
             for s in (0, 1, 2) for l in (64, 256, 1024) for p in (1, 2) for f in (0, 1)]


def _profiled():
    with open(TRAFFIC) as f:
        return json.load(f)["workloads"]


def _matching(phase, name):
    return [s for s in SCHEDULES if bench.kernel_signature(phase, s) in name]


def test_signatures_tell_the_instances_apart():
    for phase in PHASES:
        sigs = {bench.kernel_signature(phase, s) for s in SCHEDULES}
        if phase == "forward" or phase.endswith("_t0"):
            assert len(sigs) == 1          # no schedule argument in the kernel
        elif phase.endswith("_t1"):
            assert len(sigs) == 3          # one per tier-1 shape
        else:
            assert len(sigs) == 3          # one per tier-2 lane count
    # count and decrement modes are different kernels
    assert bench.kernel_signature("init_t0", {}) != bench.kernel_signature("rev_t0", {})


@pytest.mark.skipif(not os.path.exists(TRAFFIC), reason="no counter summary committed")
def test_profiled_kernels_are_recognised_by_exactly_their_schedule():
    for wl, rec in _profiled().items():
        for phase, k in rec["kernels"].items():
            m = _matching(phase, k["kernel"])
            assert m, (wl, phase, k["kernel"])
            if phase.endswith("_t1"):
                assert {s["tier1_shape"] for s in m} == {m[0]["tier1_shape"]}
            if phase.endswith("_t2"):
                assert {s["tier2_lanes"] for s in m} == {m[0]["tier2_lanes"]}


@pytest.mark.skipif(not os.path.exists(TRAFFIC), reason="no counter summary committed")
def test_load_traffic_follows_the_schedule():
    for wl, rec in _profiled().items():
        for phase, k in rec["kernels"].items():
            if k.get("source_digest") != bench.source_digest(k.get("sources", [])):
                # the kernel's source changed since the counters were taken
                assert bench.load_traffic(phase, wl, SCHEDULES[0]) is None
                continue
            prof = rec.get("schedule", {})
            for s in SCHEDULES:
                got = bench.load_traffic(phase, wl, s)
                same = bench.kernel_signature(phase, s) in k["kernel"]
                if phase.endswith("_t2"):
                    same = same and s["tier1_shape"] == prof.get("tier1_shape", 0)
                if phase in ("rev_t1", "rev_t2"):
                    same = same and s["rev_first_tier"] == prof.get("rev_first_tier", 0)
                if phase == "rev_t2":
                    same = same and s["rev_split"] == prof.get("rev_split", 1)
                if same:
                    assert got == k["hbm_bytes_per_launch"], (wl, phase, s)
                else:
                    assert got is None, (wl, phase, s)
        assert bench.load_traffic("rev_t0", wl + "_other", SCHEDULES[0]) is None


def test_signatures_follow_the_launch_code():
    # the instances run_tiers launches for each schedule value, read from the
    # library source: tier-0 and tier-1 template arguments, tier-2 lanes
    import re
    with open(os.path.join(ROOT, "paper_1212_4779_amd", "csrc", "im.hip")) as f:
        src = f.read()
    const = {k: int(v) for k, v in re.findall(r"\b(T[012][A-Z]*_[A-Z]+) = (\d+)", src)}
    body = src[src.index("static void run_tiers("):]
    body = body[:body.index("\n}\n")]
    shapes = {0: (const["T1_T"], const["T1_CS"], const["T1_LIM"])}
    for case, t, cs, lim in re.findall(
            r"case (\d+): \{\s*auto k1 = k_lds_bfs<MODE, T1_NT, (\d+), (\d+), (\d+),", body):
        shapes[int(case)] = (int(t), int(cs), int(lim))
    assert sorted(shapes) == [0, 1, 2]
    for mode, pre in ((0, "init"), (1, "rev")):
        assert bench.kernel_signature(pre + "_t0", {}) == (
            f"k_lds_bfs<{mode}, 64, {const['T0_T']}, {const['T0_CS']}, {const['T0_LIM']},")
        for s, (t, cs, lim) in shapes.items():
            assert bench.kernel_signature(pre + "_t1", {"tier1_shape": s}) == (
                f"k_lds_bfs<{mode}, {const['T1_NT']}, {t}, {cs}, {lim},")
        for lanes in (const["T2W_NT"], const["T2S_NT"], const["T2_NT"]):
            assert bench.kernel_signature(pre + "_t2", {"tier2_lanes": lanes}) == (
                f"k_block_bfs<{mode}, {lanes}, {const['T2_U']},")
