"""Pins for the oracle's work counters (CPU only).

The oracle's counters are the numerator of the benchmark's throughput and
the reference the GPU tests hold the library's own counters to, so each is
recomputed here by brute force from its definition, on snapshots built from
the pinned live bits (Sec. 3.1: snapshot r keeps arc e iff its coin is live):

  trav_init        sum over u, r and x in R_r(u) of outdeg(x)
  word_reach_deg   sum over (u, word) of outdeg(x) over the union of R_r(u),
                   r in the word's snapshots
  word_reach_nodes sum over (u, word) of the size of that union
  live_pairs       live (arc, snapshot) pairs
  trav_fwd         per round t and snapshot r: sum of outdeg(x) over the
                   newly covered set N_r = R_r(s_t) minus R_r(s_1..s_{t-1})
  trav_rev         per round, r and w in N_r: sum of indeg(x) over U_r(w),
                   the nodes that reach w in snapshot r (Sec. 4, Algorithm 2
                   delete loop)
  decrements       per round, r and w in N_r: |U_r(w)|
  celf_evals       exact re-evaluations of a lazy greedy whose queue is
                   ordered by (bound desc, id asc) (Sec. 5, StaticGreedyCELF)

Degrees are those of the stored graph (every arc, live or not): the
per-snapshot search examines every stored arc of an expanded node.
"""
import heapq

import numpy as np
import pytest

import oracle
from test_oracle_pins import _f, _greedy_by_definition, _random_graph, _reach, _snapshots


def _degrees(row_ptr, col, n):
    outdeg = np.diff(row_ptr.astype(np.int64))
    indeg = np.bincount(col.astype(np.int64), minlength=n)
    return outdeg, indeg


def _reverse(adj, n):
    radj = [[[] for _ in range(n)] for _ in range(len(adj))]
    for r, a in enumerate(adj):
        for u in range(n):
            for v in a[u]:
                radj[r][v].append(u)
    return radj


def _case(case, nmin=5, nmax=14):
    rng = np.random.default_rng(900 + case)
    n = int(rng.integers(nmin, nmax + 1))
    m = int(rng.integers(n, min(3 * n, n * (n - 1)) + 1))
    R = int(rng.choice([1, 5, 64, 70, 130]))
    seed = int(rng.integers(0, 2 ** 63))
    row_ptr, col, prob = _random_graph(rng, n, m, 0.1, 0.8)
    return n, R, seed, row_ptr, col, prob


def _initial_counters(adj, n, R, outdeg):
    trav = wdeg = wnodes = 0
    for u in range(n):
        for r in range(R):
            trav += sum(int(outdeg[x]) for x in _reach(adj[r], [u]))
        for w in range((R + 63) // 64):
            union = set()
            for r in range(64 * w, min(R, 64 * w + 64)):
                union |= _reach(adj[r], [u])
            wdeg += sum(int(outdeg[x]) for x in union)
            wnodes += len(union)
    return trav, wdeg, wnodes


def _round_counters(adj, radj, S, t, outdeg, indeg):
    """(trav_fwd, trav_rev, decrements) of round t (0-based) for seeds S."""
    fwd = rev = dec = 0
    for r in range(len(adj)):
        covered = _reach(adj[r], S[:t]) if t else set()
        newly = _reach(adj[r], [S[t]]) - covered
        fwd += sum(int(outdeg[x]) for x in newly)
        for w in newly:
            up = _reach(radj[r], [w])
            dec += len(up)
            rev += sum(int(indeg[x]) for x in up)
    return fwd, rev, dec


@pytest.mark.parametrize("case", range(10))
def test_initial_counters_bruteforce(case):
    n, R, seed, row_ptr, col, prob = _case(case)
    adj = _snapshots(row_ptr, col, prob, R, seed)
    outdeg, _ = _degrees(row_ptr, col, n)
    trav, wdeg, wnodes = _initial_counters(adj, n, R, outdeg)
    _, st = oracle.initial_gains(row_ptr, col, prob, R, seed)
    assert st["trav_init"] == trav
    assert st["word_reach_deg"] == wdeg
    assert st["word_reach_nodes"] == wnodes
    bits = oracle.live_bits(prob, R, seed)
    assert st["live_pairs"] == sum(bin(int(x)).count("1") for x in bits.ravel())
    # the oracle's initial loop reports the same counters inside the selection
    _, _, _, st_du = oracle.select_du(row_ptr, col, prob, R, 1, seed)
    for key in ("trav_init", "word_reach_deg", "word_reach_nodes", "live_pairs"):
        assert st_du[key] == st[key], key


@pytest.mark.parametrize("case", range(10))
def test_round_counters_bruteforce_per_round(case):
    n, R, seed, row_ptr, col, prob = _case(case)
    adj = _snapshots(row_ptr, col, prob, R, seed)
    radj = _reverse(adj, n)
    outdeg, indeg = _degrees(row_ptr, col, n)
    k = min(n, 5)
    S, _ = _greedy_by_definition(adj, n, k)
    prev = dict(trav_fwd=0, trav_rev=0, decrements=0)
    # the rounds of a k-seed selection are those of the (k+1)-seed one, so the
    # counters of round t are the difference of two prefix selections
    for t in range(k):
        seeds, _, _, st = oracle.select_du(row_ptr, col, prob, R, t + 1, seed)
        assert list(seeds) == S[: t + 1]
        fwd, rev, dec = _round_counters(adj, radj, S, t, outdeg, indeg)
        assert st["trav_fwd"] - prev["trav_fwd"] == fwd, ("trav_fwd", t)
        assert st["trav_rev"] - prev["trav_rev"] == rev, ("trav_rev", t)
        assert st["decrements"] - prev["decrements"] == dec, ("decrements", t)
        prev = st


@pytest.mark.parametrize("case", range(6))
def test_decrements_equal_the_drop_of_the_gain_vector(case):
    # every decrement lowers one entry of s by one, and s of a selected node
    # ends at 0: sum of decrements = sum_u trace[0][u] - sum_u trace[k][u]
    n, R, seed, row_ptr, col, prob = _case(case, 8, 30)
    k = int(np.random.default_rng(case).integers(1, n + 1))
    seeds, gains, tr, st = oracle.select_du(row_ptr, col, prob, R, k, seed, trace=True)
    tr = tr.astype(np.int64)
    assert st["decrements"] == int(tr[0].sum() - tr[k].sum())
    # the selected nodes' entries are 0 from the round after their pick
    for t in range(k):
        assert tr[t + 1, seeds[: t + 1]].sum() == 0
    # and the whole coverage gained is the sum of the gains
    assert int(tr[0].sum() - tr[k].sum()) >= int(gains.sum())


def _celf_by_definition(adj, n, k):
    """Lazy greedy with a (bound desc, id asc) queue; returns (S, gains, evals).
    Round 0's bounds are the exact single-node spreads, so they are fresh."""
    fresh_round = [0] * n
    heap = [(-_f(adj, [u]), u) for u in range(n)]
    heapq.heapify(heap)
    S, gains, evals, fS = [], [], 0, 0
    for t in range(k):
        while True:
            key, u = heapq.heappop(heap)
            if fresh_round[u] == t:
                break
            val = _f(adj, S + [u]) - fS
            evals += 1
            fresh_round[u] = t
            heapq.heappush(heap, (-val, u))
        S.append(u)
        gains.append(-key)
        fS += -key
    return S, gains, evals


@pytest.mark.parametrize("case", range(10))
def test_celf_evaluation_count_bruteforce(case):
    n, R, seed, row_ptr, col, prob = _case(case)
    adj = _snapshots(row_ptr, col, prob, R, seed)
    k = n
    S, gains, evals = _celf_by_definition(adj, n, k)
    s, g, st = oracle.select_celf(row_ptr, col, prob, R, k, seed)
    assert list(s) == S and list(g) == gains
    assert st["celf_evals"] == evals
    # a lazy greedy never evaluates more than the plain one would
    assert evals <= sum(n - t for t in range(1, k))


def test_the_pins_tell_plausible_misreadings_apart():
    # the brute-force definitions above would fail an oracle that counted
    # in-degrees in the forward searches, only live arcs, or out-degrees in
    # the reverse ones: on these graphs every such variant gives other totals
    differ = dict(indeg_fwd=0, live_only=0, outdeg_rev=0)
    for case in range(10):
        n, R, seed, row_ptr, col, prob = _case(case)
        adj = _snapshots(row_ptr, col, prob, R, seed)
        radj = _reverse(adj, n)
        outdeg, indeg = _degrees(row_ptr, col, n)
        _, st = oracle.initial_gains(row_ptr, col, prob, R, seed)
        alt = sum(int(indeg[x]) for u in range(n) for r in range(R) for x in _reach(adj[r], [u]))
        differ["indeg_fwd"] += alt != st["trav_init"]
        alt = sum(len(adj[r][x]) for u in range(n) for r in range(R) for x in _reach(adj[r], [u]))
        differ["live_only"] += alt != st["trav_init"]
        S, _ = _greedy_by_definition(adj, n, 2)
        _, _, _, st2 = oracle.select_du(row_ptr, col, prob, R, 2, seed)
        _, rev, _ = _round_counters(adj, radj, S, 0, indeg, outdeg)
        _, rev1, _ = _round_counters(adj, radj, S, 1, indeg, outdeg)
        differ["outdeg_rev"] += rev + rev1 != st2["trav_rev"]
    assert all(v >= 5 for v in differ.values()), differ
