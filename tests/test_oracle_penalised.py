"""Pins for the oracle's penalised mode (no GPU).

Penalised mode scores every move by dD + w_L dL_V + w_T dT_V over the
touched routes (Section 5.3.3 attribute deltas, eq. scoring_tensor; the
feasible and infeasible search of Alg. A2).  Pinned against: a hand-computed
example, the paper's concatenation rules for time warp (Section 4.3.3, a
different algorithm from the oracle's forward simulation), whole-solution
recomputation over an independent brute-force neighbour enumeration,
zero weights (the distance delta), inverse moves and the local search's
monotone objective.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2506_17357_amd import workload as W
from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden():
    with open(os.path.join(GOLDEN, "timewarp_line.json")) as f:
        g = json.load(f)
    inst = W.Instance(g["n"], np.asarray(g["dist"], np.int32), np.asarray(g["node4"], np.int32),
                      g["capacity"], g["has_tw"], np.zeros((g["n"] + 1, 2), np.int64), "golden", 0)
    return g, inst, W.Solution.from_routes(g["routes"])


def concat(s1, s2, t):
    """Concatenation of two subsequence summaries (T_D, T_E, T_L, T_V) joined
    by an edge of travel time t, as Section 4.3.3 states it, with the
    garbled shift read as T_D(s1) - T_V(s1) + t."""
    D1, E1, L1, V1 = s1
    D2, E2, L2, V2 = s2
    dt = D1 - V1 + t
    dw = max(E2 - dt - L1, 0)
    dv = max(E1 + dt - L2, 0)
    return (D1 + t + dw + D2, max(E1, E2 - dt) - dw, min(L1, L2 - dt) + dv, V1 + dv + V2)


def route_tv_by_concatenation(inst, r):
    nd, D = inst.node4, inst.dist
    if not inst.has_tw:
        return 0
    seq = [0] + [int(c) for c in r] + [0]
    s = (int(nd[0][3]), int(nd[0][1]), int(nd[0][2]), 0)
    for a, b in zip(seq[:-1], seq[1:]):
        s = concat(s, (int(nd[b][3]), int(nd[b][1]), int(nd[b][2]), 0), int(D[a][b]))
    return s[3]


def penalised_cost(inst, routes, wl, wt):
    """Whole-solution penalised objective from the brute-force helpers and
    the concatenation rules (nothing from the oracle)."""
    c = 0
    for r in routes:
        load = sum(int(inst.node4[x][0]) for x in r)
        c += brute.route_cost(inst.dist, r) + wl * max(load - inst.capacity, 0) + wt * route_tv_by_concatenation(inst, r)
    return c


def tight_instance(n, seed, has_tw=True):
    inst = W.tiny_instance(n, seed, has_tw, span=100)
    rng = np.random.default_rng(seed)
    if has_tw:
        inst.node4[1:, 2] = inst.node4[1:, 1] + rng.integers(0, 40, size=n)
        inst.node4[0, 2] = int(rng.integers(150, 700))
    inst.capacity = int(inst.node4[:, 0].sum() // 3 + 1)
    return inst


def test_golden_timewarp_hand_computed():
    g, inst, sol = golden()
    wl, wt = g["weights"]
    assert oracle.cost(inst, sol)[0] == g["expected_distance"]
    assert oracle.violations(inst, sol) == (g["expected_load_excess"], g["expected_time_warp"])
    best, dd, df = oracle.eval_neighbourhood(inst, sol, dump=True, threads=1, penalty=(wl, wt))
    for m in g["moves"]:
        assert (int(dd[m["id"]]), int(df[m["id"]])) == (m["score"], m["feas"]), m["why"]


def test_time_warp_equals_concatenation_rules():
    """The oracle's forward simulation against the paper's concatenation
    algebra on random routes with tight windows (warps at customers and at
    the depot)."""
    seen_warp = 0
    for seed in range(200):
        inst = tight_instance(9, 500 + seed)
        sol = W.random_solution(inst, 3, seed)
        routes = [sol.customers[sol.offsets[r]:sol.offsets[r + 1]] for r in range(sol.R)]
        tv = sum(route_tv_by_concatenation(inst, r) for r in routes)
        assert oracle.violations(inst, sol)[1] == tv, seed
        seen_warp += tv > 0
    assert seen_warp > 150


@pytest.mark.parametrize("has_tw", [0, 1])
@pytest.mark.parametrize("n,R", [(4, 1), (5, 2), (6, 3), (7, 2)])
def test_scores_equal_whole_solution_difference(has_tw, n, R):
    """Every move's score equals F(S') - F(S) over an independent brute-force
    enumeration, for several weight pairs; the hard bits are unchanged."""
    inst = tight_instance(n, 70 + 7 * n + R + 100 * has_tw, bool(has_tw))
    sol = W.random_solution(inst, R, 80 + n + R)
    routes = [list(map(int, sol.customers[sol.offsets[r]:sol.offsets[r + 1]])) for r in range(R)]
    for wl, wt in ((0, 0), (1, 0), (0, 1), (3, 7)):
        base = penalised_cost(inst, routes, wl, wt)
        best, dd, df = oracle.eval_neighbourhood(inst, sol, dump=True, threads=1, penalty=(wl, wt))
        ids = set()
        exp_best = None
        for mid, new, touched in brute.neighbours(inst, routes):
            ids.add(mid)
            score = penalised_cost(inst, new, wl, wt) - base
            assert int(dd[mid]) == score, (mid, oracle.decode(n + R, mid), wl, wt)
            feas = int(all(brute.route_ok_cap(inst, new[r]) for r in touched)) | \
                (int(all(brute.route_ok_tw(inst, new[r]) for r in touched)) << 1)
            assert int(df[mid]) == feas
            if exp_best is None or (score, mid) < exp_best:
                exp_best = (score, mid)
        assert set(np.nonzero(df != oracle.NOT_A_MOVE)[0].tolist()) == ids
        assert best.found == (exp_best is not None)
        if best.found:
            assert (best.delta, best.id) == exp_best


def test_zero_weights_score_is_the_distance_delta():
    inst = tight_instance(40, 9)
    sol = W.random_solution(inst, 5, 10)
    _, d0, f0 = oracle.eval_neighbourhood(inst, sol, dump=True, threads=2)
    best, dp, fp = oracle.eval_neighbourhood(inst, sol, dump=True, threads=2, penalty=(0, 0))
    assert np.array_equal(d0, dp) and np.array_equal(f0, fp)
    valid = f0 != oracle.NOT_A_MOVE
    ids = np.nonzero(valid)[0]
    k = np.lexsort((ids, d0[ids]))[0]
    assert (best.delta, best.id) == (int(d0[ids[k]]), int(ids[k]))


def test_inverse_moves_cancel():
    inst = tight_instance(12, 13)
    sol = W.random_solution(inst, 3, 14)
    pen = (2, 5)
    _, dd, df = oracle.eval_neighbourhood(inst, sol, dump=True, threads=1, penalty=pen)
    Q = inst.n + sol.R
    rng = np.random.default_rng(0)
    ids = np.nonzero(df != oracle.NOT_A_MOVE)[0]
    checked = 0
    for mid in rng.choice(ids, size=min(200, ids.size), replace=False):
        op, k, a, b = oracle.decode(Q, int(mid))
        if op not in (1, 2, 3):  # self-inverse on the same refs
            continue
        s2 = oracle.apply_move(inst, sol, int(mid))
        _, d2, _ = oracle.eval_neighbourhood(inst, s2, dump=True, threads=1, penalty=pen)
        assert int(dd[mid]) + int(d2[mid]) == 0, (op, k, a, b)
        checked += 1
    assert checked > 30


def test_penalised_local_search_descends():
    inst = tight_instance(30, 21)
    sol = W.random_solution(inst, 4, 22)
    pen = (3, 2)
    final, ids, scores, mv = oracle.local_search(inst, sol, max_steps=200, penalty=pen)
    assert len(ids) > 5 and (scores < 0).all()

    def F(s):
        d = oracle.cost(inst, s)[0]
        lv, tv = oracle.violations(inst, s)
        return d + pen[0] * lv + pen[1] * tv

    cur = sol
    for mid, sc in zip(ids, scores):
        nxt = oracle.apply_move(inst, cur, int(mid))
        assert F(nxt) - F(cur) == int(sc)
        cur = nxt
    best = oracle.eval_neighbourhood(inst, final, penalty=pen)
    assert best.delta >= 0  # a local optimum of the penalised objective
