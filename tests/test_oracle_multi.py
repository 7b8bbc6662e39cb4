"""Pins for the oracle's multi-move step (no GPU): several independent moves
per local-search iteration (Section 7, after Dynasearch).  The selection is
pinned by an independent implementation over the brute-force enumeration
(each move's touched routes come from the enumerator itself), by the
additivity that independence implies (applying the selection changes the
objective by exactly the sum of its deltas, and every selected move keeps
its delta after the earlier ones are applied), by route-disjointness, and by
the multi-move search ending at a local optimum of the single-move
neighbourhood."""
import itertools

import numpy as np
import pytest

import oracle
from paper_2506_17357_amd import workload as W
from tests import brute


def brute_select(inst, routes, op_mask):
    """Greedy route-disjoint selection over per-route-pair bests, from the
    brute-force enumeration (hard feasibility)."""
    base = brute.total_cost(inst, routes)
    best = {}
    gen = itertools.chain(brute.neighbours(inst, routes, op_mask & 0x1F), brute.neighbours_ext(inst, routes, op_mask))
    for mid, new, touched in gen:
        if not all(brute.route_ok_cap(inst, new[r]) and brute.route_ok_tw(inst, new[r]) for r in touched):
            continue
        delta = brute.total_cost(inst, new) - base
        if delta >= 0:
            continue
        key = (min(touched), max(touched))
        if key not in best or (delta, mid) < best[key]:
            best[key] = (delta, mid)
    used, out = set(), []
    for (delta, mid), key in sorted((v, k) for k, v in best.items()):
        if key[0] in used or key[1] in used:
            continue
        used.update(key)
        out.append((mid, delta))
    return out


@pytest.mark.parametrize("has_tw", [0, 1])
@pytest.mark.parametrize("n,R,mask", [(6, 3, 0x1F), (7, 4, 0x1F), (8, 4, 0x1F), (7, 4, 0xFF)])
def test_selection_equals_brute_force(has_tw, n, R, mask):
    found = 0
    for seed in range(12):
        inst = W.tiny_instance(n, 3000 + 10 * seed + n + R + has_tw, bool(has_tw), dup=seed % 2 == 0)
        sol = W.random_solution(inst, R, 3100 + seed + n)
        routes = [list(map(int, sol.customers[sol.offsets[r]:sol.offsets[r + 1]])) for r in range(R)]
        sel, _ = oracle.multi_select(inst, sol, mask, threads=1)
        assert sel == brute_select(inst, routes, mask)
        found += len(sel) > 1
    assert found > 0 or R < 4, "no case with more than one selected move"


def routes_of(sol):
    return [list(map(int, sol.customers[sol.offsets[r]:sol.offsets[r + 1]])) for r in range(sol.R)]


def touched_routes(Q, n, sol, mid):
    """Route slots a move touches, from its refs (ops 3 and 4 stay in one route)."""
    op, k, a, b = oracle.decode(Q, mid)
    route_of = {}
    for r, cs in enumerate(routes_of(sol)):
        for c in cs:
            route_of[c - 1] = r
    def rt(ref):
        return ref - n if ref >= n else route_of[ref]
    return {rt(a)} if op in (3, 4) else {rt(a), rt(b)}


@pytest.mark.parametrize("pen", [None, (5, 3)])
@pytest.mark.parametrize("mask", [0x1F, 0xFF])
@pytest.mark.parametrize("has_tw", [False, True])
def test_independence_and_additivity(pen, mask, has_tw):
    inst = W.tiny_instance(60, 3200, has_tw, span=300)
    inst.capacity = int(inst.node4[:, 0].sum() // 6)
    sol = W.random_solution(inst, 9, 3201)
    Q = inst.n + sol.R
    sel, _ = oracle.multi_select(inst, sol, mask, penalty=pen)
    assert len(sel) >= 2
    used = set()
    for mid, _ in sel:
        t = touched_routes(Q, inst.n, sol, mid)
        assert not (t & used), "selected moves share a route"
        used |= t

    def objective(s):
        c = oracle.cost(inst, s)[0]
        if pen is None:
            return c
        lv, tv = oracle.violations(inst, s)
        return c + pen[0] * lv + pen[1] * tv

    cur = sol
    for mid, delta in sel:
        # the move keeps its delta (score) after the earlier selections
        _, dd, df = oracle.eval_neighbourhood(inst, cur, mask, dump=True, penalty=pen)
        assert int(dd[mid]) == delta
        if pen is None:
            assert int(df[mid]) == 3
        cur = oracle.apply_move(inst, cur, mid)
    assert objective(cur) - objective(sol) == sum(d for _, d in sel)
    # each selected move is the best improving move of its route pair
    _, dd, df = oracle.eval_neighbourhood(inst, sol, mask, dump=True, penalty=pen)
    ok = (df != oracle.NOT_A_MOVE) & (dd < 0)
    if pen is None:
        ok &= df == 3
    ids = np.nonzero(ok)[0]
    for mid, delta in sel:
        t = touched_routes(Q, inst.n, sol, mid)
        rivals = [(int(dd[i]), int(i)) for i in ids if touched_routes(Q, inst.n, sol, int(i)) == t]
        assert min(rivals) == (delta, mid)


def test_multi_search_reaches_a_single_move_local_optimum():
    inst, sol = W.c1()
    final, applied, per, mv = oracle.local_search_multi(inst, sol, max_steps=200)
    assert sum(per) == len(applied) and len(per) < len(applied)
    assert oracle.cost(inst, final)[0] - oracle.cost(inst, sol)[0] == sum(d for _, d in applied)
    b = oracle.eval_neighbourhood(inst, final)
    assert not b.found or b.delta >= 0
    # one selected move per step reduces to the single-move search
    inst2 = W.tiny_instance(12, 3300, False)
    sol2 = W.random_solution(inst2, 1, 3301)
    f2, ap2, per2, _ = oracle.local_search_multi(inst2, sol2, max_steps=50)
    f1, ids1, d1, _ = oracle.local_search(inst2, sol2, max_steps=50)
    assert all(p == 1 for p in per2)
    assert [m for m, _ in ap2] == ids1.tolist() and [d for _, d in ap2] == d1.tolist()
    assert f2.offsets.tolist() == f1.offsets.tolist() and f2.customers.tolist() == f1.customers.tolist()
