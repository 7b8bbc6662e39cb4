"""Pins for the oracle with pickups (VRPSPDTW, no GPU).

With a pickup amount per customer the vehicle leaves the depot with all of
its route's deliveries and, at each customer, unloads the delivery and loads
the pickup; capacity holds when the largest load over the route does not
exceed it (Section 2; Section 4.3.2 load attributes).  Pinned by the paper's
load concatenation rules (L_I, L_O, L_M) implemented here separately, by a
hand-computed route, by zero pickups reducing to the delivery-only oracle,
by the reversal symmetry (a route driven backwards with deliveries and
pickups exchanged has the same largest load), and by brute force over an
independent neighbour enumeration in hard and penalised mode.
"""
import numpy as np
import pytest

import oracle
from paper_2506_17357_amd import workload as W
from tests import brute


def concat_load(a, b):
    """Section 4.3.2: (L_I, L_O, L_M) of a followed by b."""
    return (a[0] + b[0], a[1] + b[1], max(a[2] + b[0], a[1] + b[2]))


def peak_by_concatenation(dem, pick, route):
    s = (0, 0, 0)  # the depot: no delivery, no pickup
    for c in list(route) + [0]:
        s = concat_load(s, (int(dem[c]), int(pick[c]), max(int(dem[c]), int(pick[c]))))
    return s[2]


def with_pickups(inst, seed, hi=10):
    rng = np.random.default_rng(seed)
    inst.pickup = np.zeros(inst.n + 1, np.int32)
    inst.pickup[1:] = rng.integers(0, hi, size=inst.n)
    return inst


def test_hand_computed_route():
    """Capacity 10; customers 1, 2, 3 deliver 4, 2, 3 and pick up 1, 6, 5.
    [1, 2, 3]: leaves with 9; after 1: 6; after 2: 10; after 3: 12 -> peak 12.
    [2, 1, 3]: 9; after 2: 13 -> peak 13.  [3, 1, 2]: 9; after 3: 11; after 1:
    8; after 2: 12 -> peak 12.  [1, 3, 2]: 9, 6, 8, 12 -> peak 12.  With
    capacity 12 the excess is 0, 1, 0, 0."""
    inst = W.tiny_instance(3, 5, False, capacity=12)
    inst.node4[1:, 0] = (4, 2, 3)
    inst.pickup = np.array([0, 1, 6, 5], np.int32)
    for route, exc in (([1, 2, 3], 0), ([2, 1, 3], 1), ([3, 1, 2], 0), ([1, 3, 2], 0)):
        sol = W.Solution.from_routes([route])
        assert oracle.violations(inst, sol)[0] == exc, route
        assert W.peak_load(inst, route) - 12 == exc


def test_peak_load_equals_concatenation_rules():
    rng = np.random.default_rng(3)
    for seed in range(100):
        inst = with_pickups(W.tiny_instance(12, 40 + seed, False, capacity=1), seed)
        sol = W.random_solution(inst, 3, seed)
        exp = 0
        for r in range(sol.R):
            route = sol.customers[sol.offsets[r]:sol.offsets[r + 1]]
            exp += max(peak_by_concatenation(inst.node4[:, 0], inst.pickup, route) - inst.capacity, 0)
        assert oracle.violations(inst, sol)[0] == exp, seed


def test_reversal_symmetry():
    """Driving a route backwards with deliveries and pickups exchanged gives
    the same largest load."""
    for seed in range(30):
        inst = with_pickups(W.tiny_instance(15, 70 + seed, False, capacity=1), seed)
        mirror = W.tiny_instance(15, 70 + seed, False, capacity=1)
        mirror.node4[:, 0] = inst.pickup
        mirror.pickup = inst.node4[:, 0].astype(np.int32).copy()
        sol = W.random_solution(inst, 1, seed)
        rev = W.Solution(sol.offsets, sol.customers[::-1].copy())
        assert oracle.violations(inst, sol)[0] == oracle.violations(mirror, rev)[0]


def test_zero_pickups_equal_delivery_only():
    inst = W.tiny_instance(40, 9, True, span=300)
    sol = W.random_solution(inst, 5, 10)
    b0, d0, f0 = oracle.eval_neighbourhood(inst, sol, dump=True, threads=2)
    inst.pickup = np.zeros(inst.n + 1, np.int32)
    b1, d1, f1 = oracle.eval_neighbourhood(inst, sol, dump=True, threads=2)
    assert np.array_equal(d0, d1) and np.array_equal(f0, f1) and (b0.delta, b0.id) == (b1.delta, b1.id)


@pytest.mark.parametrize("has_tw", [0, 1])
@pytest.mark.parametrize("n,R", [(4, 1), (6, 2), (7, 3)])
def test_brute_force_hard_and_penalised(has_tw, n, R):
    inst = with_pickups(W.tiny_instance(n, 500 + n + R + has_tw, bool(has_tw)), n + R, hi=8)
    inst.capacity = int(inst.node4[:, 0].sum() // 2 + 2)
    sol = W.random_solution(inst, R, 600 + n + R)
    routes = [list(map(int, sol.customers[sol.offsets[r]:sol.offsets[r + 1]])) for r in range(R)]

    def cap_ok(r):
        return W.peak_load(inst, r) <= inst.capacity

    base_d = brute.total_cost(inst, routes)
    best, dd, df = oracle.eval_neighbourhood(inst, sol, dump=True, threads=1)
    exp = None
    for mid, new, touched in brute.neighbours(inst, routes):
        delta = brute.total_cost(inst, new) - base_d
        feas = int(all(cap_ok(new[r]) for r in touched)) | (int(all(brute.route_ok_tw(inst, new[r]) for r in touched)) << 1)
        assert (int(dd[mid]), int(df[mid])) == (delta, feas), mid
        if feas == 3 and (exp is None or (delta, mid) < exp):
            exp = (delta, mid)
    assert best.found == (exp is not None) and (not best.found or (best.delta, best.id) == exp)
    # penalised: load excess from the peak load; time warp unchanged by pickups
    w = (3, 2 if has_tw else 0)

    # time warp does not depend on loads: take it from the oracle without pickups (pinned elsewhere)
    inst_no_pick = W.Instance(inst.n, inst.dist, inst.node4, inst.capacity, inst.has_tw, inst.xy, "tiny", 0)

    def F(rs):
        lv = sum(max(W.peak_load(inst, r) - inst.capacity, 0) for r in rs)
        tv = oracle.violations(inst_no_pick, W.Solution.from_routes(rs))[1]
        return brute.total_cost(inst, rs) + w[0] * lv + w[1] * tv

    base = F(routes)
    _, sd, _ = oracle.eval_neighbourhood(inst, sol, dump=True, threads=1, penalty=w)
    for mid, new, touched in brute.neighbours(inst, routes):
        assert int(sd[mid]) == F(new) - base, mid


def test_pickup_local_search_descends():
    inst, sol = W.c6(150)
    final, ids, deltas, mv = oracle.local_search(inst, sol, max_steps=300)
    assert len(ids) > 10 and (deltas < 0).all()
    assert oracle.violations(inst, final) == (0, 0)
    assert oracle.cost(inst, final)[0] == oracle.cost(inst, sol)[0] + int(deltas.sum())
