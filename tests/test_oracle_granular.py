"""Pins for the oracle's granular mode (no GPU): the edge-based neighbourhood
reduction (Section 5.3.1 edge-based extraction; granularity threshold theta
of the experiments) restricts inter-route moves to pairs of nodes where one
is among the theta closest to the other; intra-route moves stay complete.

Pinned by an independent pure-Python selection of the theta nearest
neighbours and filter of the brute-force enumeration, by theta >= n giving
the full neighbourhood, and by the count of moves the pairs generate.
"""
import numpy as np
import pytest

import oracle
from paper_2506_17357_amd import workload as W
from tests import brute


def python_mask(inst, theta):
    N = inst.n + 1
    M = np.zeros((N, N), bool)
    for i in range(N):
        others = sorted((int(inst.dist[i][j]), j) for j in range(N) if j != i)
        for _, j in others[:theta]:
            M[i, j] = M[j, i] = True
    return M


def node_of_ref(n, ref):
    return ref + 1 if ref < n else 0


@pytest.mark.parametrize("has_tw", [0, 1])
@pytest.mark.parametrize("n,R,theta", [(5, 2, 1), (6, 3, 2), (7, 2, 3), (7, 3, 1), (8, 4, 2)])
def test_granular_equals_filtered_brute_force(has_tw, n, R, theta):
    inst = W.tiny_instance(n, 300 + n * 7 + R + theta, bool(has_tw), dup=(n % 2 == 0))
    sol = W.random_solution(inst, R, 400 + n + R)
    routes = [list(map(int, sol.customers[sol.offsets[r]:sol.offsets[r + 1]])) for r in range(R)]
    M = python_mask(inst, theta)
    assert np.array_equal(oracle.granular_mask(inst, theta).astype(bool), M)
    Q = n + R
    ref = brute.evaluate_all(inst, routes)
    best, dd, df = oracle.eval_neighbourhood(inst, sol, dump=True, threads=1, theta=theta)
    kept = {}
    for mid, (delta, feas, _) in ref.items():
        op, k, a, b = oracle.decode(Q, mid)
        ra = routes.index(next(r for r in routes if (a + 1) in r)) if a < n else a - n
        rb = routes.index(next(r for r in routes if (b + 1) in r)) if b < n else b - n
        inter = op in (0, 2) or (op == 1 and ra != rb)
        if inter and not M[node_of_ref(n, a), node_of_ref(n, b)]:
            continue
        kept[mid] = (delta, feas)
    got = {int(i) for i in np.nonzero(df != oracle.NOT_A_MOVE)[0]}
    assert got == set(kept)
    for mid, (delta, feas) in kept.items():
        assert (int(dd[mid]), int(df[mid])) == (delta, feas), mid
    adm = [(d, m) for m, (d, f) in kept.items() if f == 3]
    assert best.found == bool(adm) and best.moves == len(kept)
    if adm:
        assert (best.delta, best.id) == min(adm)


def test_theta_at_least_n_is_the_full_neighbourhood():
    """Every pair of distinct nodes is kept; the only moves left out are the
    2-opt* exchanges of two whole routes (two start depots: the depot is not
    its own neighbour), which change nothing (delta 0)."""
    inst = W.tiny_instance(30, 5, True, span=300)
    sol = W.random_solution(inst, 4, 6)
    n, R = inst.n, sol.R
    Q = n + R
    b0, d0, f0 = oracle.eval_neighbourhood(inst, sol, dump=True, threads=2)
    b1, d1, f1 = oracle.eval_neighbourhood(inst, sol, dump=True, threads=2, theta=inst.n)
    depot_pairs = [(8 * Q + a) * Q + b for a in range(n, Q) for b in range(a + 1, Q)]
    assert all(d0[i] == 0 and f1[i] == oracle.NOT_A_MOVE for i in depot_pairs)
    f1[depot_pairs] = f0[depot_pairs]
    assert np.array_equal(d0, d1) and np.array_equal(f0, f1) and (b0.delta, b0.id) == (b1.delta, b1.id)


def test_granular_move_count():
    """|N_theta(S)|: per kept pair {u, v} of nodes in different routes, the
    relocations of each customer, the swap of two customers and the 2-opt*
    (a depot node stands for the start depot of every other route), plus
    the complete intra-route neighbourhoods."""
    inst = W.make_cvrp(200, 9)
    sol = W.sweep(inst)
    theta = 10
    M = python_mask(inst, theta)
    n, R = inst.n, sol.R
    route = np.zeros(n + 1, int)
    for r in range(R):
        route[sol.customers[sol.offsets[r]:sol.offsets[r + 1]]] = r
    count = 0
    for u in range(1, n + 1):
        for v in range(u + 1, n + 1):
            if M[u, v] and route[u] != route[v]:
                count += 4  # relocate u, relocate v, swap, 2-opt*
        if M[u, 0]:
            count += 2 * (R - 1)  # relocate u after another start depot; 2-opt* with it
    L = np.diff(sol.offsets).astype(int)
    count += int((L * (L - 1) // 2).sum())  # same-route swaps
    count += int((L * (L - 1) // 2).sum())  # 2-opt
    count += sum((l - k + 1) * (l - k) for l in L for k in (1, 2, 3) if k <= l)  # or-opt
    best = oracle.eval_neighbourhood(inst, sol, theta=theta)
    assert best.moves == count


def test_granular_local_search_descends():
    inst = W.make_vrptw(150, 7)
    sol = W.sweep(inst)
    final, ids, deltas, mv = oracle.local_search(inst, sol, max_steps=500, theta=20)
    assert len(ids) > 10 and (deltas < 0).all()
    assert oracle.cost(inst, final)[0] == oracle.cost(inst, sol)[0] + int(deltas.sum())
    b = oracle.eval_neighbourhood(inst, final, theta=20)
    assert not b.found or b.delta >= 0
