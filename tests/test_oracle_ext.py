"""Pins for the oracle's operator variants (no GPU): inter-route segment
relocation of 2..3 nodes, kept (op 5) or reversed (op 6), and cross-exchange
of segments of 1..3 nodes (ops 7..9; Section 4.1 names segments of N > 1
nodes and reversal, Section 7 cross-exchange).  Pinned by an independent
brute-force enumeration by segment and insertion index, textbook
edge-exchange deltas, the move count and self-inverse exchanges."""
import numpy as np
import pytest

import oracle
from paper_2506_17357_amd import workload as W
from tests import brute


@pytest.mark.parametrize("has_tw", [0, 1])
@pytest.mark.parametrize("n,R", [(4, 2), (6, 2), (7, 3), (8, 3)])
def test_variants_equal_brute_force(has_tw, n, R):
    inst = W.tiny_instance(n, 800 + 3 * n + R + has_tw, bool(has_tw), dup=n % 2 == 0)
    sol = W.random_solution(inst, R, 850 + n + R)
    routes = [list(map(int, sol.customers[sol.offsets[r]:sol.offsets[r + 1]])) for r in range(R)]
    mask = 0xFF
    ref = brute.evaluate_all(inst, routes, mask)
    best, dd, df = oracle.eval_neighbourhood(inst, sol, mask, dump=True, threads=1)
    got = {int(i) for i in np.nonzero(df != oracle.NOT_A_MOVE)[0]}
    assert got == set(ref)
    for mid, (delta, feas, _) in ref.items():
        assert (int(dd[mid]), int(df[mid])) == (delta, feas), (mid, oracle.decode(n + R, mid))
    adm = [(d, m) for m, (d, f, _) in ref.items() if f == 3]
    assert best.found == bool(adm) and (not adm or (best.delta, best.id) == min(adm))
    assert best.moves == len(ref)


def test_textbook_deltas():
    """Segment f..g (pred p, succ w) inserted between v and v': kept adds
    c(v, f) + c(g, v'), reversed c(v, g) + c(f, v'); both remove c(p, f),
    c(g, w), c(v, v') and add c(p, w)."""
    inst = W.tiny_instance(12, 901, False, capacity=10 ** 6, span=500)
    sol = W.random_solution(inst, 3, 902)
    D = inst.dist
    n, R = inst.n, sol.R
    Q = n + R
    routes = [[0] + list(map(int, sol.customers[sol.offsets[r]:sol.offsets[r + 1]])) + [0] for r in range(R)]
    _, dd, df = oracle.eval_neighbourhood(inst, sol, 0x60, dump=True, threads=1)
    checked = 0
    for r1 in range(R):
        A = routes[r1]
        for k in (2, 3):
            for i in range(1, len(A) - k):
                p, f, g, w = A[i - 1], A[i], A[i + k - 1], A[i + k]
                for r2 in range(R):
                    if r2 == r1:
                        continue
                    B = routes[r2]
                    for j in range(len(B) - 1):
                        v, v2 = B[j], B[j + 1]
                        b = n + r2 if j == 0 else v - 1
                        common = D[p][w] - D[p][f] - D[g][w] - D[v][v2]
                        keep = common + D[v][f] + D[g][v2]
                        rev = common + D[v][g] + D[f][v2]
                        assert dd[((5 * 4 + k) * Q + f - 1) * Q + b] == keep
                        assert dd[((6 * 4 + k) * Q + f - 1) * Q + b] == rev
                        checked += 1
    assert checked > 50


def test_variant_counts():
    inst = W.make_cvrp(120, 9)
    sol = W.sweep(inst)
    n, R = inst.n, sol.R
    Q = n + R
    L = np.diff(sol.offsets).astype(int)
    route = np.zeros(n + 1, int)
    for r in range(R):
        route[sol.customers[sol.offsets[r]:sol.offsets[r + 1]]] = r
    pos = np.zeros(n + 1, int)
    for r in range(R):
        for q, c in enumerate(sol.customers[sol.offsets[r]:sol.offsets[r + 1]]):
            pos[c] = q + 1
    seg = sum(max(l - k + 1, 0) * (Q - l - 1) for l in L for k in (2, 3))
    cross = 0
    for a in range(1, n + 1):
        for b in range(a + 1, n + 1):
            if route[a] == route[b]:
                continue
            for ka in (1, 2, 3):
                for kb in (1, 2, 3):
                    if (ka, kb) != (1, 1) and pos[a] + ka - 1 <= L[route[a]] and pos[b] + kb - 1 <= L[route[b]]:
                        cross += 1
    assert oracle.eval_neighbourhood(inst, sol, 0x20).moves == seg
    assert oracle.eval_neighbourhood(inst, sol, 0x60).moves == 2 * seg
    assert oracle.eval_neighbourhood(inst, sol, 0x80).moves == cross


def test_cross_exchange_is_self_inverse():
    inst = W.tiny_instance(14, 911, True, span=300)
    sol = W.random_solution(inst, 3, 912)
    _, dd, df = oracle.eval_neighbourhood(inst, sol, 0x80, dump=True, threads=1)
    ids = np.nonzero(df != oracle.NOT_A_MOVE)[0]
    rng = np.random.default_rng(1)
    for mid in rng.choice(ids, size=min(60, ids.size), replace=False):
        s2 = oracle.apply_move(inst, sol, int(mid))
        _, d2, _ = oracle.eval_neighbourhood(inst, s2, 0x80, dump=True, threads=1)
        assert int(dd[mid]) + int(d2[mid]) == 0
        back = oracle.apply_move(inst, s2, int(mid))
        assert back.customers.tolist() == sol.customers.tolist()


def test_variant_local_search_descends():
    inst = W.make_vrptw(120, 13)
    sol = W.sweep(inst)
    final, ids, deltas, mv = oracle.local_search(inst, sol, 0xFF, max_steps=300)
    assert len(ids) > 10 and (deltas < 0).all()
    assert oracle.cost(inst, final)[0] == oracle.cost(inst, sol)[0] + int(deltas.sum())
    Q = inst.n + sol.R
    assert any(oracle.decode(Q, int(m))[0] >= 5 for m in ids)  # the variants take part
