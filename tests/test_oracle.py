"""Pins for the CPU oracle (no GPU).

The oracle is checked against things other than itself: an independent
brute-force enumerator, a hand-computed example, textbook closed-form deltas,
the move-count formula, inverse moves, whole-solution recomputation,
exhaustive global optima, and relaxations that reduce VRPTW to CVRP.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2506_17357_amd import workload as W
from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden_case(name):
    with open(os.path.join(GOLDEN, name)) as f:
        g = json.load(f)
    inst = W.Instance(g["n"], np.asarray(g["dist"], np.int32), np.asarray(g["node4"], np.int32),
                      g["capacity"], g["has_tw"], np.zeros((g["n"] + 1, 2), np.int64), "golden", 0)
    return g, inst, W.Solution.from_routes(g["routes"])


def move_count(sol, n):
    """|N(S)| by the closed count formula of the canonical move space."""
    L = np.diff(sol.offsets).astype(np.int64)
    R = len(L)
    Q = n + R
    reloc = int((L * (Q - L - 1)).sum())
    swap = n * (n - 1) // 2
    two_star = (Q * Q - int(((L + 1) ** 2).sum())) // 2
    two_opt = int((L * (L - 1) // 2).sum())
    oropt = 0
    for l in L:
        for k in (1, 2, 3):
            if k <= l:
                oropt += int((l - k + 1) * (l - k))
    return reloc + swap + two_star + two_opt + oropt


# ------------------------------------------------------------ golden ------

def test_golden_line4_hand_computed():
    g, inst, sol = golden_case("line4_vrptw.json")
    assert oracle.cost(inst, sol)[0] == g["expected_cost"]
    best, dd, df = oracle.eval_neighbourhood(inst, sol, dump=True, threads=1)
    assert best.moves == g["expected_moves"]
    assert int((df != oracle.NOT_A_MOVE).sum()) == g["expected_moves"]
    for m in g["moves"]:
        assert (int(dd[m["id"]]), int(df[m["id"]])) == (m["delta"], m["feas"]), m["why"]
    assert best.found and (best.delta, best.id) == (g["expected_best"]["delta"], g["expected_best"]["id"])


# ------------------------------------------------------------ brute -------

def _cases():
    out = []
    seed = 0
    for has_tw in (False, True):
        for n in range(1, 8):
            for R in (1, 2, 3):
                seed += 1
                out.append((n, R, has_tw, seed))
    return out


@pytest.mark.parametrize("n,R,has_tw,seed", _cases())
def test_oracle_equals_brute_force(n, R, has_tw, seed):
    inst = W.tiny_instance(n, seed, has_tw, dup=(seed % 3 == 0))
    sol = W.random_solution(inst, R, seed + 1000)
    bf = brute.evaluate_all(inst, sol.routes())
    best, dd, df = oracle.eval_neighbourhood(inst, sol, dump=True, threads=2)
    ids = set(np.nonzero(df != oracle.NOT_A_MOVE)[0].tolist())
    assert ids == set(bf.keys())
    for mid, (delta, feas, _) in bf.items():
        assert (int(dd[mid]), int(df[mid])) == (delta, feas), (mid, oracle.decode(n + R, mid))
    assert best.moves == len(bf) == move_count(sol, n)
    adm = [(d, m) for m, (d, f, _) in bf.items() if f == 3]
    if adm:
        assert best.found and (best.delta, best.id) == min(adm)
    else:
        assert not best.found


@pytest.mark.parametrize("op_bit", [1, 2, 4, 8, 16])
def test_op_mask_restricts(op_bit):
    inst = W.tiny_instance(6, 77, True)
    sol = W.random_solution(inst, 3, 78)
    bf = brute.evaluate_all(inst, sol.routes(), op_mask=op_bit)
    best, dd, df = oracle.eval_neighbourhood(inst, sol, op_mask=op_bit, dump=True, threads=1)
    assert set(np.nonzero(df != oracle.NOT_A_MOVE)[0].tolist()) == set(bf.keys())
    adm = [(d, m) for m, (d, f, _) in bf.items() if f == 3]
    assert best.found == bool(adm)
    if adm:
        assert (best.delta, best.id) == min(adm)


# ------------------------------------------------------- closed forms -----

def _pos_table(sol, n):
    R = sol.R
    seq = {}
    for r, lst in enumerate(sol.routes()):
        seq[r] = [0] + lst + [0]
    where = {}
    for r in range(R):
        for p, c in enumerate(seq[r][1:-1], start=1):
            where[c] = (r, p)
    return seq, where


@pytest.mark.parametrize("seed", range(6))
def test_textbook_deltas(seed):
    """Delta of each operator from the classical edge-exchange formulas."""
    n, R = 30, 4
    inst = W.tiny_instance(n, 500 + seed, False, span=1000)
    sol = W.random_solution(inst, R, 600 + seed)
    D = inst.dist.astype(np.int64)
    Q = n + R
    _, dd, df = oracle.eval_neighbourhood(inst, sol, dump=True, threads=2)
    seq, where = _pos_table(sol, n)

    def mid(op, k, a, b):
        return ((op * 4 + k) * Q + a) * Q + b

    def ref_at(r, p):
        return n + r if p == 0 else seq[r][p] - 1

    checked = 0
    for u in range(1, n + 1):
        r1, i = where[u]
        p, w = seq[r1][i - 1], seq[r1][i + 1]
        for r2 in range(R):
            if r2 == r1:
                continue
            for j in range(len(seq[r2]) - 1):
                v, vn = seq[r2][j], seq[r2][j + 1]
                exp = D[p, w] - D[p, u] - D[u, w] + D[v, u] + D[u, vn] - D[v, vn]
                assert dd[mid(0, 1, u - 1, ref_at(r2, j))] == exp
                checked += 1
    for u in range(1, n + 1):
        for v in range(u + 1, n + 1):
            (ru, i), (rv, j) = where[u], where[v]
            pu, wu = seq[ru][i - 1], seq[ru][i + 1]
            pv, wv = seq[rv][j - 1], seq[rv][j + 1]
            if ru == rv and abs(i - j) == 1:
                if j < i:
                    u2, v2, pu2, wv2 = v, u, pv, wu
                else:
                    u2, v2, pu2, wv2 = u, v, pu, wv
                exp = D[pu2, v2] + D[u2, wv2] - D[pu2, u2] - D[v2, wv2]
            else:
                exp = (D[pu, v] + D[v, wu] + D[pv, u] + D[u, wv]
                       - D[pu, u] - D[u, wu] - D[pv, v] - D[v, wv])
            assert dd[mid(1, 1, u - 1, v - 1)] == exp
            checked += 1
    for r1 in range(R):
        for r2 in range(r1 + 1, R):
            for i in range(len(seq[r1]) - 1):
                for j in range(len(seq[r2]) - 1):
                    x, wx = seq[r1][i], seq[r1][i + 1]
                    y, wy = seq[r2][j], seq[r2][j + 1]
                    exp = D[x, wy] + D[y, wx] - D[x, wx] - D[y, wy]
                    a, b = sorted((ref_at(r1, i), ref_at(r2, j)))
                    assert dd[mid(2, 0, a, b)] == exp
                    checked += 1
    for r in range(R):
        s = seq[r]
        L = len(s) - 2
        for i in range(1, L + 1):
            for j in range(i + 1, L + 1):
                exp = D[s[i - 1], s[j]] + D[s[i], s[j + 1]] - D[s[i - 1], s[i]] - D[s[j], s[j + 1]]
                a, b = sorted((s[i] - 1, s[j] - 1))
                assert dd[mid(3, 0, a, b)] == exp
                checked += 1
        for k in (1, 2, 3):
            for i in range(1, L - k + 2):
                f, g = s[i], s[i + k - 1]
                p, w = s[i - 1], s[i + k]
                for j in range(0, L + 1):
                    if i - 1 <= j <= i + k - 1:
                        continue
                    v, vn = s[j], s[j + 1]
                    exp = D[p, w] - D[p, f] - D[g, w] + D[v, f] + D[g, vn] - D[v, vn]
                    assert dd[mid(4, k, f - 1, ref_at(r, j))] == exp
                    checked += 1
    assert checked == move_count(sol, n)


# ------------------------------------------------------------ invariants --

def _inverse(inst, sol, mid):
    n = inst.n
    Q = n + sol.R
    op, k, a, b = oracle.decode(Q, mid)
    seq, where = _pos_table(sol, n)
    if op == 0:
        r, p = where[a + 1]
        pred = n + r if p == 1 else seq[r][p - 1] - 1
        return ((0 * 4 + 1) * Q + a) * Q + pred
    if op in (1, 2, 3):
        return mid
    r, p = where[a + 1]
    pred = n + r if p == 1 else seq[r][p - 1] - 1
    return ((4 * 4 + k) * Q + a) * Q + pred


@pytest.mark.parametrize("has_tw", [False, True])
def test_move_then_inverse(has_tw):
    inst = W.tiny_instance(12, 31 + has_tw, has_tw)
    sol = W.random_solution(inst, 3, 32)
    _, dd, df = oracle.eval_neighbourhood(inst, sol, dump=True, threads=2)
    ids = np.nonzero(df != oracle.NOT_A_MOVE)[0]
    rng = np.random.default_rng(5)
    for mid in rng.choice(ids, size=min(300, ids.size), replace=False):
        s1 = oracle.apply_move(inst, sol, int(mid))
        inv = _inverse(inst, sol, int(mid))
        _, dd1, df1 = oracle.eval_neighbourhood(inst, s1, dump=True, threads=1)
        assert df1[inv] != oracle.NOT_A_MOVE
        assert int(dd[mid]) + int(dd1[inv]) == 0
        s2 = oracle.apply_move(inst, s1, inv)
        assert s2.routes() == sol.routes()


@pytest.mark.parametrize("has_tw", [False, True])
def test_delta_equals_full_recompute(has_tw):
    inst = W.tiny_instance(25, 41 + has_tw, has_tw)
    sol = W.random_solution(inst, 4, 42)
    _, dd, df = oracle.eval_neighbourhood(inst, sol, dump=True, threads=2)
    assert oracle.check_full(inst, sol, dd, df) == 0


def test_capacity_infinite_all_bit0():
    inst = W.tiny_instance(20, 9, True, capacity=10 ** 6)
    sol = W.random_solution(inst, 3, 10)
    _, dd, df = oracle.eval_neighbourhood(inst, sol, dump=True, threads=2)
    mv = df[df != oracle.NOT_A_MOVE]
    assert np.all(mv & 1)


def test_capacity_at_max_load_blocks_load_increase():
    inst = W.tiny_instance(20, 19, False)
    sol = W.random_solution(inst, 3, 20)
    loads = [int(inst.node4[r, 0].sum()) for r in sol.routes()]
    inst.capacity = max(loads)
    rmax = int(np.argmax(loads))
    n, Q = inst.n, inst.n + sol.R
    _, dd, df = oracle.eval_neighbourhood(inst, sol, dump=True, threads=1)
    seq, where = _pos_table(sol, n)
    for u in range(1, n + 1):
        if where[u][0] == rmax:
            continue
        for j in range(len(seq[rmax]) - 1):
            b = n + rmax if j == 0 else seq[rmax][j] - 1
            assert df[((0 * 4 + 1) * Q + u - 1) * Q + b] & 1 == 0


def test_relaxed_windows_reduce_to_cvrp():
    base = W.tiny_instance(15, 61, True)
    sol = W.random_solution(base, 3, 62)
    relaxed = W.Instance(base.n, base.dist, base.node4.copy(), base.capacity, 1, base.xy, "r", 0)
    relaxed.node4[:, 1] = 0
    relaxed.node4[:, 2] = 1 << 26
    cvrp = W.Instance(base.n, base.dist, base.node4.copy(), base.capacity, 0, base.xy, "c", 0)
    b1, d1, f1 = oracle.eval_neighbourhood(relaxed, sol, dump=True, threads=1)
    b2, d2, f2 = oracle.eval_neighbourhood(cvrp, sol, dump=True, threads=1)
    mv = f1 != oracle.NOT_A_MOVE
    assert np.all(f1[mv] & 2) and np.array_equal(d1, d2) and np.array_equal(f1, f2)
    assert (b1.delta, b1.id) == (b2.delta, b2.id)


def test_tight_window_blocks_earlier_insertion():
    """A node reached exactly at its due time: any insertion before it that
    adds travel time makes its route infeasible."""
    g, inst, sol = golden_case("line4_vrptw.json")
    _, dd, df = oracle.eval_neighbourhood(inst, sol, dump=True, threads=1)
    n, Q = 4, 6
    # relocating 4 to before 3 in slot 0 (after depot, 1 or 2) breaks 3's window
    for b in (4, 0, 1):
        assert df[((0 * 4 + 1) * Q + 3) * Q + b] & 2 == 0


def test_removal_can_break_windows_without_triangle_inequality():
    """Rounded distances need not satisfy the triangle inequality, so removing
    a node can make its route late.  Hand-built: route [2, 1] reaches 1 at
    time 2 through 2; without 2 the direct edge 0 -> 1 costs 30 and misses
    1's due time 10."""
    D = np.array([[0, 30, 1], [30, 0, 1], [1, 1, 0]], np.int32)
    node4 = np.array([[0, 0, 1000, 0], [1, 0, 10, 0], [1, 0, 100, 0]], np.int32)
    inst = W.Instance(2, D, node4, 10, 1, np.zeros((3, 2), np.int64), "tri", 0)
    sol = W.Solution.from_routes([[2, 1], []])
    _, dd, df = oracle.eval_neighbourhood(inst, sol, dump=True, threads=1)
    Q = 4
    mid = ((0 * 4 + 1) * Q + 1) * Q + 3  # relocate customer 2 (ref 1) into slot 1
    assert df[mid] == 1  # capacity holds, windows fail
    # slot 0 becomes [1] (30 + 30), slot 1 becomes [2] (1 + 1); before: 1 + 1 + 30
    assert dd[mid] == (30 + 30) + (1 + 1) - (1 + 1 + 30)


# --------------------------------------------------------- optimality -----

@pytest.mark.parametrize("has_tw,seed", [(False, 1), (False, 2), (True, 3), (True, 4)])
def test_no_improving_move_at_global_optimum(has_tw, seed):
    inst = W.tiny_instance(6, 900 + seed, has_tw)
    inst.capacity = int(inst.node4[:, 0].sum())  # every customer fits one vehicle
    opt = brute.global_optimum(inst, 2)
    if opt is None:
        pytest.skip("no feasible solution for this seed")
    cost, routes = opt
    sol = W.Solution.from_routes(routes)
    best = oracle.eval_neighbourhood(inst, sol, threads=1)
    assert best.found and best.delta >= 0
    start = W.random_solution(inst, 2, seed)
    final, ids, deltas, _ = oracle.local_search(inst, start, max_steps=200, threads=1)
    c0 = oracle.cost(inst, start)[0]
    c1 = oracle.cost(inst, final)[0]
    assert c1 == c0 + int(deltas.sum())
    assert np.all(deltas < 0)
    if oracle.cost(inst, start)[1:] == (0, 0):
        assert c1 >= cost
    bf = brute.evaluate_all(inst, final.routes())
    assert not any(d < 0 and f == 3 for d, f, _ in bf.values())


def test_ties_resolved_by_lowest_id():
    """Duplicate coordinates create exact ties; the oracle returns the
    smallest id among the minimal admissible deltas, found by brute force."""
    for seed in range(20):
        inst = W.tiny_instance(7, 300 + seed, seed % 2 == 1, dup=True, span=20)
        sol = W.random_solution(inst, 2, 400 + seed)
        bf = brute.evaluate_all(inst, sol.routes())
        adm = sorted((d, m) for m, (d, f, _) in bf.items() if f == 3)
        best = oracle.eval_neighbourhood(inst, sol, threads=3)
        if not adm:
            assert not best.found
            continue
        assert (best.delta, best.id) == adm[0]


def test_local_search_c1_monotone():
    inst, sol = W.c1()
    final, ids, deltas, mv = oracle.local_search(inst, sol, max_steps=100, threads=4)
    c0 = oracle.cost(inst, sol)[0]
    c1, cb, tb = oracle.cost(inst, final)
    assert len(ids) > 0 and np.all(deltas < 0)
    assert c1 == c0 + int(deltas.sum())
    assert cb == 0 and tb == 0


def test_threads_do_not_change_result():
    inst, sol = W.c1()
    a = oracle.eval_neighbourhood(inst, sol, threads=1, dump=True)
    b = oracle.eval_neighbourhood(inst, sol, threads=7, dump=True)
    assert (a[0].delta, a[0].id, a[0].moves) == (b[0].delta, b[0].id, b[0].moves)
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


@pytest.mark.parametrize("has_tw", [0, 1])
@pytest.mark.parametrize("n,R,mask", [(5, 2, 0x1F), (6, 3, 0x1F), (7, 3, 0xFF)])
def test_apply_equals_brute_force_routes(has_tw, n, R, mask):
    """The oracle's list edits give, for every move of N(S), exactly the new
    routes the independent brute-force enumerator builds."""
    import itertools
    inst = W.tiny_instance(n, 4100 + n + R + has_tw, bool(has_tw))
    sol = W.random_solution(inst, R, 4200 + n + R)
    routes = [list(map(int, sol.customers[sol.offsets[r]:sol.offsets[r + 1]])) for r in range(R)]
    gen = itertools.chain(brute.neighbours(inst, routes, mask & 0x1F), brute.neighbours_ext(inst, routes, mask))
    count = 0
    for mid, new, _ in gen:
        got = oracle.apply_move(inst, sol, int(mid)).routes()
        assert got == [list(r) for r in new], (mid, oracle.decode(n + R, mid))
        count += 1
    assert count > 20
