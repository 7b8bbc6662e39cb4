"""Independent brute-force neighbour generator for tiny instances.

Pure Python, written separately from the C oracle: it enumerates neighbours by
insertion index / cut index rather than by ref, edits Python lists, and
computes cost and feasibility with its own functions.  Used only to pin the
oracle on tiny inputs.
"""
from __future__ import annotations

import itertools


def route_cost(D, r):
    seq = [0] + list(r) + [0]
    return sum(int(D[seq[i]][seq[i + 1]]) for i in range(len(seq) - 1))


def route_ok_cap(inst, r):
    return sum(int(inst.node4[c][0]) for c in r) <= inst.capacity


def route_ok_tw(inst, r):
    if not inst.has_tw:
        return True
    nd, D = inst.node4, inst.dist
    time = int(nd[0][1])
    prev = 0
    for c in r:
        arr = time + int(nd[prev][3]) + int(D[prev][c])
        if arr > int(nd[c][2]):
            return False
        time = max(arr, int(nd[c][1]))
        prev = c
    return time + int(nd[prev][3]) + int(D[prev][0]) <= int(nd[0][2])


def total_cost(inst, routes):
    return sum(route_cost(inst.dist, r) for r in routes)


def ref_of_customer(c):
    return c - 1


def neighbours(inst, routes, op_mask=0x1F):
    """Yield (id, new_routes, touched_slots) for every move of N(S)."""
    n = inst.n
    R = len(routes)
    Q = n + R

    def mid(op, k, a, b):
        return ((op * 4 + k) * Q + a) * Q + b

    def before_ref(r, lst, idx):
        # ref of the node right before insertion index idx of list lst in route r
        return n + r if idx == 0 else ref_of_customer(lst[idx - 1])

    where = {}
    for r, lst in enumerate(routes):
        for p, c in enumerate(lst):
            where[c] = (r, p)

    if op_mask & 1:  # relocate into another route, by insertion index
        for u in range(1, n + 1):
            r1, p1 = where[u]
            for r2 in range(R):
                if r2 == r1:
                    continue
                for idx in range(len(routes[r2]) + 1):
                    new = [list(x) for x in routes]
                    new[r1].remove(u)
                    b = before_ref(r2, routes[r2], idx)
                    new[r2].insert(idx, u)
                    yield mid(0, 1, u - 1, b), new, (r1, r2)
    if op_mask & 2:  # swap any two customers
        for u, v in itertools.combinations(range(1, n + 1), 2):
            new = [list(x) for x in routes]
            (ru, pu), (rv, pv) = where[u], where[v]
            new[ru][pu] = v
            new[rv][pv] = u
            yield mid(1, 1, u - 1, v - 1), new, tuple(sorted({ru, rv}))
    if op_mask & 4:  # 2-opt*: cut index i in route r1, j in route r2
        for r1, r2 in itertools.combinations(range(R), 2):
            A, B = routes[r1], routes[r2]
            for i in range(len(A) + 1):
                for j in range(len(B) + 1):
                    x = before_ref(r1, A, i)
                    y = before_ref(r2, B, j)
                    new = [list(t) for t in routes]
                    new[r1] = A[:i] + B[j:]
                    new[r2] = B[:j] + A[i:]
                    yield mid(2, 0, min(x, y), max(x, y)), new, (r1, r2)
    if op_mask & 8:  # 2-opt: reverse lst[i..j], i < j
        for r, lst in enumerate(routes):
            for i in range(len(lst)):
                for j in range(i + 1, len(lst)):
                    new = [list(t) for t in routes]
                    new[r] = lst[:i] + lst[i:j + 1][::-1] + lst[j + 1:]
                    a, b = sorted((lst[i] - 1, lst[j] - 1))
                    yield mid(3, 0, a, b), new, (r,)
    if op_mask & 16:  # or-opt: move a k-segment to right after another node
        for r, lst in enumerate(routes):
            for k in (1, 2, 3):
                for s in range(len(lst) - k + 1):
                    seg = lst[s:s + k]
                    rest = lst[:s] + lst[s + k:]
                    orig_pred = 0 if s == 0 else lst[s - 1]
                    for idx in range(len(rest) + 1):
                        pred = 0 if idx == 0 else rest[idx - 1]
                        if pred == orig_pred:
                            continue
                        new = [list(t) for t in routes]
                        new[r] = rest[:idx] + seg + rest[idx:]
                        b = n + r if idx == 0 else pred - 1
                        yield mid(4, k, seg[0] - 1, b), new, (r,)


def neighbours_ext(inst, routes, op_mask):
    """Operator variants (ops 5..9), enumerated by segment start index and
    insertion index: (id, new_routes, touched_slots)."""
    n = inst.n
    R = len(routes)
    Q = n + R

    def mid(op, k, a, b):
        return ((op * 4 + k) * Q + a) * Q + b

    for r1 in range(R):
        A = routes[r1]
        for k in (2, 3):
            for s0 in range(len(A) - k + 1):
                seg = A[s0:s0 + k]
                for r2 in range(R):
                    if r2 == r1:
                        continue
                    B = routes[r2]
                    for idx in range(len(B) + 1):
                        b = n + r2 if idx == 0 else B[idx - 1] - 1
                        for op, piece in ((5, seg), (6, seg[::-1])):
                            if not op_mask & (32 if op == 5 else 64):
                                continue
                            new = [list(x) for x in routes]
                            new[r1] = A[:s0] + A[s0 + k:]
                            new[r2] = B[:idx] + list(piece) + B[idx:]
                            yield mid(op, k, seg[0] - 1, b), new, (r1, r2)
    if op_mask & 128:
        for r1 in range(R):
            for r2 in range(R):
                if r1 == r2:
                    continue
                A, B = routes[r1], routes[r2]
                for i in range(len(A)):
                    for j in range(len(B)):
                        if A[i] >= B[j]:
                            continue  # the segment starting at the lower customer comes first
                        for ka in (1, 2, 3):
                            for kb in (1, 2, 3):
                                if (ka, kb) == (1, 1) or i + ka > len(A) or j + kb > len(B):
                                    continue
                                new = [list(x) for x in routes]
                                new[r1] = A[:i] + B[j:j + kb] + A[i + ka:]
                                new[r2] = B[:j] + A[i:i + ka] + B[j + kb:]
                                yield mid(6 + ka, kb, A[i] - 1, B[j] - 1), new, (r1, r2)


def evaluate_all(inst, routes, op_mask=0x1F):
    """dict id -> (delta, feas, new_routes)."""
    base = total_cost(inst, routes)
    out = {}
    gen = itertools.chain(neighbours(inst, routes, op_mask), neighbours_ext(inst, routes, op_mask))
    for mid, new, touched in gen:
        feas = 0
        if all(route_ok_cap(inst, new[r]) for r in touched):
            feas |= 1
        if all(route_ok_tw(inst, new[r]) for r in touched):
            feas |= 2
        assert mid not in out, "duplicate move id %d" % mid
        out[mid] = (total_cost(inst, new) - base, feas, new)
    return out


def all_solutions(n, R):
    """Every assignment of customers 1..n to R ordered route slots."""
    for perm in itertools.permutations(range(1, n + 1)):
        for cuts in itertools.combinations_with_replacement(range(n + 1), R - 1):
            bounds = (0,) + cuts + (n,)
            yield [list(perm[bounds[i]:bounds[i + 1]]) for i in range(R)]


def global_optimum(inst, R):
    """Cheapest fully feasible solution with R route slots (None if none)."""
    best = None
    for sol in all_solutions(inst.n, R):
        if not all(route_ok_cap(inst, r) and route_ok_tw(inst, r) for r in sol):
            continue
        c = total_cost(inst, sol)
        if best is None or c < best[0]:
            best = (c, sol)
    return best
