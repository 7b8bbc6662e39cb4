"""Batched form: one persistent launch per step over many solutions of
uneven sizes, CVRP and VRPTW mixed, the step loop captured in a HIP graph.
Each solution's result must equal its plain (one-solution-per-launch) result
and the oracle's."""
import numpy as np
import pytest

import oracle
from paper_2506_17357_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tga():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_17357_amd import tga as T
    T.lib()
    print("device limits", T.device_limits(), flush=True)
    return T


def small_mix(count=10, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        n = int(rng.integers(20, 260))
        inst = W.make_cvrp(n, 100 + b) if b % 2 == 0 else W.make_vrptw(n, 100 + b)
        out.append((inst, W.sweep(inst)))
    return out


def make_solutions(T, pairs):
    insts = [T.Instance.from_workload(i) for i, _ in pairs]
    sols = [T.Solution(I, s.offsets, s.customers) for I, (_, s) in zip(insts, pairs)]
    return insts, sols


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_ls_equals_oracle(tga, use_graph):
    pairs = small_mix()
    insts, sols = make_solutions(tga, pairs)
    B = tga.Batch(sols)
    steps, moves, cost = B.ls_run(40, use_graph=use_graph)
    for b, (inst, sol) in enumerate(pairs):
        final, ids, deltas, mv = oracle.local_search(inst, sol, max_steps=40)
        assert steps[b] == len(ids), b
        assert cost[b] == oracle.cost(inst, final)[0], b
        assert moves[b] == mv, b
    B.close()
    for b, s in enumerate(sols):
        off, cust, c = s.get()
        ref, _, _, _ = oracle.local_search(pairs[b][0], pairs[b][1], max_steps=40)
        assert off.tolist() == ref.offsets.tolist() and cust.tolist() == ref.customers.tolist()


def test_batch_mixed_distance_widths(tga):
    """Solutions whose matrices stream at 16 and at 32 bits share a launch."""
    pairs = small_mix(6, seed=5)
    for k in range(3):
        inst = W.tiny_instance(150 + 40 * k, 930 + k, bool(k % 2), span=100000)
        pairs.append((inst, W.random_solution(inst, 6 + k, 940 + k)))
    insts, sols = make_solutions(tga, pairs)
    assert sorted({I.dist_bytes for I in insts}) == [2, 4]
    B = tga.Batch(sols)
    steps, moves, cost = B.ls_run(25)
    B.close()
    for b, (inst, sol) in enumerate(pairs):
        final, ids, _, mv = oracle.local_search(inst, sol, max_steps=25)
        assert (steps[b], moves[b], cost[b]) == (len(ids), mv, oracle.cost(inst, final)[0]), b


def test_batch_graph_replay_and_reset(tga):
    """A captured graph replayed twice from fresh solutions gives the same
    result; begin/step_part/collect gives the same result too."""
    pairs = small_mix(6, seed=1)
    results = []
    for mode in ("graph", "graph", "parts"):
        insts, sols = make_solutions(tga, pairs)
        B = tga.Batch(sols)
        if mode == "graph":
            r = B.ls_run(30, use_graph=True)
        else:
            B.begin(30)
            for _ in range(30):
                B.step_part(0)
                B.step_part(1)
            r = B.collect()
        results.append(tuple(x.tolist() for x in r))
        B.close()
    assert results[0] == results[1] == results[2]


def test_batch_eval_equals_single(tga):
    pairs = small_mix(8, seed=2)
    insts, sols = make_solutions(tga, pairs)
    B = tga.Batch(sols, rows_per_item=3, sub_rows=2)
    best, status = B.eval()
    for b, (inst, sol) in enumerate(pairs):
        ob = oracle.eval_neighbourhood(inst, sol)
        assert status[b] == (0 if ob.found else 1)
        if ob.found:
            assert (best[b].delta, best[b].id) == (ob.delta, ob.id), b


def test_batch_eval_after_ls_run(tga):
    """A record evaluation after a batched local search covers the converged
    solutions too and leaves their flags and counters as they were."""
    pairs = small_mix(8, seed=6)
    insts, sols = make_solutions(tga, pairs)
    B = tga.Batch(sols)
    steps, moves, cost = B.ls_run(600, use_graph=False)
    done = B.poll()
    assert done.all()
    best, status = B.eval()
    assert (B.poll() == done).all()
    assert B.collect()[0].tolist() == steps.tolist()
    for b, s in enumerate(sols):
        off, cust, _ = s.get()
        ob = oracle.eval_neighbourhood(pairs[b][0], W.Solution(off, cust))
        assert status[b] == (0 if ob.found else 1), b
        if ob.found:
            assert (best[b].delta, best[b].id) == (ob.delta, ob.id), b
            assert best[b].delta >= 0, b


@pytest.mark.parametrize("rows_per_item,sub_rows", [(1, 1), (2, 3), (5, 1), (0, 2), (7, 3), (0, 0), (100, 8)])
def test_schedule_does_not_change_results(tga, rows_per_item, sub_rows):
    pairs = small_mix(6, seed=3)
    insts, sols = make_solutions(tga, pairs)
    B = tga.Batch(sols, rows_per_item=rows_per_item, sub_rows=sub_rows)
    steps, moves, cost = B.ls_run(25, use_graph=False)
    for b, (inst, sol) in enumerate(pairs):
        final, ids, _, _ = oracle.local_search(inst, sol, max_steps=25)
        assert steps[b] == len(ids) and cost[b] == oracle.cost(inst, final)[0]


@pytest.mark.parametrize("lds_kb,split", [(40, 0), (52, 1), (78, 0), (79, 0), (24, 1)])
def test_config_does_not_change_results(tga, lds_kb, split):
    pairs = small_mix(6, seed=4)
    insts, sols = make_solutions(tga, pairs)
    B = tga.Batch(sols)
    B.set_config(lds_kb, split)
    c = B.config()
    assert (c["lds_kb"], c["split"]) == (lds_kb, split)
    steps, moves, cost = B.ls_run(25, use_graph=True)
    for b, (inst, sol) in enumerate(pairs):
        final, ids, _, mv = oracle.local_search(inst, sol, max_steps=25)
        assert (steps[b], moves[b], cost[b]) == (len(ids), mv, oracle.cost(inst, final)[0]), b


def test_autotune_picks_a_candidate_and_keeps_results(tga):
    pairs = small_mix(8, seed=6)
    insts, sols = make_solutions(tga, pairs)
    B = tga.Batch(sols)
    cfg = B.autotune(launches=2)
    print("autotuned", cfg, flush=True)
    whole = tga.device_limits()[1] // 1024  # the whole-LDS candidate (one workgroup per compute unit)
    assert cfg["lds_kb"] in (40, 52, 64, 78, 79, whole) and cfg["split"] in (0, 1) and cfg["us_per_eval"] > 0
    assert B.config() == cfg
    steps, moves, cost = B.ls_run(30)
    for b, (inst, sol) in enumerate(pairs):
        final, ids, _, mv = oracle.local_search(inst, sol, max_steps=30)
        assert (steps[b], moves[b], cost[b]) == (len(ids), mv, oracle.cost(inst, final)[0]), b
    with pytest.raises(tga.TGAError) as e:
        B.set_config(200, 0)
    assert e.value.code == tga.TGA_ERANGE
    assert B.config() == cfg


def test_full_batched_workload_sampled(tga):
    """The 256-solution mix (100..2000 customers) for 200 steps: every
    solution equals its plain form; a sample equals the oracle."""
    pairs = W.c4()
    insts, sols = make_solutions(tga, pairs)
    B = tga.Batch(sols)
    steps, moves, cost = B.ls_run(200, use_graph=True)
    B.close()
    finals = [s.get() for s in sols]
    print("batched: total steps", int(steps.sum()), "moves", int(moves.sum()), flush=True)
    # plain form on fresh copies
    _, plain = make_solutions(tga, pairs)
    for b, s in enumerate(plain):
        st, mv, c = s.ls_run(200)
        assert (st, mv, c) == (steps[b], moves[b], cost[b]), b
    ns = np.array([i.n for i, _ in pairs])
    sample = list(np.argsort(ns)[:6])
    for b in sample:
        inst, sol = pairs[b]
        final, ids, _, mv = oracle.local_search(inst, sol, max_steps=200)
        assert steps[b] == len(ids) and moves[b] == mv
        assert finals[b][0].tolist() == final.offsets.tolist()
        assert finals[b][1].tolist() == final.customers.tolist()


def test_slot_batch_members_come_and_go(tga):
    """A slot batch whose members are replaced while it runs (served form):
    every solution ends exactly where the oracle's local search ends, with
    the same counters, whatever slot it had and whoever it shared the
    launches with; empty slots are skipped."""
    import torch
    pairs = small_mix(9, seed=7)
    insts, sols = make_solutions(tga, pairs)
    caps = [15, 40, 7, 25, 60, 3, 33, 18, 50]
    B = tga.SlotBatch(4, 1 << 14, 1 << 10)
    members = [None] * 4
    queue = list(range(len(sols)))
    result = {}
    st = torch.cuda.current_stream()
    joined = {}
    ticks = 0
    while queue or any(m is not None for m in members):
        changed = False
        for k in range(4):
            if members[k] is None and queue and k != 2:  # slot 2 stays empty
                b = queue.pop(0)
                sols[b].begin(caps[b])
                members[k] = b
                joined[b] = ticks
                changed = True
        if changed:
            B.set_members([sols[b] if b is not None else None for b in members])
        t = B.tick(3)
        ticks += 1
        st.synchronize()
        tick, conv, steps, moves, cost = B.status()
        assert tick == t
        assert conv[2] == 1 and steps[2] == 0
        for k, b in enumerate(members):
            if b is not None and conv[k]:
                result[b] = (int(steps[k]), int(moves[k]), int(cost[k]))
                members[k] = None
                changed = True
        if changed:
            B.set_members([sols[b] if b is not None else None for b in members])
    st.synchronize()
    B.close()
    for b, (inst, sol) in enumerate(pairs):
        final, ids, _, mv = oracle.local_search(inst, sol, max_steps=caps[b])
        assert result[b] == (len(ids), mv, oracle.cost(inst, final)[0]), b
        off, cust, c = sols[b].get()
        assert off.tolist() == final.offsets.tolist() and cust.tolist() == final.customers.tolist(), b


def test_slot_batch_other_calls_skip_empty_slots(tga):
    pairs = small_mix(3, seed=8)
    insts, sols = make_solutions(tga, pairs)
    B = tga.SlotBatch(5, 1 << 12, 1 << 8)
    B.set_members([None, sols[0], None, sols[1], sols[2]])
    best, status = B.eval()
    assert status[0] == 1 and status[2] == 1
    for k, b in ((1, 0), (3, 1), (4, 2)):
        ob = oracle.eval_neighbourhood(*pairs[b])
        assert (best[k].delta, best[k].id) == (ob.delta, ob.id)
    steps, moves, cost = B.ls_run(12, use_graph=False)
    assert steps[0] == steps[2] == 0 and cost[0] == 0
    for k, b in ((1, 0), (3, 1), (4, 2)):
        final, ids, _, mv = oracle.local_search(*pairs[b], max_steps=12)
        assert (steps[k], moves[k], cost[k]) == (len(ids), mv, oracle.cost(pairs[b][0], final)[0])
    assert B.poll().tolist()[0] == 1
    B.close()


def inter_pairs(sol):
    """Slot pairs of different routes (start depots included as slots)."""
    P = np.diff(np.asarray(sol.offsets, np.int64)) + 1
    return (int(P.sum()) ** 2 - int((P * P).sum())) // 2


def screen_expectation(inst, sol, cap):
    """(pairs visited by the inter-route screens over the oracle's
    trajectory, accepted moves that are necessarily inter-route)."""
    _, ids, _, _ = oracle.local_search(inst, sol, max_steps=cap)
    Q = inst.n + sol.R
    evals = min(len(ids) + 1, cap)
    cur, visited, inter = sol, 0, 0
    for k in range(evals):
        visited += inter_pairs(cur)
        if k < len(ids):
            op = int(ids[k]) // (Q * Q) // 4
            inter += op in (0, 2)
            cur = oracle.apply_move(inst, cur, int(ids[k]))
    return visited, inter


@pytest.mark.parametrize("use_graph", [False, True])
def test_screen_counters(tga, use_graph):
    """The screening counters (the counting instantiation of the batched
    launch): pairs visited equal the slot pairs of different routes summed
    over the evaluated states of the oracle's trajectory; pairs evaluated in
    full cover at least every accepted inter-route move and stay a small
    share of the visited ones; the results are those without counting."""
    pairs = small_mix(6, seed=4)
    insts, sols = make_solutions(tga, pairs)
    B = tga.Batch(sols)
    plain = B.ls_run(40, use_graph=use_graph)
    assert B.screen_stats() == (0, 0)
    for s, (_, sol) in zip(sols, pairs):
        s.reload(sol.offsets, sol.customers)
    counted = B.ls_run(40, tga.OPS_ALL | tga.OP_COUNT_FULL, use_graph=use_graph)
    for a, b in zip(plain, counted):
        assert np.array_equal(a, b)
    full, visited = B.screen_stats()
    exp = [screen_expectation(i, s, 40) for i, s in pairs]
    assert visited == sum(v for v, _ in exp)
    assert sum(a for _, a in exp) <= full < visited // 4
    per = [s.screen_stats() for s in sols]
    assert (sum(f for f, _ in per), sum(v for _, v in per)) == (full, visited)
    assert [v for _, v in per] == [v for v, _ in exp]
    B.eval()  # a record-mode evaluation leaves the counters alone
    assert B.screen_stats() == (full, visited)
    B.close()
    inst, sol = W.c1()
    I = tga.Instance.from_workload(inst)
    S = tga.Solution(I, sol.offsets, sol.customers)
    with pytest.raises(tga.TGAError):
        S.ls_run(10, tga.OPS_ALL | tga.OP_COUNT_FULL)  # the batched form only
    B = tga.Batch([S])
    B.ls_run(1000, tga.OPS_ALL | tga.OP_COUNT_FULL)
    full, visited = B.screen_stats()
    v, a = screen_expectation(inst, sol, 1000)
    assert visited == v and a <= full < visited // 4
    B.close()


def shaped_solution(inst, lengths, seed):
    """The customers in random order, cut into routes of the given lengths."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(np.arange(1, inst.n + 1)).astype(np.int32)
    off = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int32)
    assert off[-1] == inst.n
    return W.Solution(off, perm)


def test_batch_intra_route_shapes(tga):
    """Route shapes that take every intra-route path of the batched launch:
    groups that fit their wavefront's LDS region (one cell per lane for CVRP,
    walks for VRPTW, empty routes among them), a group beyond the region's 64
    first positions (its routes staged one at a time), a route too long to
    stage (read from the slot arrays), and routes over capacity."""
    shapes = [[70], [38, 30, 12, 10, 10], [0, 14, 9, 0, 16, 11, 0, 10]]
    pairs = []
    for k, lens in enumerate(shapes):
        for tw in (False, True):
            inst = W.tiny_instance(sum(lens), 5100 + 10 * k + tw, tw)
            if k == 1:
                inst.capacity = int(inst.node4[:, 0].sum() // 3)
            pairs.append((inst, shaped_solution(inst, lens, 5200 + 10 * k + tw)))
    insts, sols = make_solutions(tga, pairs)
    print("intra-route shapes", [s.R for s in sols], flush=True)
    B = tga.Batch(sols)
    steps, moves, cost = B.ls_run(30)
    B.close()
    for b, (inst, sol) in enumerate(pairs):
        final, ids, _, mv = oracle.local_search(inst, sol, max_steps=30)
        assert (steps[b], moves[b], cost[b]) == (len(ids), mv, oracle.cost(inst, final)[0]), b
        off, cust, _ = sols[b].get()
        assert off.tolist() == final.offsets.tolist() and cust.tolist() == final.customers.tolist(), b
