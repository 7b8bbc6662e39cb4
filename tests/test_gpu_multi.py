"""GPU parity of the multi-move step (several independent moves per
local-search iteration, Section 7): the selection after one evaluation and
whole multi-move local searches against the oracle, with hard feasibility,
penalties, pickups and the operator variants; the path that selects without
sorting (more improving route pairs than the sort holds).  Integer path, so
the bar is equality."""
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
    return T


def vrptw400():
    inst = W.make_vrptw(400, 2800)
    return inst, W.sweep(inst)


def gpu_multi(T, inst, sol, pen=None):
    I = T.Instance.from_workload(inst)
    S = T.Solution(I, sol.offsets, sol.customers)
    S.set_multi(True)
    if pen is not None:
        S.set_penalty(*pen)
    return I, S


def check_select(T, inst, sol, mask, pen=None, tag=""):
    print("multi select", tag, "n=%d R=%d mask=0x%x pen=%s" % (inst.n, sol.R, mask, pen), flush=True)
    I, S = gpu_multi(T, inst, sol, pen)
    ref, _ = oracle.multi_select(inst, sol, mask, penalty=pen)
    b = S.eval(mask | T.OP_MULTI)
    got = [(m.id, m.delta) for m in S.select_moves()]
    assert got == ref
    ob = oracle.eval_neighbourhood(inst, sol, mask, penalty=pen)
    assert (b is None) == (not ob.found)
    if b is not None:
        assert (b.delta, b.id) == (ob.delta, ob.id)
    return S


@pytest.mark.parametrize("which,mask,pen", [("c1", 0x1F, None), ("vrptw400", 0x1F, None), ("vrptw400", 0xFF, None),
                                            ("vrptw400", 0xFF, (5, 5)), ("c3", 0x1F, None)])
def test_select_matches_oracle(tga, which, mask, pen):
    inst, sol = W.c1() if which == "c1" else (W.c3() if which == "c3" else vrptw400())
    check_select(tga, inst, sol, mask, pen, which)


def test_select_pickups(tga):
    inst, sol = W.c6(300)
    check_select(tga, inst, sol, 0x1F, None, "pickups")
    check_select(tga, inst, sol, 0xFF, (5, 5), "pickups pen")


def test_select_random_solutions(tga):
    for seed in range(3):
        inst = W.tiny_instance(80, 3400 + seed, seed % 2 == 1, span=400)
        inst.capacity = int(inst.node4[:, 0].sum() // 6)
        sol = W.random_solution(inst, 10, 3410 + seed)
        S = check_select(tga, inst, sol, 0xFF, None, "random")
        # the table starts empty at every evaluation: a second call selects the same
        S.eval(0xFF | tga.OP_MULTI)
        again = [(m.id, m.delta) for m in S.select_moves()]
        assert again == oracle.multi_select(inst, sol, 0xFF)[0]


@pytest.mark.parametrize("which,mask,pen", [("c1", 0x1F, None), ("vrptw400", 0xFF, None), ("vrptw400", 0x1F, (5, 5))])
def test_multi_local_search_matches_oracle(tga, which, mask, pen):
    inst, sol = W.c1() if which == "c1" else vrptw400()
    steps = 40
    final, applied, per, mv = oracle.local_search_multi(inst, sol, mask, max_steps=steps, penalty=pen)
    assert len(applied) > len(per) > 3
    I, S = gpu_multi(tga, inst, sol, pen)
    st, moves, cost = S.ls_run(steps, mask | tga.OP_MULTI)
    assert (st, moves) == (len(per), mv)
    assert S.multi_stats() == (len(per), len(applied))
    assert cost == oracle.cost(inst, final)[0]
    off, cust, _ = S.get()
    assert off.tolist() == final.offsets.tolist() and cust.tolist() == final.customers.tolist()
    # step by step: the selections, then their application
    S.reload(sol.offsets, sol.customers)
    k = 0
    for cnt in per[:5]:
        S.eval(mask | tga.OP_MULTI)
        got = S.select_moves()
        assert [(m.id, m.delta) for m in got] == applied[k:k + cnt]
        for m in got:
            m.version = S.version
            S.apply(m)
        k += cnt


def test_select_without_sorting(tga):
    """More improving route pairs than the sorted selection holds (4096):
    the repeated-minimum path must give the same selection."""
    inst = W.make_cvrp(1500, 3500)
    sol = W.random_solution(inst, 200, 3501)
    ref, _, ncand = oracle.multi_select(inst, sol, 0x1F, candidates=True)
    assert ncand > 4096
    I, S = gpu_multi(tga, inst, sol)
    S.eval(0x1F | tga.OP_MULTI)
    got = [(m.id, m.delta) for m in S.select_moves()]
    assert got == ref and len(ref) > 50
    final, applied, per, mv = oracle.local_search_multi(inst, sol, 0x1F, max_steps=2)
    S.reload(sol.offsets, sol.customers)
    st, moves, cost = S.ls_run(2, 0x1F | tga.OP_MULTI)
    assert (st, moves, cost) == (len(per), mv, oracle.cost(inst, final)[0])


def test_multi_errors(tga):
    inst = W.tiny_instance(20, 3600, False)
    sol = W.random_solution(inst, 3, 3601)
    I = tga.Instance.from_workload(inst)
    S = tga.Solution(I, sol.offsets, sol.customers)
    with pytest.raises(tga.TGAError) as e:
        S.eval(0x1F | tga.OP_MULTI)
    assert e.value.code == tga.TGA_EINVAL
    with pytest.raises(tga.TGAError):
        S.select_moves()
    S.set_multi(True)
    assert S.eval(0x1F | tga.OP_MULTI) is not None
    S.select_moves()
    S.set_multi(False)
    with pytest.raises(tga.TGAError):
        S.ls_run(5, 0x1F | tga.OP_MULTI)


def test_large_selection_applied_move_by_move(tga):
    """A selection larger than the one-pass apply holds (more than 546
    moves) is applied move by move; the step must still equal the oracle's."""
    inst = W.make_cvrp(3000, 3700)
    sol = W.random_solution(inst, 1500, 3701)
    ref, _ = oracle.multi_select(inst, sol, 0x1F, threads=4)
    assert len(ref) > 546
    final, applied, per, mv = oracle.local_search_multi(inst, sol, 0x1F, max_steps=1, threads=4)
    assert per == [len(ref)]
    I, S = gpu_multi(tga, inst, sol)
    st, moves, cost = S.ls_run(1, 0x1F | tga.OP_MULTI)
    assert (st, moves, cost) == (1, mv, oracle.cost(inst, final)[0])
    off, cust, _ = S.get()
    assert off.tolist() == final.offsets.tolist() and cust.tolist() == final.customers.tolist()
