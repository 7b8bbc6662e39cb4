"""GPU parity with pickups (VRPSPDTW): per-move delta / score and feasibility
bits, best moves and local-search trajectories against the oracle with
pickups, in hard and penalised mode.  Integer path, so the bar is equality."""
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


def with_pickups(inst, seed, hi=10):
    rng = np.random.default_rng(seed)
    inst.pickup = np.zeros(inst.n + 1, np.int32)
    inst.pickup[1:] = rng.integers(0, hi, size=inst.n)
    return inst


def check_dump(T, inst, sol, pen=None, op_mask=0x1F, tag=""):
    print("pickup dump", tag, "n=%d R=%d tw=%d pen=%s" % (inst.n, sol.R, inst.has_tw, pen), flush=True)
    I = T.Instance.from_workload(inst)
    S = T.Solution(I, sol.offsets, sol.customers)
    if pen is not None:
        S.set_penalty(*pen)
        assert S.violations() == oracle.violations(inst, sol)
    ob, odd, odf = oracle.eval_neighbourhood(inst, sol, op_mask, dump=True, threads=0, penalty=pen)
    gb, gdd, gdf = S.eval(op_mask, dump=True)
    gdd = gdd.cpu().numpy()
    gdf = gdf.cpu().numpy()
    bad = np.nonzero(gdf != odf)[0]
    assert bad.size == 0, ("feas/move-set mismatch", [(int(i), oracle.decode(S.Q, i), int(odf[i]), int(gdf[i])) for i in bad[:8]])
    bad = np.nonzero(gdd != odd)[0]
    assert bad.size == 0, ("delta mismatch", [(int(i), oracle.decode(S.Q, i), int(odd[i]), int(gdd[i])) for i in bad[:8]])
    if ob.found:
        assert gb is not None and (gb.delta, gb.id) == (ob.delta, ob.id)
        m = S.eval(op_mask)
        assert (m.delta, m.id) == (ob.delta, ob.id)
    else:
        assert gb is None
    return I, S


@pytest.mark.parametrize("has_tw", [0, 1])
@pytest.mark.parametrize("n,R", [(1, 2), (5, 2), (8, 3), (30, 4)])
def test_pickup_dump_tiny(tga, has_tw, n, R):
    inst = with_pickups(W.tiny_instance(n, 1100 + 5 * n + R + has_tw, bool(has_tw), span=200), n + R)
    inst.capacity = int(inst.node4[:, 0].sum() // 2 + 2)
    sol = W.random_solution(inst, R, 1200 + n + R)
    check_dump(tga, inst, sol, tag="tiny")
    check_dump(tga, inst, sol, pen=(3, 2 if has_tw else 0), tag="tiny pen")


@pytest.mark.parametrize("op_mask", [1, 2, 4, 8, 16, 0x1F])
def test_pickup_dump_op_masks(tga, op_mask):
    inst = with_pickups(W.tiny_instance(80, 1300, True, span=400), 7)
    inst.capacity = int(inst.node4[:, 0].sum() // 6)
    sol = W.random_solution(inst, 8, 1301)
    check_dump(tga, inst, sol, op_mask=op_mask, tag="mask")


@pytest.mark.parametrize("pen", [None, (10, 10)])
def test_pickup_dump_full_size(tga, pen):
    inst, sol = W.c6()
    check_dump(tga, inst, sol, pen=pen, tag="c6")


@pytest.mark.parametrize("pen", [None, (5, 5)])
def test_pickup_local_search_matches_oracle(tga, pen):
    inst, sol = W.c6(300)
    final, ids, deltas, mv = oracle.local_search(inst, sol, max_steps=200, penalty=pen)
    assert len(ids) > 10
    I = tga.Instance.from_workload(inst)
    S = tga.Solution(I, sol.offsets, sol.customers)
    if pen is not None:
        S.set_penalty(*pen)
    st, moves, cost = S.ls_run(200)
    assert (st, moves, cost) == (len(ids), mv, oracle.cost(inst, final)[0])
    off, cust, _ = S.get()
    assert off.tolist() == final.offsets.tolist() and cust.tolist() == final.customers.tolist()
    S.reload(sol.offsets, sol.customers)
    for k in range(min(30, len(ids))):
        m = S.eval()
        assert (m.id, m.delta) == (int(ids[k]), int(deltas[k])), k
        S.apply(m)


def test_pickup_errors(tga):
    inst = W.tiny_instance(10, 1400, False)
    I = tga.Instance.from_workload(inst)
    bad = np.zeros(11, np.int32)
    bad[3] = -1
    with pytest.raises(tga.TGAError) as e:
        I.set_pickups(bad)
    assert e.value.code == tga.TGA_EINVAL
    bad[3], bad[0] = 1, 2
    with pytest.raises(tga.TGAError) as e:
        I.set_pickups(bad)
    assert e.value.code == tga.TGA_EINVAL
    inst = with_pickups(inst, 3)
    I = tga.Instance.from_workload(inst)
    sol = W.random_solution(inst, 3, 1401)
    S = tga.Solution(I, sol.offsets, sol.customers)
    with pytest.raises(tga.TGAError) as e:
        tga.Batch([S])
    assert e.value.code == tga.TGA_EINVAL
