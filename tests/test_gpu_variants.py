"""GPU parity of the operator variants (segment relocation of 2..3 nodes,
kept or reversed; cross-exchange of segments of 1..3 nodes; Sections 4.1 and
7) on the general path: per-move delta and feasibility bits, best moves,
local-search trajectories and the application of every variant, against the
oracle.  Integer path, so the bar is equality."""
import numpy as np
import pytest

import oracle
from paper_2506_17357_amd import workload as W

pytestmark = pytest.mark.gpu

ALL = 0xFF


@pytest.fixture(scope="module")
def tga():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_17357_amd import tga as T
    T.lib()
    return T


def gpu_general(T, inst, sol, pen=None):
    I = T.Instance.from_workload(inst)
    S = T.Solution(I, sol.offsets, sol.customers)
    S.set_general(True)
    if pen is not None:
        S.set_penalty(*pen)
    return I, S


def check_dump(T, inst, sol, op_mask=ALL, pen=None, tag=""):
    print("variants dump", tag, "n=%d R=%d tw=%d mask=0x%x pen=%s" % (inst.n, sol.R, inst.has_tw, op_mask, pen),
          flush=True)
    I, S = gpu_general(T, inst, sol, pen)
    ob, odd, odf = oracle.eval_neighbourhood(inst, sol, op_mask, dump=True, threads=0, penalty=pen)
    gb, gdd, gdf = S.eval(op_mask, dump=True)
    gdd = gdd.cpu().numpy()
    gdf = gdf.cpu().numpy()
    assert gdd.shape == odd.shape
    bad = np.nonzero(gdf != odf)[0]
    assert bad.size == 0, ("feas/move-set mismatch", [(int(i), oracle.decode(S.Q, i), int(odf[i]), int(gdf[i])) for i in bad[:8]])
    bad = np.nonzero(gdd != odd)[0]
    assert bad.size == 0, ("delta mismatch", [(int(i), oracle.decode(S.Q, i), int(odd[i]), int(gdd[i])) for i in bad[:8]])
    if ob.found:
        assert gb is not None and (gb.delta, gb.id) == (ob.delta, ob.id)
        assert (gb.op, gb.k, gb.a, gb.b) == oracle.decode(S.Q, ob.id)
    else:
        assert gb is None
    return I, S, ob


@pytest.mark.parametrize("has_tw", [0, 1])
@pytest.mark.parametrize("n,R", [(1, 2), (4, 2), (7, 3), (12, 4), (40, 5)])
def test_variants_dump_tiny(tga, has_tw, n, R):
    inst = W.tiny_instance(n, 2100 + 7 * n + R + has_tw, bool(has_tw), dup=n % 2 == 0, span=250)
    sol = W.random_solution(inst, R, 2200 + n + R)
    check_dump(tga, inst, sol, tag="tiny")


@pytest.mark.parametrize("op_mask", [0x20, 0x40, 0x80, 0x21, 0xE0, 0xE3, ALL])
def test_variants_dump_op_masks(tga, op_mask):
    inst = W.tiny_instance(90, 2300, True, span=400)
    sol = W.random_solution(inst, 9, 2301)
    check_dump(tga, inst, sol, op_mask=op_mask, tag="mask")


def test_variants_dump_ragged_tiles(tga):
    """Q = 37 + 3 (not a multiple of the 16-slot pair tiles), short and empty
    routes among long ones."""
    inst = W.tiny_instance(37, 2400, True, span=300)
    routes = [list(range(1, 20)), [], [20], list(range(21, 38))]
    sol = W.Solution.from_routes(routes)
    check_dump(tga, inst, sol, tag="ragged")


@pytest.mark.parametrize("pen", [(3, 2), (10, 0)])
def test_variants_dump_penalised(tga, pen):
    inst = W.tiny_instance(60, 2500, True, span=300)
    inst.capacity = int(inst.node4[:, 0].sum() // 7)
    sol = W.random_solution(inst, 6, 2501)
    check_dump(tga, inst, sol, pen=pen, tag="pen")


def test_variants_dump_pickups(tga):
    inst, sol = W.c6(200)
    check_dump(tga, inst, sol, tag="pickups")
    check_dump(tga, inst, sol, pen=(5, 5), tag="pickups pen")


@pytest.mark.parametrize("which", ["c1", "c3"])
def test_variants_dump_full_size(tga, which):
    inst, sol = getattr(W, which)()
    check_dump(tga, inst, sol, tag=which)


def test_base_operators_identical_on_general_path(tga):
    """The five base operators give the same dump on the general path as on
    the plain path."""
    inst, sol = W.c3()
    I = tga.Instance.from_workload(inst)
    S = tga.Solution(I, sol.offsets, sol.customers)
    b1, d1, f1 = S.eval(dump=True)
    S.set_general(True)
    b2, d2, f2 = S.eval(dump=True)
    assert (b1.delta, b1.id) == (b2.delta, b2.id)
    assert np.array_equal(d1.cpu().numpy(), d2.cpu().numpy())
    assert np.array_equal(f1.cpu().numpy(), f2.cpu().numpy())
    S.set_general(False)
    b3 = S.eval()
    assert (b3.delta, b3.id) == (b1.delta, b1.id)


def test_apply_every_variant_matches_oracle(tga):
    """Moves of every variant operator, admissible or not, apply as the
    oracle applies them; the attributes rebuilt afterwards give the dump of
    a freshly loaded solution."""
    inst = W.tiny_instance(40, 2600, True, span=300)
    sol = W.random_solution(inst, 5, 2601)
    _, odd, odf = oracle.eval_neighbourhood(inst, sol, ALL, dump=True)
    Q = inst.n + sol.R
    ids = np.nonzero(odf != oracle.NOT_A_MOVE)[0]
    ops = ids // (Q * Q) // 4
    rng = np.random.default_rng(5)
    picks = []
    for op in range(5, 10):
        cand = ids[ops == op]
        assert cand.size > 0, op
        picks += rng.choice(cand, size=min(12, cand.size), replace=False).tolist()
    I = tga.Instance.from_workload(inst)
    for mid in picks:
        S = tga.Solution(I, sol.offsets, sol.customers)
        S.set_general(True)
        op, k, a, b = oracle.decode(Q, int(mid))
        m = tga.Move(op, k, a, b, int(odd[mid]), int(odf[mid]), int(mid), S.version)
        cost = S.apply(m)
        ref = oracle.apply_move(inst, sol, int(mid))
        off, cust, c = S.get()
        assert off.tolist() == ref.offsets.tolist() and cust.tolist() == ref.customers.tolist(), (mid, op, k, a, b)
        assert cost == oracle.cost(inst, ref)[0] == c
        _, rd, rf = oracle.eval_neighbourhood(inst, ref, ALL, dump=True)
        _, gd, gf = S.eval(ALL, dump=True)
        assert np.array_equal(gd.cpu().numpy(), rd) and np.array_equal(gf.cpu().numpy(), rf), (mid, op, k)


def vrptw400():
    inst = W.make_vrptw(400, 2800)
    return inst, W.sweep(inst)


@pytest.mark.parametrize("which,pen", [("c1", None), ("vrptw400", None), ("vrptw400", (5, 5))])
def test_variants_local_search_matches_oracle(tga, which, pen):
    inst, sol = W.c1() if which == "c1" else vrptw400()
    steps = 120
    final, ids, deltas, mv = oracle.local_search(inst, sol, ALL, max_steps=steps, penalty=pen)
    assert len(ids) > 10
    Q = inst.n + sol.R
    assert any(int(i) // (Q * Q) // 4 >= 5 for i in ids), "no variant move on the trajectory"
    I, S = gpu_general(tga, inst, sol, pen)
    st, moves, cost = S.ls_run(steps, ALL)
    assert (st, moves, cost) == (len(ids), mv, oracle.cost(inst, final)[0])
    off, cust, _ = S.get()
    assert off.tolist() == final.offsets.tolist() and cust.tolist() == final.customers.tolist()
    S.reload(sol.offsets, sol.customers)
    for k in range(min(25, len(ids))):
        m = S.eval(ALL)
        assert (m.id, m.delta) == (int(ids[k]), int(deltas[k])), k
        S.apply(m)


def test_variant_errors(tga):
    inst = W.tiny_instance(10, 2700, False)
    sol = W.random_solution(inst, 3, 2701)
    I = tga.Instance.from_workload(inst)
    S = tga.Solution(I, sol.offsets, sol.customers)
    for mask in (0x20, 0x40, 0x80):
        with pytest.raises(tga.TGAError) as e:
            S.eval(mask)
        assert e.value.code == tga.TGA_EINVAL
    with pytest.raises(tga.TGAError) as e:
        S.eval(1 << 8)
    assert e.value.code == tga.TGA_EINVAL
    S.set_general(True)
    with pytest.raises(tga.TGAError) as e:
        S.eval(tga.OPS_ALL | tga.OP_GRANULAR)
    assert e.value.code == tga.TGA_EINVAL
    with pytest.raises(tga.TGAError) as e:
        tga.Batch([S])
    assert e.value.code == tga.TGA_EINVAL
    assert S.eval(ALL) is not None
