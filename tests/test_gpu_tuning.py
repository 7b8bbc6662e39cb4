"""Per-size schedules (rows per inter-route item of the single-solution and
batched forms): every schedule gives the oracle's results, and the autotuner
writes a table whose schedules do too."""
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
    yield T
    if T.TUNE_PATH and __import__("os").path.exists(T.TUNE_PATH):
        T.load_tuning(T.TUNE_PATH)
    else:
        T.set_tuning([])


@pytest.mark.parametrize("which", ["c1", "vrptw300"])
@pytest.mark.parametrize("rows", [1, 2, 5, 64])
def test_plain_rows_keep_the_dump(tga, which, rows):
    inst = W.make_vrptw(300, 3300) if which == "vrptw300" else W.c1()[0]
    sol = W.sweep(inst)
    print("plain rows", which, rows, flush=True)
    I = tga.Instance.from_workload(inst)
    S = tga.Solution(I, sol.offsets, sol.customers)
    S.set_rows(rows, 0)
    assert S.rows()[0] == rows
    ob, odd, odf = oracle.eval_neighbourhood(inst, sol, dump=True)
    gb, gdd, gdf = S.eval(dump=True)
    assert np.array_equal(gdd.cpu().numpy(), odd) and np.array_equal(gdf.cpu().numpy(), odf)
    assert (gb.delta, gb.id) == (ob.delta, ob.id)
    st, mv, cost = S.ls_run(60)
    final, ids, _, omv = oracle.local_search(inst, sol, max_steps=60)
    assert (st, mv, cost) == (len(ids), omv, oracle.cost(inst, final)[0])


@pytest.mark.parametrize("item_rows", [1, 3, 40, 200])
def test_batched_item_rows_keep_results(tga, item_rows):
    rng = np.random.default_rng(9)
    pairs = []
    for b in range(6):
        n = int(rng.integers(40, 400))
        inst = W.make_cvrp(n, 3400 + b) if b % 2 == 0 else W.make_vrptw(n, 3400 + b)
        pairs.append((inst, W.sweep(inst)))
    insts = [tga.Instance.from_workload(i) for i, _ in pairs]
    sols = [tga.Solution(I, s.offsets, s.customers) for I, (_, s) in zip(insts, pairs)]
    for s in sols:
        s.set_rows(0, item_rows)
    B = tga.Batch(sols)
    st, mv, cost = B.ls_run(40)
    for b, (inst, sol) in enumerate(pairs):
        final, ids, _, omv = oracle.local_search(inst, sol, max_steps=40)
        assert (st[b], mv[b], cost[b]) == (len(ids), omv, oracle.cost(inst, final)[0]), b
    B.close()


def test_autotuner_table_round_trip(tga, tmp_path):
    from paper_2506_17357_amd import autotune
    entries, meas = autotune.run(buckets=(80, 160), kinds=("cvrp", "vrptw"), steps_plain=5, steps_batch=3, mix=False)
    assert len(entries) == 4 and len(meas) == 4
    for e in entries:
        assert e["plain_rows"] >= 1 and e["item_rows"] >= 0
    assert [e["n_max"] for e in entries[:2]] == [113, 14654]
    tga.set_tuning(entries)
    inst = W.make_vrptw(150, 3500)
    sol = W.sweep(inst)
    I = tga.Instance.from_workload(inst)
    S = tga.Solution(I, sol.offsets, sol.customers)
    e = [x for x in entries if x["kind"] == "vrptw" and x["n_max"] >= 150][0]
    assert S.rows() == (min(e["plain_rows"], 64), e["item_rows"])
    ob = oracle.eval_neighbourhood(inst, sol)
    m = S.eval()
    assert (m.delta, m.id) == (ob.delta, ob.id)
