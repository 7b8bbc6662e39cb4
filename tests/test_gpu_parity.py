"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Integer work, so the bar is bit-exactness: every per-move delta and
feasibility mask, the best move (delta, id), trajectories and final
solutions.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2506_17357_amd import workload as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tga():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_17357_amd import tga as T
    T.lib()
    return T


def gpu_solution(T, inst, sol):
    I = T.Instance.from_workload(inst)
    return I, T.Solution(I, sol.offsets, sol.customers)


def check_dump(T, inst, sol, op_mask=0x1F, tag=""):
    say("dump parity", tag, "limits", T.device_limits(), "n=%d R=%d tw=%d mask=%d" % (inst.n, sol.R, inst.has_tw, op_mask))
    ob, odd, odf = oracle.eval_neighbourhood(inst, sol, op_mask, dump=True, threads=0)
    I, S = gpu_solution(T, inst, sol)
    gb, gdd, gdf = S.eval(op_mask, dump=True)
    gdd = gdd.cpu().numpy()
    gdf = gdf.cpu().numpy()
    bad = np.nonzero(gdf != odf)[0]
    assert bad.size == 0, ("feas/move-set mismatch", [(int(i), oracle.decode(S.Q, i), int(odf[i]), int(gdf[i])) for i in bad[:8]])
    bad = np.nonzero(gdd != odd)[0]
    assert bad.size == 0, ("delta mismatch", [(int(i), oracle.decode(S.Q, i), int(odd[i]), int(gdd[i])) for i in bad[:8]])
    if ob.found:
        assert gb is not None and (gb.delta, gb.id, gb.feas) == (ob.delta, ob.id, 3)
        op, k, a, b = oracle.decode(S.Q, ob.id)
        assert (gb.op, gb.k, gb.a, gb.b) == (op, k, a, b)
    else:
        assert gb is None
    assert int(S.move_counts().sum()) == ob.moves or op_mask != 0x1F
    return S


def tiny_cases():
    out = []
    seed = 0
    for has_tw in (0, 1):
        for n in (1, 2, 3, 5, 8):
            for R in (1, 2, 3, 4):
                seed += 1
                out.append((n, R, has_tw, seed))
    return out


@pytest.mark.parametrize("n,R,has_tw,seed", tiny_cases())
def test_dump_tiny(tga, n, R, has_tw, seed):
    inst = W.tiny_instance(n, 7000 + seed, bool(has_tw), dup=seed % 4 == 0)
    sol = W.random_solution(inst, R, 8000 + seed)
    check_dump(tga, inst, sol, tag="tiny")


def test_dump_golden_line4(tga):
    with open(os.path.join(GOLDEN, "line4_vrptw.json")) as f:
        g = json.load(f)
    inst = W.Instance(g["n"], np.asarray(g["dist"], np.int32), np.asarray(g["node4"], np.int32),
                      g["capacity"], g["has_tw"], np.zeros((g["n"] + 1, 2), np.int64), "golden", 0)
    sol = W.Solution.from_routes(g["routes"])
    S = check_dump(tga, inst, sol, tag="golden")
    best = S.eval()
    assert (best.delta, best.id) == (g["expected_best"]["delta"], g["expected_best"]["id"])


@pytest.mark.parametrize("op_mask", [1, 2, 4, 8, 16, 3, 12, 0x1F])
def test_dump_op_masks(tga, op_mask):
    inst = W.tiny_instance(40, 11, True, span=200)
    sol = W.random_solution(inst, 5, 12)
    check_dump(tga, inst, sol, op_mask, tag="mask")


@pytest.mark.parametrize("has_tw", [0, 1])
def test_dump_medium_random(tga, has_tw):
    """Several row tiles and column chunks with a ragged tail; random routes
    (empty, infeasible and long ones)."""
    inst = W.tiny_instance(333, 21 + has_tw, bool(has_tw), span=1000)
    sol = W.random_solution(inst, 17, 22)
    check_dump(tga, inst, sol, tag="medium")


@pytest.mark.parametrize("has_tw", [0, 1])
def test_dump_wide_distances(tga, has_tw):
    """Distances above 2^16: the inter-route kernels stream the int32 matrix
    (the generators' instances all fit the 16-bit copy)."""
    inst = W.tiny_instance(333, 91 + has_tw, bool(has_tw), span=100000)
    assert int(inst.dist.max()) >= 1 << 16
    sol = W.random_solution(inst, 17, 92)
    S = check_dump(tga, inst, sol, tag="wide")
    assert S.inst.dist_bytes == 4


@pytest.mark.parametrize("dmax,width", [(65535, 2), (65536, 4)])
def test_distance_width_boundary(tga, dmax, width):
    """The largest distance decides the streamed width; 65535 must survive
    the 16-bit copy exactly."""
    inst = W.tiny_instance(60, 97, True, span=300)
    inst.dist[0, 7] = inst.dist[7, 0] = dmax
    inst.dist[3, 9] = inst.dist[9, 3] = dmax - 1
    sol = W.random_solution(inst, 5, 98)
    S = check_dump(tga, inst, sol, tag="width%d" % width)
    assert S.inst.dist_bytes == width


def test_dump_c1(tga):
    inst, sol = W.c1()
    check_dump(tga, inst, sol, tag="C1")


@pytest.mark.parametrize("which", ["c2", "c3"])
def test_dump_full_size(tga, which):
    """Every move of a 1000-customer neighbourhood (about 2.1e6 moves)."""
    inst, sol = getattr(W, which)()
    check_dump(tga, inst, sol, tag=which)


def test_dump_2000_vrptw(tga):
    """The largest size of the batched mix."""
    inst = W.make_vrptw(2000, 4001)
    sol = W.sweep(inst)
    check_dump(tga, inst, sol, tag="vrptw2000")


@pytest.mark.parametrize("op_mask", [0x1F, 8 | 16])
def test_dump_long_routes(tga, op_mask):
    """Routes longer than a wavefront (intra-route lanes wrap, and a route
    too long for LDS is read from global memory), with all operators and
    with the intra-route ones alone (their own launch)."""
    inst = W.tiny_instance(300, 31, True, capacity=10 ** 6, span=1000)
    inst.node4[:, 2] = np.maximum(inst.node4[:, 2], 1 << 20)  # loose windows
    inst.node4[0, 2] = 1 << 22
    sol = W.random_solution(inst, 2, 32)
    check_dump(tga, inst, sol, op_mask, tag="long")


@pytest.mark.parametrize("has_tw", [0, 1])
def test_route_block_cache_follows_route_changes(tga, has_tw):
    """Intra-route distance blocks cached per route are reused only for the
    same nodes in the same order.  Routes are reordered in place and
    customers exchanged between routes of equal length, by applied moves
    (the cache then holds the old routes) and by reloads; every state is
    compared with the oracle."""
    inst = W.tiny_instance(240, 77 + has_tw, bool(has_tw), capacity=10 ** 6, span=1000)
    if has_tw:
        inst.node4[:, 2] = np.maximum(inst.node4[:, 2], 1 << 20)
        inst.node4[0, 2] = 1 << 22
    off = np.arange(0, 241, 20, dtype=np.int32)  # 12 routes of 20 customers (22 positions, cached)
    rng = np.random.Generator(np.random.PCG64(5))
    cust_a = rng.permutation(np.arange(1, 241)).astype(np.int32)
    cust_b = cust_a.copy()
    cust_b[0:20] = cust_b[0:20][::-1]                  # route 0 reversed
    cust_b[40:60], cust_b[80:100] = cust_a[80:100], cust_a[40:60]  # routes 2 and 4 exchanged
    cust_b[120:140] = np.roll(cust_b[120:140], 3)      # route 6 rotated
    A, B = W.Solution(off, cust_a), W.Solution(off, cust_b)
    I, S = gpu_solution(tga, inst, A)

    def same_as_oracle(sol, tag):
        ob, odd, odf = oracle.eval_neighbourhood(inst, sol, 0x1F, dump=True, threads=0)
        gb, gdd, gdf = S.eval(0x1F, dump=True)
        assert np.array_equal(gdf.cpu().numpy(), odf), tag
        assert np.array_equal(gdd.cpu().numpy(), odd), tag
        assert (gb.delta, gb.id) == (ob.delta, ob.id), tag
        m = S.eval()  # the non-dump path skips moves that cannot win
        assert (m.delta, m.id) == (ob.delta, ob.id), tag
        return m

    for tag, sol in [("a", A), ("b", B), ("a again", A)]:
        S.reload(sol.offsets, sol.customers)
        cur = sol
        for step in range(4):  # applied moves rewrite one or two routes each
            m = same_as_oracle(cur, "%s step %d" % (tag, step))
            S.apply(m)
            cur = oracle.apply_move(inst, cur, m.id)
        same_as_oracle(cur, tag + " end")


def test_c1_trajectory_step_by_step(tga):
    inst, sol = W.c1()
    _, ids, deltas, _ = oracle.local_search(inst, sol, max_steps=100)
    I, S = gpu_solution(tga, inst, sol)
    c0 = oracle.cost(inst, sol)[0]
    cost = c0
    for step in range(len(ids)):
        m = S.eval()
        assert (m.id, m.delta) == (int(ids[step]), int(deltas[step])), step
        cost = S.apply(m)
        assert cost == c0 + int(deltas[:step + 1].sum())
    m = S.eval()
    assert m is None or m.delta >= 0


@pytest.mark.parametrize("which", ["c1", "c2", "c3"])
def test_device_ls_matches_oracle(tga, which):
    """The device-resident loop reaches the oracle's local optimum (stored
    trajectory written by tests/golden/make_trajectories.py)."""
    inst, sol = getattr(W, which)()
    path = os.path.join(GOLDEN, "traj_%s.json" % which)
    with open(path) as f:
        g = json.load(f)
    assert g["instance_sha256"] == inst.sha256()
    I, S = gpu_solution(tga, inst, sol)
    steps, moves, cost = S.ls_run(100000)
    say(which, "steps", steps, "cost", cost, "moves", moves)
    assert steps == len(g["ids"]) and cost == g["final_cost"] and moves == g["moves_evaluated"]
    off, cust, c = S.get()
    assert off.tolist() == g["final_offsets"] and cust.tolist() == g["final_customers"]


@pytest.mark.parametrize("which", ["c2", "c3"])
def test_host_loop_trajectory_full_size(tga, which):
    """Best move (id, delta) at every step of the 1000-customer runs."""
    inst, sol = getattr(W, which)()
    with open(os.path.join(GOLDEN, "traj_%s.json" % which)) as f:
        g = json.load(f)
    I, S = gpu_solution(tga, inst, sol)
    for step, (mid, d) in enumerate(zip(g["ids"], g["deltas"])):
        m = S.eval()
        assert (m.id, m.delta) == (mid, d), step
        S.apply(m)
    m = S.eval()
    assert m is None or m.delta >= 0


def test_apply_rebuild_equals_fresh_build(tga):
    inst = W.tiny_instance(120, 41, True, span=500)
    sol = W.sweep(inst)
    I, S = gpu_solution(tga, inst, sol)
    for _ in range(25):
        m = S.eval()
        if m is None or m.delta >= 0:
            break
        S.apply(m)
    off, cust, cost = S.get()
    fresh = tga.Solution(I, off, cust)
    _, d1, f1 = S.eval(dump=True)
    _, d2, f2 = fresh.eval(dump=True)
    assert np.array_equal(d1.cpu().numpy(), d2.cpu().numpy())
    assert np.array_equal(f1.cpu().numpy(), f2.cpu().numpy())
    assert cost == oracle.cost(inst, W.Solution(off, cust))[0]


def test_apply_any_move_matches_oracle(tga):
    """Non-improving and inadmissible moves apply exactly as the oracle
    applies them, for every operator."""
    inst = W.tiny_instance(30, 51, True, span=300)
    sol = W.random_solution(inst, 4, 52)
    _, odd, odf = oracle.eval_neighbourhood(inst, sol, dump=True)
    ids = np.nonzero(odf != oracle.NOT_A_MOVE)[0]
    rng = np.random.default_rng(3)
    I = tga.Instance.from_workload(inst)
    for mid in rng.choice(ids, size=60, replace=False):
        S = tga.Solution(I, sol.offsets, sol.customers)
        op, k, a, b = oracle.decode(S.Q, int(mid))
        m = tga.Move(op, k, a, b, int(odd[mid]), int(odf[mid]), int(mid), S.version)
        cost = S.apply(m)
        ref = oracle.apply_move(inst, sol, int(mid))
        off, cust, c = S.get()
        assert off.tolist() == ref.offsets.tolist() and cust.tolist() == ref.customers.tolist()
        assert cost == oracle.cost(inst, ref)[0] == c


def test_errors(tga):
    T = tga
    inst = W.tiny_instance(10, 61, False)
    sol = W.random_solution(inst, 3, 62)
    I, S = gpu_solution(T, inst, sol)
    m = S.eval()
    stale = T.Move(m.op, m.k, m.a, m.b, m.delta, m.feas, m.id, m.version + 1)
    with pytest.raises(T.TGAError) as e:
        S.apply(stale)
    assert e.value.code == T.TGA_ESTALE
    bad = T.Move(0, 1, 0, 0, 0, 3, (1 * S.Q + 0) * S.Q + 0, S.version)  # relocate 1 after itself
    with pytest.raises(T.TGAError) as e:
        S.apply(bad)
    assert e.value.code == T.TGA_EINVAL
    with pytest.raises(T.TGAError) as e:
        T.Solution(I, [0, 5, 9], list(range(1, 11)))  # offsets do not end at n
    assert e.value.code == T.TGA_EINVAL
    with pytest.raises(T.TGAError) as e:
        T.Solution(I, [0, 5, 10], [1, 1, 2, 3, 4, 5, 6, 7, 8, 9])  # not a permutation
    assert e.value.code == T.TGA_EINVAL
    asym = inst.dist.copy()
    asym[1, 2] += 1
    with pytest.raises(T.TGAError) as e:
        T.Instance(inst.n, asym, inst.node4, inst.capacity, 0)
    assert e.value.code == T.TGA_EINVAL
    tw = inst.node4.copy()
    tw[3, 1], tw[3, 2] = 50, 10  # e > l
    with pytest.raises(T.TGAError) as e:
        T.Instance(inst.n, inst.dist, tw, inst.capacity, 1)
    assert e.value.code == T.TGA_EINVAL
    # an instance workspace that is not 256-byte aligned is refused
    import ctypes
    import torch
    L = T.lib()
    dd = torch.from_numpy(inst.dist).cuda()
    nd = torch.from_numpy(inst.node4).cuda()
    nb = L.tga_instance_workspace_bytes(inst.n)
    ws = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    rc = L.tga_load_instance(inst.n, dd.data_ptr(), nd.data_ptr(), inst.capacity, 0, ws.data_ptr() + 16, nb,
                             T._stream(None), ctypes.byref(h))
    assert rc == T.TGA_EINVAL and h.value is None
    assert S.eval() is not None  # still usable after the errors


def test_no_admissible_move(tga):
    """Capacity below every route load: nothing is admissible."""
    inst = W.tiny_instance(6, 71, False, capacity=0)
    sol = W.random_solution(inst, 2, 72)
    ob = oracle.eval_neighbourhood(inst, sol)
    I, S = gpu_solution(tga, inst, sol)
    assert not ob.found and S.eval() is None
    steps, moves, cost = S.ls_run(10)
    assert steps == 0


def test_single_customer(tga):
    inst = W.tiny_instance(1, 81, True)
    for R in (1, 3):
        sol = W.random_solution(inst, R, 82)
        check_dump(tga, inst, sol, tag="n1")


@pytest.mark.parametrize("has_tw", [0, 1])
@pytest.mark.parametrize("cap", [7, 100000])
def test_eval_after_ls_run(tga, has_tw, cap):
    """An evaluation after a device local search (stopped at the step cap or
    at the local optimum) still covers every move of the current routes."""
    inst = W.make_vrptw(150, 33) if has_tw else W.make_cvrp(150, 33)
    sol = W.sweep(inst)
    I, S = gpu_solution(tga, inst, sol)
    steps, _, cost = S.ls_run(cap)
    assert (steps == cap) == (cap == 7)
    off, cust, _ = S.get()
    cur = W.Solution(off, cust)
    ob, odd, odf = oracle.eval_neighbourhood(inst, cur, 0x1F, dump=True, threads=0)
    gb, gdd, gdf = S.eval(0x1F, dump=True)
    assert np.array_equal(gdf.cpu().numpy(), odf) and np.array_equal(gdd.cpu().numpy(), odd)
    assert ob.found and (gb.delta, gb.id) == (ob.delta, ob.id)
    if cap > steps:
        assert gb.delta >= 0  # a local optimum
    m = S.eval()
    assert (m.delta, m.id) == (ob.delta, ob.id)
    assert S.stats()[0] == steps  # the evaluation leaves the run's counters alone
