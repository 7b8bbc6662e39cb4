"""Served form: continuous batching under an HBM budget.  Each request's
result must be the same alone and in the mix (tolerance 0: integer path), and
equal the oracle's."""
import numpy as np
import pytest

import oracle
from paper_2506_17357_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_17357_amd import tga, serve
    tga.lib()
    return tga, serve


def make_requests(serve, count=10, seed=0, gap_s=0.002, max_steps=60, lo=30, hi=300):
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(count):
        n = int(rng.integers(lo, hi))
        inst = W.make_cvrp(n, 900 + k) if k % 2 == 0 else W.make_vrptw(n, 900 + k)
        reqs.append(serve.ServeRequest(k, k * gap_s, inst, W.sweep(inst), max_steps))
    return reqs


def alone(tga, req):
    I = tga.Instance.from_workload(req.inst)
    S = tga.Solution(I, req.sol.offsets, req.sol.customers)
    steps, moves, cost = S.ls_run(req.max_steps)
    off, cust, _ = S.get()
    return steps, moves, cost, off, cust


def test_mix_equals_alone_and_oracle(env):
    tga, serve = env
    reqs = make_requests(serve)
    srv = serve.Server(hbm_budget_bytes=1 << 32)
    res = srv.run(reqs)
    assert [r.rid for r in res] == list(range(len(reqs)))
    assert srv.peak_active > 1, "requests never overlapped on the device"
    for r, req in zip(res, reqs):
        steps, moves, cost, off, cust = alone(tga, req)
        assert (r.steps, r.moves, r.cost) == (steps, moves, cost), r.rid
        assert r.offsets.tolist() == off.tolist() and r.customers.tolist() == cust.tolist()
        final, ids, _, mv = oracle.local_search(req.inst, req.sol, max_steps=req.max_steps)
        assert r.steps == len(ids) and r.moves == mv
        assert r.cost == oracle.cost(req.inst, final)[0]
        assert r.latency_s >= 0 and r.admitted_s >= req.arrival_s - 1e-3


@pytest.mark.parametrize("steps_per_tick", [1, 7])
def test_tick_length_does_not_change_results(env, steps_per_tick):
    tga, serve = env
    reqs = make_requests(serve, count=6, seed=4, max_steps=30)
    res = serve.Server(hbm_budget_bytes=1 << 32, steps_per_tick=steps_per_tick).run(reqs)
    for r, req in zip(res, reqs):
        steps, moves, cost, off, cust = alone(tga, req)
        assert (r.steps, r.moves, r.cost) == (steps, moves, cost), (steps_per_tick, r.rid)
        assert r.customers.tolist() == cust.tolist()


@pytest.mark.parametrize("half", [False, True])
def test_engine_schedule_does_not_change_results(env, half):
    """The engine on the whole LDS (the default) and on half of it (two
    inter-route workgroups per compute unit, fewer rows per sub-block), with
    requests that arrive together (taken largest first): results equal each
    request's own run."""
    tga, serve = env
    reqs = make_requests(serve, count=6, seed=5, gap_s=0.0, max_steps=30, lo=200, hi=1200)
    whole = tga.device_limits()[1] // 1024
    sch = {"lds_kb": whole // 2 if half else whole, "split": 0}
    print("engine schedule", sch, flush=True)
    srv = serve.Server(hbm_budget_bytes=1 << 32, schedule=sch)
    res = srv.run(reqs)
    assert srv.config["lds_kb"] == sch["lds_kb"]
    for r, req in zip(res, reqs):
        steps, moves, cost, off, cust = alone(tga, req)
        assert (r.steps, r.moves, r.cost) == (steps, moves, cost), (sch, r.rid)
        assert r.customers.tolist() == cust.tolist()


def test_admission_respects_budget(env):
    tga, serve = env
    reqs = make_requests(serve, count=8, seed=1, gap_s=0.0, max_steps=40)
    sizes = sorted(serve.device_bytes(r.inst, r.sol.R) for r in reqs)
    budget = sizes[-1] + sizes[-2]  # at most about two requests at a time
    srv = serve.Server(hbm_budget_bytes=budget)
    res = srv.run(reqs)
    assert srv.peak_used <= budget
    assert len(res) == len(reqs)
    for r, req in zip(res, reqs):
        steps, moves, cost, off, cust = alone(tga, req)
        assert (r.steps, r.moves, r.cost) == (steps, moves, cost)


def test_request_larger_than_budget_is_refused(env):
    tga, serve = env
    reqs = make_requests(serve, count=1, seed=2)
    srv = serve.Server(hbm_budget_bytes=1024)
    with pytest.raises(ValueError):
        srv.run(reqs)


def test_large_request_in_the_mix(env):
    """A 10000-customer request (400 MB matrix, one staged row per LDS
    sub-block) served next to small ones; its first steps equal its plain
    form."""
    tga, serve = env
    reqs = make_requests(serve, count=4, seed=3, max_steps=5)
    big = W.make_cvrp(10000, 5003)
    reqs.append(serve.ServeRequest(99, 0.0, big, W.sweep(big), 5))
    srv = serve.Server(hbm_budget_bytes=1 << 34)
    res = {r.rid: r for r in srv.run(reqs)}
    for req in reqs:
        steps, moves, cost, off, cust = alone(tga, req)
        r = res[req.rid]
        assert (r.steps, r.moves, r.cost) == (steps, moves, cost), req.rid


def test_largest_requests_served_equal_oracle_goldens(env):
    """The four largest served cases (about 10^4 customers, Q about 10.5k)
    admitted next to small requests: each result equals the oracle's stored
    trajectory (tests/golden/traj_c5_large.json)."""
    import hashlib
    import json
    import os
    from tests import large_requests
    tga, serve = env
    path = os.path.join(os.path.dirname(__file__), "golden", "traj_c5_large.json")
    if not os.path.exists(path):
        pytest.skip("golden traj_c5_large.json not written")
    with open(path) as f:
        g = json.load(f)["entries"]
    reqs = make_requests(serve, count=6, seed=9, max_steps=20)
    labels = {}
    for j, (label, _) in enumerate(large_requests.cases()):
        inst, sol, req = large_requests.instance(label)
        assert inst.sha256() == g[label]["instance_sha256"]
        rid = 100 + j
        labels[rid] = label
        reqs.insert(2 * j, serve.ServeRequest(rid, 0.001 * j, inst, sol, req.max_steps))
    srv = serve.Server(hbm_budget_bytes=1 << 34)
    res = {r.rid: r for r in srv.run(reqs)}
    assert srv.peak_active > 1
    for rid, label in labels.items():
        r, e = res[rid], g[label]
        assert (r.steps, r.moves, r.cost) == (e["steps"], e["moves_evaluated"], e["final_cost"]), label
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(r.offsets, dtype="<i4").tobytes())
        h.update(np.ascontiguousarray(r.customers, dtype="<i4").tobytes())
        assert h.hexdigest() == e["final_routes_sha256"], label
    for req in reqs:
        if req.rid < 100:
            steps, moves, cost, off, cust = alone(tga, req)
            assert (res[req.rid].steps, res[req.rid].moves, res[req.rid].cost) == (steps, moves, cost)
