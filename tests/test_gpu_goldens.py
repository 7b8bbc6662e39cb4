"""Every configuration of the batched and served workloads against stored
oracle trajectories (tests/golden/traj_c4.json, traj_c4_1000.json,
traj_c5_large.json, written by tests/golden/make_batch_goldens.py, which
calls only oracle/ and the input generators).

Integer path, so the bar is equality: accepted moves, moves evaluated,
final cost and the final routes (sha256 of the int32 offsets then
customers), for the batched form (HIP graph), the plain form (one solution
per launch sequence) and, for the largest requests, the step-by-step best
move (id, delta) of the host loop.
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

from paper_2506_17357_amd import workload as W
from tests import large_requests

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def load(name):
    path = os.path.join(GOLDEN, "traj_%s.json" % name)
    if not os.path.exists(path):
        pytest.skip("golden %s not written" % name)
    with open(path) as f:
        return json.load(f)


def routes_sha256(offsets, customers) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(offsets, dtype="<i4").tobytes())
    h.update(np.ascontiguousarray(customers, dtype="<i4").tobytes())
    return h.hexdigest()


@pytest.fixture(scope="module")
def tga():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_17357_amd import tga as T
    T.lib()
    return T


def c4_pairs():
    return W.c4()


def c4_1000_pairs():
    return W.c4_uniform()


def check_entry(g, b, steps, moves, cost, S):
    assert (int(steps), int(moves), int(cost)) == (g["steps"], g["moves_evaluated"], g["final_cost"]), \
        (b, int(steps), int(moves), int(cost), g["steps"], g["moves_evaluated"], g["final_cost"])
    off, cust, _ = S.get()
    assert routes_sha256(off, cust) == g["final_routes_sha256"], b


@pytest.fixture(scope="module")
def c4_env(tga):
    g = load("c4")
    pairs = c4_pairs()
    for (inst, _), e in zip(pairs, g["entries"]):
        assert inst.sha256() == e["instance_sha256"]
    insts = [tga.Instance.from_workload(i) for i, _ in pairs]
    sols = [tga.Solution(I, s.offsets, s.customers) for I, (_, s) in zip(insts, pairs)]
    return g, pairs, insts, sols


@pytest.mark.parametrize("autotune", [False, True])
def test_c4_batched_equals_oracle(tga, c4_env, autotune):
    """All 256 solutions of the batched mix, 200 steps in one captured step
    loop, against the oracle."""
    g, pairs, insts, sols = c4_env
    for s, (_, sol) in zip(sols, pairs):
        s.reload(sol.offsets, sol.customers)
    B = tga.Batch(sols)
    if autotune:
        say("autotuned", B.autotune(launches=2))
        for s, (_, sol) in zip(sols, pairs):
            s.reload(sol.offsets, sol.customers)
    steps, moves, cost = B.ls_run(g["entries"][0]["max_steps"], use_graph=True)
    B.close()
    say("c4 batched: accepted", int(steps.sum()), "moves", int(moves.sum()))
    for b, e in enumerate(g["entries"]):
        check_entry(e, b, steps[b], moves[b], cost[b], sols[b])


def test_c4_plain_equals_oracle(tga, c4_env):
    g, pairs, insts, sols = c4_env
    for b, (s, (_, sol)) in enumerate(zip(sols, pairs)):
        s.reload(sol.offsets, sol.customers)
        e = g["entries"][b]
        steps, moves, cost = s.ls_run(e["max_steps"])
        check_entry(e, b, steps, moves, cost, s)


def test_c4_1000_batched_and_plain_equal_oracle(tga):
    g = load("c4_1000")
    pairs = c4_1000_pairs()
    insts = [tga.Instance.from_workload(i) for i, _ in pairs]
    sols = [tga.Solution(I, s.offsets, s.customers) for I, (_, s) in zip(insts, pairs)]
    B = tga.Batch(sols)
    steps, moves, cost = B.ls_run(g["entries"][0]["max_steps"], use_graph=True)
    B.close()
    for b, e in enumerate(g["entries"]):
        assert pairs[b][0].sha256() == e["instance_sha256"]
        check_entry(e, b, steps[b], moves[b], cost[b], sols[b])
    for b, (s, (_, sol)) in enumerate(zip(sols, pairs)):
        s.reload(sol.offsets, sol.customers)
        e = g["entries"][b]
        st, mv, c = s.ls_run(e["max_steps"])
        check_entry(e, b, st, mv, c, s)


@pytest.fixture(scope="module")
def c5_golden():
    return load("c5_large")


@pytest.mark.parametrize("label", [c[0] for c in large_requests.cases()])
def test_c5_large_requests_step_by_step(tga, c5_golden, label):
    """The largest requests (about 10^4 customers, Q about 10.5k: one or two
    rows per LDS sub-block): best move of every step through the host loop,
    then the device loop, against the oracle."""
    e = c5_golden["entries"][label]
    inst, sol, req = large_requests.instance(label)
    assert inst.sha256() == e["instance_sha256"], label
    say(label, "n", inst.n, "R", sol.R, "Q", inst.n + sol.R)
    I = tga.Instance.from_workload(inst)
    S = tga.Solution(I, sol.offsets, sol.customers)
    for step, (mid, d) in enumerate(zip(e["ids"], e["deltas"])):
        m = S.eval()
        assert (m.id, m.delta) == (mid, d), (label, step)
        S.apply(m)
    off, cust, cost = S.get()
    assert cost == e["final_cost"] and routes_sha256(off, cust) == e["final_routes_sha256"]
    S.reload(sol.offsets, sol.customers)
    st, mv, c = S.ls_run(e["max_steps"])
    check_entry(e, label, st, mv, c, S)
