"""Input generators (no GPU): reproducible, well-formed, feasible starts."""
import numpy as np
import pytest

import oracle
from paper_2506_17357_amd import workload as W


def test_seeds_reproduce_identical_instances():
    a, b = W.make_vrptw(300, 7), W.make_vrptw(300, 7)
    assert a.sha256() == b.sha256()
    assert W.make_cvrp(300, 7).sha256() != W.make_cvrp(300, 8).sha256()


@pytest.mark.parametrize("maker", [W.make_cvrp, W.make_vrptw])
def test_distance_matrix_well_formed(maker):
    inst = maker(400, 3)
    D = inst.dist
    assert D.dtype == np.int32 and D.shape == (401, 401)
    assert np.array_equal(D, D.T) and not np.any(np.diag(D))
    # round(Euclid) never sits near a .5 tie for integer coordinates
    dx = inst.xy[:, None, 0] - inst.xy[None, :, 0]
    dy = inst.xy[:, None, 1] - inst.xy[None, :, 1]
    e = np.sqrt((dx * dx + dy * dy).astype(np.float64))
    frac = e - np.floor(e)
    assert np.min(np.abs(frac - 0.5)) > 1e-5
    assert np.array_equal(D, np.floor(e + 0.5).astype(np.int32))


@pytest.mark.parametrize("which", ["c1", "c2", "c3"])
def test_sweep_is_a_feasible_partition(which):
    inst, sol = getattr(W, which)()
    assert sol.offsets[0] == 0 and sol.offsets[-1] == inst.n
    assert sorted(sol.customers.tolist()) == list(range(1, inst.n + 1))
    cost, cap_bad, tw_bad = oracle.cost(inst, sol)
    assert cap_bad == 0 and tw_bad == 0 and cost > 0


def test_vrptw_windows_admit_out_and_back_routes():
    inst = W.make_vrptw(500, 11)
    D, nd = inst.dist.astype(np.int64), inst.node4.astype(np.int64)
    arrive = D[0, 1:]
    start = np.maximum(arrive, nd[1:, 1])
    assert np.all(arrive <= nd[1:, 2])
    assert np.all(start + nd[1:, 3] + D[1:, 0] <= nd[0, 2])


def test_batch_and_request_distributions():
    sizes = W.batch_sizes(256)
    assert len(sizes) == 256 and min(sizes) >= 100 and max(sizes) <= 2000
    assert sizes == W.batch_sizes(256)
    reqs = W.request_stream(200, qps=5.0)
    t = [r.arrival_s for r in reqs]
    assert all(b > a for a, b in zip(t, t[1:]))
    assert all(200 <= r.n <= 10000 for r in reqs)
    assert [r.kind for r in reqs[:4]] == ["cvrp", "vrptw", "cvrp", "vrptw"]
    assert 20 < len(reqs) / t[-1] * 4 < 80  # about 5 per second (loose)


def test_random_solution_has_empty_routes_sometimes():
    inst = W.tiny_instance(5, 1, False)
    seen_empty = any(np.any(np.diff(W.random_solution(inst, 6, s).offsets) == 0) for s in range(10))
    assert seen_empty
