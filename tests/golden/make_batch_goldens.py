"""Write the expected local-search trajectories of the batched and served
workloads by running the CPU oracle (test infrastructure).  Calls only
oracle/ and the input generators; the device library is never involved.

  c4        the batched mix: 256 solutions, 100..2000 customers log-uniform,
            even b CVRP / odd b clustered VRPTW (seeds 4000 + b), sweep
            start, 200 local-search steps each (or the local optimum).
  c4_1000   256 CVRP solutions of exactly 1000 customers (seeds 4500 + b),
            20 steps each (the batched-versus-plain comparison at n = 1000).
  c5_large  the largest CVRP and the largest VRPTW request of the served
            stream (200 requests, 200..10000 customers) plus one request of
            exactly 10000 customers of each kind, 5 steps each.

Each entry holds the accepted move ids and deltas, the moves evaluated, the
final cost and a sha256 of the final routes (offsets then customers, int32
little-endian).  One solution per worker process, single-threaded oracle.

    python tests/golden/make_batch_goldens.py [c4 c4_1000 c5_large] [--workers N]
"""
import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2506_17357_amd import workload as W  # noqa: E402
from tests import large_requests  # noqa: E402

C4_STEPS = 200
C4_1000_STEPS = 20
C5_STEPS = large_requests.STEPS


def routes_sha256(offsets, customers) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(offsets, dtype="<i4").tobytes())
    h.update(np.ascontiguousarray(customers, dtype="<i4").tobytes())
    return h.hexdigest()


def served_requests():
    """(label, Request) of the large served cases."""
    return large_requests.cases()


def make_case(task):
    which, key = task
    if which == "c4":
        n = W.batch_sizes()[key]
        inst = W.batch_instance(key, n)
        steps = C4_STEPS
    elif which == "c4_1000":
        inst = W.make_cvrp(1000, 4500 + key, demand_max=100, capacity=1000)
        steps = C4_1000_STEPS
    else:
        req = dict(served_requests())[key]
        inst = W.request_instance(req)
        steps = req.max_steps
    return inst, W.sweep(inst), steps


def run_case(task):
    t0 = time.time()
    inst, sol, steps = make_case(task)
    threads = 1 if task[0] != "c5_large" else 0
    final, ids, deltas, moves = oracle.local_search(inst, sol, max_steps=steps, threads=threads)
    return task, {
        "n": inst.n,
        "has_tw": int(inst.has_tw),
        "R": sol.R,
        "seed": int(inst.seed),
        "instance_sha256": inst.sha256(),
        "max_steps": steps,
        "initial_cost": oracle.cost(inst, sol)[0],
        "steps": int(len(ids)),
        "moves_evaluated": int(moves),
        "final_cost": oracle.cost(inst, final)[0],
        "final_routes_sha256": routes_sha256(final.offsets, final.customers),
        "ids": [int(x) for x in ids],
        "deltas": [int(x) for x in deltas],
    }, time.time() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="*", default=["c4", "c4_1000", "c5_large"])
    ap.add_argument("--workers", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    args = ap.parse_args()
    for which in args.which:
        if which == "c4":
            sizes = W.batch_sizes()
            tasks = sorted(((which, b) for b in range(len(sizes))), key=lambda t: -sizes[t[1]])
        elif which == "c4_1000":
            tasks = [(which, b) for b in range(256)]
        else:
            tasks = [(which, label) for label, _ in served_requests()]
        results = {}
        t0 = time.time()
        if which == "c5_large":  # few, large: one at a time, all threads
            it = map(run_case, tasks)
            for task, res, dt in it:
                results[task[1]] = res
                print(which, task[1], "n", res["n"], "steps", res["steps"], "%.1f s" % dt, flush=True)
        else:
            with mp.Pool(args.workers) as pool:
                for k, (task, res, dt) in enumerate(pool.imap_unordered(run_case, tasks)):
                    results[task[1]] = res
                    print(which, "%d/%d" % (k + 1, len(tasks)), "b", task[1], "n", res["n"],
                          "steps", res["steps"], "%.1f s" % dt, "(%.0f s total)" % (time.time() - t0),
                          flush=True)
        if which == "c5_large":
            entries = {label: results[label] for label, _ in served_requests()}
        else:
            entries = [results[b] for b in sorted(results)]
        out = {
            "what": "best-improvement local search, all five operators, computed by the CPU oracle "
                    "(test infrastructure); final_routes_sha256 hashes the int32 offsets then customers",
            "workload": which,
            "entries": entries,
        }
        with open(os.path.join(HERE, "traj_%s.json" % which), "w") as f:
            json.dump(out, f, separators=(",", ":"))
        print(which, "done in %.0f s" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
