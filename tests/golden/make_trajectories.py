"""Write the expected local-search trajectories of the three single-solution
workloads (100-customer CVRP, 1000-customer CVRP, 1000-customer clustered
VRPTW) by running the CPU oracle.  Calls only oracle/ and the input
generators; the device library is never involved.

    python tests/golden/make_trajectories.py [c1 c2 c3]
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2506_17357_amd import workload as W  # noqa: E402


def main(which):
    for w in which:
        inst, sol = getattr(W, w)()
        final, ids, deltas, moves = oracle.local_search(inst, sol, max_steps=1_000_000, threads=0)
        out = {
            "what": "best-improvement local search to a local optimum, all five operators, "
                    "computed by the CPU oracle (test infrastructure)",
            "workload": w,
            "instance_sha256": inst.sha256(),
            "initial_cost": oracle.cost(inst, sol)[0],
            "final_cost": oracle.cost(inst, final)[0],
            "moves_evaluated": moves,
            "ids": [int(x) for x in ids],
            "deltas": [int(x) for x in deltas],
            "final_offsets": final.offsets.tolist(),
            "final_customers": final.customers.tolist(),
        }
        with open(os.path.join(HERE, "traj_%s.json" % w), "w") as f:
            json.dump(out, f)
        print(w, "steps", len(ids), "final", out["final_cost"], flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1", "c2", "c3"])
