"""The largest requests of the served workload, shared by the golden writer
(tests/golden/make_batch_goldens.py) and the GPU tests: the largest CVRP and
the largest VRPTW request of the 200-request stream (200..10000 customers,
seeds 5000 + k) and one request of exactly 10000 customers of each kind,
5 local-search steps each."""
import functools

from paper_2506_17357_amd import workload as W

STEPS = 5


def cases():
    """[(label, workload.Request)] in a fixed order."""
    stream = W.request_stream(200, qps=1.0)
    out = []
    for kind in ("cvrp", "vrptw"):
        big = max((r for r in stream if r.kind == kind), key=lambda r: r.n)
        out.append(("stream_k%d" % big.k, W.Request(big.k, 0.0, big.n, kind, STEPS)))
    out.append(("n10000_cvrp", W.Request(10000, 0.0, 10000, "cvrp", STEPS)))
    out.append(("n10000_vrptw", W.Request(10001, 0.0, 10000, "vrptw", STEPS)))
    return out


@functools.lru_cache(maxsize=None)
def instance(label):
    """(Instance, sweep Solution, Request) of one case, generated once per process."""
    req = dict(cases())[label]
    inst = W.request_instance(req)
    return inst, W.sweep(inst), req
