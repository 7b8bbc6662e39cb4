"""Seeded synthetic workloads: CVRP / VRPTW instances, sweep starting solutions,
the batched mix and the Poisson request stream.

This module builds inputs only.  It contains no move evaluation, no move
application and no best-move selection; the device library and the CPU oracle
both consume what it produces and neither depends on it for correctness (a
starting solution that happened to be infeasible would be handled by both
sides through the same definitions).

Instance families (Section 2 defines the problems; the paper's own benchmark
suites X and Gehring-Homberger are not available, so these seeded generators
stand in for them with the shapes the paper's experiments use: uniform CVRP up
to 1000 customers, clustered VRPTW):

* ``make_cvrp``: integer coordinates uniform in [0, 1000]^2, depot at
  (500, 500), integer demands, one capacity.
* ``make_vrptw``: 8 Gaussian clusters (sigma 60, clipped to the square),
  service time 10, depot window [0, 5000], a window per customer whose centre
  is uniform over the range that keeps the out-and-back route feasible.

Distances are round(Euclidean) = floor(sqrt(dx^2 + dy^2) + 0.5) computed in
float64 and stored as int32.  For integer dx, dy the square root of an integer
is never within 8e-5 of m + 0.5 for the sizes used here, so the rounding mode
cannot change a value.  Travel time equals distance.
"""
from __future__ import annotations

import functools
import hashlib
import math
from dataclasses import dataclass, field

import numpy as np

BIG_WINDOW = 1 << 26  # "no time window" upper bound used for CVRP node data


@dataclass
class Instance:
    """One routing instance.

    ``dist`` is (n+1) x (n+1) int32, row-major, node 0 is the depot.
    ``node4`` is (n+1) x 4 int32 holding (demand, e, l, s) per node.
    """
    n: int
    dist: np.ndarray
    node4: np.ndarray
    capacity: int
    has_tw: int
    xy: np.ndarray
    kind: str
    seed: int
    meta: dict = field(default_factory=dict)
    pickup: np.ndarray | None = None  # (n+1,) int32 pickup amounts (VRPSPDTW), node 0 = 0

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64([self.n, self.capacity, self.has_tw]).tobytes())
        h.update(np.ascontiguousarray(self.dist).tobytes())
        h.update(np.ascontiguousarray(self.node4).tobytes())
        if self.pickup is not None:
            h.update(np.ascontiguousarray(self.pickup, dtype=np.int32).tobytes())
        return h.hexdigest()


@dataclass
class Solution:
    """Routes as CSR: route r holds customers[offsets[r]:offsets[r+1]]."""
    offsets: np.ndarray  # int32, R+1
    customers: np.ndarray  # int32, n (ids 1..n)

    @property
    def R(self) -> int:
        return int(self.offsets.shape[0] - 1)

    def routes(self) -> list[list[int]]:
        o = self.offsets
        return [self.customers[o[r]:o[r + 1]].tolist() for r in range(self.R)]

    @staticmethod
    def from_routes(routes: list[list[int]]) -> "Solution":
        off = [0]
        cust: list[int] = []
        for r in routes:
            cust.extend(int(c) for c in r)
            off.append(len(cust))
        return Solution(np.asarray(off, np.int32), np.asarray(cust, np.int32))


def round_euclid(xy: np.ndarray) -> np.ndarray:
    """int32 matrix of floor(|p_i - p_j| + 0.5), built in row blocks."""
    m = xy.shape[0]
    out = np.empty((m, m), np.int32)
    x = xy[:, 0].astype(np.float64)
    y = xy[:, 1].astype(np.float64)
    blk = max(1, (1 << 24) // max(m, 1))
    for r0 in range(0, m, blk):
        r1 = min(m, r0 + blk)
        dx = x[r0:r1, None] - x[None, :]
        dy = y[r0:r1, None] - y[None, :]
        out[r0:r1] = np.floor(np.sqrt(dx * dx + dy * dy) + 0.5).astype(np.int32)
    return out


def make_cvrp(n: int, seed: int, demand_max: int = 100, capacity: int = 1000) -> Instance:
    rng = np.random.Generator(np.random.PCG64(seed))
    xy = np.empty((n + 1, 2), np.int64)
    xy[0] = (500, 500)
    xy[1:] = rng.integers(0, 1001, size=(n, 2))
    node4 = np.zeros((n + 1, 4), np.int32)
    node4[1:, 0] = rng.integers(1, demand_max + 1, size=n)
    node4[:, 1] = 0
    node4[:, 2] = BIG_WINDOW
    node4[:, 3] = 0
    return Instance(n, round_euclid(xy), node4, capacity, 0, xy, "cvrp", seed,
                    {"demand_max": demand_max})


def make_vrptw(n: int, seed: int, clusters: int = 8, sigma: float = 60.0,
               service: int = 10, horizon: int = 5000, demand_max: int = 30,
               capacity: int = 200) -> Instance:
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.integers(0, 1001, size=(clusters, 2))
    which = rng.integers(0, clusters, size=n)
    pts = centres[which].astype(np.float64) + rng.normal(0.0, sigma, size=(n, 2))
    pts = np.clip(np.floor(pts + 0.5), 0, 1000).astype(np.int64)
    xy = np.empty((n + 1, 2), np.int64)
    xy[0] = (500, 500)
    xy[1:] = pts
    dist = round_euclid(xy)
    node4 = np.zeros((n + 1, 4), np.int32)
    node4[1:, 0] = rng.integers(1, demand_max + 1, size=n)
    node4[0] = (0, 0, horizon, 0)
    d0 = dist[0, 1:].astype(np.int64)
    lo = d0
    hi = horizon - service - d0
    centre = lo + np.floor(rng.random(n) * (hi - lo + 1)).astype(np.int64)
    width = rng.integers(100, 601, size=n)
    node4[1:, 1] = np.maximum(0, centre - width // 2)
    node4[1:, 2] = centre + (width + 1) // 2
    node4[1:, 3] = service
    return Instance(n, dist, node4, capacity, 1, xy, "vrptw", seed,
                    {"clusters": clusters, "sigma": sigma, "horizon": horizon})


def make_vrpspdtw(n: int, seed: int, pickup_max: int = 30, **kw) -> Instance:
    """Clustered VRPTW (as make_vrptw) with a pickup amount per customer,
    uniform 1..pickup_max: simultaneous pickup and delivery with windows."""
    inst = make_vrptw(n, seed, **kw)
    rng = np.random.Generator(np.random.PCG64(seed + (1 << 20)))
    pick = np.zeros(n + 1, np.int32)
    pick[1:] = rng.integers(1, pickup_max + 1, size=n)
    inst.pickup = pick
    inst.kind = "vrpspdtw"
    inst.meta["pickup_max"] = pickup_max
    return inst


def peak_load(inst: Instance, route: list[int]) -> int:
    """Largest load the vehicle carries on the route: all deliveries at the
    depot, then at each customer its delivery off and its pickup on."""
    q = sum(int(inst.node4[c, 0]) for c in route)
    if inst.pickup is None:
        return q
    peak = q
    for c in route:
        q += int(inst.pickup[c]) - int(inst.node4[c, 0])
        peak = max(peak, q)
    return peak


# ---------------------------------------------------------------- sweep -----

def _angle_order(inst: Instance) -> list[int]:
    """Customers sorted by polar angle about the depot, starting at +x,
    counter-clockwise, with an exact integer comparator (half-plane, cross
    product, squared radius, id)."""
    x0, y0 = inst.xy[0]
    vec = [(int(inst.xy[i, 0] - x0), int(inst.xy[i, 1] - y0)) for i in range(inst.n + 1)]

    def half(v):
        dx, dy = v
        return 0 if (dy > 0 or (dy == 0 and dx >= 0)) else 1

    def cmp(i, j):
        a, b = vec[i], vec[j]
        ha, hb = half(a), half(b)
        if ha != hb:
            return ha - hb
        cr = a[0] * b[1] - a[1] * b[0]
        if cr != 0:
            return -1 if cr > 0 else 1
        ra = a[0] * a[0] + a[1] * a[1]
        rb = b[0] * b[0] + b[1] * b[1]
        if ra != rb:
            return -1 if ra < rb else 1
        return i - j

    return sorted(range(1, inst.n + 1), key=functools.cmp_to_key(cmp))


def _tw_schedule_ok(inst: Instance, route: list[int]) -> bool:
    """Construction-time check used only to build a sensible starting point."""
    D, nd = inst.dist, inst.node4
    t = int(nd[0, 1])
    prev = 0
    for c in route:
        a = t + int(nd[prev, 3]) + int(D[prev, c])
        if a > int(nd[c, 2]):
            return False
        t = max(a, int(nd[c, 1]))
        prev = c
    return t + int(nd[prev, 3]) + int(D[prev, 0]) <= int(nd[0, 2])


def sweep(inst: Instance) -> Solution:
    """Sweep construction.  CVRP: fill routes in angle order up to capacity.
    VRPTW (and VRPSPDTW): insert each customer (angle order) at the cheapest
    position of the current route that keeps capacity (the peak load with
    pickups) and windows, else open a new route."""
    order = _angle_order(inst)
    dem = inst.node4[:, 0]
    D = inst.dist
    routes: list[list[int]] = []
    cur: list[int] = []
    load = 0
    for c in order:
        d = int(dem[c])
        if not inst.has_tw:
            if cur and load + d > inst.capacity:
                routes.append(cur)
                cur, load = [], 0
            cur.append(c)
            load += d
            continue
        best = None
        if cur and load + d <= inst.capacity:
            seq = [0] + cur + [0]
            for p in range(len(cur) + 1):
                a, b = seq[p], seq[p + 1]
                inc = int(D[a, c]) + int(D[c, b]) - int(D[a, b])
                if best is not None and inc >= best[0]:
                    continue
                cand = cur[:p] + [c] + cur[p:]
                if _tw_schedule_ok(inst, cand) and (inst.pickup is None or peak_load(inst, cand) <= inst.capacity):
                    best = (inc, p)
        if best is None:
            if cur:
                routes.append(cur)
            cur, load = [c], d
        else:
            cur.insert(best[1], c)
            load += d
    if cur:
        routes.append(cur)
    return Solution.from_routes(routes)


# ------------------------------------------------------------ workloads -----

def c1() -> tuple[Instance, Solution]:
    """Plain CVRP, 100 customers, demand 1..10, capacity 50, seed 101."""
    inst = make_cvrp(100, 101, demand_max=10, capacity=50)
    return inst, sweep(inst)


def c6(n: int = 1000) -> tuple[Instance, Solution]:
    """VRPSPDTW, n customers (default 1000), the clustered VRPTW generator
    with pickups 1..30, seed 106."""
    inst = make_vrpspdtw(n, 106)
    return inst, sweep(inst)


def c2() -> tuple[Instance, Solution]:
    """Plain CVRP, 1000 customers, demand 1..100, capacity 1000, seed 102."""
    inst = make_cvrp(1000, 102, demand_max=100, capacity=1000)
    return inst, sweep(inst)


def c3() -> tuple[Instance, Solution]:
    """Plain clustered VRPTW, 1000 customers, seed 103."""
    inst = make_vrptw(1000, 103)
    return inst, sweep(inst)


def batch_sizes(count: int = 256, lo: int = 100, hi: int = 2000, seed: int = 3999) -> list[int]:
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random(count)
    return [int(round(math.exp(math.log(lo) + x * (math.log(hi) - math.log(lo))))) for x in u]


def batch_instance(b: int, n: int) -> Instance:
    """Solution b of the batched mix: even b uses the 1000-customer CVRP
    generator parameters, odd b the VRPTW generator; seed 4000 + b."""
    if b % 2 == 0:
        return make_cvrp(n, 4000 + b, demand_max=100, capacity=1000)
    return make_vrptw(n, 4000 + b)


def c4(count: int = 256) -> list[tuple[Instance, Solution]]:
    out = []
    for b, n in enumerate(batch_sizes(count)):
        inst = batch_instance(b, n)
        out.append((inst, sweep(inst)))
    return out


def c4_uniform(count: int = 256, n: int = 1000) -> list[tuple[Instance, Solution]]:
    """256 CVRP solutions of exactly n customers (seed 4500 + b): the
    plain-versus-batched comparison at n = 1000."""
    out = []
    for b in range(count):
        inst = make_cvrp(n, 4500 + b, demand_max=100, capacity=1000)
        out.append((inst, sweep(inst)))
    return out


@dataclass
class Request:
    k: int
    arrival_s: float
    n: int
    kind: str
    max_steps: int


def request_stream(count: int, qps: float, lo: int = 200, hi: int = 10000,
                   max_steps: int = 500, seed: int = 5999) -> list[Request]:
    """Poisson arrivals at ``qps``; sizes log-uniform over [lo, hi];
    CVRP and VRPTW alternate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / qps, size=count)
    u = rng.random(count)
    t = 0.0
    out = []
    for k in range(count):
        t += float(gaps[k])
        n = int(round(math.exp(math.log(lo) + u[k] * (math.log(hi) - math.log(lo)))))
        out.append(Request(k, t, n, "cvrp" if k % 2 == 0 else "vrptw", max_steps))
    return out


def request_instance(req: Request) -> Instance:
    if req.kind == "cvrp":
        return make_cvrp(req.n, 5000 + req.k, demand_max=100, capacity=1000)
    return make_vrptw(req.n, 5000 + req.k)


def random_solution(inst: Instance, R: int, seed: int) -> Solution:
    """A random partition of the customers into R ordered routes (some may be
    empty); used for edge-case tests, not for benchmarks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    perm = rng.permutation(np.arange(1, inst.n + 1))
    cuts = np.sort(rng.integers(0, inst.n + 1, size=R - 1))
    off = np.concatenate([[0], cuts, [inst.n]]).astype(np.int32)
    return Solution(off, perm.astype(np.int32))


def tiny_instance(n: int, seed: int, has_tw: bool, capacity: int | None = None,
                  span: int = 100, dup: bool = False) -> Instance:
    """Small random instance for exhaustive tests.  ``dup`` forces repeated
    coordinates so that exact ties between moves occur."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xy = np.empty((n + 1, 2), np.int64)
    xy[0] = (span // 2, span // 2)
    if dup:
        base = rng.integers(0, span + 1, size=(max(1, n // 2), 2))
        xy[1:] = base[rng.integers(0, base.shape[0], size=n)]
    else:
        xy[1:] = rng.integers(0, span + 1, size=(n, 2))
    dist = round_euclid(xy)
    node4 = np.zeros((n + 1, 4), np.int32)
    node4[1:, 0] = rng.integers(1, 10, size=n)
    cap = int(capacity) if capacity is not None else int(node4[:, 0].sum() // 2 + 5)
    if has_tw:
        horizon = 8 * span
        node4[0] = (0, 0, horizon, 0)
        c = rng.integers(0, horizon // 2, size=n)
        w = rng.integers(span // 4, span * 2, size=n)
        node4[1:, 1] = np.maximum(0, c - w // 2)
        node4[1:, 2] = c + w
        node4[1:, 3] = rng.integers(0, 5, size=n)
    else:
        node4[:, 2] = BIG_WINDOW
    return Instance(n, dist, node4, cap, int(has_tw), xy, "tiny", seed)
