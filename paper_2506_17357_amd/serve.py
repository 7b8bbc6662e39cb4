"""Served form: continuous batching of local-search requests on one GPU.

Requests (an instance, a starting solution, a step cap) arrive over time.
A request is admitted when its device bytes (distance matrix, node data,
instance and solution workspaces) fit in the HBM budget still free; its data
are uploaded on a copy stream while the compute stream keeps stepping the
requests already on the device.  Every engine tick runs `steps_per_tick`
batched steps (each one persistent evaluation launch + one finalize launch;
two by default, which halves the host polls at the cost of at most one
step of latency) over all admitted requests; a request leaves when it reaches a local optimum or its cap, its
memory is returned, and queued requests are admitted.  Results do not depend
on what else is in the batch: each solution's step only reads its own data.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import tga


@dataclass
class ServeRequest:
    rid: int
    arrival_s: float
    inst: object          # workload.Instance
    sol: object           # workload.Solution (starting routes)
    max_steps: int


@dataclass
class ServeResult:
    rid: int
    n: int
    kind: str
    arrival_s: float
    admitted_s: float
    done_s: float
    steps: int
    moves: int
    cost: int
    offsets: np.ndarray = field(repr=False)
    customers: np.ndarray = field(repr=False)

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


def device_bytes(inst, R: int) -> int:
    """Device bytes one request keeps resident while it is served."""
    L = tga.lib()
    return (4 * (inst.n + 1) ** 2 + 16 * (inst.n + 1) + int(L.tga_instance_workspace_bytes(inst.n))
            + int(L.tga_solution_workspace_bytes(inst.n, R)))


class Server:
    def __init__(self, hbm_budget_bytes: int, max_slots: int = 256, op_mask: int = tga.OPS_ALL,
                 device: str = "cuda", steps_per_tick: int = 2):
        self.budget = int(hbm_budget_bytes)
        self.max_slots = int(max_slots)
        self.steps_per_tick = int(steps_per_tick)
        self.op_mask = op_mask
        self.device = device
        self.compute = torch.cuda.Stream(device=device)
        self.copy = torch.cuda.Stream(device=device)
        self.used = 0
        self.peak_used = 0
        self.peak_active = 0
        self.ticks = 0
        self.rebuilds = 0
        self.rebuild_s = 0.0

    def _admit(self, req: ServeRequest, t0: float):
        with torch.cuda.stream(self.copy):
            I = tga.Instance.from_workload(req.inst, device=self.device, stream=self.copy)
            S = tga.Solution(I, req.sol.offsets, req.sol.customers, stream=self.copy)
            S.begin(req.max_steps, stream=self.copy)
        self.copy.synchronize()
        return {"req": req, "inst": I, "sol": S, "bytes": device_bytes(req.inst, req.sol.R),
                "admitted": time.perf_counter() - t0}

    def run(self, requests: list[ServeRequest], log=None) -> list[ServeResult]:
        """Serve every request in real time (arrival_s relative to the start)."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival_s))
        queue: collections.deque = collections.deque()
        active: list[dict] = []
        results: list[ServeResult] = []
        batch = None
        dirty = False
        t0 = time.perf_counter()
        while pending or queue or active:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival_s <= now:
                queue.append(pending.popleft())
            while queue and len(active) < self.max_slots:
                need = device_bytes(queue[0].inst, queue[0].sol.R)
                if need > self.budget:
                    raise ValueError("request %d needs %d bytes, more than the whole budget"
                                     % (queue[0].rid, need))
                if self.used + need > self.budget:
                    break
                req = queue.popleft()
                active.append(self._admit(req, t0))
                self.used += need
                dirty = True
            self.peak_used = max(self.peak_used, self.used)
            self.peak_active = max(self.peak_active, len(active))
            if not active:
                if pending:
                    time.sleep(max(0.0, min(0.001, pending[0].arrival_s - (time.perf_counter() - t0))))
                continue
            if dirty:
                tb = time.perf_counter()
                if batch is not None:
                    batch.close()
                with torch.cuda.stream(self.compute):
                    batch = tga.Batch([a["sol"] for a in active], stream=self.compute)
                dirty = False
                self.rebuilds += 1
                self.rebuild_s += time.perf_counter() - tb
            for _ in range(self.steps_per_tick):  # a finished solution skips the rest of a tick
                batch.step_part(0, self.op_mask, stream=self.compute)
                batch.step_part(1, self.op_mask, stream=self.compute)
            self.ticks += 1
            done = batch.poll(stream=self.compute)
            if done.any():
                t_done = time.perf_counter() - t0
                keep = []
                for a, d in zip(active, done):
                    if not d:
                        keep.append(a)
                        continue
                    S, req = a["sol"], a["req"]
                    steps, _, moves, cost = S.stats(stream=self.compute)
                    off, cust, _ = S.get(stream=self.compute)
                    results.append(ServeResult(req.rid, req.inst.n, req.inst.kind, req.arrival_s,
                                               a["admitted"], t_done, steps, moves, cost, off, cust))
                    self.used -= a["bytes"]
                    if log:
                        log("request %d (n=%d) done: %d steps, latency %.3f s"
                            % (req.rid, req.inst.n, steps, t_done - req.arrival_s))
                batch.close()
                batch = None
                active = keep
                dirty = bool(active)
        if batch is not None:
            batch.close()
        return sorted(results, key=lambda r: r.rid)
