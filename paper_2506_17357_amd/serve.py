"""Served form: continuous batching of local-search requests on one GPU.

Requests (an instance, a starting solution, a step cap) arrive over time.
A request is admitted, first come first served, when its device bytes
(distance matrix, node data, instance and solution workspaces) fit in the
HBM budget still free and a slot of the engine is free.  Requests that
arrive at the same time are taken largest first (most distance-matrix
entries times step cap: the longest runs start first, so none of them
starts late and runs on alone at the end).  Upload threads
(each with its own copy stream) copy its data to the device while the
compute stream keeps stepping the requests already there.

The engine is one slot batch (tga_batch_create_slots): a fixed number of
slots whose members change while it runs.  Every tick enqueues
`steps_per_tick` batched local-search steps of all members (one captured
graph, replayed) plus a copy of the per-slot results into pinned memory;
the host keeps up to two ticks in flight and reads the newest finished
tick's results without waiting.  A member that reached its local optimum or
step cap is skipped by the kernels; the host reads its routes back on a
separate stream (nothing writes a converged solution), frees its slot with
an asynchronous plan update, and returns its memory once the device is past
the last tick that could read it.  Results do not depend on what else is in
the batch: each solution's step reads only its own data.
"""
from __future__ import annotations

import collections
import queue as queue_mod
import threading
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


def admission_order(requests):
    """Requests in the order they are considered for admission: by arrival
    time, and among requests that arrive together the largest first (most
    distance-matrix entries times step cap), then by request id."""
    return sorted(requests, key=lambda r: (r.arrival_s, -(r.inst.n + 1) ** 2 * r.max_steps, r.rid))


class Server:
    def __init__(self, hbm_budget_bytes: int, max_slots: int = 256, op_mask: int = tga.OPS_ALL,
                 device: str = "cuda", steps_per_tick: int = 4, max_sum_q: int = 1 << 20,
                 max_sum_r: int = 1 << 17, autotune: bool = False, ticks_ahead: int = 2,
                 upload_workers: int = 4, schedule: dict | None = None):
        self.budget = int(hbm_budget_bytes)
        self.max_slots = int(max_slots)
        self.steps_per_tick = int(steps_per_tick)
        self.op_mask = op_mask
        self.device = device
        self.max_sum_q = int(max_sum_q)
        self.max_sum_r = int(max_sum_r)
        # Engine schedule: by default the whole LDS for one inter-route
        # workgroup per compute unit, one launch per step.  Requests of 5000
        # to 10^4 customers then get two to three times the rows per
        # sub-block that half the LDS gives (at 10^4: 6 against 2), which
        # matters more for the served mix than a second workgroup per compute
        # unit.  Autotuning the engine on the few members present early in a
        # run had picked smaller budgets that were slower once the engine
        # filled up; autotune=True tunes once instead, when eight members are
        # present.
        if schedule is None and not autotune:
            schedule = {"lds_kb": tga.device_limits()[1] // 1024, "split": 0}
        self.autotune = autotune and schedule is None
        self.schedule = schedule
        self.ticks_ahead = int(ticks_ahead)
        self.compute = torch.cuda.Stream(device=device)
        self.copies = [torch.cuda.Stream(device=device) for _ in range(max(1, int(upload_workers)))]
        self.readback = torch.cuda.Stream(device=device)
        self._stat_lock = threading.Lock()
        self.used = 0
        self.peak_used = 0
        self.peak_active = 0
        self.ticks = 0
        self.rebuilds = 0       # plan updates (membership changes)
        self.rebuild_s = 0.0    # host time spent in them
        self.upload_s = 0.0     # upload worker busy time (all workers)
        self.uploads = 0
        self.config = None

    # ---------------------------------------------------------------- upload
    def _upload_loop(self, copy, todo: queue_mod.Queue, ready: queue_mod.Queue, t0: float):
        while True:
            req = todo.get()
            if req is None:
                return
            try:
                tu = time.perf_counter()
                with torch.cuda.stream(copy):
                    I = tga.Instance.from_workload(req.inst, device=self.device, stream=copy)
                    S = tga.Solution(I, req.sol.offsets, req.sol.customers, stream=copy)
                now = time.perf_counter()
                with self._stat_lock:
                    self.upload_s += now - tu
                    self.uploads += 1
                ready.put((req, I, S, now - t0, None))
            except Exception as e:  # handed to the serving loop, which raises it
                ready.put((req, None, None, 0.0, e))

    # ------------------------------------------------------------------ run
    def run(self, requests: list[ServeRequest], log=None) -> list[ServeResult]:
        """Serve every request in real time (arrival_s relative to the start)."""
        pending = collections.deque(admission_order(requests))
        waiting: collections.deque = collections.deque()
        todo: queue_mod.Queue = queue_mod.Queue()
        ready: queue_mod.Queue = queue_mod.Queue()
        slots = [None] * self.max_slots   # per slot: dict of the member, or None
        retiring: list = []               # (event, entry): memory kept until the event has passed
        results: list[ServeResult] = []
        uploading = 0
        q_used = r_used = 0
        tuned = not self.autotune
        B = tga.SlotBatch(self.max_slots, self.max_sum_q, self.max_sum_r, device=self.device, stream=self.compute)
        if self.schedule is not None:
            B.set_config(int(self.schedule["lds_kb"]), int(self.schedule.get("split", 0)), stream=self.compute)
            self.config = B.config()
        t0 = time.perf_counter()
        workers = [threading.Thread(target=self._upload_loop, args=(c, todo, ready, t0), daemon=True)
                   for c in self.copies]
        for w in workers:
            w.start()
        in_flight = 0      # ticks enqueued and not yet seen finished
        last_seen = -1     # newest tick whose status was processed
        next_tick = 0      # number the next tick will get
        changed = False
        try:
            while pending or waiting or uploading or any(slots) or retiring:
                now = time.perf_counter() - t0
                while pending and pending[0].arrival_s <= now:
                    waiting.append(pending.popleft())
                # release the memory of retired members the device is done with
                keep = []
                for ev, ent in retiring:
                    if ev.query():
                        self.used -= ent["bytes"]
                    else:
                        keep.append((ev, ent))
                retiring = keep
                # admission, first come first served: budget, slots, batch capacity
                free_slots = sum(s is None for s in slots) - uploading
                while waiting and free_slots > 0:
                    req = waiting[0]
                    need = device_bytes(req.inst, req.sol.R)
                    if need > self.budget:
                        raise ValueError("request %d needs %d bytes, more than the whole budget" % (req.rid, need))
                    Q, R = req.inst.n + req.sol.R, req.sol.R
                    if Q > self.max_sum_q or R > self.max_sum_r:
                        raise ValueError("request %d (Q = %d, R = %d) exceeds the engine's size" % (req.rid, Q, R))
                    if self.used + need > self.budget or q_used + Q > self.max_sum_q or r_used + R > self.max_sum_r:
                        break
                    waiting.popleft()
                    self.used += need
                    q_used += Q
                    r_used += R
                    uploading += 1
                    free_slots -= 1
                    todo.put(req)
                self.peak_used = max(self.peak_used, self.used)
                # uploaded requests join free slots
                while True:
                    try:
                        req, I, S, t_adm, err = ready.get_nowait()
                    except queue_mod.Empty:
                        break
                    uploading -= 1
                    if err is not None:
                        raise err
                    k = slots.index(None)
                    S.begin(req.max_steps, stream=self.compute)
                    slots[k] = {"req": req, "inst": I, "sol": S, "bytes": device_bytes(req.inst, req.sol.R),
                                "admitted": t_adm, "joined": next_tick, "Q": req.inst.n + req.sol.R,
                                "R": req.sol.R}
                    changed = True
                active = sum(s is not None for s in slots)
                self.peak_active = max(self.peak_active, active)
                if changed:
                    tb = time.perf_counter()
                    B.set_members([s["sol"] if s else None for s in slots], stream=self.compute)
                    changed = False
                    self.rebuilds += 1
                    self.rebuild_s += time.perf_counter() - tb
                    if not tuned and (active >= 8 or (not pending and not waiting and not uploading)):
                        self.config = B.autotune(self.op_mask, launches=2, stream=self.compute)
                        tuned = True
                if active and in_flight < self.ticks_ahead:
                    B.tick(self.steps_per_tick, self.op_mask, stream=self.compute)
                    next_tick += 1
                    in_flight += 1
                    self.ticks += 1
                tick, conv, steps, moves, cost = B.status()
                if tick > last_seen:
                    in_flight -= tick - last_seen
                    last_seen = tick
                    for k, ent in enumerate(slots):
                        if ent is None or ent["joined"] > tick or not conv[k]:
                            continue
                        S, req = ent["sol"], ent["req"]
                        off, cust, _ = S.get(stream=self.readback)
                        t_done = time.perf_counter() - t0
                        results.append(ServeResult(req.rid, req.inst.n, req.inst.kind, req.arrival_s,
                                                   ent["admitted"], t_done, int(steps[k]), int(moves[k]),
                                                   int(cost[k]), off, cust))
                        if log:
                            log("request %d (n=%d) done: %d steps, latency %.3f s"
                                % (req.rid, req.inst.n, int(steps[k]), t_done - req.arrival_s))
                        slots[k] = None
                        q_used -= ent["Q"]
                        r_used -= ent["R"]
                        changed = True
                        ent["retired"] = True
                        retiring.append((None, ent))
                    if changed:
                        tb = time.perf_counter()
                        B.set_members([s["sol"] if s else None for s in slots], stream=self.compute)
                        changed = False
                        self.rebuilds += 1
                        self.rebuild_s += time.perf_counter() - tb
                        ev = torch.cuda.Event()
                        ev.record(self.compute)
                        retiring = [(ev if e is None else e, ent) for e, ent in retiring]
                elif in_flight >= self.ticks_ahead or (not active and (uploading or retiring)):
                    time.sleep(5e-5)
                elif not active and pending and not waiting and not uploading:
                    time.sleep(max(0.0, min(0.001, pending[0].arrival_s - (time.perf_counter() - t0))))
        finally:
            for _ in workers:
                todo.put(None)
            for w in workers:
                w.join()
            torch.cuda.synchronize()
            B.close()
        return sorted(results, key=lambda r: r.rid)
