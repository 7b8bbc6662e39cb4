"""Autotuner of the per-size schedules: rows per inter-route work item of the
single-solution form (plain_rows) and of the batched form (item_rows), per
problem kind (CVRP, VRPTW) and size bucket.

For every (kind, n) bucket it builds seeded instances of that size with the
workload generators, times every candidate schedule on the device over the
same local-search steps and checks that every candidate gives the same
trajectory (steps, moves evaluated, cost: a schedule never changes a
result), then
writes the winners as a table (JSON) that tga.load_tuning / tga_set_tuning
install.  Bucket n covers sizes up to the geometric midpoint to the next
bucket.

    python -m paper_2506_17357_amd.autotune --out paper_2506_17357_amd/tune_table.json
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import tga, workload as W

BUCKETS = (100, 200, 500, 1000, 2000, 5000, 10000)
PLAIN_CANDIDATES = (1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64)
ITEM_CANDIDATES = (0, 2, 4, 8, 16, 32, 64, 128)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def instance(kind: str, n: int, seed: int):
    inst = W.make_cvrp(n, seed) if kind == "cvrp" else W.make_vrptw(n, seed)
    return inst, W.sweep(inst)


def tune_plain(kind: str, n: int, steps: int = 30, reps: int = 3):
    """Time per local-search step of the single-solution form (tga_ls_run
    from the same start, best of `reps`) per rows-per-item candidate; every
    candidate must give the same steps, moves and cost.  Returns (best rows,
    {rows: us per step}, the built-in rule's rows)."""
    inst, sol = instance(kind, n, 7000 + n + (kind != "cvrp"))
    I = tga.Instance.from_workload(inst)
    S = tga.Solution(I, sol.offsets, sol.customers)
    default = S.rows()[0]
    seen, times, ref = set(), {}, None
    for c in sorted(set(PLAIN_CANDIDATES) | {default}):
        S.set_rows(c, 0)
        eff = S.rows()[0]
        if eff in seen:
            continue
        seen.add(eff)
        best = float("inf")
        for _ in range(reps):
            S.reload(sol.offsets, sol.customers)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = S.ls_run(steps)
            torch.cuda.synchronize()
            best = min(best, (time.perf_counter() - t0) / max(1, res[0]) * 1e6)
            if ref is None:
                ref = res
            assert res == ref, ("schedule changed the trajectory", kind, n, eff, res, ref)
        times[eff] = best
    S.set_rows(0, 0)
    return min(times, key=times.get), times, default


def tune_batched(kind: str, n: int, steps: int = 20):
    """Mean evaluation-launch time (HIP events on the launching stream) over
    `steps` local-search steps of a batch of solutions of this bucket, from
    the same start, per item-rows candidate (the batch's LDS budget and
    launch split autotuned once first); every candidate must give the same
    steps, moves and costs.  Returns (best item rows, {rows: us}, schedule,
    solutions)."""
    count = int(min(64, max(2, round(2e4 / n))))
    pairs = [instance(kind, n, 7500 + 97 * b + n) for b in range(count)]
    insts = [tga.Instance.from_workload(i) for i, _ in pairs]
    sols = [tga.Solution(I, s.offsets, s.customers) for I, (_, s) in zip(insts, pairs)]
    B = tga.Batch(sols)
    cfg = B.autotune(launches=3)
    B.close()
    times, ref = {}, None
    for c in ITEM_CANDIDATES:
        for s, (_, sol) in zip(sols, pairs):
            s.set_rows(0, c)
            s.reload(sol.offsets, sol.customers)
        B = tga.Batch(sols)
        B.set_config(cfg["lds_kb"], cfg["split"])
        ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        torch.cuda.synchronize()
        B.begin(steps)
        for k in range(steps):
            ev0[k].record()
            B.step_part(0)
            ev1[k].record()
            B.step_part(1)
        torch.cuda.synchronize()
        res = tuple(x.tolist() for x in B.collect())
        if ref is None:
            ref = res
        assert res == ref, ("schedule changed a trajectory", kind, n, c)
        times[c] = float(np.mean([a.elapsed_time(b) for a, b in zip(ev0, ev1)])) * 1e3
        B.close()
    for s in sols:
        s.set_rows(0, 0)
    return min(times, key=times.get), times, cfg, count


def bucket_bounds(buckets):
    """n_max of each bucket: the geometric midpoint to the next one, the last
    one open (TGA_MAX_Q)."""
    out = []
    for k, n in enumerate(buckets):
        out.append(int(math.floor(math.sqrt(n * buckets[k + 1]))) if k + 1 < len(buckets) else 14654)
    return out


def run(buckets=BUCKETS, kinds=("cvrp", "vrptw"), steps_plain=30, steps_batch=20):
    torch.cuda.set_device(0)
    tga.set_tuning([])  # measure from the built-in rule, whatever table is installed
    entries, meas = [], []
    bounds = bucket_bounds(buckets)
    for kind in kinds:
        for n, n_max in zip(buckets, bounds):
            t0 = time.time()
            pr, pt, pdef = tune_plain(kind, n, steps_plain)
            ir, it, cfg, count = tune_batched(kind, n, steps_batch)
            entries.append({"kind": kind, "n_max": n_max, "plain_rows": pr, "item_rows": ir})
            meas.append({"kind": kind, "n": n, "plain_default_rows": pdef,
                         "plain_us_per_step": {str(k): round(v, 1) for k, v in pt.items()},
                         "batched_us_per_eval_launch": {str(k): round(v, 1) for k, v in it.items()},
                         "batch": {"solutions": count, "lds_kb": cfg["lds_kb"], "split": cfg["split"]}})
            log("%s n=%d: plain rows %d (%.1f us per step; built-in rule %d rows: %.1f us), batched item rows "
                "%d (%.1f us per launch; built-in rule %.1f us) [%.1f s]" % (
                    kind, n, pr, pt[pr], pdef, pt[pdef], ir, it[ir], it[0], time.time() - t0))
    return entries, meas


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="gpurun_out/tune_table.json")
    ap.add_argument("--buckets", default=",".join(map(str, BUCKETS)))
    ap.add_argument("--kinds", default="cvrp,vrptw")
    args = ap.parse_args()
    buckets = tuple(int(x) for x in args.buckets.split(","))
    entries, meas = run(buckets, tuple(args.kinds.split(",")))
    doc = {"device": torch.cuda.get_device_name(0),
           "command": "python -m paper_2506_17357_amd.autotune " + " ".join(sys.argv[1:]),
           "entries": entries, "measurements": meas}
    with open(args.out, "w") as f:
        json.dump(doc, f, indent=1)
    log("wrote", args.out)


if __name__ == "__main__":
    main()
