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
    count = int(min(256, max(2, round(1.5e5 / n))))
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


def _mix_launch_us(sols, pairs, rows, group_of, cfg, steps, reps, ref):
    """Mean evaluation-launch time of the batch with per-group item rows
    (best of `reps` passes of `steps` local-search steps from the start);
    checks every pass against the reference trajectory `ref` (a list that
    the first call fills)."""
    for s, (inst, sol) in zip(sols, pairs):
        s.set_rows(0, rows[group_of(inst)])
    B = tga.Batch(sols)
    B.set_config(cfg["lds_kb"], cfg["split"])
    best = float("inf")
    for _ in range(reps):
        for s, (_, sol) in zip(sols, pairs):
            s.reload(sol.offsets, sol.customers)
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
        if not ref:
            ref.append(res)
        assert res == ref[0], "schedule changed a trajectory of the mix"
        best = min(best, float(np.mean([a.elapsed_time(b) for a, b in zip(ev0, ev1)])) * 1e3)
    B.close()
    return best


def tune_mix(buckets=BUCKETS, steps=40, reps=2, gain=0.01):
    """Item rows of the batched form per (kind, bucket) in the context of the
    benchmark's mixed batch (256 solutions, 100..2000 customers, CVRP and
    VRPTW): coordinate descent over the groups, largest total work first,
    keeping a candidate only when it shortens the whole launch by more than
    `gain`.  Returns ({(kind, bucket n): rows}, launch us before, after)."""
    bounds = bucket_bounds(buckets)

    def group_of(inst):
        kind = "vrptw" if inst.has_tw else "cvrp"
        return kind, next(b for b, m in zip(buckets, bounds) if inst.n <= m)

    pairs = W.c4()
    insts = [tga.Instance.from_workload(i) for i, _ in pairs]
    sols = [tga.Solution(I, s.offsets, s.customers) for I, (_, s) in zip(insts, pairs)]
    work = {}
    for inst, _ in pairs:
        work[group_of(inst)] = work.get(group_of(inst), 0) + inst.n ** 2
    rows = {g: 0 for g in work}
    B = tga.Batch(sols)
    cfg = B.autotune(launches=3)
    B.close()
    ref = []
    base = first = _mix_launch_us(sols, pairs, rows, group_of, cfg, steps, reps, ref)
    for g in sorted(work, key=work.get, reverse=True):
        for c in ITEM_CANDIDATES[1:]:
            trial = dict(rows)
            trial[g] = c
            t = _mix_launch_us(sols, pairs, trial, group_of, cfg, steps, reps, ref)
            if t < base * (1 - gain):
                rows, base = trial, t
        log("mix: %s n~%d -> item rows %d (launch %.1f us)" % (g[0], g[1], rows[g], base))
    for s in sols:
        s.set_rows(0, 0)
    return rows, first, base


def bucket_bounds(buckets):
    """n_max of each bucket: the geometric midpoint to the next one, the last
    one open (TGA_MAX_Q)."""
    out = []
    for k, n in enumerate(buckets):
        out.append(int(math.floor(math.sqrt(n * buckets[k + 1]))) if k + 1 < len(buckets) else 14654)
    return out


def run(buckets=BUCKETS, kinds=("cvrp", "vrptw"), steps_plain=30, steps_batch=20, mix=True, gain=0.03):
    """The table: plain rows from tune_plain; batched item rows from
    tune_mix for the groups the benchmark's mix holds, else from
    tune_batched when the winner beats the built-in rule by more than
    `gain` (smaller differences are within run-to-run noise)."""
    torch.cuda.set_device(0)
    tga.set_tuning([])  # measure from the built-in rule, whatever table is installed
    entries, meas = [], []
    bounds = bucket_bounds(buckets)
    mix_rows, mix_meas = {}, None
    if mix:
        mix_rows, before, after = tune_mix(buckets)
        mix_meas = {"workload": "the benchmark's batched mix (256 solutions)", "launch_us_built_in": round(before, 1),
                    "launch_us_tuned": round(after, 1),
                    "rows": {"%s/%d" % g: r for g, r in sorted(mix_rows.items())}}
    for kind in kinds:
        for n, n_max in zip(buckets, bounds):
            t0 = time.time()
            pr, pt, pdef = tune_plain(kind, n, steps_plain)
            ir, it, cfg, count = tune_batched(kind, n, steps_batch)
            if (kind, n) in mix_rows:
                ir = mix_rows[(kind, n)]
            elif it[ir] > it[0] * (1 - gain):
                ir = 0
            entries.append({"kind": kind, "n_max": n_max, "plain_rows": pr, "item_rows": ir})
            meas.append({"kind": kind, "n": n, "plain_default_rows": pdef,
                         "plain_us_per_step": {str(k): round(v, 1) for k, v in pt.items()},
                         "batched_us_per_eval_launch": {str(k): round(v, 1) for k, v in it.items()},
                         "batch": {"solutions": count, "lds_kb": cfg["lds_kb"], "split": cfg["split"]}})
            log("%s n=%d: plain rows %d (%.1f us per step; built-in rule %d rows: %.1f us), batched item rows "
                "%d (homogeneous batch: %s) [%.1f s]" % (
                    kind, n, pr, pt[pr], pdef, pt[pdef], ir,
                    ", ".join("%d: %.1f us" % kv for kv in sorted(it.items())), time.time() - t0))
    if mix_meas:
        meas.append({"mix": mix_meas})
    return entries, meas


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="gpurun_out/tune_table.json")
    ap.add_argument("--buckets", default=",".join(map(str, BUCKETS)))
    ap.add_argument("--kinds", default="cvrp,vrptw")
    ap.add_argument("--no-mix", action="store_true", help="skip the tuning in the context of the mixed batch")
    args = ap.parse_args()
    buckets = tuple(int(x) for x in args.buckets.split(","))
    entries, meas = run(buckets, tuple(args.kinds.split(",")), mix=not args.no_mix)
    doc = {"device": torch.cuda.get_device_name(0),
           "command": "python -m paper_2506_17357_amd.autotune " + " ".join(sys.argv[1:]),
           "entries": entries, "measurements": meas}
    with open(args.out, "w") as f:
        json.dump(doc, f, indent=1)
    log("wrote", args.out)


if __name__ == "__main__":
    main()
