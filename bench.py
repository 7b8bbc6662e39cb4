#!/usr/bin/env python
"""Benchmark of the batched full-neighbourhood local search on one MI355X.

Workload (the batched configuration): 256 independent solutions, sizes
log-uniform over 100..2000 customers, even b = CVRP (demand 1..100, capacity
1000), odd b = clustered VRPTW, seeds 4000 + b, sweep starting solutions.
One step = one evaluation of every move of every active solution (one
persistent launch) + best-move reduction, apply and attribute rebuild (one
launch).  Inputs are resident in HBM before the timed region starts.

Reported: GMoves/s of the batched form (HIP graph of the K-step loop), the
same K steps run eagerly with HIP events around every evaluation launch (the
roofline figures come from those events), the plain one-solution-per-launch
form on the same solutions (same results, checked), the best-move latency
of the plain form, and the CPU oracle timed on the host.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "GMoves/s evaluated + best-move latency; batched vs plain, same GPU, bit-exact"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def eval_bytes(inst, R):
    """Algorithmic HBM bytes of one full-neighbourhood evaluation: the int32
    distance matrix read once, 4(n+1)^2, plus 36 bytes of slot attributes per
    ref (Q = n + R), 16 bytes of node data per node and 16 bytes per route."""
    Q = inst.n + R
    return 4 * (inst.n + 1) ** 2 + 36 * Q + 16 * (inst.n + 1) + 16 * R


def streamed_bytes(inst, R, dist_bytes):
    """The bytes the kernels actually stream per evaluation: the matrix at the
    width the inter-route kernels read it (2 bytes per entry when every
    distance is below 2^16, else 4) plus the slot attribute records (two int4
    per slot for CVRP, four with time windows)."""
    Q = inst.n + R
    return dist_bytes * (inst.n + 1) ** 2 + (64 if inst.has_tw else 32) * (Q + 1)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def committed_counters(name):
    """A counter summary committed under profiles/ (rocprofv3 runs of the
    default benchmark's evaluation launch); None when missing or taken on
    other kernel sources."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    from paper_2506_17357_amd.counters import kernel_source_hash
    if t.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return t


def traffic_entry(alg_bytes_per_launch):
    """HBM bytes per evaluation launch from FETCH_SIZE and WRITE_SIZE (each
    scaled by the same counter on a plain copy of known size)."""
    t = committed_counters("traffic_k_eval_batch_batched256.json")
    if t is None:
        return None
    return {"bytes_per_launch": t["bytes_per_launch"],
            "vs_algorithmic": round(t["bytes_per_launch"] / alg_bytes_per_launch, 3),
            "unscaled_bytes_per_launch": t.get("unscaled_bytes_per_launch"),
            "source": "profiles/traffic_k_eval_batch_batched256.json"}


def valu_entry(avg_launch_us):
    """VALU issue fraction of the evaluation launch: wavefront VALU
    instructions per launch (SQ_INSTS_VALU) over what the chip issues in the
    launch time (256 CUs x 4 SIMDs, one wave64 instruction per SIMD every 4
    cycles at 2.4 GHz)."""
    t = committed_counters("valu_k_eval_batch_batched256.json")
    if t is None:
        return None
    peak_per_us = 256 * 4 * 2400.0 / 4
    out = {"valu_insts_per_launch": t["valu_insts_per_launch"],
           "frac": round(t["valu_insts_per_launch"] / (avg_launch_us * peak_per_us), 4),
           "source": "profiles/valu_k_eval_batch_batched256.json"}
    q = committed_counters("sq_k_eval_batch_batched256.json")
    if q is not None and "wait_any_share" in q:
        # share of the wavefronts' cycles spent waiting (s_waitcnt, barriers)
        out["wave_cycles_waiting"] = q["wait_any_share"]
        out["wait_source"] = "profiles/sq_k_eval_batch_batched256.json"
    return out


def calibrate_copy():
    """Calibration launches for a profiler pass: a plain device copy of
    exactly 1 GiB (read) + 1 GiB (write), which scales WRITE_SIZE, and one
    read of 1 GiB through the 16-byte LDS DMA the evaluation stages its
    16-bit rows with (k_probe_stream), which scales FETCH_SIZE for that
    request type."""
    import torch
    from paper_2506_17357_amd import tga
    a = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    tga.probe_stream_read(a)
    torch.cuda.synchronize()
    del a, b


def eager_pass(B, K, ebytes, sbytes):
    """K local-search steps of batch B from its current state, launched one
    by one with HIP events (on the launching stream) around every evaluation
    launch.  ebytes / sbytes: algorithmic / streamed bytes of one evaluation
    of each solution; a launch is charged for the solutions still active in
    it."""
    import torch
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.begin(K)
    for k in range(K):
        ev0[k].record()
        B.step_part(0)
        ev1[k].record()
        B.step_part(1)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    st, mv, cost = B.collect()
    dur_ms = np.array([a.elapsed_time(b) for a, b in zip(ev0, ev1)])
    evals = np.where(st < K, st + 1, K)
    active = np.arange(K)[:, None] < evals[None, :]
    return {"seconds": t, "steps": st, "moves": mv, "cost": cost, "dur_ms": dur_ms,
            "alg_bytes": (active * ebytes[None, :]).sum(axis=1),
            "str_bytes": (active * sbytes[None, :]).sum(axis=1)}


def roofline_entry(ev, kernel="k_eval_batch<3>"):
    secs = ev["dur_ms"].sum() * 1e-3
    alg = ev["alg_bytes"].sum() / secs / 1e9
    streamed = ev["str_bytes"].sum() / secs / 1e9
    return {
        "bound": "hbm", "kernel": kernel,
        "achieved": round(alg, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(alg / HBM_PEAK_GBS, 4),
        "bytes_model": "per active solution per launch: 4(n+1)^2 + 36Q + 16(n+1) + 16R",
        "avg_launch_us": round(float(ev["dur_ms"].mean() * 1e3), 2),
        "avg_bytes_per_launch": int(ev["alg_bytes"].mean()),
        "streamed": {"achieved": round(streamed, 1), "frac": round(streamed / HBM_PEAK_GBS, 4),
                     "avg_bytes_per_launch": int(ev["str_bytes"].mean()),
                     "bytes_model": "w(n+1)^2 at the streamed width w (2 B below 2^16, else 4) "
                                    "+ 32 (CVRP) or 64 (VRPTW) bytes per slot"},
    }


GRANULAR_THETA = {"c1": 20, "c2": 20, "c3": 100}  # the paper's tuned thresholds: CVRP 20, VRPTW 100


def granular_config(tga, I, S, inst, sol, name):
    """Granular mode (edge-based neighbourhood reduction, theta nearest
    neighbours) on the same instance: local search to the local optimum of
    the reduced neighbourhood and the best-move latency along it."""
    import torch
    theta = GRANULAR_THETA[name]
    t0 = time.perf_counter()
    I.set_granular(theta)
    t_set = time.perf_counter() - t0
    mask = tga.OPS_ALL | tga.OP_GRANULAR
    S.reload(sol.offsets, sol.customers)
    S.ls_run(5, mask)
    S.reload(sol.offsets, sol.customers)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps, moves, cost = S.ls_run(100000 if name != "c1" else 100, mask)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    S.reload(sol.offsets, sol.customers)
    lat = []
    for _ in range(steps + 1):
        t1 = time.perf_counter()
        m = S.eval(mask)
        lat.append((time.perf_counter() - t1) * 1e6)
        if m is None or m.delta >= 0:
            break
        S.apply(m)
    lat = np.array(lat)
    S.reload(sol.offsets, sol.customers)
    log("%s granular theta=%d: %d steps in %.4f s, %.2f GMoves/s, latency p50 %.1f us" % (
        name, theta, steps, t, moves / t / 1e9, np.percentile(lat, 50)))
    return {"theta": theta, "pair_entries": I.granular_pairs, "setup_s": round(t_set, 4), "steps": int(steps),
            "moves_evaluated": int(moves), "final_cost": int(cost), "seconds": round(t, 5),
            "gmoves_s": round(moves / t / 1e9, 3),
            "best_move_latency_us": {"p50": round(float(np.percentile(lat, 50)), 1),
                                     "p99": round(float(np.percentile(lat, 99)), 1), "evals": int(lat.size)}}


PENALTY = {"c1": (10, 0), "c2": (10, 0), "c3": (10, 10)}  # (w_load, w_tw); the paper fixes no weights


def penalised_config(tga, I, inst, sol, name):
    """Penalised mode (feasible and infeasible search: every move admissible,
    scored by dD + w_L dL_V + w_T dT_V) from the same start: local search to
    its local optimum (at most 2000 steps) and the best-move latency."""
    import torch
    w = PENALTY[name]
    S = tga.Solution(I, sol.offsets, sol.customers)
    S.set_penalty(*w)
    S.ls_run(5)
    S.reload(sol.offsets, sol.customers)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps, moves, cost = S.ls_run(100 if name == "c1" else 2000)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    lv, tv = S.violations()
    S.reload(sol.offsets, sol.customers)
    lat = []
    for _ in range(min(steps, 200) + 1):
        t1 = time.perf_counter()
        m = S.eval()
        lat.append((time.perf_counter() - t1) * 1e6)
        if m is None or m.delta >= 0:
            break
        S.apply(m)
    lat = np.array(lat)
    log("%s penalised w=%s: %d steps in %.4f s, %.2f GMoves/s, latency p50 %.1f us, final distance %d, "
        "load excess %d, time warp %d" % (name, w, steps, t, moves / t / 1e9, np.percentile(lat, 50), cost, lv, tv))
    return {"weights": list(w), "steps": int(steps), "moves_evaluated": int(moves), "final_cost": int(cost),
            "final_load_excess": lv, "final_time_warp": tv, "seconds": round(t, 5),
            "gmoves_s": round(moves / t / 1e9, 3),
            "best_move_latency_us": {"p50": round(float(np.percentile(lat, 50)), 1),
                                     "p99": round(float(np.percentile(lat, 99)), 1), "evals": int(lat.size)}}


def plain_configs(log_lat=True):
    """The single-solution configurations on the plain form: moves per
    second of the device-resident loop to the local optimum (100 steps for
    the 100-customer case), and the best-move latency of a host call
    (evaluation + record copy) at every step of the same trajectory."""
    import torch
    from paper_2506_17357_amd import tga, workload as W
    out = {}
    for name, caps in (("c1", 100), ("c2", 100000), ("c3", 100000)):
        inst, sol = getattr(W, name)()
        I = tga.Instance.from_workload(inst)
        S = tga.Solution(I, sol.offsets, sol.customers)
        S.ls_run(5)  # warm the code paths
        S.reload(sol.offsets, sol.customers)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps, moves, cost = S.ls_run(caps)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        S.reload(sol.offsets, sol.customers)
        lat = []
        for _ in range(steps + 1):
            t1 = time.perf_counter()
            m = S.eval()
            lat.append((time.perf_counter() - t1) * 1e6)
            if m is None or m.delta >= 0:
                break
            S.apply(m)
        lat = np.array(lat)
        gran = granular_config(tga, I, S, inst, sol, name)
        pen = penalised_config(tga, I, inst, sol, name)
        out[name] = {"workload": "%s: n = %d %s, seed %d, sweep start, R = %d" % (
                         name, inst.n, inst.kind, inst.seed, sol.R),
                     "granular": gran,
                     "penalised": pen,
                     "steps": int(steps), "moves_evaluated": int(moves), "final_cost": int(cost),
                     "seconds": round(t, 5), "gmoves_s": round(moves / t / 1e9, 3),
                     "best_move_latency_us": {"p50": round(float(np.percentile(lat, 50)), 1),
                                              "p99": round(float(np.percentile(lat, 99)), 1),
                                              "evals": int(lat.size)}}
        log("%s: %d steps to the local optimum in %.4f s, %.2f GMoves/s, best-move latency p50 %.1f us "
            "p99 %.1f us" % (name, steps, t, out[name]["gmoves_s"], out[name]["best_move_latency_us"]["p50"],
                             out[name]["best_move_latency_us"]["p99"]))
    return out


def _ls_leg(S, sol, steps_cap, mask, lat_mask=None):
    """Device-resident local search from the start (after a short warm-up)
    and the best-move latency along the single-move trajectory."""
    import torch
    S.ls_run(3, mask)
    S.reload(sol.offsets, sol.customers)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps, moves, cost = S.ls_run(steps_cap, mask)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    out = {"steps": int(steps), "moves_evaluated": int(moves), "final_cost": int(cost), "seconds": round(t, 5),
           "gmoves_s": round(moves / t / 1e9, 3)}
    if lat_mask is not None:
        S.reload(sol.offsets, sol.customers)
        lat = []
        for _ in range(min(steps, 200) + 1):
            t1 = time.perf_counter()
            m = S.eval(lat_mask)
            lat.append((time.perf_counter() - t1) * 1e6)
            if m is None or m.delta >= 0:
                break
            S.apply(m)
        out["best_move_latency_us"] = {"p50": round(float(np.percentile(lat, 50)), 1),
                                       "p99": round(float(np.percentile(lat, 99)), 1), "evals": len(lat)}
    return out


def general_configs():
    """The general (concatenation) path on the 1000-customer instances:
    the operator variants (all ten operators), multi-move steps, and pickups
    (VRPSPDTW, hard and penalised), each a local search to its local optimum
    from the sweep start."""
    from paper_2506_17357_amd import tga, workload as W
    out = {}
    for name in ("c2", "c3"):
        inst, sol = getattr(W, name)()
        I = tga.Instance.from_workload(inst)
        S = tga.Solution(I, sol.offsets, sol.customers)
        S.set_general(True)
        row = {"base_general_path": _ls_leg(S, sol, 100000, tga.OPS_ALL),
               "variants": _ls_leg(S, sol, 100000, tga.OPS_ALL | tga.OPS_VARIANTS, tga.OPS_ALL | tga.OPS_VARIANTS)}
        S.set_multi(True)
        row["multi_move"] = _ls_leg(S, sol, 100000, tga.OPS_ALL | tga.OP_MULTI)
        row["multi_move"]["moves_applied"] = S.multi_stats()[1]
        out[name] = row
        log("%s general path: base %d steps %.4f s (%.1f GMoves/s); variants %d steps %.4f s (%.1f GMoves/s, "
            "latency p50 %.1f us, final %d vs %d); multi-move %d steps / %d moves %.4f s (final %d)" % (
                name, row["base_general_path"]["steps"], row["base_general_path"]["seconds"],
                row["base_general_path"]["gmoves_s"], row["variants"]["steps"], row["variants"]["seconds"],
                row["variants"]["gmoves_s"], row["variants"]["best_move_latency_us"]["p50"],
                row["variants"]["final_cost"], row["base_general_path"]["final_cost"], row["multi_move"]["steps"],
                row["multi_move"]["moves_applied"], row["multi_move"]["seconds"], row["multi_move"]["final_cost"]))
    inst, sol = W.c6()
    I = tga.Instance.from_workload(inst)
    S = tga.Solution(I, sol.offsets, sol.customers)
    row = {"workload": "c6: n = %d vrpspdtw, seed 106, sweep start, R = %d" % (inst.n, sol.R),
           "hard": _ls_leg(S, sol, 100000, tga.OPS_ALL, tga.OPS_ALL)}
    S.set_penalty(10, 10)
    row["penalised"] = _ls_leg(S, sol, 100000, tga.OPS_ALL, tga.OPS_ALL)
    row["penalised"]["weights"] = [10, 10]
    out["c6"] = row
    log("c6 pickups: hard %d steps %.4f s (%.1f GMoves/s, latency p50 %.1f us); penalised %d steps %.4f s" % (
        row["hard"]["steps"], row["hard"]["seconds"], row["hard"]["gmoves_s"],
        row["hard"]["best_move_latency_us"]["p50"], row["penalised"]["steps"], row["penalised"]["seconds"]))
    return out


def oracle_configs(threads):
    """The oracle on one full-neighbourhood evaluation of each
    single-solution configuration's starting state, at `threads` threads and
    at one thread."""
    import oracle
    from paper_2506_17357_amd import workload as W
    out = {}
    for name in ("c1", "c2", "c3"):
        inst, sol = getattr(W, name)()
        row = {}
        for T in (threads, 1):
            t0 = time.perf_counter()
            r = oracle.eval_neighbourhood(inst, sol, threads=T)
            t = time.perf_counter() - t0
            row["t%d" % T] = {"gmoves_s": round(r.moves / t / 1e9, 5), "seconds": round(t, 4)}
        row["moves"] = int(r.moves)
        theta = GRANULAR_THETA[name]
        mask = oracle.granular_mask(inst, theta)
        t0 = time.perf_counter()
        rg = oracle.eval_neighbourhood(inst, sol, threads=threads, mask=mask)
        tg = time.perf_counter() - t0
        row["granular"] = {"theta": theta, "moves": int(rg.moves), "t%d" % threads: {
            "gmoves_s": round(rg.moves / tg / 1e9, 5), "seconds": round(tg, 4)}}
        out[name] = row
    return out


def n1000_comparison(steps):
    """Batched against plain at n = 1000: 256 CVRP solutions of exactly 1000
    customers (seeds 4500 + b), sweep start, `steps` local-search steps, both
    forms timed from the same initial solutions and compared bit for bit."""
    import torch
    from paper_2506_17357_amd import tga, workload as W
    t = time.time()
    pairs = W.c4_uniform()
    insts = [tga.Instance.from_workload(i) for i, _ in pairs]
    sols = [tga.Solution(I, s.offsets, s.customers) for I, (_, s) in zip(insts, pairs)]

    def reload_all():
        for s, (_, sol) in zip(sols, pairs):
            s.reload(sol.offsets, sol.customers)
        torch.cuda.synchronize()

    B = tga.Batch(sols)
    B.autotune(launches=3)
    reload_all()
    ebytes = np.array([eval_bytes(i, s.R) for i, s in pairs], np.float64)
    sbytes = np.array([streamed_bytes(i, s.R, I.dist_bytes) for I, (i, s) in zip(insts, pairs)], np.float64)
    ev = eager_pass(B, steps, ebytes, sbytes)
    reload_all()
    B.ls_run(steps, use_graph=True)  # capture + first replay, untimed
    reload_all()
    t0 = time.perf_counter()
    st_b, mv_b, cost_b = B.ls_run(steps, use_graph=True)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    B.close()
    assert np.array_equal(st_b, ev["steps"]) and np.array_equal(cost_b, ev["cost"])
    reload_all()
    t0 = time.perf_counter()
    res = [s.ls_run(steps) for s in sols]
    torch.cuda.synchronize()
    t_p = time.perf_counter() - t0
    same = (np.array_equal([r[0] for r in res], st_b) and np.array_equal([r[1] for r in res], mv_b) and
            np.array_equal([r[2] for r in res], cost_b))
    out = {"workload": "256 CVRP solutions of n = 1000 (seeds 4500+b), sweep start, %d steps" % steps,
           "batched_gmoves_s": round(int(mv_b.sum()) / t_b / 1e9, 3),
           "plain_gmoves_s": round(int(sum(r[1] for r in res)) / t_p / 1e9, 3),
           "bit_exact": bool(same)}
    out["batched_over_plain"] = round(out["batched_gmoves_s"] / out["plain_gmoves_s"], 2)
    out["roofline"] = roofline_entry(ev)
    log("n = 1000: batched %.1f GMoves/s, plain %.2f GMoves/s, bit-exact %s (%.1f s)" % (
        out["batched_gmoves_s"], out["plain_gmoves_s"], same, time.time() - t))
    return out


def served_run(args, count):
    """Served form: a Poisson stream of `count` local-search requests
    (200..10000 customers log-uniform, CVRP / VRPTW alternating, seeds
    5000 + k, arrivals seed 5999, <= --served-steps steps each) served by
    continuous batching under an HBM budget.  A closed loop (every request
    queued at t = 0) measures the capacity; the open loop offers 0.7 x that
    rate and must give every request the closed loop's result."""
    import torch
    from paper_2506_17357_amd import serve, workload as W
    torch.cuda.set_device(0)
    t = time.time()
    base = W.request_stream(count, qps=1.0, max_steps=args.served_steps)
    reqs = []
    for r in base:
        inst = W.request_instance(r)
        reqs.append(serve.ServeRequest(r.k, 0.0, inst, W.sweep(inst), r.max_steps))
    log("served: %d requests generated in %.1f s (sum n = %d)" % (len(reqs), time.time() - t,
                                                                  sum(q.inst.n for q in reqs)))
    budget = int(args.hbm_budget_gb * (1 << 30))
    srv = serve.Server(budget, steps_per_tick=args.steps_per_tick)
    srv.run(reqs[: min(8, len(reqs))])  # warm: code paths
    srv = serve.Server(budget, steps_per_tick=args.steps_per_tick)
    t0 = time.perf_counter()
    res0 = srv.run(reqs)
    t_closed = time.perf_counter() - t0
    moves0 = sum(r.moves for r in res0)
    cap_qps = len(reqs) / t_closed
    qps = 0.7 * cap_qps
    log("served closed loop: %.2f s, %.1f GMoves/s, capacity %.2f requests/s -> offered %.2f requests/s "
        "(%d plan updates, %.3f s; uploads busy %.2f s; peak %d requests on the device; %d ticks)" % (
            t_closed, moves0 / t_closed / 1e9, cap_qps, qps, srv.rebuilds, srv.rebuild_s, srv.upload_s,
            srv.peak_active, srv.ticks))
    arrivals = W.request_stream(count, qps=qps, max_steps=args.served_steps)
    for q, a in zip(reqs, arrivals):
        q.arrival_s = a.arrival_s
    srv = serve.Server(budget, steps_per_tick=args.steps_per_tick)
    t0 = time.perf_counter()
    res = srv.run(reqs)
    t_open = time.perf_counter() - t0
    same = all((a.steps, a.moves, a.cost) == (b.steps, b.moves, b.cost) and
               a.customers.tolist() == b.customers.tolist() for a, b in zip(res0, res))
    lat = np.array([r.latency_s for r in res]) * 1e3
    moves = sum(r.moves for r in res)
    out = {
        "metric": "served: aggregate GMoves/s + p50/p99 request latency (continuous batching)",
        "value": round(moves / t_open / 1e9, 4),
        "unit": "GMoves/s",
        "closed_loop_gmoves_s": round(moves0 / t_closed / 1e9, 4),
        "workload": "served: %d requests, 200..10000 customers log-uniform, CVRP/VRPTW alternating, "
                    "<= %d steps each, Poisson arrivals at 0.7 x the closed-loop capacity" % (
                        len(reqs), args.served_steps),
        "qps": round(qps, 3), "capacity_qps": round(cap_qps, 3),
        "hbm_budget_bytes": budget, "moves_evaluated": moves,
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 2),
                       "p99": round(float(np.percentile(lat, 99)), 2),
                       "max": round(float(lat.max()), 2)},
        "makespan_s": round(t_open, 3),
        "steps_per_tick": srv.steps_per_tick,
        "engine_schedule": srv.config,
        "upload_busy_s": round(srv.upload_s, 3),
        "plan_updates": srv.rebuilds,
        "plan_update_s": round(srv.rebuild_s, 3),
        "peak_active_requests": srv.peak_active,
        "peak_resident_bytes": srv.peak_used,
        "ticks": srv.ticks,
        "same_results_as_closed_loop": bool(same),
    }
    log("served open loop: %.1f GMoves/s, p50 %.1f ms, p99 %.1f ms, same results %s" % (
        out["value"], out["latency_ms"]["p50"], out["latency_ms"]["p99"], same))
    return out


def large_run(args):
    """One request of exactly args.large customers (the served stream's
    largest size; seeds as the large oracle-checked requests: 15000 CVRP,
    15001 VRPTW) as a batch of one: args.steps local-search steps from the
    sweep start, HIP events around every evaluation launch.  The single-GPU
    view of the largest instances (one row-sliced D per evaluation)."""
    import torch
    from paper_2506_17357_amd import tga, workload as W
    kind = args.large_kind
    req = W.Request(10000 + (kind != "cvrp"), 0.0, args.large, kind, args.steps)
    t = time.time()
    inst = W.request_instance(req)
    sol = W.sweep(inst)
    log("large: %s n = %d generated in %.1f s (R = %d)" % (kind, inst.n, time.time() - t, sol.R))
    I = tga.Instance.from_workload(inst)
    S = tga.Solution(I, sol.offsets, sol.customers)
    if args.large_item_rows:
        S.set_rows(0, args.large_item_rows)
    B = tga.Batch([S])
    if args.large_lds_kb:
        B.set_config(args.large_lds_kb, 0)
        schedule = B.config()
    else:
        schedule = B.autotune(launches=3)
    ebytes = np.array([eval_bytes(inst, sol.R)], np.float64)
    sbytes = np.array([streamed_bytes(inst, sol.R, I.dist_bytes)], np.float64)
    S.reload(sol.offsets, sol.customers)
    ev = eager_pass(B, args.steps, ebytes, sbytes)
    roof = roofline_entry(ev)
    line = {"metric": "large request: evaluation launch vs the HBM roofline", "value": roof["achieved"],
            "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "higher_is_better": True, "dtype": "int32",
            "data": "synthetic", "config": {"workload": "one %s request of %d customers (seed %d), batch of one, "
                                                        "%d local-search steps" % (kind, inst.n, 5000 + req.k,
                                                                                   args.steps),
                                            "R": sol.R, "schedule": schedule, "rows": S.rows(),
                                            "accepted_moves": int(ev["steps"][0]),
                                            "moves_evaluated": int(ev["moves"][0])},
            "roofline": roof}
    log("large: eval launch avg %.1f us, %.0f GB/s algorithmic (%.3f), %.0f GB/s streamed" % (
        roof["avg_launch_us"], roof["achieved"], roof["frac"], roof["streamed"]["achieved"]))
    B.close()
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--count", type=int, default=256)
    ap.add_argument("--served", action="store_true", help="benchmark the served form instead")
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--served-steps", type=int, default=500)
    ap.add_argument("--steps-per-tick", type=int, default=4,
                    help="served form: local-search steps per scheduling tick (one poll per tick)")
    ap.add_argument("--hbm-budget-gb", type=float, default=64.0)
    ap.add_argument("--served-leg-requests", type=int, default=100,
                    help="requests of the served leg of the default run (0 = none)")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--plain-only", action="store_true",
                    help="instead: only the single-solution legs (configs, general path)")
    ap.add_argument("--large", type=int, default=0,
                    help="instead: one request of this many customers as a batch of one (evaluation roofline)")
    ap.add_argument("--large-kind", default="cvrp", choices=("cvrp", "vrptw"))
    ap.add_argument("--large-item-rows", type=int, default=0, help="rows per inter-route item (0: the table)")
    ap.add_argument("--large-lds-kb", type=int, default=0, help="LDS budget per workgroup (0: autotuned)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="start with a 1 GiB device copy (profiler scaling of FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        log("bench.py: measures one GPU only (the batched solutions are independent, so more GPUs "
            "would each take a share of the solutions); run with --gpus 1")
        sys.exit(2)
    K, Wm = args.steps, args.warmup
    from paper_2506_17357_amd import build_lib
    build_lib.ensure_built(verbose=True)
    if args.plain_only:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps({"plain_configs": plain_configs(), "general_path": general_configs()}), flush=True)
        return
    if args.large:
        import torch
        torch.cuda.set_device(0)
        if args.calibrate_copy:
            calibrate_copy()
        print(json.dumps(large_run(args)), flush=True)
        return
    if args.served:
        line = served_run(args, args.requests)
        line.update({"n_gpus": 1, "higher_is_better": True, "dtype": "int32", "data": "synthetic"})
        print(json.dumps(line), flush=True)
        return
    import torch
    from paper_2506_17357_amd import tga, workload as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        calibrate_copy()
    cus, lds = tga.device_limits()
    log("device: %s, %d CUs, %d B LDS per evaluation workgroup" % (torch.cuda.get_device_name(0), cus, lds))

    t = time.time()
    sizes = W.batch_sizes(args.count)
    pairs = []
    for b, n in enumerate(sizes):
        inst = W.batch_instance(b, n)
        pairs.append((inst, W.sweep(inst)))
    log("workload generated in %.1f s: %d solutions, sum n = %d" % (time.time() - t, len(pairs), sum(sizes)))
    insts = [tga.Instance.from_workload(i) for i, _ in pairs]
    sols = [tga.Solution(I, s.offsets, s.customers) for I, (_, s) in zip(insts, pairs)]
    ebytes = np.array([eval_bytes(i, s.R) for i, s in pairs], np.float64)
    sbytes = np.array([streamed_bytes(i, s.R, I.dist_bytes) for I, (i, s) in zip(insts, pairs)], np.float64)
    B = tga.Batch(sols)
    torch.cuda.synchronize()
    t = time.time()
    schedule = B.autotune(launches=5)  # untimed: picks tile shapes and launch split
    log("autotuned schedule in %.2f s: %s" % (time.time() - t, schedule))
    log("uploaded: %.1f MB of distance matrices resident, %d of %d streamed at 16 bits" % (
        sum(4 * (i.n + 1) ** 2 for i, _ in pairs) / 1e6, sum(I.dist_bytes == 2 for I in insts), len(insts)))

    def reload_all():
        for s, (_, sol) in zip(sols, pairs):
            s.reload(sol.offsets, sol.customers)
        torch.cuda.synchronize()

    # ---- warmup: W eager steps from the initial state
    reload_all()
    B.begin(Wm)
    for _ in range(Wm):
        B.step_part(0)
        B.step_part(1)
    B.collect()
    log("warmup: %d steps" % Wm)

    # ---- eager pass with events around every evaluation launch
    reload_all()
    ev = eager_pass(B, K, ebytes, sbytes)
    st_e, mv_e, cost_e = ev["steps"], ev["moves"], ev["cost"]
    moves_total = int(mv_e.sum())
    roof = roofline_entry(ev)
    log("eager: %.3f s for %d steps, %d moves, eval launch avg %.1f us (first %.1f us, last %.1f us), "
        "%.0f GB/s algorithmic (%.3f of peak), %.0f GB/s streamed" % (
            ev["seconds"], K, moves_total, roof["avg_launch_us"], ev["dur_ms"][0] * 1e3, ev["dur_ms"][-1] * 1e3,
            roof["achieved"], roof["frac"], roof["streamed"]["achieved"]))

    # ---- graph pass (the step loop captured once, replayed from the initial state)
    reload_all()
    B.ls_run(K, use_graph=True)  # capture + first replay, untimed
    reload_all()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st_g, mv_g, cost_g = B.ls_run(K, use_graph=True)
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t0
    assert np.array_equal(st_g, st_e) and np.array_equal(mv_g, mv_e) and np.array_equal(cost_g, cost_e), \
        "graph and eager passes disagree"
    value = moves_total / t_graph / 1e9
    log("graph: %.3f s -> %.1f GMoves/s" % (t_graph, value))
    # ---- screening statistics: the same steps with the counting instantiation (untimed)
    reload_all()
    st_c, mv_c, cost_c = B.ls_run(K, tga.OPS_ALL | tga.OP_COUNT_FULL, use_graph=False)
    assert np.array_equal(st_c, st_e) and np.array_equal(mv_c, mv_e) and np.array_equal(cost_c, cost_e), \
        "counting pass disagrees"
    screen = B.screen_stats()
    log("screens: %d of %d inter-route slot pairs evaluated in full (%.5f)" % (
        screen[0], screen[1], screen[0] / max(1, screen[1])))
    B.close()

    out_plain = None
    bit_exact = None
    if not args.no_plain:
        # ---- plain form: one solution per launch sequence, same solutions
        reload_all()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = [s.ls_run(K) for s in sols]
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        st_p = np.array([r[0] for r in res])
        mv_p = np.array([r[1] for r in res])
        cost_p = np.array([r[2] for r in res])
        bit_exact = bool(np.array_equal(st_p, st_e) and np.array_equal(mv_p, mv_e) and
                         np.array_equal(cost_p, cost_e))
        plain_value = int(mv_p.sum()) / t_plain / 1e9
        log("plain: %.3f s -> %.2f GMoves/s, bit-exact with batched: %s" % (t_plain, plain_value, bit_exact))
        out_plain = {
            "value": round(plain_value, 4), "unit": "GMoves/s", "seconds": round(t_plain, 4),
            "form": "one solution per launch sequence (device-resident loop per solution)",
            "configs": plain_configs(),
            "general_path": general_configs(),
            "n1000": n1000_comparison(min(K, 50)),
        }

    out_served = None
    if not args.no_served and args.served_leg_requests > 0:
        out_served = served_run(args, args.served_leg_requests)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = len(os.sched_getaffinity(0))
        sample = list(range(0, len(pairs), 2))[:64] + list(range(1, len(pairs), 2))[:64]
        t0 = time.perf_counter()
        mv = 0
        for b in sample:
            inst, sol = pairs[b]
            r = oracle.eval_neighbourhood(inst, sol, threads=threads)
            mv += r.moves
            if time.perf_counter() - t0 > 25:
                sample = sample[:sample.index(b) + 1]
                break
        t_cpu = time.perf_counter() - t0
        cpu = {"value": round(mv / t_cpu / 1e9, 5), "unit": "GMoves/s", "cores": threads, "kind": "oracle",
               "sample": "one full-neighbourhood evaluation of the initial state of %d of the 256 solutions "
                         "(%d moves, %.1f s)" % (len(sample), mv, t_cpu),
               "cpu_model": cpu_model(),
               "configs": oracle_configs(threads)}
        log("cpu oracle: %.4f GMoves/s on %d threads (%s)" % (cpu["value"], threads, cpu["cpu_model"]))

    roof["traffic"] = traffic_entry(roof["avg_bytes_per_launch"])
    roof["valu"] = valu_entry(roof["avg_launch_us"])
    line = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "GMoves/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": round(t_graph / K * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": "batched: 256 solutions, 100..2000 customers log-uniform, CVRP (even b) / "
                        "clustered VRPTW (odd b), seeds 4000+b, sweep start, %d local-search steps, "
                        "all five operators" % K,
            "global_batch": len(pairs),
            "sum_customers": int(sum(sizes)),
            "dist_bytes_resident": int(sum(4 * (i.n + 1) ** 2 for i, _ in pairs)),
            "dist_bytes_streamed_per_eval": int(sum(I.dist_bytes * (i.n + 1) ** 2 for I, (i, _) in zip(insts, pairs))),
            "moves_evaluated": moves_total,
            "moves_counted": "every move of N(S) per evaluation (delta of each; feasibility and id only "
                             "where the delta can still be the step's best)",
            "accepted_moves": int(st_e.sum()),
            "full_eval_fraction": round(screen[0] / max(1, screen[1]), 5),
            "full_eval_fraction_means": "share of the inter-route slot pairs visited whose RELOCATE / SWAP / "
                                        "2OPT* moves were evaluated in full (feasibility and ids); the others "
                                        "were dropped by their deltas or the capacity screen, which never "
                                        "drops the step's best move (%d of %d pairs; counted in an untimed "
                                        "pass of the same steps)" % screen,
            "form": "batched: persistent evaluation launch(es) + one finalize launch per step, "
                    "step loop captured in a HIP graph",
            "schedule": schedule,
            "rows_per_item_table": (os.path.relpath(tga.TUNE_PATH, os.path.dirname(os.path.abspath(__file__)))
                                    if tga.TUNE_PATH and os.path.exists(tga.TUNE_PATH) else None),
        },
        "roofline": roof,
        "eager_value": round(moves_total / ev["seconds"] / 1e9, 4),
        "plain": out_plain,
        "batched_over_plain": round(value / out_plain["value"], 3) if out_plain else None,
        "bit_exact_batched_vs_plain": bit_exact,
        "served": out_served,
        "served_closed_loop_over_batched": (round(out_served["closed_loop_gmoves_s"] / value, 3)
                                            if out_served else None),
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
