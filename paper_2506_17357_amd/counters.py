"""Summaries of rocprofv3 hardware-counter runs of the benchmark (the
figures committed under profiles/ and read back by bench.py).

Traffic: two runs of the same benchmark command, one with --pmc FETCH_SIZE
and one with --pmc WRITE_SIZE, started with --calibrate-copy so that each
process also runs the calibration launches: a 1 GiB device copy (scales
WRITE_SIZE) and a 1 GiB read through the 16-byte LDS DMA of k_probe_stream
(scales FETCH_SIZE for the request type the evaluation stages its rows
with).  The evaluation launch's figures are the mean over its last `last`
dispatches, one whole local-search pass of the benchmark.

VALU: one run with --pmc SQ_INSTS_VALU; wavefront VALU instructions per
launch, the same dispatches.

SQ: runs with --pmc and up to eight SQ_ counters each; the mean of every
counter over the same dispatches, and the shares of wave cycles spent
waiting (SQ_WAIT_ANY, SQ_WAIT_INST_ANY over SQ_WAVE_CYCLES) and issuing VALU
instructions (SQ_ACTIVE_INST_VALU over SQ_WAVE_CYCLES; both in the same
units).

    python -m paper_2506_17357_amd.counters traffic <fetch dir> <write dir> --last 200 --out <json>
    python -m paper_2506_17357_amd.counters valu <dir> --last 200 --out <json>
    python -m paper_2506_17357_amd.counters sq <dir> [<dir> ...] --last 200 --out <json>
    python -m paper_2506_17357_amd.counters trace <kernel-trace results.db> --last 200
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GIB = 1 << 30


def kernel_source_hash() -> str:
    """sha256 over the device library's sources: a committed counter summary
    applies only to the kernels it was taken on."""
    h = hashlib.sha256()
    for f in ("kernels.hip", "api.hip", "tga_internal.h"):
        with open(os.path.join(ROOT, "paper_2506_17357_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def load(path: str, counter: str):
    """[(dispatch id, kernel name, value)] of one counter, in dispatch order,
    from every counter_collection CSV under `path`."""
    rows = {}
    files = sorted(glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True))
    if not files:
        raise FileNotFoundError("no counter_collection.csv under %s" % path)
    for fn in files:
        with open(fn, newline="") as f:
            for r in csv.DictReader(f):
                if r.get("Counter_Name") != counter:
                    continue
                key = (fn, int(r.get("Dispatch_Id") or r.get("Correlation_Id")))
                name = r.get("Kernel_Name", "")
                v = float(r["Counter_Value"])
                if key in rows:
                    rows[key] = (rows[key][0], rows[key][1] + v)
                else:
                    rows[key] = (name, v)
    return [(k[1], n, v) for k, (n, v) in sorted(rows.items())]


def _match(name: str, kernel: str) -> bool:
    """Kernel names come demangled ("tga::k_eval_batch<3>(...)") or not."""
    if kernel in name:
        return True
    m = re.match(r"(\w+)<(\d+)>$", kernel)
    return bool(m) and ("%d%sILi%sE" % (len(m.group(1)), m.group(1), m.group(2))) in name


def dispatch_values(rows, kernel: str, last: int):
    vals = [v for _, n, v in rows if _match(n, kernel)]
    if len(vals) < last:
        raise ValueError("%d dispatches of %s, fewer than %d" % (len(vals), kernel, last))
    return vals[-last:]


def traffic(fetch_dir: str, write_dir: str, kernel: str = "k_eval_batch<3>", last: int = 200) -> dict:
    fr = load(fetch_dir, "FETCH_SIZE")
    wr = load(write_dir, "WRITE_SIZE")
    fv = dispatch_values(fr, kernel, last)
    wv = dispatch_values(wr, kernel, last)
    probe = [v for _, n, v in fr if "k_probe_stream" in n]
    if len(probe) != 1:
        raise ValueError("expected one k_probe_stream dispatch in the FETCH_SIZE run, found %d" % len(probe))
    others = [v for _, n, v in wr if "tga" not in n]  # the torch copy
    if not others:
        raise ValueError("no calibration copy in the WRITE_SIZE run")
    copy_w = max(others)
    fetch_scale = GIB / (probe[0] * 1024.0)
    write_scale = GIB / (copy_w * 1024.0)
    f_kib = sum(fv) / len(fv)
    w_kib = sum(wv) / len(wv)
    return {
        "kernel": kernel,
        "dispatches": last,
        "fetch_kib_per_dispatch": round(f_kib, 1),
        "write_kib_per_dispatch": round(w_kib, 1),
        "calibration": {"read_bytes": GIB, "fetch_kib_for_probe_read": round(probe[0], 1),
                        "fetch_scale": round(fetch_scale, 4), "write_bytes": GIB,
                        "write_kib_for_copy": round(copy_w, 1), "write_scale": round(write_scale, 4),
                        "fetch_probe": "k_probe_stream: 1 GiB through 16-byte global_load_lds",
                        "write_probe": "1 GiB device copy"},
        "fetch_bytes_per_launch": int(f_kib * 1024 * fetch_scale),
        "write_bytes_per_launch": int(w_kib * 1024 * write_scale),
        "bytes_per_launch": int(f_kib * 1024 * fetch_scale + w_kib * 1024 * write_scale),
        "unscaled_bytes_per_launch": int((f_kib + w_kib) * 1024),
        "kernel_source_sha256": kernel_source_hash(),
    }


def valu(path: str, kernel: str = "k_eval_batch<3>", last: int = 200) -> dict:
    v = dispatch_values(load(path, "SQ_INSTS_VALU"), kernel, last)
    return {"kernel": kernel, "dispatches": last, "valu_insts_per_launch": int(sum(v) / len(v)),
            "kernel_source_sha256": kernel_source_hash()}


def sq(paths, kernel: str = "k_eval_batch<3>", last: int = 200) -> dict:
    means = {}
    for path in paths:
        names = set()
        for fn in glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True):
            with open(fn, newline="") as f:
                names.update(r["Counter_Name"] for r in csv.DictReader(f))
        for c in sorted(names):
            v = dispatch_values(load(path, c), kernel, last)
            means[c] = sum(v) / len(v)
    out = {"kernel": kernel, "dispatches": last, "means_per_launch": {k: round(v, 1) for k, v in means.items()}}
    cyc = means.get("SQ_WAVE_CYCLES")
    if cyc:
        for num, name in (("SQ_WAIT_ANY", "wait_any_share"), ("SQ_WAIT_INST_ANY", "wait_inst_any_share"),
                          ("SQ_ACTIVE_INST_VALU", "valu_active_share")):
            if num in means:
                out[name] = round(means[num] / cyc, 4)
    out["kernel_source_sha256"] = kernel_source_hash()
    return out


def trace(db: str, kernel: str = "k_eval_batch<3>", last: int = 200, top: int = 12) -> str:
    """Markdown summary of a rocprofv3 --kernel-trace database: the mean
    duration of the last `last` dispatches of `kernel` (one pass of the
    benchmark; dispatch durations are in ns) and the per-kernel totals of
    the whole run."""
    import sqlite3
    c = sqlite3.connect(db)
    rows = c.execute("select name, duration from kernels order by start").fetchall()
    durs = [d for n, d in rows if _match(n, kernel)]
    if len(durs) < last:
        raise ValueError("%d dispatches of %s, fewer than %d" % (len(durs), kernel, last))
    tail = durs[-last:]
    out = ["| quantity | value |", "|---|---|",
           "| %s: dispatches in the run | %d |" % (kernel, len(durs)),
           "| mean of the last %d dispatches (us) | %.2f |" % (last, sum(tail) / len(tail) / 1e3),
           "| median of the last %d (us) | %.2f |" % (last, sorted(tail)[len(tail) // 2] / 1e3),
           "| min / max of the last %d (us) | %.2f / %.2f |" % (last, min(tail) / 1e3, max(tail) / 1e3),
           "", "| kernel (whole run) | calls | total (us) | mean (us) |", "|---|---|---|---|"]
    for name, calls, total, avg, _ in c.execute("select * from top_kernels limit %d" % int(top)):
        short = name.split("(")[0]
        out.append("| `%s` | %d | %.1f | %.2f |" % (short, calls, total, avg))  # the view is in us
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    tr = sub.add_parser("trace")
    tr.add_argument("db")
    tr.add_argument("--kernel", default="k_eval_batch<3>")
    tr.add_argument("--last", type=int, default=200)
    tr.add_argument("--top", type=int, default=12)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    v = sub.add_parser("valu")
    v.add_argument("dir")
    q = sub.add_parser("sq")
    q.add_argument("dirs", nargs="+")
    for p in (t, v, q):
        p.add_argument("--kernel", default="k_eval_batch<3>")
        p.add_argument("--last", type=int, default=200)
        p.add_argument("--out", required=True)
        p.add_argument("--workload", default="")
        p.add_argument("--command", action="append", default=[])
    a = ap.parse_args()
    if a.what == "trace":
        print(trace(a.db, a.kernel, a.last, a.top))
        return
    if a.what == "traffic":
        doc = traffic(a.fetch_dir, a.write_dir, a.kernel, a.last)
    elif a.what == "sq":
        doc = sq(a.dirs, a.kernel, a.last)
    else:
        doc = valu(a.dir, a.kernel, a.last)
    doc["workload"] = a.workload
    doc["commands"] = a.command
    with open(a.out, "w") as f:
        json.dump(doc, f, indent=1)
    print(json.dumps(doc, indent=1))


if __name__ == "__main__":
    main()
