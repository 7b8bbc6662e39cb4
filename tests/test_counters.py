"""The counter summariser (paper_2506_17357_amd/counters.py) on synthetic
rocprofv3 outputs: dispatch selection by kernel name (demangled or not),
the calibration scales of FETCH_SIZE and WRITE_SIZE, the VALU and SQ
summaries, and the kernel-trace summary.  Host logic only."""
import csv
import os
import sqlite3

import pytest

from paper_2506_17357_amd import counters

GIB = 1 << 30
EVAL = "void tga::k_eval_batch<3>(tga::SolDev const*, tga::InterItem const*, int const*)"
EVAL_MANGLED = "_ZN3tga12k_eval_batchILi3EEEvPKNS_6SolDevE"


def write_csv(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "p_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], r)))


def test_traffic_scales_and_selects_the_last_dispatches(tmp_path):
    fetch, write = str(tmp_path / "f"), str(tmp_path / "w")
    # the probe reads 1 GiB and reports half of it in KiB: scale 2
    rows = [(1, "tga::k_probe_stream(int const*)", "FETCH_SIZE", GIB / 1024 / 2)]
    # an early dispatch that must be left out, then three counted ones (one
    # counter value split over two rows of the same dispatch)
    rows += [(2, EVAL, "FETCH_SIZE", 9999.0), (3, EVAL, "FETCH_SIZE", 100.0), (4, EVAL_MANGLED, "FETCH_SIZE", 150.0),
             (4, EVAL_MANGLED, "FETCH_SIZE", 50.0), (5, EVAL, "FETCH_SIZE", 300.0)]
    write_csv(fetch, rows)
    wrows = [(1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", GIB / 1024),  # the 1 GiB copy: scale 1
             (2, EVAL, "WRITE_SIZE", 7.0), (3, EVAL, "WRITE_SIZE", 10.0), (4, EVAL, "WRITE_SIZE", 20.0),
             (5, EVAL, "WRITE_SIZE", 30.0)]
    write_csv(write, wrows)
    t = counters.traffic(fetch, write, last=3)
    assert t["calibration"]["fetch_scale"] == 2.0 and t["calibration"]["write_scale"] == 1.0
    assert t["fetch_kib_per_dispatch"] == 200.0 and t["write_kib_per_dispatch"] == 20.0
    assert t["fetch_bytes_per_launch"] == 200 * 1024 * 2 and t["write_bytes_per_launch"] == 20 * 1024
    assert t["bytes_per_launch"] == t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"]
    assert t["unscaled_bytes_per_launch"] == 220 * 1024
    assert t["kernel_source_sha256"] == counters.kernel_source_hash()
    with pytest.raises(ValueError):
        counters.traffic(fetch, write, last=5)  # fewer dispatches than asked for


def test_valu_and_sq_summaries(tmp_path):
    a, b = str(tmp_path / "a"), str(tmp_path / "b")
    write_csv(a, [(d, EVAL, c, v) for d in (1, 2) for c, v in
                  (("SQ_WAVE_CYCLES", 1000.0 * d), ("SQ_WAIT_ANY", 500.0 * d), ("SQ_WAIT_INST_ANY", 100.0 * d))])
    write_csv(b, [(d, EVAL, c, v) for d in (1, 2) for c, v in
                  (("SQ_ACTIVE_INST_VALU", 250.0 * d), ("SQ_INSTS_VALU", 40.0 * d))])
    q = counters.sq([a, b], last=2)
    assert q["means_per_launch"]["SQ_WAVE_CYCLES"] == 1500.0
    assert (q["wait_any_share"], q["wait_inst_any_share"], q["valu_active_share"]) == (0.5, 0.1, 0.25)
    assert counters.valu(b, last=2)["valu_insts_per_launch"] == 60


def test_trace_summary(tmp_path):
    db = str(tmp_path / "trace_results.db")
    c = sqlite3.connect(db)
    c.execute("create table kernels (name text, duration integer, start integer)")
    durs = [5000, 1000, 2000, 3000]  # ns; the first one is not among the last three
    for k, d in enumerate(durs):
        c.execute("insert into kernels values (?, ?, ?)", (EVAL, d, k))
    c.execute("insert into kernels values (?, ?, ?)", ("tga::k_finalize(int)", 700, 10))
    c.execute("create view top_kernels as select name, count(*) as calls, sum(duration) / 1000.0 as total, "
              "avg(duration) / 1000.0 as average, 0 as pct from kernels group by name order by total desc")
    c.commit()
    c.close()
    md = counters.trace(db, last=3, top=4)
    assert "| k_eval_batch<3>: dispatches in the run | 4 |" in md
    assert "| mean of the last 3 dispatches (us) | 2.00 |" in md
    assert "| min / max of the last 3 (us) | 1.00 / 3.00 |" in md
    assert "`void tga::k_eval_batch<3>` | 4 | 11.0 | 2.75 |" in md
