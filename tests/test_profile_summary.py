"""The profile summariser (rocprofv3 databases -> per-kernel time and HBM
traffic) on small databases written here, whose answers are known: the
counters are scaled by the calibration copies, and a group averages bytes over
its launches."""
from __future__ import annotations

import sqlite3
import subprocess
import sys

KIB = 262144.0  # the calibration copy, 256 MiB


def _trace(path):
    con = sqlite3.connect(path)
    con.execute("create table kernels (name text, start integer, end integer)")
    rows = [("__amd_rocclr_copyBuffer", 0, 100_000)] * 3 + [
        ("void ck::k_plan_search<8, 2, 0, false>(ck::Geo, ck::Round)", 200_000, 230_000),
        ("void ck::k_plan_search<8, 2, 0, false>(ck::Geo, ck::Round)", 300_000, 310_000),
        ("void ck::k_plan_walk<8, 2, false>(ck::Geo, ck::Round)", 400_000, 420_000),
        ("void ck::k_plan_walk<8, 2, false>(ck::Geo, ck::Round)", 500_000, 520_000),
        ("void ck::k_commit<false>(ck::Geo, ck::Round)", 600_000, 640_000)]
    con.executemany("insert into kernels values (?, ?, ?)", rows)
    con.commit()


def _counters(path, counter, copy_kib, per_kernel):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, counter_name text, "
                "value real, dispatch_id integer)")
    rows = [("__amd_rocclr_copyBuffer", counter, copy_kib, d) for d in (1, 2, 3)]
    d = 4
    for name, v in per_kernel:
        rows.append((name, counter, v, d))
        d += 1
    con.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
    con.commit()


def test_group_traffic_and_calibration(tmp_path):
    s0 = "void ck::k_plan_search<8, 2, 0, false>(ck::Geo, ck::Round)"
    w0 = "void ck::k_plan_walk<8, 2, false>(ck::Geo, ck::Round)"
    c0 = "void ck::k_commit<false>(ck::Geo, ck::Round)"
    _trace(tmp_path / "t.db")
    # FETCH_SIZE reads half of a copy's bytes (x2), WRITE_SIZE all of them (x1)
    _counters(tmp_path / "f.db", "FETCH_SIZE", KIB / 2,
              [(s0, 1000.0), (s0, 1000.0), (w0, 500.0), (w0, 500.0), (c0, 7.0)])
    _counters(tmp_path / "w.db", "WRITE_SIZE", KIB,
              [(s0, 100.0), (s0, 100.0), (w0, 50.0), (w0, 50.0), (c0, 9.0)])
    out = subprocess.run(
        [sys.executable, "-m", "paper_1605_05236_amd.rocprof_summary",
         "--trace", str(tmp_path / "t.db"), "--fetch", str(tmp_path / "f.db"),
         "--write", str(tmp_path / "w.db"), "--group", "evict=k_plan_(search|walk)"],
        capture_output=True, text=True, check=True).stdout
    assert "FETCH_SIZE x2.000, WRITE_SIZE x1.000" in out
    line = [x for x in out.splitlines() if x.startswith("group evict")][0]
    # 4 launches of 30, 10, 20 and 20 us
    assert "4 launches, 20.00 us average" in line
    # read (2000 + 1000) KiB x 2 over 4 launches, write (200 + 100) KiB x 1 over 4
    assert "read 1536000, write 76800, total 1612800" in line
    search = [x for x in out.splitlines() if "k_plan_search" in x and x.startswith("|")][0]
    cells = [c.strip() for c in search.split("|")]
    assert cells[2] == "2" and cells[4] == "20.0"  # calls, average us
    assert cells[6] == "1.95" and cells[7] == "0.10"  # MiB read and written per launch
