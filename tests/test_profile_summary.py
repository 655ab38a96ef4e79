"""The profile summariser (rocprofv3 databases -> per-kernel time and HBM
traffic) on small databases written here, whose answers are known: the
counters are scaled by the calibration copies, a group averages bytes over
its launches, and a run's timed window (from its log) cuts every database to
the dispatches inside it."""
from __future__ import annotations

import sqlite3
import subprocess
import sys

KIB = 262144.0  # the calibration copy, 256 MiB


# (name, start ns, end ns) of the dispatches, in dispatch order (ids 1, 2, ...)
DISPATCHES = [("__amd_rocclr_copyBuffer", 0, 100_000)] * 3 + [
    ("void ck::k_plan_search<8, 2, 0, false>(ck::Geo, ck::Round)", 200_000, 230_000),
    ("void ck::k_plan_search<8, 2, 0, false>(ck::Geo, ck::Round)", 300_000, 310_000),
    ("void ck::k_plan_walk<8, 2, false>(ck::Geo, ck::Round)", 400_000, 420_000),
    ("void ck::k_plan_walk<8, 2, false>(ck::Geo, ck::Round)", 500_000, 520_000),
    ("void ck::k_commit<false>(ck::Geo, ck::Round)", 600_000, 640_000)]


def _trace(path):
    con = sqlite3.connect(path)
    con.execute("create table kernels (name text, start integer, end integer, "
                "dispatch_id integer)")
    con.executemany("insert into kernels values (?, ?, ?, ?)",
                    [(n, s, e, d) for d, (n, s, e) in enumerate(DISPATCHES, 1)])
    con.commit()


def _counters(path, counter, copy_kib, per_kernel, timestamps=True, shift=0):
    """Counter rows in dispatch order; their start and end are the trace's
    (moved by `shift`, as another run's clock would be), or 0 without them."""
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, counter_name text, "
                "value real, dispatch_id integer, start integer, end integer)")
    vals = [copy_kib] * 3 + [v for _, v in per_kernel]
    rows = []
    for d, ((name, s, e), v) in enumerate(zip(DISPATCHES, vals), 1):
        rows.append((name, counter, v, d, s + shift if timestamps else 0,
                     e + shift if timestamps else 0))
    con.executemany("insert into counters_collection values (?, ?, ?, ?, ?, ?)", rows)
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


def _summary(tmp_path, *extra):
    return subprocess.run(
        [sys.executable, "-m", "paper_1605_05236_amd.rocprof_summary",
         "--trace", str(tmp_path / "t.db"), "--fetch", str(tmp_path / "f.db"),
         "--write", str(tmp_path / "w.db"), "--group", "evict=k_plan_(search|walk)", *extra],
        capture_output=True, text=True, check=True).stdout


def _window_log(path, a, b):
    path.write_text(f"# warmup 0 done\n# profiler window ns: {a} {b}\n{{}}\n")
    return str(path)


PER_KERNEL_F = [("s", 1000.0), ("s", 3000.0), ("w", 500.0), ("w", 900.0), ("c", 7.0)]
PER_KERNEL_W = [("s", 100.0), ("s", 300.0), ("w", 50.0), ("w", 90.0), ("c", 9.0)]


def test_timed_window_cuts_trace_and_counters(tmp_path):
    # the window holds the two searches and the first walk only
    _trace(tmp_path / "t.db")
    _counters(tmp_path / "f.db", "FETCH_SIZE", KIB / 2, PER_KERNEL_F, shift=7_000_000)
    _counters(tmp_path / "w.db", "WRITE_SIZE", KIB, PER_KERNEL_W, shift=9_000_000)
    out = _summary(tmp_path,
                   "--trace-log", _window_log(tmp_path / "t.log", 150_000, 450_000),
                   "--fetch-log", _window_log(tmp_path / "f.log", 7_150_000, 7_450_000),
                   "--write-log", _window_log(tmp_path / "w.log", 9_150_000, 9_450_000))
    assert "trace cut to the timed window: 3 dispatches" in out
    assert "FETCH_SIZE own timed window, WRITE_SIZE own timed window" in out
    line = [x for x in out.splitlines() if x.startswith("group evict")][0]
    # 3 launches of 30, 10 and 20 us
    assert "3 launches, 20.00 us average" in line
    # read (1000 + 3000 + 500) KiB x 2 over 3 launches, write (100 + 300 + 50) x 1 over 3
    assert "read 3072000, write 153600, total 3225600" in line
    assert not [x for x in out.splitlines() if "k_commit" in x]


def test_window_by_dispatch_ids_when_counters_have_no_timestamps(tmp_path):
    _trace(tmp_path / "t.db")
    _counters(tmp_path / "f.db", "FETCH_SIZE", KIB / 2, PER_KERNEL_F, timestamps=False)
    _counters(tmp_path / "w.db", "WRITE_SIZE", KIB, PER_KERNEL_W, timestamps=False)
    out = _summary(tmp_path, "--trace-log", _window_log(tmp_path / "t.log", 150_000, 450_000))
    assert "FETCH_SIZE dispatch ids of the trace's window" in out
    line = [x for x in out.splitlines() if x.startswith("group evict")][0]
    assert "3 launches" in line and "total 3225600" in line


def test_window_refuses_a_different_dispatch_sequence(tmp_path):
    _trace(tmp_path / "t.db")
    bad = [("s", 1000.0)] * 5
    _counters(tmp_path / "f.db", "FETCH_SIZE", KIB / 2, bad, timestamps=False)
    con = sqlite3.connect(tmp_path / "f.db")
    con.execute("update counters_collection set kernel_name = 'other' where dispatch_id = 5")
    con.commit()
    _counters(tmp_path / "w.db", "WRITE_SIZE", KIB, PER_KERNEL_W, timestamps=False)
    r = subprocess.run(
        [sys.executable, "-m", "paper_1605_05236_amd.rocprof_summary",
         "--trace", str(tmp_path / "t.db"), "--fetch", str(tmp_path / "f.db"),
         "--write", str(tmp_path / "w.db"),
         "--trace-log", _window_log(tmp_path / "t.log", 150_000, 450_000)],
        capture_output=True, text=True)
    assert r.returncode != 0 and "dispatch sequence differs" in r.stderr + r.stdout
