"""Per-kernel summary of rocprofv3 result databases (SQLite, rocpd format).

    python -m paper_1605_05236_amd.rocprof_summary --trace K.db \
        [--fetch F.db --write W.db] [--kernels REGEX] [--calibration-kib 262144]
        [--group NAME=REGEX ...]

* --trace: a `rocprofv3 --kernel-trace` database: calls, total and average
  duration per kernel.
* --fetch / --write: `--pmc FETCH_SIZE` and `--pmc WRITE_SIZE` databases of
  the same command.  The counters are scaled by what they read for the plain
  device copies of --calibration-kib KiB that the command ran first (the
  benchmark's --pmc-calibration option): the first copyBuffer dispatches whose
  WRITE_SIZE is at least half the copy size.  Output: HBM MiB per launch and
  the achieved HBM rate of every kernel.
* --group NAME=REGEX: one more line per group of kernels taken together (for
  example the planners that share one role): launches, average duration, and
  HBM bytes per launch averaged over the group's launches.
* --trace-log / --fetch-log / --write-log: the stderr of each profiled run.
  When it holds the benchmark's `# profiler window ns: A B` line (its timed
  region, in the profiler's clock), that run's kernels are cut to the ones
  that started and ended inside the window.  A counter database whose
  dispatches carry no timestamps is cut to the dispatch ids of the trace's
  window instead (the runs dispatch the same sequence: give every run
  --pmc-calibration), and the kernel names at those ids are checked.
"""
from __future__ import annotations

import argparse
import collections
import re
import sqlite3


def _short(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "")
    return name.split("(")[0].replace("void ", "").strip()


def window(log):
    """(start, end) ns of the benchmark's timed region from a run's log, or None."""
    if not log:
        return None
    found = None
    with open(log, errors="replace") as fh:
        for line in fh:
            m = re.search(r"# profiler window ns: (\d+) (\d+)", line)
            if m:
                found = (int(m.group(1)), int(m.group(2)))
    if found is None:
        raise SystemExit(f"{log}: no profiler window line")
    return found


def kernel_times(db: str, win=None):
    """(kernel -> [calls, total microseconds], {dispatch id: kernel}) of the
    dispatches inside `win` (all when None)."""
    out = collections.defaultdict(lambda: [0, 0.0])
    ids = {}
    con = sqlite3.connect(db)
    for name, s, e, d in con.execute("select name, start, end, dispatch_id from kernels"):
        if win is not None and not (s >= win[0] and e <= win[1]):
            continue
        k = _short(name)
        out[k][0] += 1
        out[k][1] += (e - s) / 1e3
        ids[d] = k
    return dict(out), ids


def counter_totals(db: str, counter: str, win=None, trace_ids=None):
    """(kernel -> [dispatches, KiB total], [(dispatch id, kernel, KiB)], how):
    all rows, or those inside `win` by their own timestamps, or (when the
    database holds none) those at the dispatch ids of the trace's window."""
    rows = []
    con = sqlite3.connect(db)
    for name, v, d, s, e in con.execute(
            "select kernel_name, value, dispatch_id, start, end from counters_collection "
            "where counter_name = ? order by dispatch_id", (counter,)):
        rows.append((d, _short(name), v, s, e))
    how = "all dispatches"
    keep = rows
    if win is not None and any(s for _, _, _, s, _ in rows):
        keep = [r for r in rows if r[3] >= win[0] and r[4] <= win[1]]
        how = "own timed window"
    elif trace_ids is not None:
        keep = [r for r in rows if r[0] in trace_ids]
        bad = sum(1 for r in keep if trace_ids[r[0]] != r[1])
        if bad or len(keep) != len(trace_ids):
            raise SystemExit(f"{db}: dispatch sequence differs from the trace's "
                             f"({bad} names differ, {len(keep)} of {len(trace_ids)} ids found)")
        how = "dispatch ids of the trace's window"
    out = collections.defaultdict(lambda: [0, 0.0])
    for d, k, v, _, _ in keep:
        out[k][0] += 1
        out[k][1] += v
    return dict(out), [(d, k, v) for d, k, v, _, _ in rows], how


def calibration(write_rows, fetch_rows, kib: float):
    """Scale factors (fetch, write) from the calibration copies: the first
    copyBuffer dispatches that wrote at least half the copy size."""
    ids = [d for d, k, v in write_rows if k == "__amd_rocclr_copyBuffer" and v >= kib / 2][:3]
    if not ids:
        raise SystemExit("no calibration copy found (run the command with --pmc-calibration)")
    w = [v for d, k, v in write_rows if d in ids]
    f = [v for d, k, v in fetch_rows if d in ids]
    # the two runs dispatch the same sequence, so the ids line up
    return kib / (sum(f) / len(f)), kib / (sum(w) / len(w))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--kernels", default=".*")
    ap.add_argument("--calibration-kib", type=float, default=262144.0)
    ap.add_argument("--top", type=int, default=25)
    ap.add_argument("--group", action="append", default=[])
    ap.add_argument("--trace-log")
    ap.add_argument("--fetch-log")
    ap.add_argument("--write-log")
    a = ap.parse_args()
    tw = window(a.trace_log)
    t, ids = kernel_times(a.trace, tw)
    if tw is not None:
        print(f"trace cut to the timed window: {sum(v[0] for v in t.values())} dispatches")
    f = w = None
    if a.fetch and a.write:
        tid = ids if tw is not None else None
        f, frows, fhow = counter_totals(a.fetch, "FETCH_SIZE", window(a.fetch_log), tid)
        w, wrows, whow = counter_totals(a.write, "WRITE_SIZE", window(a.write_log), tid)
        cf, cw = calibration(wrows, frows, a.calibration_kib)
        print(f"calibration: FETCH_SIZE x{cf:.3f}, WRITE_SIZE x{cw:.3f} "
              f"(plain copy of {a.calibration_kib / 1024:.0f} MiB)")
        print(f"counter dispatches: FETCH_SIZE {fhow}, WRITE_SIZE {whow}")
    pat = re.compile(a.kernels)
    total = sum(v[1] for v in t.values())
    hdr = f"| kernel | calls | total ms | avg us | % time |"
    if f is not None:
        hdr += " HBM read MiB/launch | HBM write MiB/launch | HBM GB/s |"
    print(hdr)
    print("|" + "---|" * (hdr.count("|") - 1))
    for k, (n, us) in sorted(t.items(), key=lambda kv: -kv[1][1])[:a.top]:
        if not pat.search(k):
            continue
        line = f"| `{k}` | {n} | {us / 1e3:.2f} | {us / n:.1f} | {100 * us / total:.1f} |"
        if f is not None:
            fm = f.get(k, [1, 0.0])
            wm = w.get(k, [1, 0.0])
            rd = fm[1] * cf / 1024 / max(fm[0], 1)
            wr = wm[1] * cw / 1024 / max(wm[0], 1)
            gbs = (rd + wr) * n * 1048576 / (us * 1e-6) / 1e9 if us else 0.0
            line += f" {rd:.2f} | {wr:.2f} | {gbs:.0f} |"
        print(line)
    for spec in a.group:
        name, rx = spec.split("=", 1)
        g = re.compile(rx)
        ks = [k for k in t if g.search(k)]
        n = sum(t[k][0] for k in ks)
        us = sum(t[k][1] for k in ks)
        if not n:
            print(f"group {name}: no launches")
            continue
        line = f"group {name} ({', '.join(sorted(ks))}): {n} launches, {us / n:.2f} us average"
        if f is not None:
            rd = sum(f.get(k, [0, 0.0])[1] for k in ks) * cf * 1024
            wr = sum(w.get(k, [0, 0.0])[1] for k in ks) * cw * 1024
            nf = sum(f.get(k, [0, 0.0])[0] for k in ks)
            nw = sum(w.get(k, [0, 0.0])[0] for k in ks)
            line += (f", HBM bytes per launch: read {rd / max(nf, 1):.0f}, "
                     f"write {wr / max(nw, 1):.0f}, "
                     f"total {rd / max(nf, 1) + wr / max(nw, 1):.0f}")
        print(line)


if __name__ == "__main__":
    main()
