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
"""
from __future__ import annotations

import argparse
import collections
import re
import sqlite3


def _short(name: str) -> str:
    return name.split("(")[0].replace("void ", "").strip()


def kernel_times(db: str) -> dict:
    """kernel -> [calls, total microseconds]."""
    out = collections.defaultdict(lambda: [0, 0.0])
    con = sqlite3.connect(db)
    for name, s, e in con.execute("select name, start, end from kernels"):
        k = _short(name)
        out[k][0] += 1
        out[k][1] += (e - s) / 1e3
    return dict(out)


def counter_totals(db: str, counter: str):
    """(kernel -> [dispatches, KiB total], [(dispatch id, kernel, KiB)])."""
    out = collections.defaultdict(lambda: [0, 0.0])
    rows = []
    con = sqlite3.connect(db)
    for name, v, d in con.execute(
            "select kernel_name, value, dispatch_id from counters_collection "
            "where counter_name = ? order by dispatch_id", (counter,)):
        k = _short(name)
        out[k][0] += 1
        out[k][1] += v
        rows.append((d, k, v))
    return dict(out), rows


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
    a = ap.parse_args()
    t = kernel_times(a.trace)
    f = w = None
    if a.fetch and a.write:
        f, frows = counter_totals(a.fetch, "FETCH_SIZE")
        w, wrows = counter_totals(a.write, "WRITE_SIZE")
        cf, cw = calibration(wrows, frows, a.calibration_kib)
        print(f"calibration: FETCH_SIZE x{cf:.3f}, WRITE_SIZE x{cw:.3f} "
              f"(plain copy of {a.calibration_kib / 1024:.0f} MiB)")
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
