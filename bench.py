"""Benchmark: batched cuckoo insertion to 95% load, lookups and deletes on one
MI355X (2^24 bins x 8 slots, 64-bit keys and values, 2 hash functions).

One step is one pass of the whole hot path on synthetic inputs that are
already resident in HBM:
  1. for each scheme (BFS, sorted search, queue-kicking): empty the table and
     insert 0.95 * 2^27 = 127,506,841 keys in sub-batches of 2^20 (phased
     rounds: fresh placement, kick-out planning, claims, reverse-order commit,
     metadata and spawn counts, per-band statistics);
  2. 2^26 lookups at a 90% hit rate on the last table;
  3. 2^20 overwrites of stored keys, 2^21 upserts (those keys again,
     interleaved with as many absent ones), then 2^20 deletes of the stored
     keys, on that table.
`value` is inserts per second over the three fills.  Lookup and delete rates,
bins viewed per insert around 95% load, the roofline of the dominant kernel
and the CPU oracle's rate on a bounded sample are reported beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
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

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E

# Measured HBM traffic of the eviction planners (k_plan_search, k_plan_walk)
# per launch in the default fill workload: FETCH_SIZE + WRITE_SIZE from two
# rocprofv3 --pmc runs of this benchmark (--steps 1 --warmup 1
# --pmc-calibration), each scaled by its reading for a plain 256 MiB device
# copy, over the launches of the timed step (the class the benchmark times).  It describes the library source it was taken on (kernels, launch
# shapes, host loop); once that source changes the benchmark reports null
# until the counters are taken again.
MEASURED_EVICT_TRAFFIC = {
    "sources_sha256": "f6f24c022b8b0bef9d2f3e10bab2d3ab49f32bb69b82d03505a0be48b6d0edbe",
    "bytes_per_launch": 35111708,
    "profile": "profiles/evict_planners__fill95_2e24x8.md",
}
_SOURCES = ("ck_kernels.hip", "ck_api.hip", "ck_internal.h")


def _sources_sha256() -> str:
    """sha256 over the library's sources, in the order of _SOURCES."""
    import hashlib
    h = hashlib.sha256()
    for name in _SOURCES:
        with open(os.path.join(ROOT, "paper_1605_05236_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def pmc_calibration_copies():
    """Three plain device copies of 256 MiB (the yardstick of the HBM counters)."""
    import torch
    a = torch.ones(1 << 25, dtype=torch.int64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--bins-log2", type=int, default=24)
    p.add_argument("--slots", type=int, default=8)
    p.add_argument("--load", type=float, default=0.95)
    p.add_argument("--schemes", default="bfs,sorted,queue")
    p.add_argument("--batch-log2", type=int, default=20)
    p.add_argument("--lookups-log2", type=int, default=26)
    p.add_argument("--hit-rate", type=float, default=0.9)
    p.add_argument("--deletes-log2", type=int, default=20)
    p.add_argument("--max-search", type=int, default=500)
    p.add_argument("--spawn-k", type=int, default=0,
                   help="fill: BFS and sorted search spawn this many records at a time "
                        "(Sec. 5, Prefetching; 0 = one at a time)")
    p.add_argument("--lpp", type=int, default=0,
                   help="lookup lanes per probe (1 or slots per bin; 0 = slots per bin)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--pmc-calibration", action="store_true",
                   help="first run three plain 256 MiB device copies (the yardstick "
                        "for rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    p.add_argument("--cpu-bins-log2", type=int, default=19)
    p.add_argument("--workload", default="fill",
                   choices=["fill", "group", "serve", "mixed", "dary", "bias", "stash",
                            "ceilings", "small", "txn"],
                   help="fill: one 2^24 x 8 table (default); group: 4096 tables of "
                        "2^10..2^20 bins x 4 slots, batched vs per-request launches; "
                        "serve: the same tables behind the continuous-batching server, "
                        "Poisson arrivals; mixed: steady-state lookups/inserts/deletes "
                        "with ghosts on a 2^25 x 4 table at 97%; dary: single-slot bins, "
                        "d = 3 and 4, rattle vs random walk; ceilings: random line "
                        "gathers and 64-bit atomics over 2 GiB; small: the 2^16 x 4 "
                        "random-walk table")
    p.add_argument("--mixed-steps", type=int, default=1024, help="mixed: steps of 2^18 ops")
    p.add_argument("--txn-ops", type=int, default=16, help="txn: operations per transaction")
    p.add_argument("--dary-schemes", default="rattle,random_walk", help="dary: schemes")
    p.add_argument("--rate", type=float, default=200_000.0, help="serve: requests per second")
    p.add_argument("--max-batch-ops", type=int, default=1 << 22, help="serve: ops per batch cap")
    p.add_argument("--tables", type=int, default=4096)
    p.add_argument("--requests", type=int, default=8192)
    p.add_argument("--per-request-sample", type=int, default=512)
    p.add_argument("--cpu-table-stride", type=int, default=4,
                   help="group: the all-cores oracle baseline takes every k-th table")
    p.add_argument("--group-scheme", default="queue")
    p.add_argument("--tune", action="store_true", help="autotune the group's knobs first")
    return p.parse_args()


def _cpu_model() -> dict:
    """The host CPU's model name and logical core count (from /proc/cpuinfo)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cores": os.cpu_count()}


def cpu_baseline(args, schemes):
    """The oracle (serial, one core) on a bounded sample of the same workload:
    each scheme fills a 2^cpu_bins_log2 x B table to the load, then 2^20
    lookups at the same hit rate run on the last table.  The process is
    pinned to one core for the timing (the oracle is single-threaded)."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle
    from paper_1605_05236_amd import inputs
    n = 1 << args.cpu_bins_log2
    m = inputs.target_count(n, args.slots, args.load)
    keys, vals = inputs.keys_values(2, m)
    q, _ = inputs.lookup_mix(302, keys, m, 1 << 20, args.hit_rate, key_seed=2)
    cpu = _cpu_model()
    old = os.sched_getaffinity(0)
    core = min(old)
    os.sched_setaffinity(0, {core})
    try:
        t_ins = 0.0
        total = 0
        for s in schemes:
            o = oracle.OracleTable(n, args.slots, 2, s, max_search=args.max_search, batch_ops=1,
                                   hash_seed=102, rng_seed=202)
            t0 = time.perf_counter()
            o.insert(keys, vals)
            t_ins += time.perf_counter() - t0
            total += m
        t0 = time.perf_counter()
        o.lookup(q)
        t_look = time.perf_counter() - t0
    finally:
        os.sched_setaffinity(0, old)
    return {"value": total / t_ins, "unit": "inserts/s", "cores": 1, "kind": "oracle",
            "lookups_per_s": q.size / t_look, "pinned_core": core,
            "cpu_model": cpu["model"], "host_logical_cores": cpu["logical_cores"],
            "sample": f"serial oracle (g++ -O2, one thread pinned to one core), schemes "
                      f"{','.join(schemes)}, each filling 2^{args.cpu_bins_log2} bins x "
                      f"{args.slots} slots to {args.load} ({m} inserts per scheme, same key "
                      f"stream as the GPU); then {q.size} lookups at {args.hit_rate} hits on "
                      f"the last table"}


def group_cpu_baseline(args, bins, rs, reqs, key_seed, B):
    """The oracle (serial mode) for many tables on every host core this
    process may use, up to 16: one thread per core, each pinned, over a sample
    of the tables (every --cpu-table-stride-th).  Each thread prefills its
    tables to half load and builds their requests' keys (untimed), waits for
    the others, then runs every request of the stream to its tables, a table's
    ops by kind in the order the GPU runs them (lookups, deletes, inserts).
    The oracle's C calls release the interpreter lock, so the threads run in
    parallel; the rate is the sample's ops over the slowest thread's time."""
    import threading
    import torch
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle
    from paper_1605_05236_amd import inputs
    cores = sorted(os.sched_getaffinity(0))[:16]
    nw = len(cores)
    stride = max(1, args.cpu_table_stride)
    sample = [t for t in range(len(bins)) if t % stride == 0]
    per = {t: {0: [], 1: [], 2: []} for t in sample}
    for kind, t, rec in reqs:
        if t in per:
            per[t][kind].append(rec)
    pre_start, pre = rs.prefill_records()
    # largest tables first, dealt round robin: similar prefill and op counts per thread
    order = sorted(sample, key=lambda t: -int(bins[t]))
    shares = [order[w::nw] for w in range(nw)]
    barrier = threading.Barrier(nw)
    out = [None] * nw

    def keys_of(rec):
        k, v = inputs.keys_at_torch(key_seed, torch.from_numpy(rec))
        return k.numpy().view(np.uint64), v.numpy().view(np.uint64)

    def work(w):
        os.sched_setaffinity(0, {cores[w]})  # this thread only
        tabs = []
        try:
            for t in shares[w]:
                o = oracle.OracleTable(int(bins[t]), B, 2, args.group_scheme, batch_ops=1,
                                       hash_seed=105, rng_seed=205)
                k, v = inputs.keys_values(key_seed, int(pre[t]), start=int(pre_start[t]))
                o.insert(k, v)
                calls = []
                for kind in (0, 2, 1):
                    if per[t][kind]:
                        calls.append((kind,) + keys_of(np.concatenate(per[t][kind])))
                tabs.append((o, calls))
        finally:
            barrier.wait()
        ops = 0
        t0 = time.perf_counter()
        for o, calls in tabs:
            for kind, k, v in calls:
                if kind == 0:
                    o.lookup(k)
                elif kind == 2:
                    o.delete(k)
                else:
                    o.insert(k, v)
                ops += k.size
        out[w] = (ops, time.perf_counter() - t0)

    old = os.sched_getaffinity(0)
    threads = [threading.Thread(target=work, args=(w,)) for w in range(nw)]
    try:
        for th in threads:
            th.start()
        for th in threads:
            th.join()
    finally:
        os.sched_setaffinity(0, old)
    if any(o is None for o in out):
        raise RuntimeError("a baseline thread failed")
    ops = sum(o for o, _ in out)
    span = max(s for _, s in out)
    cpu = _cpu_model()
    return {"value": ops / span, "unit": "ops/s", "cores": nw, "kind": "oracle",
            "cpu_model": cpu["model"], "host_logical_cores": cpu["logical_cores"],
            "thread_seconds": [round(s, 4) for _, s in out],
            "sample": f"serial oracle (g++ -O2), one thread pinned per core on {nw} cores, "
                      f"every {stride}th table ({len(sample)} tables, "
                      f"{int(sum(int(bins[t]) for t in sample))} bins x {B} slots) prefilled "
                      f"to 0.5 untimed, then the stream's {ops} ops to those tables"}


def measure_ceilings(gib=2, line_bytes=128, ops_log2=26, reps=5):
    """The device's random-access ceilings: random whole-line gathers and random
    64-bit atomicMin over a `gib` GiB buffer (best of `reps` launches each)."""
    import ctypes
    import torch
    from paper_1605_05236_amd import build
    if not os.path.exists(build.CEIL_LIB):
        raise RuntimeError(f"{build.CEIL_LIB} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(build.CEIL_LIB)
    vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
    L.ckc_gather_threads.restype = u64
    L.ckc_gather.argtypes = [vp, u64, u32, u64, u64, vp, vp]
    L.ckc_atomic_min.argtypes = [vp, u64, u64, u64, vp]
    words = (gib << 30) // 8
    buf = torch.randint(0, 1 << 62, (words,), dtype=torch.int64, device="cuda")
    out = torch.empty(int(L.ckc_gather_threads()), dtype=torch.int64, device="cuda")
    s = torch.cuda.current_stream()
    sp = ctypes.c_void_p(s.cuda_stream)
    n = 1 << ops_log2
    lines = (gib << 30) // line_bytes

    def best(fn):
        fn(0)
        t = []
        for r in range(reps):
            t.append(_timed(lambda: fn(r + 1)))
        return min(t)

    def gather(seed):
        assert L.ckc_gather(ctypes.c_void_p(buf.data_ptr()), lines, line_bytes, n, seed,
                            ctypes.c_void_p(out.data_ptr()), sp) == 0

    def amin(seed):
        assert L.ckc_atomic_min(ctypes.c_void_p(buf.data_ptr()), words, n, seed, sp) == 0

    tg = best(gather)
    ta = best(amin)
    del buf, out
    torch.cuda.empty_cache()
    return {"buffer_gib": gib, "ops": n,
            "gather_line_bytes": line_bytes, "gather_lines_per_s": n / tg,
            "gather_GBs": n * line_bytes / tg / 1e9,
            "atomic_min_u64_per_s": n / ta,
            "note": "random whole-line loads (lanes of a group load 16 bytes each) and random "
                    "64-bit atomicMin, addresses drawn in-kernel; best of "
                    f"{reps} launches after one warm-up"}


def run_small(args):
    """The single small table: 2^16 bins x 4 slots, two hash functions, random
    walk capped at 500 kicks, filled to 0.95 in sub-batches of 2^12, then 2^16
    lookups (half present, half absent).  4 MiB of slots: the table stays in
    the 256 MiB last-level cache, so its HBM-roofline fraction can pass 1."""
    import torch
    from paper_1605_05236_amd import inputs
    from paper_1605_05236_amd.table import CuckooTable, as_device_keys
    n, B = 1 << 16, 4
    m = inputs.target_count(n, B, 0.95)
    keys, vals = inputs.keys_values(1, m)
    dk, dv = as_device_keys(keys), as_device_keys(vals)
    q, present, src = inputs.lookup_mix(301, keys, m, 1 << 16, 0.5, key_seed=1,
                                        return_index=True)
    dq = as_device_keys(q)
    t = CuckooTable(n, B, 2, "random_walk", max_chain=500, batch_ops=1 << 12, hash_seed=101,
                    rng_seed=201)
    fills, looks = [], []
    for r in range(4):
        t.clear()
        fills.append(_timed(lambda: t.insert(dk, dv, diagnostics=False)))
        t.lookup(dq)
        looks.append(_timed(lambda: t.lookup(dq)))
    st = t.stats()
    v, f = t.lookup(dq)
    f = f.cpu().numpy().astype(bool)
    v = v.cpu().numpy().view(np.uint64)
    assert np.array_equal(f, present) and np.array_equal(v[present], vals[src[present]])
    band = 189  # [94.5%, 95%)
    fill_s, look_s = float(np.median(fills[1:])), float(np.median(looks[1:]))
    probes = st["lookup_probes"] / max(1, st["lookups"])
    bpq = 17 + probes * B * 16
    return {"workload": "2^16 bins x 4 slots, 2 hash functions, random walk (max chain 500), "
                        "fill to 0.95 in sub-batches of 2^12; 2^16 lookups at 0.5 hits",
            "inserts_per_s": m / fill_s, "lookups_per_s": q.size / look_s,
            "bins_viewed_per_insert_at_95": float(st["band_views"][band] /
                                                  max(1, st["band_inserts"][band])),
            "bins_viewed_per_insert_cumulative": st["views"] / max(1, st["inserts_ok"]),
            "failed_inserts": st["inserts_failed"], "lookup_probes_per_query": probes,
            "lookup_hbm_frac": q.size * bpq / look_s / 1e9 / PEAK_HBM_GBS,
            "note": "cache-resident (4.5 MiB): the fraction is against HBM peak and may pass 1; "
                    "times are medians of three repeats after one warm-up"}


def _profiler_ns():
    """The profiler's clock in ns when the program runs under rocprofv3 (its
    SDK is then loaded in this process), else None.  The fill workload prints
    its timed region in this clock, so a kernel trace of the same command can
    be cut to that region."""
    import ctypes
    for name in ("librocprofiler-sdk.so.1", "librocprofiler-sdk.so"):
        try:
            lib = ctypes.CDLL(name, mode=os.RTLD_NOLOAD | os.RTLD_LAZY)
        except OSError:
            continue
        ts = ctypes.c_uint64(0)
        if lib.rocprofiler_get_timestamp(ctypes.byref(ts)) == 0:
            return int(ts.value)
    return None


def _timed(fn):
    import torch
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3


def run_group(args):
    """Many tables: one group serves a stream of requests (lookups 70% at 90%
    hits, inserts 20% of fresh keys, deletes 10% of stored keys; sizes
    log-uniform on [1, 65536]; tables uniform), prefilled to half load.
    Batched: every request's ops go through one launch sequence per op type.
    Per-request: one call per request (its ops all in one table), the way a
    table-per-call library would be driven."""
    import torch
    from paper_1605_05236_amd import inputs
    from paper_1605_05236_amd.table import CuckooGroup
    torch.cuda.set_device(0)
    B, seed = 4, 5
    bins = inputs.group_tables(seed, args.tables, 10, 20)
    knobs = {"evict_wgs_per_cu": 0, "lanes_per_probe": 0}
    if args.tune:
        from paper_1605_05236_amd import autotune
        knobs = autotune.tune_group(bins, B, 2, args.group_scheme, load=0.5, verbose=True)
    g = CuckooGroup(bins, B, 2, args.group_scheme, batch_ops=1 << 22, hash_seed=105,
                    rng_seed=205, evict_wgs_per_cu=knobs["evict_wgs_per_cu"])
    rs = inputs.RequestStream(300 + seed, bins, B, 0.5, key_seed=seed)
    starts, counts = rs.prefill_records()
    total = int(counts.sum())
    t0 = time.time()
    chunk = 1 << 25
    for c0 in range(0, total, chunk):
        c1 = min(total, c0 + chunk)
        rec = torch.arange(c0, c1, dtype=torch.int64, device="cuda")
        tid = (torch.searchsorted(torch.from_numpy(starts).cuda(), rec, right=True) - 1).to(
            torch.int32)
        k, v = inputs.keys_at_torch(seed, rec)
        st = g.insert(tid, k, v, diagnostics=False)["status"]
        assert bool((st == 1).all()), "prefill insert failed"
    torch.cuda.synchronize()
    print(f"# prefilled {args.tables} tables ({int(bins.sum())} bins, {total} keys) in "
          f"{time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    reqs = [rs.next() for _ in range(args.requests)]

    def pack(sel):
        kinds = {0: [], 1: [], 2: []}
        for i in sel:
            kind, t, rec = reqs[i]
            kinds[kind].append((t, rec))
        out = {}
        for kind, lst in kinds.items():
            if not lst:
                out[kind] = None
                continue
            rec = np.concatenate([r for _, r in lst])
            tid = np.concatenate([np.full(r.size, t, np.int32) for t, r in lst])
            rr = torch.from_numpy(rec).cuda()
            k, v = inputs.keys_at_torch(seed, rr)
            out[kind] = (torch.from_numpy(tid).cuda(), k, v, rec)
        return out

    def run_batched(packed):
        res = {}
        if packed[0] is not None:
            tid, k, _, _ = packed[0]
            res[0] = g.lookup(tid, k, lanes_per_probe=knobs["lanes_per_probe"])
        if packed[2] is not None:
            tid, k, _, _ = packed[2]
            res[2] = g.delete(tid, k)
        if packed[1] is not None:
            tid, k, v, _ = packed[1]
            res[1] = g.insert(tid, k, v, diagnostics=False)["status"]
        return res

    nops = sum(r[2].size for r in reqs)
    sample = list(range(min(args.per_request_sample, len(reqs))))
    sample_ops = sum(reqs[i][2].size for i in sample)
    # batched: the whole request set (the per-request sample is run on the
    # table state it leaves; both rates are per op)
    packed = pack(range(len(reqs)))
    res = {}
    sec_b = _timed(lambda: res.update(run_batched(packed)))
    # answers: lookups hit exactly where the stream says; deletes and inserts succeed
    if packed[0] is not None:
        _, found = res[0]
        exp = packed[0][3] < rs.miss_start
        assert np.array_equal(found.cpu().numpy().astype(bool), exp), "lookup answers differ"
    if packed[2] is not None:
        assert bool((res[2] == 1).all()), "a delete missed"
    if packed[1] is not None:
        assert bool((res[1] == 1).all()), "an insert failed"
    # per-request launches on a sample of further requests (fresh records)
    more = [rs.next() for _ in range(len(sample))]
    reqs.extend(more)
    idx = list(range(len(reqs) - len(more), len(reqs)))
    per_packs = [pack([i]) for i in idx]
    sec_p = _timed(lambda: [run_batched(pk) for pk in per_packs])
    more_ops = sum(reqs[i][2].size for i in idx)
    batched = nops / sec_b
    per_req = more_ops / sec_p
    out = {
        "metric": "ops/s of many tables: batched launches vs per-request launches",
        "value": batched, "unit": "ops/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": sec_b * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic (splitmix64 keys, seeded)",
        "config": {"workload": f"{args.tables} tables, bins log-uniform 2^10..2^20 x {B} slots "
                               f"({int(bins.sum())} bins), prefilled to 0.5; {len(reqs) - len(more)} "
                               "requests of 1..65536 ops (70% lookup, 20% insert, 10% delete)",
                   "scheme": args.group_scheme, "ops": int(nops), "knobs": knobs},
        "per_request_ops_per_s": per_req,
        "per_request_sample": {"requests": len(more), "ops": int(more_ops)},
        "speedup_batched_vs_per_request": batched / per_req,
    }
    if not args.no_cpu_baseline:
        print("# group cpu baseline (oracle, all cores)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = group_cpu_baseline(args, bins, rs, reqs[:len(reqs) - len(more)],
                                                 seed, B)
    print(json.dumps(out), flush=True)


def run_serve(args):
    """Open-loop serving: Poisson arrivals of requests (1..65536 ops; 70%
    lookups at 90% hits, 20% inserts, 10% deletes) to many tables prefilled to
    half load, through the continuous-batching server.  Request payloads sit
    in pinned host memory (the receive buffer); answers return to it."""
    import torch
    from paper_1605_05236_amd import inputs
    from paper_1605_05236_amd.serve import RequestSet, Server, latency_summary
    torch.cuda.set_device(0)
    B, seed = 4, 5
    bins = inputs.group_tables(seed, args.tables, 10, 20)
    srv = Server(bins, B, 2, args.group_scheme, slab_tables=args.tables,
                 max_batch_ops=args.max_batch_ops, lanes_per_probe=args.lpp or 0,
                 hash_seed=105, rng_seed=205)
    rs = inputs.RequestStream(300 + seed, bins, B, 0.5, key_seed=seed)
    starts, counts = rs.prefill_records()
    t0 = time.time()
    g, _ = srv.table(0)
    total = int(counts.sum())
    chunk = 1 << 25
    for c0 in range(0, total, chunk):
        c1 = min(total, c0 + chunk)
        rec = torch.arange(c0, c1, dtype=torch.int64, device="cuda")
        tid = (torch.searchsorted(torch.from_numpy(starts).cuda(), rec, right=True) - 1).to(
            torch.int32)
        k, v = inputs.keys_at_torch(seed, rec)
        assert bool((g.insert(tid, k, v, diagnostics=False)["status"] == 1).all())
    torch.cuda.synchronize()
    req = rs.take(args.requests)
    keys, vals, expect = rs.payload(req)
    if args.rate > 0:
        arrivals = inputs.poisson_arrivals(400 + seed, args.requests, args.rate)
    else:  # every request at once: the server's capacity (closed burst)
        arrivals = np.zeros(args.requests)
    rset = RequestSet(req["kind"], req["table"], req["n"], arrivals, keys, vals)
    nops = int(rset.off[-1])
    print(f"# prefilled {args.tables} tables ({total} keys); {args.requests} requests "
          f"({nops} ops) ready in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    res = srv.run(rset)
    summ = latency_summary(res)
    # answers: lookups hit exactly where the stream says, with the stored
    # values; inserts and deletes succeed
    served_ops = np.repeat(~res.unserved, rset.n)
    got = res.flags_in_request_order()
    wrong = int((got[served_ops] != expect.numpy()[:nops][served_ops]).sum())
    samp = np.nonzero((rset.kind == 0) & ~res.unserved)[0][::16]
    for i in samp:
        v, f = res.result(i)
        o0 = rset.off[i]
        want = vals.numpy()[o0:o0 + rset.n[i]].view(np.uint64)
        wrong += int((v[f == 1] != want[f == 1]).sum())
    out = {
        "metric": "served ops/s with p50/p99 request latency (open loop)",
        "value": summ["ops_per_s"], "unit": "ops/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": summ["span_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic (splitmix64 keys, seeded)",
        "config": {"workload": f"{args.tables} tables, bins log-uniform 2^10..2^20 x {B} slots "
                               f"({int(bins.sum())} bins), prefilled to 0.5; {args.requests} "
                               f"requests of 1..65536 ops ({nops} ops; 70% lookup, 20% insert, "
                               f"10% delete), " + (f"Poisson arrivals at {args.rate:.0f} req/s" if args.rate > 0
                                                   else "all arriving at once"),
                   "scheme": args.group_scheme, "max_batch_ops": args.max_batch_ops},
        "latency": summ, "batches": res.stats["batches"], "wrong_answers": wrong,
        "host_issue_s": res.stats["host_issue_s"],
        "host_issue_frac_of_span": res.stats["host_issue_s"] / summ["span_s"] if summ["span_s"] else None,
        "host_slot_wait_s": res.stats["host_slot_wait_s"],
        "device_calls_s": res.stats["device_calls_s"],
        "offered_ops_per_s": nops / float(arrivals[-1]) if arrivals[-1] > 0 else None,
    }
    print(json.dumps(out), flush=True)
    if wrong:
        sys.exit("served answers differ from the request stream's expectations")


def run_mixed(args):
    """Steady state with ghost insertions and claims: a 2^25 x 4 table prefilled
    to 97% with queue-kicking, then steps of 2^18 ops (90% lookups drawn
    Zipf(0.99) over the stored keys, 5% inserts of fresh keys, 5% deletes of
    random stored keys; per step: lookups, deletes, inserts).  The op stream is
    generated before timing, assuming every insert succeeds (a failed insert
    only turns later lookups or deletes of its key into misses)."""
    import torch
    from paper_1605_05236_amd import inputs
    from paper_1605_05236_amd.table import CuckooTable
    torch.cuda.set_device(0)
    if args.pmc_calibration:
        pmc_calibration_copies()
    n, B, seed = 1 << 25, 4, 4
    step_ops = 1 << 18
    steps = args.mixed_steps
    n_look, n_ins = int(step_ops * 0.9), int(step_ops * 0.05)
    n_del = step_ops - n_look - n_ins
    t = CuckooTable(n, B, 2, "queue", ghost=True, batch_ops=step_ops, hash_seed=104,
                    rng_seed=204)
    m = inputs.target_count(n, B, 0.97)
    t0 = time.time()
    rec = torch.arange(m, dtype=torch.int64, device="cuda")
    k, v = inputs.keys_at_torch(seed, rec)
    st = t.insert(k, v, diagnostics=False)["status"]
    stored = torch.empty(m + steps * n_ins, dtype=torch.int64, device="cuda")
    ok = rec[st == 1]
    size = ok.numel()
    stored[:size] = ok
    del k, v, st, rec, ok
    # the op stream: record ids per step
    zipf = inputs.ZipfTorch(size, 0.99)
    gen = torch.Generator(device="cuda").manual_seed(504)
    look = torch.empty(steps, n_look, dtype=torch.int64, device="cuda")
    dels = torch.empty(steps, n_del, dtype=torch.int64, device="cuda")
    ins = torch.empty(steps, n_ins, dtype=torch.int64, device="cuda")
    fresh = m
    for s in range(steps):
        look[s] = stored[zipf.sample(gen, n_look).clamp_(max=size - 1)]
        # n_del distinct uniform positions (unique() sorts, so shuffle before cutting)
        pos = torch.unique(torch.randint(0, size, (n_del + n_del // 4,), generator=gen,
                                         device="cuda"))
        pos = pos[torch.randperm(pos.numel(), generator=gen, device="cuda")][:n_del]
        d = pos.numel()
        if d < n_del:
            raise RuntimeError("too few distinct delete positions")
        dels[s] = stored[pos]
        # swap-remove: holes below the new size take the tail's survivors
        new_size = size - d
        tail = torch.arange(new_size, size, device="cuda")
        is_del = torch.zeros(size - new_size, dtype=torch.bool, device="cuda")
        in_tail = pos >= new_size
        is_del[pos[in_tail] - new_size] = True
        movers = tail[~is_del]
        holes = pos[~in_tail]
        stored[holes] = stored[movers]
        size = new_size
        ins[s] = torch.arange(fresh, fresh + n_ins, device="cuda")
        stored[size:size + n_ins] = ins[s]
        size += n_ins
        fresh += n_ins
    lk, _ = inputs.keys_at_torch(seed, look)
    dk, _ = inputs.keys_at_torch(seed, dels)
    ik, iv = inputs.keys_at_torch(seed, ins)
    del look, dels, ins, stored
    torch.cuda.synchronize()
    print(f"# prefilled {m} keys; {steps} steps of {step_ops} ops ready in "
          f"{time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    before = t.stats()
    vout = torch.empty(n_look, dtype=torch.int64, device="cuda")
    fout = torch.empty(n_look, dtype=torch.uint8, device="cuda")
    hits = torch.zeros((), dtype=torch.int64, device="cuda")
    dfound = torch.zeros((), dtype=torch.int64, device="cuda")
    iok = torch.zeros((), dtype=torch.int64, device="cuda")

    def run():
        for s in range(steps):
            t.lookup(lk[s], out=vout, found=fout)
            hits.add_(fout.sum())
            dfound.add_((t.delete(dk[s]) == 1).sum())
            iok.add_((t.insert(ik[s], iv[s], diagnostics=False)["status"] == 1).sum())

    p_start = _profiler_ns()
    sec = _timed(run)
    p_end = _profiler_ns()
    if p_start is not None and p_end is not None:
        print(f"# profiler window ns: {p_start} {p_end}", file=sys.stderr, flush=True)
    after = t.stats()
    ops = steps * step_ops
    diff = {f: after[f] - before[f] for f in ("inserts_ok", "inserts_failed", "inserts_aborted",
                                              "retries", "delete_retries", "twin_updates",
                                              "kicks", "rounds", "lookups", "lookup_probes")}
    # algorithmic bytes of one step's lookup launch: key, value and found flag
    # per query, plus one 64-byte bin line per probe
    ppq = diff["lookup_probes"] / max(1, diff["lookups"])
    out = {
        "metric": "steady-state ops/s (lookup/insert/delete mix) with abort and retry counts",
        "value": ops / sec, "unit": "ops/s", "n_gpus": 1, "steps": steps, "warmup": 0,
        "ms_per_step": sec * 1e3 / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic (splitmix64 keys, seeded)",
        "config": {"workload": f"2^25 bins x 4 slots prefilled to 0.97 ({m} keys), queue-kicking "
                               f"with ghost insertions; {steps} steps of 2^18 ops (90% Zipf(0.99) "
                               "lookups of stored keys, 5% fresh inserts, 5% deletes of stored "
                               "keys)", "ops": ops},
        "lookup_hit_rate": float(hits) / (steps * n_look),
        "deletes_found": int(dfound), "deletes": steps * n_del,
        "inserts_ok": int(iok), "inserts": steps * n_ins,
        "counts": diff,
        "aborts_per_insert": diff["inserts_aborted"] / (steps * n_ins),
        "lost_rounds_per_insert": diff["retries"] / (steps * n_ins),
        "delete_retries_per_delete": diff["delete_retries"] / (steps * n_del),
        "lookup_probes_per_query": ppq,
        "lookup_algorithmic_bytes_per_launch": n_look * (17 + ppq * B * 16),
    }
    print(json.dumps(out), flush=True)


def run_dary(args):
    """Single-slot bins with d = 3 and d = 4 hash functions, 2^26 slots of
    uint64 key + uint32 value, chains capped at 1000, sub-batches of 2^20:
    rattle-kicking against random-walk kicking, filled to 0.90 then 0.95
    (d = 3) and to 0.97 (d = 4)."""
    import torch
    from paper_1605_05236_amd import inputs
    from paper_1605_05236_amd.table import CuckooTable
    torch.cuda.set_device(0)
    n = 1 << 26
    cases = [(3, (0.90, 0.95)), (4, (0.97,))]
    schemes = [s for s in args.dary_schemes.split(",") if s]
    res = {}
    total_ins, total_s = 0, 0.0
    for d, loads in cases:
        mt = inputs.target_count(n, 1, loads[-1])
        keys, vals = inputs.keys_values_torch(3, mt, value_bits=32)
        vals = vals.to(torch.int32)
        for scheme in schemes:
            t = CuckooTable(n, 1, d, scheme, max_chain=1000, batch_ops=1 << 20, hash_seed=103,
                            rng_seed=203)
            done, out = 0, {}
            st0 = t.stats()
            for load in loads:
                m = inputs.target_count(n, 1, load)
                sec = _timed(lambda: t.insert(keys[done:m], vals[done:m], diagnostics=False))
                st = t.stats()
                # d-ary byte model: 17 bytes in and out per insert, plus one
                # access granule per bin viewed and per bin written (kicks + 1);
                # G = 64 bytes, the line a 16-byte slot access fetches
                v_leg = st["views"] - st0["views"]
                w_leg = (st["kicks"] - st0["kicks"]) + (st["inserts_ok"] - st0["inserts_ok"])
                alg = 17 * (m - done) + 64 * (v_leg + w_leg)
                st0 = st
                bands = st["band_inserts"].astype(np.float64)
                bv = st["band_views"].astype(np.float64)
                top = int(np.floor(load * 200 - 1e-9))  # the band just below `load`
                out[f"{load:.2f}"] = {
                    "inserts_per_s": (m - done) / sec, "seconds": sec,
                    "bins_viewed_per_insert_in_last_band": float(bv[top] / max(bands[top], 1)),
                    "bins_viewed_per_insert_cumulative": float(st["views"] / max(st["inserts_ok"]
                                                                              + st["inserts_failed"], 1)),
                    "failed_inserts": st["inserts_failed"], "stored": st["stored"],
                    "rounds": st["rounds"], "lost_rounds": st["retries"],
                    "algorithmic_bytes_per_insert": alg / max(m - done, 1),
                    "roofline": {"bound": "hbm", "achieved": alg / sec / 1e9,
                                 "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                 "frac": alg / sec / 1e9 / PEAK_HBM_GBS,
                                 "model": "17 + 64 (V + W) per insert, G = 64"}}
                total_ins += m - done
                total_s += sec
                done = m
                print(f"# d={d} {scheme} to {load}: {out[f'{load:.2f}']}", file=sys.stderr,
                      flush=True)
            res[f"d{d}_{scheme}"] = out
            t.close()
        del keys, vals
    print(json.dumps({
        "metric": "d-ary inserts/s and bins viewed per insert: rattle vs random walk",
        "value": total_ins / total_s, "unit": "inserts/s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": total_s * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic (splitmix64 keys, seeded)",
        "config": {"workload": "2^26 single-slot bins (uint64 key + uint32 value), d = 3 to "
                               "0.90/0.95 and d = 4 to 0.97, max chain 1000, sub-batches of 2^20",
                   "schemes": schemes},
        "by_case": res}), flush=True)


def run_bias(args):
    """Biased hashes (Sec. 9's open question): the fill of 2^22 bins x 4 slots
    (two hash functions, 64-bit keys and values, sub-batches of 2^20) to 0.90
    with random kicking, BFS, sorted search and queue-kicking, at bias levels
    0 (uniform), 1 and 2.  Bins viewed per insert in the bands just below 0.80
    and 0.90, failures and insert rates per case."""
    import torch
    from paper_1605_05236_amd import inputs
    from paper_1605_05236_amd.table import CuckooTable
    torch.cuda.set_device(0)
    n, B, load = 1 << 22, 4, 0.90
    m = inputs.target_count(n, B, load)
    keys, vals = inputs.keys_values_torch(4, m)
    res, total_ins, total_s = {}, 0, 0.0
    for bias in (0, 1, 2):
        for scheme in ("random_walk", "bfs", "sorted", "queue"):
            t = CuckooTable(n, B, 2, scheme, max_chain=500, max_search=500, batch_ops=1 << 20,
                            hash_seed=104, rng_seed=204, hash_bias=bias)
            sec = _timed(lambda: t.insert(keys, vals, diagnostics=False))
            st = t.stats()
            bands = st["band_inserts"].astype(np.float64)
            bv = st["band_views"].astype(np.float64)
            out = {"inserts_per_s": m / sec, "seconds": sec,
                   "failed_inserts": st["inserts_failed"], "stored": st["stored"]}
            for edge in (0.80, 0.90):
                top = int(np.floor(edge * 200 - 1e-9))
                out[f"bins_viewed_per_insert_below_{edge:.2f}"] = (
                    float(bv[top] / bands[top]) if bands[top] else None)
            res[f"bias{bias}_{scheme}"] = out
            total_ins += m
            total_s += sec
            print(f"# bias {bias} {scheme}: {out}", file=sys.stderr, flush=True)
            t.close()
    print(json.dumps({
        "metric": "inserts/s and bins viewed per insert with biased hashes",
        "value": total_ins / total_s, "unit": "inserts/s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": total_s * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic (splitmix64 keys, seeded)",
        "config": {"workload": "2^22 bins x 4 slots, 2 hash functions, fill to 0.90 in "
                               "sub-batches of 2^20, hash bias levels 0, 1, 2",
                   "schemes": ["random_walk", "bfs", "sorted", "queue"]},
        "by_case": res}), flush=True)


def run_txn(args):
    """Transactional batches (Sec. 8): a 2^22 x 8 table (random kicking with
    load balancing, as in the paper's transactional experiments) prefilled to
    0.5, then transactions of --txn-ops operations in the paper's two mixes
    (inserts : deletes : overwrites : reads = 1:0:1:1, delete-light, and
    2:1:2:2, delete-heavy) until 0.9 load; reads, deletes and overwrites pick
    uniformly among the keys inserted so far (stored or since deleted).  The
    transactions go in calls of 2^14 (one sub-batch each)."""
    import torch
    from paper_1605_05236_amd import inputs
    from paper_1605_05236_amd.table import CuckooTable, as_device_keys
    torch.cuda.set_device(0)
    n, B, chunk = 1 << 22, 8, 1 << 14
    out = {}
    total_ops, total_s = 0, 0.0
    for name, ratio in (("delete_light", (1, 0, 1, 1)), ("delete_heavy", (2, 1, 2, 2))):
        t = CuckooTable(n, B, 2, "random_walk", load_balance=True, max_chain=500,
                        batch_ops=chunk, hash_seed=106, rng_seed=206)
        m0 = inputs.target_count(n, B, 0.5)
        pk, pv = inputs.keys_values(6, m0)
        t.insert(as_device_keys(pk), as_device_keys(pv), diagnostics=False)
        # enough ops that the inserts (net of deletes) bring the load to 0.9
        net = (ratio[0] - ratio[1]) / sum(ratio)
        nops = int((inputs.target_count(n, B, 0.9) - m0) / net)
        nops -= nops % args.txn_ops
        rng = np.random.default_rng(306)
        kind = rng.choice(4, nops, p=np.array([ratio[3], ratio[0], ratio[1], ratio[2]]) /
                          sum(ratio)).astype(np.uint8)  # 0 read, 1 insert, 2 delete, 3 overwrite
        ins = kind == 1
        nins = int(ins.sum())
        fk, fv = inputs.keys_values(6, nins, start=m0)
        keys = np.empty(nops, np.uint64)
        vals = rng.integers(0, 1 << 63, nops, dtype=np.uint64)
        keys[ins] = fk
        vals[ins] = fv
        # the others: a uniform pick among the keys inserted before them
        before = np.cumsum(ins) - ins  # inserts earlier in the stream
        pool = np.concatenate([pk, fk])
        pick = (rng.random(nops) * (m0 + before)).astype(np.int64)
        keys[~ins] = pool[pick[~ins]]
        del pool, pick, before
        off = np.arange(0, nops + 1, args.txn_ops, dtype=np.int32)
        dk, dv = as_device_keys(keys), as_device_keys(vals)
        dkind = torch.from_numpy(kind).cuda()
        doff = torch.from_numpy(off).cuda()
        ntx = off.size - 1
        before_stats = t.stats()
        sec, aborted, rsum, late = 0.0, 0, 0, 0
        for c0 in range(0, ntx, chunk):
            c1 = min(ntx, c0 + chunk)
            box = {}
            sec += _timed(lambda: box.update(r=t.transact(dkind, dk, dv, doff[c0:c1 + 1])))
            st = box["r"]["status"][int(off[c0]):int(off[c1])].cpu().numpy()
            rd = box["r"]["round"].cpu().numpy()
            aborted += int((st[::args.txn_ops] == 3).sum())
            rsum += int(rd.sum())
            late += int((rd > 0).sum())
            if (c0 // chunk) % 32 == 0:
                print(f"# txn {name}: {c1}/{ntx} transactions, {sec:.2f}s", file=sys.stderr,
                      flush=True)
        after = t.stats()
        out[name] = {"transactions": ntx, "ops": nops, "transactions_per_s": ntx / sec,
                     "ops_per_s": nops / sec, "seconds": sec,
                     "aborted_transactions": aborted,
                     "mean_commit_round": rsum / ntx,
                     "transactions_committed_after_losing_a_round": late,
                     "rounds": after["rounds"] - before_stats["rounds"],
                     "load_after": after["stored"] / (n * B),
                     "failed_inserts": after["inserts_failed"] - before_stats["inserts_failed"]}
        total_ops += nops
        total_s += sec
        print(f"# txn {name}: {out[name]}", file=sys.stderr, flush=True)
        t.close()
        del dk, dv, dkind, doff
    print(json.dumps({
        "metric": "transactional batches: transactions/s, ops/s, rounds lost and aborts",
        "value": total_ops / total_s, "unit": "ops/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": total_s * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic (splitmix64 keys, seeded)",
        "config": {"workload": f"2^22 bins x 8 slots, random kicking with load balancing, "
                               f"prefilled to 0.5, transactions of {args.txn_ops} ops to 0.9 "
                               "load, mixes 1:0:1:1 and 2:1:2:2 (insert:delete:overwrite:read), "
                               f"calls of {chunk} transactions"},
        "by_mix": out}), flush=True)


def run_stash(args):
    """The stash (Sec. 2): a 2^22 x 4 table (two hash functions, 64-bit keys and
    values, sub-batches of 2^20) filled to 0.97 by random kicking with chains
    capped at 20 kicks, so chains fail near the top, without a stash and with
    64 entries; then 2^24 lookups at 0.9 hits, whose misses also search the
    stash when there is one."""
    import torch
    from paper_1605_05236_amd import inputs
    from paper_1605_05236_amd.table import CuckooTable, as_device_keys
    torch.cuda.set_device(0)
    n, B, load = 1 << 22, 4, 0.97
    m = inputs.target_count(n, B, load)
    keys, vals = inputs.keys_values(5, m)
    dkeys, dvals = as_device_keys(keys), as_device_keys(vals)
    nq = 1 << 24
    q, present = inputs.lookup_mix(305, keys, m, nq, 0.9, key_seed=5)
    dq = as_device_keys(q)
    res, total_ins, total_s = {}, 0, 0.0
    for stash in (0, 64):
        t = CuckooTable(n, B, 2, "random_walk", max_chain=20, batch_ops=1 << 20, hash_seed=105,
                        rng_seed=205, stash=stash)
        t.insert(dkeys, dvals, diagnostics=False)  # warm-up fill
        t.clear()
        sec = _timed(lambda: t.insert(dkeys, dvals, diagnostics=False))
        st = t.stats()
        t.lookup(dq)  # warm
        lsec = _timed(lambda: t.lookup(dq))
        out_v, found = t.lookup(dq)
        res[f"stash{stash}"] = {
            "inserts_per_s": m / sec, "lookups_per_s": nq / lsec,
            "failed_inserts": st["inserts_failed"], "stashed_inserts": st["inserts_stashed"],
            "lookup_hits": int(found.sum().item())}
        total_ins += m
        total_s += sec
        print(f"# stash {stash}: {res[f'stash{stash}']}", file=sys.stderr, flush=True)
        t.close()
    print(json.dumps({
        "metric": "inserts/s and lookups/s with and without a stash",
        "value": total_ins / total_s, "unit": "inserts/s", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": total_s * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic (splitmix64 keys, seeded)",
        "config": {"workload": "2^22 bins x 4 slots, 2 hash functions, random kicking with "
                               "chains capped at 20, fill to 0.97 in sub-batches of 2^20, "
                               "stash of 0 and 64 entries; 2^24 lookups at 0.9 hits"},
        "by_case": res}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; the table shards by key "
                                   "hash across GPUs but no multi-GPU path is built"}))
        sys.exit(2)
    if args.workload == "group":
        run_group(args)
        return
    if args.workload == "serve":
        run_serve(args)
        return
    if args.workload == "mixed":
        run_mixed(args)
        return
    if args.workload == "dary":
        run_dary(args)
        return
    if args.workload == "bias":
        run_bias(args)
        return
    if args.workload == "stash":
        run_stash(args)
        return
    if args.workload == "txn":
        run_txn(args)
        return
    if args.workload in ("ceilings", "small"):
        import torch
        torch.cuda.set_device(0)
        if args.workload == "ceilings":
            c = measure_ceilings()
            line = {"metric": "random-access ceilings: line gathers/s and 64-bit atomicMin/s",
                    "value": c["gather_lines_per_s"], "unit": "lines/s", "ceilings": c}
        else:
            c = run_small(args)
            line = {"metric": "inserts/s and bins viewed per insert at 95% load, small table",
                    "value": c["inserts_per_s"], "unit": "inserts/s", "small_table": c}
        line.update({"n_gpus": 1, "higher_is_better": True, "dtype": "u64",
                     "data": "synthetic"})
        print(json.dumps(line), flush=True)
        return
    import torch
    from paper_1605_05236_amd import inputs
    from paper_1605_05236_amd.table import CuckooTable, as_device_keys

    torch.cuda.set_device(0)
    if args.pmc_calibration:
        pmc_calibration_copies()
    schemes = [s for s in args.schemes.split(",") if s]
    n, B = 1 << args.bins_log2, args.slots
    m = inputs.target_count(n, B, args.load)
    # keys up to 98% load: the fills use the first m; after the timed steps each
    # table is taken on from 95% to 98% (the top of the loads reported)
    m_top = max(m, inputs.target_count(n, B, 0.98))
    t0 = time.time()
    keys_all, vals_all = inputs.keys_values(2, m_top)
    keys, vals = keys_all[:m], vals_all[:m]
    dkeys_all, dvals_all = as_device_keys(keys_all), as_device_keys(vals_all)
    dkeys, dvals = dkeys_all[:m], dvals_all[:m]
    nq = 1 << args.lookups_log2
    q, present, q_src = inputs.lookup_mix(302, keys, m, nq, args.hit_rate, key_seed=2,
                                          return_index=True)
    dq = as_device_keys(q)
    rng = np.random.default_rng(402)
    dels = keys[rng.choice(m, 1 << args.deletes_log2, replace=False)]
    ddel = as_device_keys(dels)
    # the same stored keys get new values first (overwrites), then go
    dnew = torch.from_numpy(rng.integers(0, 1 << 63, dels.size, dtype=np.int64)).cuda()
    # then upserts: the same stored keys (new values again) and as many absent
    # keys, interleaved
    fresh, fresh_v = inputs.keys_values(3, dels.size)
    ups = np.empty(2 * dels.size, np.uint64)
    ups[0::2], ups[1::2] = dels, fresh
    ups_v = np.empty(2 * dels.size, np.uint64)
    ups_v[0::2], ups_v[1::2] = rng.integers(0, 1 << 63, dels.size, dtype=np.uint64), fresh_v
    dups, dups_v = as_device_keys(ups), as_device_keys(ups_v)
    del q
    print(f"# inputs ready in {time.time() - t0:.1f}s: {m} inserts, {nq} lookups, "
          f"{dels.size} deletes", file=sys.stderr, flush=True)
    tables = {s: CuckooTable(n, B, 2, s, max_search=args.max_search,
                             batch_ops=1 << args.batch_log2, hash_seed=102, rng_seed=202,
                             spawn_k=args.spawn_k if s in ("bfs", "sorted") else 0)
              for s in schemes}
    stream = torch.cuda.current_stream()
    vout = torch.empty(nq, dtype=torch.int64, device="cuda")
    fout = torch.empty(nq, dtype=torch.uint8, device="cuda")

    def step(record, timed):
        """One step; `timed` = kernel classes to time with HIP events."""
        res = {"fill_s": {}, "stats": {}, "timing": {}}
        for s in schemes:
            tables[s].timing(enable=timed)
        for s in schemes:
            t = tables[s]
            t.clear()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            t.insert(dkeys, dvals, diagnostics=False)
            e1.record(stream)
            e1.synchronize()
            res["fill_s"][s] = e0.elapsed_time(e1) / 1e3
            if record:
                res["stats"][s] = t.stats()
            if timed:
                res["timing"][s] = t.timing()
        t = tables[schemes[-1]]
        e0, e1, e2, e3 = (torch.cuda.Event(enable_timing=True) for _ in range(4))
        e0.record(stream)
        t.lookup(dq, out=vout, found=fout, lanes_per_probe=args.lpp)
        e1.record(stream)
        fw = t.overwrite(ddel, dnew)
        e2.record(stream)
        ru = t.upsert(dups, dups_v, diagnostics=False)["status"]
        e4 = torch.cuda.Event(enable_timing=True)
        e4.record(stream)
        t.delete(ddel)
        e3.record(stream)
        e3.synchronize()
        res["lookup_s"] = e0.elapsed_time(e1) / 1e3
        res["overwrite_s"] = e1.elapsed_time(e2) / 1e3
        res["upsert_s"] = e2.elapsed_time(e4) / 1e3
        res["delete_s"] = e4.elapsed_time(e3) / 1e3
        res["overwrites_found"] = bool((fw == 1).all())
        # stored keys are updated (5), absent ones inserted (1)
        res["upserts_as_expected"] = bool((ru[0::2] == 5).all() and (ru[1::2] == 1).all())
        if timed:
            res["lookup_timing"] = t.timing()["lookup"]
        return res

    # Warm-up: the first warm-up step times every kernel class to find the
    # dominant one; the timed steps then time only that class (two HIP events
    # per launch of it), so the instrumentation hardly touches the timed rate.
    dominant, warm_ms = "plan_evict", None
    for w in range(args.warmup):
        res = step(False, True if w == 0 else False)
        if w == 0:
            warm_ms = {}
            for s in schemes:
                for c, v in res["timing"][s].items():
                    if isinstance(v, dict) and c != "lookup":
                        warm_ms[c] = warm_ms.get(c, 0.0) + v["ms"]
            warm_ms["lookup"] = res["lookup_timing"]["ms"]
            dominant = max(warm_ms, key=warm_ms.get)
        print(f"# warmup {w} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    p_start = _profiler_ns()
    t_start = time.perf_counter()
    results = []
    for k in range(args.steps):
        results.append(step(k == args.steps - 1, [dominant]))
        print(f"# step {k}: fills {results[-1]['fill_s']} lookup {results[-1]['lookup_s']:.4f}s "
              f"overwrite {results[-1]['overwrite_s']:.4f}s upsert {results[-1]['upsert_s']:.4f}s "
              f"delete {results[-1]['delete_s']:.4f}s",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    p_end = _profiler_ns()
    if p_start is not None and p_end is not None:
        print(f"# profiler window ns: {p_start} {p_end}", file=sys.stderr, flush=True)

    # correctness guard on the timed output: every probe answered as generated,
    # and every stored key's value is the one inserted
    found = fout.cpu().numpy().astype(bool)
    assert np.array_equal(found, present), "lookup answers differ from the generated mix"
    got = vout.cpu().numpy().view(np.uint64)
    assert np.array_equal(got[present], vals[q_src[present]]), "a lookup returned a wrong value"

    # after the timed region: the same steps with no kernel timing at all, to
    # show what the two HIP events around every launch of the dominant class
    # (which `roofline` needs) cost the fills
    plain = [step(False, False) for _ in range(args.steps)]
    plain_rate = len(schemes) * m / sum(float(np.mean([r["fill_s"][s] for r in plain]))
                                        for s in schemes)

    # probes per lookup, counted by the lookup kernel (before the tables are
    # refilled below)
    lt = tables[schemes[-1]].stats()
    probes_per_q = lt["lookup_probes"] / max(1, lt["lookups"])

    # bins viewed per insert at each load of the configuration: the bands just
    # below 0.90 and 0.95 come from the timed fills; for 0.98 each table is
    # filled to 0.95 again (untimed) and taken on to 0.98 in one more call
    by_load = {}
    for lo in (0.90, args.load, 0.98):
        by_load[f"{lo:.2f}"] = {}
    top_rate = {}
    for s in schemes:
        t = tables[s]
        t.timing(enable=False)
        t.clear()
        t.insert(dkeys, dvals, diagnostics=False)
        st_lo = t.stats()
        if m_top > m:
            sec = _timed(lambda: t.insert(dkeys_all[m:], dvals_all[m:], diagnostics=False))
            top_rate[s] = (m_top - m) / sec
        st_hi = t.stats()
        for lo in by_load:
            band = int(round(float(lo) * 200)) - 1
            src = st_lo if float(lo) <= args.load else st_hi
            bi, bvv = src["band_inserts"][band], src["band_views"][band]
            by_load[lo][s] = {"band": float(bvv / bi) if bi else None,
                              "cumulative_to_here": float(
                                  src["band_views"][:band + 1].sum() /
                                  max(1, src["band_inserts"][:band + 1].sum())),
                              "failed": int(src["band_fails"][:band + 1].sum())}

    fill = {s: float(np.mean([r["fill_s"][s] for r in results])) for s in schemes}
    lookup_s = float(np.mean([r["lookup_s"] for r in results]))
    delete_s = float(np.mean([r["delete_s"] for r in results]))
    overwrite_s = float(np.mean([r["overwrite_s"] for r in results]))
    upsert_s = float(np.mean([r["upsert_s"] for r in results]))
    assert all(r["overwrites_found"] for r in results), "an overwrite missed a stored key"
    assert all(r["upserts_as_expected"] for r in results), "an upsert gave an unexpected status"
    ins_rate = len(schemes) * m / sum(fill.values())
    st = results[-1]["stats"]
    band = int(round(args.load * 200)) - 1  # the [load - 0.5%, load) band
    bv95, cum, fails, rounds, retries = {}, {}, {}, {}, {}
    for s in schemes:
        rounds[s] = st[s]["rounds"] / max(1, -(-m // (1 << args.batch_log2)))
        retries[s] = st[s]["retries"] / max(1, m)
        bi, bvv = st[s]["band_inserts"], st[s]["band_views"]
        bv95[s] = float(bvv[band] / max(1, bi[band]))
        cum[s] = st[s]["views"] / max(1, st[s]["inserts_ok"] + st[s]["inserts_failed"])
        fails[s] = st[s]["inserts_failed"]
    # The whole insert path against the HBM roofline, under two byte models.
    # Line model (the primary figure): per insert 17 bytes of key, value and
    # status; V bins viewed, each a whole line L; V_m of them also read the
    # bin's metadata word, counted as a 64-byte line (sorted search and the
    # hybrid read spawn counts, queue-kicking hit counters, ghosts duplicate
    # marks); W = kicks + 1 bins written, each a line and its metadata line.
    # Line-and-word model (the secondary figure): a view is a line and a
    # 4-byte word, a write a 16-byte slot and an 8-byte claim word.
    L = B * 16

    def reads_meta(s):
        return s in ("sorted", "hybrid", "queue")

    ins_bytes, ins_bytes_lw, ins_total, ins_total_lw = {}, {}, 0.0, 0.0
    for s in schemes:
        done = max(1, st[s]["inserts_ok"] + st[s]["inserts_failed"])
        kicks = st[s]["kicks"] / done
        vm = cum[s] if reads_meta(s) else 0.0
        ins_bytes[s] = 17 + cum[s] * L + vm * 64 + (kicks + 1) * (L + 64)
        ins_bytes_lw[s] = 17 + cum[s] * (L + 4) + (kicks + 1) * (16 + 8)
        ins_total += ins_bytes[s] * m
        ins_total_lw += ins_bytes_lw[s] * m
    ins_ach = ins_total / sum(fill.values()) / 1e9
    ins_ach_lw = ins_total_lw / sum(fill.values()) / 1e9
    insert_roof = {"bound": "hbm", "achieved": ins_ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                   "frac": ins_ach / PEAK_HBM_GBS, "bytes_per_insert": ins_bytes,
                   "model": "17 + V*L + V_m*64 + W*(L+64) per insert",
                   "line_and_word_model": {"achieved": ins_ach_lw, "frac": ins_ach_lw / PEAK_HBM_GBS,
                                           "bytes_per_insert": ins_bytes_lw,
                                           "model": "17 + V*(L+4) + W*(16+8) per insert"},
                   "scope": "whole fill (all kernels), algorithmic bytes"}
    # lookup roofline: algorithmic bytes per query = key 8 + value 8 + found 1
    # + probes * 128-byte bin line (probes counted by the kernel itself)
    bytes_per_q = 17 + probes_per_q * B * 16
    achieved = nq * bytes_per_q / lookup_s / 1e9
    lpp = args.lpp or B
    lookup_roof = {"bound": "hbm", "kernel": f"k_lookup<{B},{lpp},2>", "achieved": achieved,
                   "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                   "bytes_per_query": bytes_per_q}
    # the dominant kernel class, timed with HIP events over every timed step
    kt_ms, kt_launch = 0.0, 0
    views_by = {s: 0 for s in schemes}
    for r in results:
        if dominant == "lookup":
            kt_ms += r["lookup_timing"]["ms"]
            kt_launch += r["lookup_timing"]["launches"]
            continue
        for s in schemes:
            tm = r["timing"][s]
            kt_ms += tm[dominant]["ms"]
            kt_launch += tm[dominant]["launches"]
            views_by[s] += tm["evict_views"]
    evict_views = sum(views_by.values())
    if dominant == "lookup":
        ach = nq * args.steps * bytes_per_q / (kt_ms / 1e3) / 1e9
        roofline = dict(lookup_roof, achieved=ach, frac=ach / PEAK_HBM_GBS, traffic=None)
    else:
        # eviction planners: a bin viewed is one bin line (L bytes) and, for the
        # schemes that read it, the bin's metadata word counted as a 64-byte
        # line (the line model, the primary figure); the line-and-word model
        # counts the word as 4 bytes.  A launch's bytes are its plans' views.
        alg = sum(v * (L + (64 if reads_meta(s) else 0)) for s, v in views_by.items())
        alg_lw = evict_views * (L + 4)
        ach = alg / (kt_ms / 1e3) / 1e9 if kt_ms else 0.0
        ach_lw = alg_lw / (kt_ms / 1e3) / 1e9 if kt_ms else 0.0
        traffic = None
        if MEASURED_EVICT_TRAFFIC["sources_sha256"] == _sources_sha256():
            traffic = MEASURED_EVICT_TRAFFIC["bytes_per_launch"]
        roofline = {"bound": "hbm", "kernel": "k_plan_search<8,2> (bfs, sorted) / "
                                              "k_plan_walk<8,2> (queue)",
                    "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": ach / PEAK_HBM_GBS, "traffic": traffic,
                    "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE)",
                    "algorithmic_bytes_per_launch": alg / max(1, kt_launch),
                    "model": "per view: L, plus 64 when the scheme reads the bin's metadata",
                    "line_and_word_model": {"achieved": ach_lw, "frac": ach_lw / PEAK_HBM_GBS,
                                            "algorithmic_bytes_per_launch":
                                                alg_lw / max(1, kt_launch),
                                            "bytes_per_view": L + 4},
                    "views_per_step": evict_views / args.steps,
                    "views_per_step_by_scheme": {s: v / args.steps for s, v in views_by.items()},
                    "launches_per_step": kt_launch / args.steps,
                    "avg_launch_us": kt_ms * 1e3 / max(1, kt_launch)}
    ceilings = measure_ceilings()
    lookup_roof["lines_per_s"] = nq * probes_per_q / lookup_s
    lookup_roof["frac_of_gather_ceiling"] = lookup_roof["lines_per_s"] / \
        ceilings["gather_lines_per_s"]
    # claim atomics of the fills, a lower bound: every committed plan claimed
    # each bin it writes (kicks + 1), and every lost round at least one
    claims = sum((st[s]["inserts_ok"] + st[s]["kicks"]) + st[s]["retries"] for s in schemes)
    claims_per_s = claims / sum(fill.values())
    small = run_small(args)
    out = {
        "metric": "inserts/s & bins viewed/insert at 95% load; lookups/s vs HBM roofline",
        "value": ins_rate,
        "unit": "inserts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic (splitmix64 keys/values, seeded)",
        "config": {"workload": f"2^{args.bins_log2} bins x {B} slots (16-byte slots, "
                               f"{n * B * 16 / 2**30:.0f} GiB), 2 hash functions, "
                               f"fill to {args.load} in sub-batches of 2^{args.batch_log2} "
                               f"with {','.join(schemes)}; 2^{args.lookups_log2} lookups at "
                               f"{args.hit_rate} hits; 2^{args.deletes_log2} overwrites of "
                               f"stored keys, 2^{args.deletes_log2 + 1} upserts (half stored, "
                               f"half absent), then deletes of the stored keys",
                   "bins": n, "slots_per_bin": B, "inserts_per_fill": m,
                   "lookups": nq, "deletes": int(dels.size), "max_search": args.max_search,
                   "spawn_k": args.spawn_k},
        "inserts_per_s_by_scheme": {s: m / fill[s] for s in schemes},
        "bins_viewed_per_insert_at_95": bv95,
        "bins_viewed_per_insert_by_load": by_load,
        "inserts_per_s_95_to_98": top_rate,
        "bins_viewed_per_insert_cumulative": cum,
        "failed_inserts": fails,
        "rounds_per_sub_batch": rounds,
        "lost_rounds_per_insert": retries,
        "inserts_per_s_without_kernel_events": plain_rate,
        "lookups_per_s": nq / lookup_s,
        "deletes_per_s": dels.size / delete_s,
        "overwrites_per_s": dels.size / overwrite_s,
        "upserts_per_s": ups.size / upsert_s,
        "lookup_probes_per_query": probes_per_q,
        "roofline": roofline,
        "lookup_roofline": lookup_roof,
        "insert_roofline": insert_roof,
        "ceilings": ceilings,
        "claim_atomics_per_s_lower_bound": claims_per_s,
        "claim_atomics_frac_of_ceiling": claims_per_s / ceilings["atomic_min_u64_per_s"],
        "small_table": small,
        "kernel_ms_warmup_step": warm_ms,
        "dominant_kernel_class": dominant,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, schemes)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
