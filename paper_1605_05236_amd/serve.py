"""Continuous-batching request server over device-resident cuckoo tables.

Requests (lookup, insert or delete of a key batch in one table) arrive over
time, open loop.  Their payloads sit back to back in host memory in arrival
order (a receive buffer), so every arrival range is one contiguous copy.

* Upload: at the top of every loop iteration the newly arrived range of keys
  and values is copied to the device on the marshalling stream.
* Overlap: batch b + 1 is selected and marshalled (on the marshalling
  stream, by the calling thread) while batch b's table calls run on the
  compute stream (driven by a worker thread); up to `depth` batches are in
  flight, each with its own gather buffers.
* Batching: each batch takes, per table, the longest run of consecutive
  requests of one kind at the head of that table's queue (coalescing them).
  A table thus contributes one kind per batch, so running a batch's lookups,
  deletes and inserts as three launch sequences keeps every table's FIFO order.
  A batch holds at most `max_batch_ops` ops (at least one request); cutting in
  arrival order keeps each table's taken requests a prefix of its queue.
* Admission by HBM footprint: tables live in slabs (one table group per slab).
  A slab is allocated when a request first needs it and its footprint fits the
  budget; requests for a slab that does not fit are reported unserved (until
  memory is released with `release_slab`, between runs).
* Marshalling: the batch's ops are gathered from the device copy of the
  receive buffer by segment (offset, length, table) lists.  Answers are
  written in batch order to the next range of an answer buffer, and one copy
  per batch returns exactly that range to host memory; each request records
  where its answers start.
* Latency is the host's completion time minus the scheduled arrival time.

All table work runs in libck's kernels through the C ABI (table groups); the
server's own device work is index arithmetic, gathers and scatters.
"""
from __future__ import annotations

import time

import numpy as np

LOOKUP, INSERT, DELETE = 0, 1, 2


def _head_runs(kind, table, pending):
    """Mask over `pending` (arrival order): requests in their table's head run
    (no earlier pending request of the table has another kind)."""
    t, k = table[pending], kind[pending]
    order = np.argsort(t, kind="stable")
    ts, ks = t[order], k[order]
    new_grp = np.ones(ts.size, bool)
    new_grp[1:] = ts[1:] != ts[:-1]
    chg = new_grp.copy()
    chg[1:] |= ks[1:] != ks[:-1]
    run = np.cumsum(chg)
    first = np.maximum.accumulate(np.where(new_grp, run, 0))
    head = np.zeros(pending.size, bool)
    head[order[run == first]] = True
    return head


def take_batch(kind, table, n, pending, max_ops):
    """Split `pending` (request indices in arrival order) into one batch and
    the rest: per table, the run of same-kind requests at the head of its
    queue; then the arrival-order prefix of those whose ops fit `max_ops`
    (always at least one request).  Returns (taken, rest), both in arrival
    order.  Whether a request is in its table's head run depends only on the
    requests before it, so only a prefix of `pending` is scanned: it grows
    until its head-run requests hold more than `max_ops` ops."""
    w = min(pending.size, 256)
    while True:
        win = pending[:w]
        head = _head_runs(kind, table, win)
        if w == pending.size or int(n[win[head]].sum()) > max_ops:
            break
        w = min(pending.size, 4 * w)
    cand = np.nonzero(head)[0]
    keep = np.cumsum(n[win[cand]]) <= max_ops
    keep[0] = True
    pick = cand[keep]
    mask = np.ones(w, bool)
    mask[pick] = False
    return win[pick], np.concatenate([win[mask], pending[w:]])


class RequestSet:
    """Requests in arrival order.  `kind`, `table`, `n` are per-request arrays,
    `arrival` seconds from the start (non-decreasing).  `keys` and `vals` are
    int64 tensors (uint64 bit patterns; pinned host memory for asynchronous
    uploads) holding request i's ops at [off[i], off[i] + n[i]); values are read
    for inserts only."""

    def __init__(self, kind, table, n, arrival, keys, vals):
        self.kind = np.asarray(kind, np.int64)
        self.table = np.asarray(table, np.int64)
        self.n = np.asarray(n, np.int64)
        self.arrival = np.asarray(arrival, np.float64)
        if not (self.kind.size == self.table.size == self.n.size == self.arrival.size):
            raise ValueError("per-request arrays differ in length")
        if self.arrival.size and np.any(np.diff(self.arrival) < 0):
            raise ValueError("arrivals must be non-decreasing")
        self.off = np.concatenate([[0], np.cumsum(self.n)]).astype(np.int64)
        self.keys, self.vals = keys, vals
        if keys.numel() < self.off[-1] or vals.numel() < self.off[-1]:
            raise ValueError("payload buffers are shorter than the requests")

    def __len__(self):
        return self.kind.size

    def slice(self, i, j, arrival=None):
        """Requests [i, j) as their own set (payload views, no copy)."""
        o0, o1 = int(self.off[i]), int(self.off[j])
        arr = self.arrival[i:j] - (self.arrival[i] if j > i else 0.0) if arrival is None \
            else np.asarray(arrival, np.float64)
        return RequestSet(self.kind[i:j], self.table[i:j], self.n[i:j], arr,
                          self.keys[o0:max(o1, o0 + 1)], self.vals[o0:max(o1, o0 + 1)])

    @classmethod
    def from_lists(cls, requests, arrivals=None, pin=True):
        """From (kind, table, keys, vals or None) tuples with numpy uint64 keys."""
        import torch
        kind = [r[0] for r in requests]
        table = [r[1] for r in requests]
        n = [np.asarray(r[2]).size for r in requests]
        total = int(np.sum(n)) if requests else 0
        keys = torch.empty(max(total, 1), dtype=torch.int64, pin_memory=pin)
        vals = torch.zeros(max(total, 1), dtype=torch.int64, pin_memory=pin)
        kn, vn = keys.numpy(), vals.numpy()
        o = 0
        for r, m in zip(requests, n):
            kn[o:o + m] = np.asarray(r[2], np.uint64).view(np.int64)
            if r[3] is not None:
                vn[o:o + m] = np.asarray(r[3], np.uint64).view(np.int64)
            o += m
        arr = np.zeros(len(requests)) if arrivals is None else np.asarray(arrivals, np.float64)
        return cls(kind, table, n, arr, keys, vals)


class Results:
    """Answers of one run.  `done[i]`: completion time of request i in seconds
    from the start (NaN when unserved).  Request i's answers are at
    [aoff[i], aoff[i] + n[i]) of `flag` (lookup: found; insert: status;
    delete: found) and `value` (lookups that hit)."""

    def __init__(self, rs, done, aoff, flag, value, stats):
        self.rs, self.done, self.aoff = rs, done, aoff
        self.flag, self.value = flag, value
        self.stats = stats

    @property
    def unserved(self):
        return np.isnan(self.done)

    def flags_in_request_order(self):
        """Every op's flag, ops in request order (unserved requests: 0)."""
        out = np.zeros(int(self.rs.off[-1]), np.uint8)
        for i in np.nonzero(~self.unserved)[0]:
            out[self.rs.off[i]:self.rs.off[i + 1]] = self.flag[self.aoff[i]:self.aoff[i] + self.rs.n[i]]
        return out

    def result(self, i):
        o0 = self.aoff[i]
        o1 = o0 + self.rs.n[i]
        if self.rs.kind[i] == LOOKUP:
            return self.value[o0:o1].view(np.uint64), self.flag[o0:o1]
        return self.flag[o0:o1]

    def latency(self):
        return self.done - self.rs.arrival


class Server:
    def __init__(self, bins, slots_per_bin=4, d=2, scheme="queue", slab_tables=512,
                 budget_bytes=None, max_batch_ops=1 << 22, lanes_per_probe=0, **table_kw):
        from .table import CuckooGroup, load_library
        import ctypes
        import torch
        self._CuckooGroup = CuckooGroup
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.bins = np.asarray(bins, dtype=np.uint64)
        self.B, self.d, self.scheme = slots_per_bin, d, scheme
        self.slab_tables = slab_tables
        self.max_batch_ops = max_batch_ops
        self.lpp = lanes_per_probe
        self.table_kw = dict(table_kw)
        self.table_kw.setdefault("batch_ops", max(1 << 16, max_batch_ops))
        nslabs = (self.bins.size + slab_tables - 1) // slab_tables
        self.slabs = [None] * nslabs
        self.slab_bytes = []
        L = load_library()
        for s in range(nslabs):
            b = np.ascontiguousarray(self.bins[s * slab_tables:(s + 1) * slab_tables])
            out = ctypes.c_size_t()
            rc = L.ck_group_storage_bytes(b.size, b.ctypes.data_as(ctypes.c_void_p),
                                          slots_per_bin, d, ctypes.byref(out))
            if rc != 0:
                raise ValueError("bad table geometry")
            self.slab_bytes.append(int(out.value))
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = int(free * 0.8)
        self.budget = budget_bytes
        self.used = 0
        self.stats = {"batches": 0, "ops": 0, "admitted_slabs": 0, "deferred": 0}

    # ---- admission ---------------------------------------------------------
    def slab_of(self, table):
        return table // self.slab_tables

    def _admit_slab(self, s) -> bool:
        if self.slabs[s] is not None:
            return True
        if self.used + self.slab_bytes[s] > self.budget:
            return False
        b = self.bins[s * self.slab_tables:(s + 1) * self.slab_tables]
        self.slabs[s] = self._CuckooGroup(b, self.B, self.d, self.scheme, **self.table_kw)
        self.used += self.slab_bytes[s]
        self.stats["admitted_slabs"] += 1
        return True

    def release_slab(self, s):
        """Free a slab's memory (its tables' contents are dropped)."""
        if self.slabs[s] is not None:
            self.slabs[s].close()
            self.slabs[s] = None
            self.used -= self.slab_bytes[s]

    def table(self, t):
        """The group holding table t and t's index in it (admitting the slab)."""
        s = self.slab_of(t)
        if not self._admit_slab(s):
            raise MemoryError("slab does not fit the HBM budget")
        return self.slabs[s], t - s * self.slab_tables

    # ---- batching ----------------------------------------------------------
    def _take(self, rs, pending):
        return take_batch(rs.kind, rs.table, rs.n, pending, self.max_batch_ops)

    def _plan(self, rs, taken, cursor, aoff):
        """A batch's launch groups: (kind, slab, requests, answer offset, ops) per
        kind (lookups, deletes, inserts, in that order) and slab; every
        request's answers get the next range of the answer buffers."""
        kinds = rs.kind[taken]
        slabs = self.slab_of(rs.table[taken])
        groups = []
        for kind in (LOOKUP, DELETE, INSERT):
            for s in np.unique(slabs[kinds == kind]):
                sel = taken[(kinds == kind) & (slabs == s)]
                ln = rs.n[sel]
                aoff[sel] = cursor + np.cumsum(ln) - ln
                tot = int(ln.sum())
                if tot:
                    groups.append((kind, int(s), sel, cursor, tot))
                    cursor += tot
        return groups, cursor

    def _marshal(self, rs, groups, slot, d_keys, d_vals):
        """Gather a batch's keys, values and table ids from the device copy of
        the receive buffer into the slot's buffers (segment lists go up in one
        pinned copy).  Enqueued on the current stream."""
        import torch
        m = sum(g[2].size for g in groups)
        if slot["staging"] is None or slot["staging"].numel() < 3 * m:
            slot["staging"] = torch.empty(max(3 * m, 1 << 14), dtype=torch.int64,
                                          pin_memory=True)
        tot_all = sum(g[4] for g in groups)
        if slot["keys"] is None or slot["keys"].numel() < tot_all:
            size = max(tot_all, self.max_batch_ops, 1 << 16)
            slot["keys"] = torch.empty(size, dtype=torch.int64, device=self.device)
            slot["vals"] = torch.empty(size, dtype=torch.int64, device=self.device)
            slot["tids"] = torch.empty(size, dtype=torch.int32, device=self.device)
        h = slot["staging"].numpy()
        o = 0
        for kind, s, sel, c0, tot in groups:
            k = sel.size
            h[o:o + k] = rs.n[sel]
            h[o + k:o + 2 * k] = rs.off[sel]
            h[o + 2 * k:o + 3 * k] = rs.table[sel] - s * self.slab_tables
            o += 3 * k
        dh = slot["staging"][:3 * m].to(self.device, non_blocking=True)
        o = b = 0
        for kind, s, sel, c0, tot in groups:
            k = sel.size
            dln, dsrc, dtab = dh[o:o + k], dh[o + k:o + 2 * k], dh[o + 2 * k:o + 3 * k]
            o += 3 * k
            seg = torch.repeat_interleave(torch.arange(k, device=self.device), dln,
                                          output_size=tot)
            first = torch.cumsum(dln, 0) - dln
            pos = torch.arange(tot, device=self.device) - first[seg] + dsrc[seg]
            torch.index_select(d_keys, 0, pos, out=slot["keys"][b:b + tot])
            if kind == INSERT:
                torch.index_select(d_vals, 0, pos, out=slot["vals"][b:b + tot])
            slot["tids"][b:b + tot].copy_(dtab[seg])
            b += tot

    def _execute(self, groups, slot, d_flag, d_val, stream):
        """The table calls of one marshalled batch, on `stream` (lookups first,
        then deletes, then inserts: each table's FIFO order)."""
        b = 0
        for kind, s, sel, c0, tot in groups:
            g = self.slabs[s]
            keys, tids = slot["keys"][b:b + tot], slot["tids"][b:b + tot]
            c1 = c0 + tot
            if kind == LOOKUP:
                g.lookup(tids, keys, lanes_per_probe=self.lpp, out=d_val[c0:c1],
                         found=d_flag[c0:c1], stream=stream)
            elif kind == DELETE:
                d_flag[c0:c1].copy_(g.delete(tids, keys, stream=stream))
            else:
                d_flag[c0:c1].copy_(g.insert(tids, keys, slot["vals"][b:b + tot],
                                             diagnostics=False, stream=stream)["status"])
            b += tot

    # ---- the request loop --------------------------------------------------
    def run(self, rs: RequestSet, depth: int = 2) -> Results:
        """Serve the request set, each request becoming visible at its arrival
        time (seconds from the start of the call).

        Two threads and two streams keep up to `depth` batches in flight.  The
        calling thread uploads arrivals, selects batch b + 1 and marshals it on
        the marshalling stream (gathers into one of `depth` buffer slots) while
        batch b's table calls run on the compute stream, driven by a worker
        thread (the table calls return once their rounds are done).  The
        worker runs batches in selection order, so every table's requests keep
        their FIFO order; a batch's answers go back to host memory with one copy
        on the compute stream, and its requests complete when that copy has."""
        import queue
        import threading
        import torch
        R = len(rs)
        total = int(rs.off[-1])
        cap = max(total, 1)
        dev = self.device
        d_keys = torch.empty(cap, dtype=torch.int64, device=dev)
        d_vals = torch.empty(cap, dtype=torch.int64, device=dev)
        d_flag = torch.zeros(cap, dtype=torch.uint8, device=dev)
        d_val = torch.zeros(cap, dtype=torch.int64, device=dev)
        h_flag = torch.zeros(cap, dtype=torch.uint8, pin_memory=True)
        h_val = torch.zeros(cap, dtype=torch.int64, pin_memory=True)
        torch.cuda.current_stream(dev).synchronize()  # the buffers exist before other streams use them
        done = np.full(R, np.nan)
        aoff = np.zeros(R, np.int64)
        comp = torch.cuda.Stream(dev)   # table calls and answer copies (worker)
        prep = torch.cuda.Stream(dev)   # uploads and marshalling (calling thread)
        free = queue.Queue()
        # each slot's buffers exist before the clock starts (a warm server)
        size = max(self.max_batch_ops, 1 << 16)
        for _ in range(max(1, depth)):
            free.put({"staging": torch.empty(3 << 16, dtype=torch.int64, pin_memory=True),
                      "keys": torch.empty(size, dtype=torch.int64, device=dev),
                      "vals": torch.empty(size, dtype=torch.int64, device=dev),
                      "tids": torch.empty(size, dtype=torch.int32, device=dev)})
        torch.cuda.current_stream(dev).synchronize()
        work = queue.Queue()
        failure = []
        busy = [0.0]
        ready_evt = threading.Event()
        start = 0.0

        def worker():
            try:
                torch.cuda.set_device(dev)
                with torch.cuda.stream(comp):
                    ready_evt.set()
                    while True:
                        item = work.get()
                        if item is None:
                            return
                        slot, groups, taken, ready, c0, c1 = item
                        t0 = time.perf_counter()
                        comp.wait_event(ready)
                        self._execute(groups, slot, d_flag, d_val, comp)
                        if c1 > c0:
                            h_flag[c0:c1].copy_(d_flag[c0:c1], non_blocking=True)
                            h_val[c0:c1].copy_(d_val[c0:c1], non_blocking=True)
                        fin = torch.cuda.Event()
                        fin.record(comp)
                        fin.synchronize()
                        done[taken] = time.perf_counter() - start
                        busy[0] += time.perf_counter() - t0
                        free.put(slot)
            except BaseException as e:  # surfaced by the calling thread
                failure.append(e)
                ready_evt.set()
                free.put(None)

        # the two threads hand the interpreter lock back and forth at every
        # call; the default 5 ms switch interval would make the calling thread
        # wait for the worker's Python steps (and the other way round)
        import sys
        old_switch = sys.getswitchinterval()
        sys.setswitchinterval(5e-5)
        th = threading.Thread(target=worker, daemon=True)
        th.start()
        ready_evt.wait()
        start = time.perf_counter()
        up = 0  # requests uploaded
        pending = np.empty(0, np.int64)
        admitted = np.zeros(len(self.slabs), bool)
        batches = ops = cursor = 0
        host_s = wait_s = 0.0
        try:
            while not failure:
                now = time.perf_counter() - start
                a = int(np.searchsorted(rs.arrival, now, side="right"))
                if a > up:
                    new = np.arange(up, a, dtype=np.int64)
                    sl = self.slab_of(rs.table[new])
                    fresh = False
                    for s in np.unique(sl):
                        if self.slabs[s] is None:
                            admitted[s] = self._admit_slab(int(s))
                            fresh |= bool(admitted[s])
                        else:
                            admitted[s] = True
                    if fresh:  # a new slab's initialisation is done before any stream uses it
                        torch.cuda.current_stream(dev).synchronize()
                    o0, o1 = int(rs.off[up]), int(rs.off[a])
                    if o1 > o0:
                        with torch.cuda.stream(prep):
                            d_keys[o0:o1].copy_(rs.keys[o0:o1], non_blocking=True)
                            d_vals[o0:o1].copy_(rs.vals[o0:o1], non_blocking=True)
                    up = a
                    ok = admitted[sl]
                    self.stats["deferred"] += int((~ok).sum())
                    pending = np.concatenate([pending, new[ok]])
                if pending.size == 0:
                    if up == R:
                        break
                    time.sleep(min(max(rs.arrival[up] - now, 0.0), 0.0005))
                    continue
                t0 = time.perf_counter()
                slot = free.get()  # at most `depth` batches in flight
                if slot is None:
                    break
                t1 = time.perf_counter()
                taken, pending = self._take(rs, pending)
                c0 = cursor
                groups, cursor = self._plan(rs, taken, cursor, aoff)
                with torch.cuda.stream(prep):
                    self._marshal(rs, groups, slot, d_keys, d_vals)
                    ready = torch.cuda.Event()
                    ready.record(prep)
                work.put((slot, groups, taken, ready, c0, cursor))
                t2 = time.perf_counter()
                wait_s += t1 - t0
                host_s += t2 - t1
                batches += 1
                ops += int(rs.n[taken].sum())
        finally:
            work.put(None)
            th.join()
            sys.setswitchinterval(old_switch)
            prep.synchronize()  # uploads of never-served requests end here
        if failure:
            raise failure[0]
        self.stats["batches"] += batches
        self.stats["ops"] += ops
        return Results(rs, done, aoff, h_flag.numpy()[:total], h_val.numpy()[:total],
                       {"batches": batches, "ops": ops, "host_issue_s": host_s,
                        "host_slot_wait_s": wait_s, "device_calls_s": busy[0]})

    def close(self):
        for s in range(len(self.slabs)):
            self.release_slab(s)


def latency_summary(res: Results) -> dict:
    served = ~res.unserved
    lat = res.latency()[served]
    ops = int(res.rs.n[served].sum())
    span = float(np.max(res.done[served]) - np.min(res.rs.arrival)) if lat.size else 0.0
    pct = (lambda q: float(np.percentile(lat, q) * 1e3)) if lat.size else (lambda q: None)
    return {"p50_ms": pct(50), "p99_ms": pct(99), "max_ms": pct(100),
            "mean_ms": float(lat.mean() * 1e3) if lat.size else None,
            "served": int(lat.size), "unserved": int((~served).sum()), "ops": ops,
            "span_s": span, "ops_per_s": ops / span if span > 0 else None}
