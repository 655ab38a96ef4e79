"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no part of the cuckoo-table method: it only draws keys,
values and operation mixes.  Keys and values come from one splitmix64 stream
(Steele, Lea, Flood 2014): key_i = s[2i], value_i = s[2i+1].  Outputs of one
stream are pairwise distinct (distinct states through a bijective mixer), so
keys are distinct without deduplication, and "absent" query keys are simply
later draws of the same stream.  The paper's experiments use uniformly random
hashes and random integer payloads (Sec. 3, Sec. 8.3); uniform 64-bit keys
under a seeded multiply-shift hash stand in for them.
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs ``start .. start+count-1`` of the splitmix64 stream of ``seed``."""
    out = np.empty(count, dtype=np.uint64)
    chunk = 1 << 22
    with np.errstate(over="ignore"):
        for c0 in range(0, count, chunk):
            c1 = min(count, c0 + chunk)
            idx = np.arange(start + c0 + 1, start + c1 + 1, dtype=np.uint64)
            z = np.uint64(seed) + idx * GOLDEN
            z = (z ^ (z >> np.uint64(30))) * _M1
            z = (z ^ (z >> np.uint64(27))) * _M2
            out[c0:c1] = z ^ (z >> np.uint64(31))
    return out


def keys_values(seed: int, count: int, start: int = 0, value_bits: int = 64):
    """``count`` distinct keys with their values, from record index ``start``."""
    s = splitmix64(seed, 2 * start, 2 * count)
    keys = s[0::2].copy()
    vals = s[1::2].copy()
    if value_bits == 32:
        vals &= np.uint64(0xFFFFFFFF)
    if np.any(keys == EMPTY):  # probability 2^-64 per key; refuse rather than alter
        raise ValueError("key stream hit the reserved empty key")
    return keys, vals


def target_count(bins: int, slots_per_bin: int, load: float) -> int:
    """Number of keys that fills ``bins * slots_per_bin`` slots to ``load``."""
    return int(np.floor(load * bins * slots_per_bin))


def lookup_mix(seed: int, stored_keys: np.ndarray, absent_start: int, count: int,
               hit_rate: float, key_seed: int, return_index: bool = False):
    """``count`` query keys: a ``hit_rate`` share drawn uniformly from
    ``stored_keys`` and the rest fresh (never inserted) keys from record index
    ``absent_start`` of the key stream ``key_seed``; shuffled together.
    Returns (queries, expected_present), and with ``return_index`` also each
    query's index into ``stored_keys`` (-1 for an absent key), so a caller can
    check returned values against the values it stored."""
    rng = np.random.default_rng(seed)
    n_hit = int(round(hit_rate * count))
    src = rng.integers(0, stored_keys.size, n_hit)
    hits = stored_keys[src]
    absent, _ = keys_values(key_seed, count - n_hit, start=absent_start)
    q = np.concatenate([hits, absent])
    present = np.concatenate([np.ones(n_hit, bool), np.zeros(count - n_hit, bool)])
    perm = rng.permutation(count)
    if return_index:
        idx = np.concatenate([src, np.full(count - n_hit, -1, np.int64)])
        return q[perm], present[perm], idx[perm]
    return q[perm], present[perm]


def zipf_ranks(seed: int, n_items: int, count: int, s: float = 0.99) -> np.ndarray:
    """``count`` ranks in [0, n_items) with P(rank k) proportional to 1/(k+1)^s."""
    rng = np.random.default_rng(seed)
    w = 1.0 / np.power(np.arange(1, n_items + 1, dtype=np.float64), s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    return np.minimum(np.searchsorted(cdf, rng.random(count)), n_items - 1)


class ZipfTorch:
    """Ranks in [0, n_items) with P(rank k) proportional to 1/(k+1)^s, drawn on
    a torch device from a seeded generator (inverse CDF by binary search)."""

    def __init__(self, n_items: int, s: float = 0.99, device="cuda"):
        import torch
        self.n = int(n_items)
        w = torch.arange(1, self.n + 1, dtype=torch.float64, device=device).pow_(-s)
        self.cdf = torch.cumsum(w, 0)
        self.cdf /= self.cdf[-1].clone()
        self.device = device

    def sample(self, gen, count: int):
        import torch
        u = torch.rand(count, generator=gen, dtype=torch.float64, device=self.device)
        return torch.searchsorted(self.cdf, u).clamp_(max=self.n - 1)


def poisson_arrivals(seed: int, count: int, rate_per_s: float) -> np.ndarray:
    """Open-loop arrival times in seconds (exponential gaps of mean 1/rate)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, count))


def log_uniform_int(seed: int, count: int, lo_exp: float, hi_exp: float) -> np.ndarray:
    """round(2^(lo + (hi-lo) u)) for uniform u."""
    rng = np.random.default_rng(seed)
    return np.round(np.power(2.0, lo_exp + (hi_exp - lo_exp) * rng.random(count))).astype(
        np.int64)


# ---------------------------------------------------------------------------
# device-side generation for large workloads (bit-identical to splitmix64())
# ---------------------------------------------------------------------------
def _i64(c: int) -> int:
    return c - (1 << 64) if c >= (1 << 63) else c


def splitmix64_torch(seed: int, start: int, count: int, device="cuda"):
    """Same outputs as splitmix64(seed, start, count), as an int64 tensor holding
    the uint64 bit patterns, computed on `device` (two's-complement wrap)."""
    import torch
    idx = torch.arange(start + 1, start + count + 1, dtype=torch.int64, device=device)
    z = _i64(seed & ((1 << 64) - 1)) + idx * _i64(int(GOLDEN))
    lo34 = (1 << 34) - 1
    lo37 = (1 << 37) - 1
    lo33 = (1 << 33) - 1
    z = (z ^ ((z >> 30) & lo34)) * _i64(int(_M1))
    z = (z ^ ((z >> 27) & lo37)) * _i64(int(_M2))
    return z ^ ((z >> 31) & lo33)


def keys_values_torch(seed: int, count: int, start: int = 0, device="cuda", value_bits=64):
    """keys_values() on the device: (keys, values) int64 tensors."""
    s = splitmix64_torch(seed, 2 * start, 2 * count, device)
    keys = s[0::2].contiguous()
    vals = s[1::2].contiguous()
    if value_bits == 32:
        vals = vals & 0xFFFFFFFF
    if bool((keys == -1).any()):
        raise ValueError("key stream hit the reserved empty key")
    return keys, vals


# ---------------------------------------------------------------------------
# many tables: bin counts and request streams
# ---------------------------------------------------------------------------
def group_tables(seed: int, count: int, lo_exp: float, hi_exp: float, min_bins: int = 4):
    """Bin counts round(2^(lo + (hi-lo) u)), u uniform."""
    return np.maximum(log_uniform_int(seed, count, lo_exp, hi_exp), min_bins).astype(np.uint64)


class RequestStream:
    """Seeded requests to many tables prefilled from one key stream.

    Table t is prefilled with records [pre_start[t], pre_start[t] + pre[t]) of
    the key stream `key_seed`: the first half is the lookup target (never
    deleted), the second half is consumed in order by deletes.  Inserts take
    fresh records from a per-table range beyond every prefill; lookup misses are
    fresh records nobody inserts.  Requests: a table (uniform), a type (lookup,
    insert, delete with the given shares), a size log-uniform on [1, max_ops].

    `take(count)` draws requests as arrays; `records_torch` expands them into
    the record index of every op, on any torch device.  A lookup op with
    global lookup index g draws u = splitmix64 output g of `lookup_seed`: it
    hits (record pre_start[t] + floor(lo32(u) * half / 2^32)) when
    hi53(u) / 2^53 < hit_rate, else it misses (record miss_start + g).
    """

    def __init__(self, seed, bins, slots_per_bin, prefill_load, key_seed, shares=(0.7, 0.2, 0.1),
                 max_ops=65536, hit_rate=0.9):
        self.rng = np.random.default_rng(seed)
        self.lookup_seed = int(self.rng.integers(0, 1 << 62))
        self.bins = np.asarray(bins, dtype=np.int64)
        self.nt = self.bins.size
        self.pre = np.floor(prefill_load * self.bins * slots_per_bin).astype(np.int64)
        self.pre_start = np.concatenate([[0], np.cumsum(self.pre)[:-1]]).astype(np.int64)
        self.half = np.maximum(1, self.pre // 2)
        total_pre = int(self.pre.sum())
        cap = (self.bins * slots_per_bin - self.pre).astype(np.int64)
        self.fresh_start = total_pre + np.concatenate([[0], np.cumsum(cap)[:-1]]).astype(np.int64)
        self.fresh_cap = cap
        self.miss_start = total_pre + int(cap.sum())
        self.key_seed = key_seed
        self.shares = np.asarray(shares, dtype=np.float64) / np.sum(shares)
        self.max_ops = max_ops
        self.hit_rate = hit_rate
        self.fresh_used = np.zeros(self.nt, np.int64)
        self.del_used = np.zeros(self.nt, np.int64)
        self.lookup_used = 0

    def prefill_records(self):
        """(start, count) of the prefill records of every table, in table order."""
        return self.pre_start, self.pre

    def take(self, count):
        """`count` requests: dict of int64 arrays kind (0 lookup, 1 insert,
        2 delete), table, n (ops; inserts and deletes are clipped to what the
        table has left) and base (the first op's index within its kind's
        per-table range, or the first global lookup index)."""
        rng = self.rng
        table = rng.integers(0, self.nt, count).astype(np.int64)
        kind = rng.choice(3, size=count, p=self.shares).astype(np.int64)
        n = np.round(np.exp(rng.uniform(0.0, np.log(self.max_ops), count))).astype(np.int64)
        n = np.clip(n, 1, self.max_ops)
        base = np.zeros(count, np.int64)
        fresh_left = self.fresh_cap // 2 - self.fresh_used
        del_left = self.pre - self.pre // 2 - self.del_used
        for i in range(count):  # per-table budgets make clipping sequential
            t, k = table[i], kind[i]
            if k == 1:
                m = min(n[i], max(0, fresh_left[t]))
                base[i] = self.fresh_used[t]
                self.fresh_used[t] += m
                fresh_left[t] -= m
                n[i] = m
            elif k == 2:
                m = min(n[i], max(0, del_left[t]))
                base[i] = self.del_used[t]
                self.del_used[t] += m
                del_left[t] -= m
                n[i] = m
            else:
                base[i] = self.lookup_used
                self.lookup_used += n[i]
        return {"kind": kind, "table": table, "n": n, "base": base}

    def records_torch(self, req, r0=0, r1=None, device="cuda"):
        """Record index of every op of requests [r0, r1) of `req` (from take),
        concatenated in request order, as an int64 tensor on `device`."""
        import torch
        r1 = req["n"].size if r1 is None else r1
        n = torch.from_numpy(req["n"][r0:r1]).to(device)
        total = int(req["n"][r0:r1].sum())
        seg = torch.repeat_interleave(torch.arange(r1 - r0, device=device), n, output_size=total)
        first = torch.cumsum(n, 0) - n
        j = torch.arange(total, device=device) - first[seg]
        t = torch.from_numpy(req["table"][r0:r1]).to(device)[seg]
        k = torch.from_numpy(req["kind"][r0:r1]).to(device)[seg]
        b = torch.from_numpy(req["base"][r0:r1]).to(device)[seg] + j
        pre_start = torch.from_numpy(self.pre_start).to(device)
        half = torch.from_numpy(self.half).to(device)
        fresh_start = torch.from_numpy(self.fresh_start).to(device)
        ins = fresh_start[t] + b
        dele = pre_start[t] + (torch.from_numpy(self.pre).to(device) // 2)[t] + b
        u = _mix_torch(_i64(self.lookup_seed) + (b + 1) * _i64(int(GOLDEN)))
        hit = ((u >> 11) & ((1 << 53) - 1)).to(torch.float64) < self.hit_rate * float(1 << 53)
        pos = ((u & 0xFFFFFFFF) * half[t]) >> 32
        look = torch.where(hit, pre_start[t] + pos, self.miss_start + b)
        return torch.where(k == 1, ins, torch.where(k == 2, dele, look))

    def payload(self, req, device="cuda", chunk_ops=1 << 25, pin=True):
        """Keys and values of every op of `req` in request order, as int64
        tensors in host memory (pinned when `pin`), generated on `device` chunk
        by chunk, and per op the expected answer (uint8): 1 for inserts,
        deletes and lookups that hit, 0 for lookup misses."""
        import torch
        off = np.concatenate([[0], np.cumsum(req["n"])]).astype(np.int64)
        total = int(off[-1])
        keys = torch.empty(max(total, 1), dtype=torch.int64, pin_memory=pin)
        vals = torch.empty(max(total, 1), dtype=torch.int64, pin_memory=pin)
        expect = torch.empty(max(total, 1), dtype=torch.uint8, pin_memory=pin)
        r0, R = 0, off.size - 1
        while r0 < R:
            r1 = int(np.searchsorted(off, off[r0] + chunk_ops, side="right")) - 1
            r1 = min(max(r1, r0 + 1), R)
            o0, o1 = int(off[r0]), int(off[r1])
            if o1 > o0:
                rec = self.records_torch(req, r0, r1, device)
                k, v = keys_at_torch(self.key_seed, rec)
                keys[o0:o1].copy_(k)
                vals[o0:o1].copy_(v)
                expect[o0:o1].copy_((rec < self.miss_start).to(torch.uint8))
            r0 = r1
        return keys, vals, expect

    def prefill_payload(self, device="cuda", chunk_ops=1 << 25, pin=True):
        """Keys and values of every prefill record, table after table (the
        records are 0 .. sum(pre) - 1), as int64 tensors in host memory."""
        import torch
        total = int(self.pre.sum())
        keys = torch.empty(max(total, 1), dtype=torch.int64, pin_memory=pin)
        vals = torch.empty(max(total, 1), dtype=torch.int64, pin_memory=pin)
        for c0 in range(0, total, chunk_ops):
            c1 = min(total, c0 + chunk_ops)
            k, v = keys_at_torch(self.key_seed,
                                 torch.arange(c0, c1, dtype=torch.int64, device=device))
            keys[c0:c1].copy_(k)
            vals[c0:c1].copy_(v)
        return keys, vals

    def next(self):
        """One request: (kind, table, record indices into the key stream)."""
        r = self.take(1)
        rec = self.records_torch(r, device="cpu").numpy()
        return int(r["kind"][0]), int(r["table"][0]), rec


def _mix_torch(z):
    lo34, lo37, lo33 = (1 << 34) - 1, (1 << 37) - 1, (1 << 33) - 1
    z = (z ^ ((z >> 30) & lo34)) * _i64(int(_M1))
    z = (z ^ ((z >> 27) & lo37)) * _i64(int(_M2))
    return z ^ ((z >> 31) & lo33)


def keys_at_torch(seed: int, records, value_bits=64):
    """Key and value of arbitrary record indices (int64 tensor) of the stream
    keys_values(seed, ...): record r is splitmix64 outputs 2r and 2r+1."""
    s0 = _i64(seed & ((1 << 64) - 1))
    g = _i64(int(GOLDEN))
    keys = _mix_torch(s0 + (2 * records + 1) * g)
    vals = _mix_torch(s0 + (2 * records + 2) * g)
    if value_bits == 32:
        vals = vals & 0xFFFFFFFF
    return keys, vals
