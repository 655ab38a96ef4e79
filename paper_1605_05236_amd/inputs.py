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
               hit_rate: float, key_seed: int):
    """``count`` query keys: a ``hit_rate`` share drawn uniformly from
    ``stored_keys`` and the rest fresh (never inserted) keys from record index
    ``absent_start`` of the key stream ``key_seed``; shuffled together.
    Returns (queries, expected_present)."""
    rng = np.random.default_rng(seed)
    n_hit = int(round(hit_rate * count))
    hits = stored_keys[rng.integers(0, stored_keys.size, n_hit)]
    absent, _ = keys_values(key_seed, count - n_hit, start=absent_start)
    q = np.concatenate([hits, absent])
    present = np.concatenate([np.ones(n_hit, bool), np.zeros(count - n_hit, bool)])
    perm = rng.permutation(count)
    return q[perm], present[perm]


def zipf_ranks(seed: int, n_items: int, count: int, s: float = 0.99) -> np.ndarray:
    """``count`` ranks in [0, n_items) with P(rank k) proportional to 1/(k+1)^s."""
    rng = np.random.default_rng(seed)
    w = 1.0 / np.power(np.arange(1, n_items + 1, dtype=np.float64), s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    return np.minimum(np.searchsorted(cdf, rng.random(count)), n_items - 1)


def poisson_arrivals(seed: int, count: int, rate_per_s: float) -> np.ndarray:
    """Open-loop arrival times in seconds (exponential gaps of mean 1/rate)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, count))


def log_uniform_int(seed: int, count: int, lo_exp: float, hi_exp: float) -> np.ndarray:
    """round(2^(lo + (hi-lo) u)) for uniform u."""
    rng = np.random.default_rng(seed)
    return np.round(np.power(2.0, lo_exp + (hi_exp - lo_exp) * rng.random(count))).astype(
        np.int64)
