"""Autotuner for libck's performance knobs.

Only knobs that leave every result unchanged are tuned:
  * lanes per probe of the lookup kernel (1 lane loads a whole bin, or one
    lane per slot with a ballot),
  * workgroups per compute unit of the kick-out planners (their LDS footprint
    sets the ceiling).
The sub-batch size changes the round schedule and therefore the table layout,
so it is tuned only on request (``tune_batch=True``) and never in parity runs;
the chain and search caps are part of the method and are never tuned.

Each candidate is timed with HIP events on a sample table of the target
geometry (at most 2^22 bins, results being size-independent per Sec. 3 of the
paper), filled to the target load with seeded keys.  Choices are cached as
JSON keyed by (bins, slots per bin, d, scheme, ghost, load, arch).
"""
from __future__ import annotations

import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tune_cache.json")


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name)


def _key(bins, B, d, scheme, ghost, load, arch) -> str:
    return f"{int(bins)}|{B}|{d}|{scheme}|{int(bool(ghost))}|{load:.3f}|{arch}"


def _load_cache() -> dict:
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            return json.load(f)
    return {}


def _save_cache(c: dict):
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def _elapsed(fn) -> float:
    import torch
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3


def tune(bins, slots_per_bin=4, d=2, scheme="queue", ghost=False, load=0.95,
         sample_bins_log2=22, wgs_choices=(4, 8, 16, 32), batch_choices=(1 << 18, 1 << 20),
         tune_batch=False, max_chain=500, max_search=500, force=False, verbose=False) -> dict:
    """Pick the fastest knobs for this geometry; cached unless `force`."""
    from . import inputs
    from .table import CuckooTable
    arch = _arch()
    key = _key(bins, slots_per_bin, d, scheme, ghost, load, arch)
    cache = _load_cache()
    if key in cache and not force:
        return cache[key]
    n = int(min(int(bins), 1 << sample_bins_log2))
    m = inputs.target_count(n, slots_per_bin, load)
    keys, vals = inputs.keys_values_torch(77, m, value_bits=32 if slots_per_bin == 1 else 64)
    nq = min(1 << 22, 4 * m)
    q = keys[np.random.default_rng(3).integers(0, m, nq)]
    results = {"fill": {}, "lookup": {}}
    best = None
    batches = batch_choices if tune_batch else (1 << 20,)
    for b in batches:
        for w in wgs_choices:
            t = CuckooTable(n, slots_per_bin, d, scheme, ghost=ghost, max_chain=max_chain,
                            max_search=max_search, batch_ops=b, evict_wgs_per_cu=w,
                            hash_seed=7, rng_seed=8)
            t.insert(keys[: m // 4], vals[: m // 4], diagnostics=False)  # warm the code paths
            t.clear()
            sec = _elapsed(lambda: t.insert(keys, vals, diagnostics=False))
            results["fill"][f"{b}:{w}"] = m / sec
            if verbose:
                print(f"# tune fill batch={b} wgs/cu={w}: {m / sec / 1e6:.1f} M inserts/s",
                      flush=True)
            if best is None or m / sec > best[0]:
                best = (m / sec, b, w, t)
            else:
                t.close()
    t = best[3]
    lpp_best = None
    for lpp in sorted({1, slots_per_bin}):
        t.lookup(q, lanes_per_probe=lpp)
        sec = _elapsed(lambda: t.lookup(q, lanes_per_probe=lpp))
        results["lookup"][str(lpp)] = nq / sec
        if verbose:
            print(f"# tune lookup lanes/probe={lpp}: {nq / sec / 1e9:.2f} G lookups/s", flush=True)
        if lpp_best is None or nq / sec > lpp_best[0]:
            lpp_best = (nq / sec, lpp)
    t.close()
    choice = {"evict_wgs_per_cu": best[2], "lanes_per_probe": lpp_best[1],
              "batch_ops": best[1] if tune_batch else None, "sample_bins": n,
              "measured": results}
    cache[key] = choice
    _save_cache(cache)
    return choice


def tune_group(bins, slots_per_bin=4, d=2, scheme="queue", ghost=False, load=0.5, **kw) -> dict:
    """Knobs for a group of tables: tuned on a sample table of the group's mean
    table size (the planners' per-op work does not depend on which table)."""
    mean_bins = int(np.mean(np.asarray(bins, dtype=np.float64)))
    return tune(max(mean_bins, 1024), slots_per_bin, d, scheme, ghost, load, **kw)
