"""Shared helpers of the GPU tests: run the same seeded op stream through the
HIP library (via its C ABI binding) and through the oracle, and compare."""
from __future__ import annotations

import numpy as np

import oracle
from paper_1605_05236_amd import inputs


def gpu_table(n, B, d, scheme, seed=1, **kw):
    from paper_1605_05236_amd.table import CuckooTable
    return CuckooTable(n, B, d, scheme, hash_seed=100 + seed, rng_seed=200 + seed, **kw)


def oracle_table(n, B, d, scheme, seed=1, **kw):
    return oracle.OracleTable(n, B, d, scheme, hash_seed=100 + seed, rng_seed=200 + seed, **kw)


def to_dev(a, dtype=np.uint64):
    from paper_1605_05236_amd.table import as_device_keys
    import torch
    a = np.ascontiguousarray(a, dtype=dtype)
    if dtype == np.uint64:
        return as_device_keys(a)
    return torch.from_numpy(a.view(np.int32)).cuda()


def dev_values(vals, B):
    if B == 1:
        return to_dev((vals & np.uint64(0xFFFFFFFF)).astype(np.uint32), np.uint32)
    return to_dev(vals)


def gpu_insert(t, keys, vals):
    r = t.insert(to_dev(keys), dev_values(vals, t.B))
    return {k: v.cpu().numpy().view(np.uint32 if k != "status" else np.uint8)
            for k, v in r.items()}


def gpu_lookup(t, keys, lpp=0):
    v, f = t.lookup(to_dev(keys), lanes_per_probe=lpp)
    v = v.cpu().numpy()
    v = v.view(np.uint32).astype(np.uint64) if t.B == 1 else v.view(np.uint64)
    return v, f.cpu().numpy()


def gpu_delete(t, keys):
    return t.delete(to_dev(keys)).cpu().numpy()


def gpu_overwrite(t, keys, vals):
    return t.overwrite(to_dev(keys), dev_values(vals, t.B)).cpu().numpy()


def assert_same_image(a, b, what=""):
    assert ("stash_keys" in a) == ("stash_keys" in b), f"{what}: one image has a stash"
    for f in ("keys", "vals", "rattle", "meta", "stash_keys", "stash_vals"):
        if f not in b:
            continue
        if not np.array_equal(a[f], b[f]):
            bad = np.nonzero(a[f] != b[f])[0]
            raise AssertionError(f"{what}: {f} differs at {bad.size} entries, first {bad[:8]} "
                                 f"gpu={a[f][bad[:4]]} oracle={b[f][bad[:4]]}")


def assert_same_stats(g, o, what=""):
    for k in o:
        if isinstance(o[k], np.ndarray):
            assert np.array_equal(g[k], o[k]), f"{what}: stats {k} differ"
        else:
            assert g[k] == o[k], f"{what}: stats {k} gpu={g[k]} oracle={o[k]}"


def assert_same_ops(g, o, what=""):
    for k in ("status", "views", "kicks", "retries"):
        ga, oa = g[k].astype(np.int64), o[k].astype(np.int64)
        if not np.array_equal(ga, oa):
            bad = np.nonzero(ga != oa)[0]
            raise AssertionError(f"{what}: per-op {k} differs at {bad.size} ops, first {bad[:8]} "
                                 f"gpu={ga[bad[:4]]} oracle={oa[bad[:4]]}")


def keys_for(n, B, load, seed):
    m = inputs.target_count(n, B, load)
    return inputs.keys_values(seed, m, value_bits=32 if B == 1 else 64)


def gpu_upsert(t, keys, vals):
    r = t.upsert(to_dev(keys), dev_values(vals, t.B))
    return {k: v.cpu().numpy().view(np.uint32 if k != "status" else np.uint8)
            for k, v in r.items()}
