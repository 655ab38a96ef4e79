"""GPU parity of table groups: many tables of uneven sizes served by the same
launches give, table by table, exactly what the oracle gives for each table on
its own (every op carries its table index; tables never interact)."""
from __future__ import annotations

import numpy as np
import pytest

import checks
import oracle
from gpu_util import assert_same_image
from paper_1605_05236_amd import inputs

pytestmark = pytest.mark.gpu


def make_group(bins, B, d, scheme, **kw):
    from paper_1605_05236_amd.table import CuckooGroup
    return CuckooGroup(bins, B, d, scheme, hash_seed=111, rng_seed=222, **kw)


def dev(a, dtype):
    import torch
    a = np.ascontiguousarray(a)
    if dtype == "u64":
        return torch.from_numpy(a.astype(np.uint64).view(np.int64)).cuda()
    if dtype == "u32":
        return torch.from_numpy(a.astype(np.uint32).view(np.int32)).cuda()
    raise ValueError(dtype)


@pytest.mark.parametrize("scheme,B,d,ghost", [("queue", 4, 2, True), ("sorted", 4, 2, False),
                                              ("random_walk", 8, 2, False),
                                              ("bfs", 2, 2, True), ("rattle", 1, 3, False),
                                              ("hybrid", 8, 2, False)])
def test_group_matches_tables_alone(scheme, B, d, ghost):
    rng = np.random.default_rng(7)
    nt = 24
    bins = inputs.log_uniform_int(5, nt, 5, 10)
    bins = np.maximum(bins, 4)
    chunk = 1500
    kw = dict(ghost=ghost, max_chain=1000, max_search=500)
    g = make_group(bins, B, d, scheme, batch_ops=chunk, **kw)
    orc = [oracle.OracleTable(int(n), B, d, scheme, batch_ops=1 << 30, hash_seed=111,
                              rng_seed=222, **kw) for n in bins]
    load = 0.9 if B > 1 else 0.85
    per_table = [inputs.target_count(int(n), B, load) for n in bins]
    # each table's keys from its own segment of one stream; ops interleaved
    keys, vals, tids = [], [], []
    start = 0
    for t, m in enumerate(per_table):
        k, v = inputs.keys_values(31, m, start=start, value_bits=32 if B == 1 else 64)
        start += m
        keys.append(k)
        vals.append(v)
        tids.append(np.full(m, t, np.uint32))
    keys, vals, tids = np.concatenate(keys), np.concatenate(vals), np.concatenate(tids)
    perm = rng.permutation(keys.size)
    keys, vals, tids = keys[perm], vals[perm], tids[perm]
    base = g.insert_count
    import torch
    r = g.insert(dev(tids, "u32"), dev(keys, "u64"),
                 dev(vals & 0xFFFFFFFF, "u32") if B == 1 else dev(vals, "u64"))
    got = {k: v.cpu().numpy().view(np.uint8 if k == "status" else np.uint32) for k, v in r.items()}
    # the oracle: per chunk of the call, each table's ops of that chunk are one sub-batch
    for c0 in range(0, keys.size, chunk):
        c1 = min(keys.size, c0 + chunk)
        for t in range(nt):
            pos = np.nonzero(tids[c0:c1] == t)[0] + c0
            if pos.size == 0:
                continue
            ro = orc[t].insert(keys[pos], vals[pos], op_ids=base + pos)
            for f in ("status", "views", "kicks", "retries"):
                assert np.array_equal(got[f][pos].astype(np.int64), ro[f].astype(np.int64)), \
                    (scheme, t, f)
    for t in range(nt):
        img = g.export_table(t)
        assert_same_image(img, orc[t].export(), f"{scheme} table {t}")
    # lookups, overwrites and deletes through the group
    q = np.concatenate([keys[::3], inputs.keys_values(32, 500)[0]])
    qt = np.concatenate([tids[::3], rng.integers(0, nt, 500).astype(np.uint32)])
    v, f = g.lookup(dev(qt, "u32"), dev(q, "u64"))
    v = v.cpu().numpy()
    v = v.view(np.uint32).astype(np.uint64) if B == 1 else v.view(np.uint64)
    f = f.cpu().numpy()
    for t in range(nt):
        pos = np.nonzero(qt == t)[0]
        vo, fo = orc[t].lookup(q[pos])
        assert np.array_equal(f[pos], fo) and np.array_equal(v[pos], vo)
    # new values through the group (stored keys and a few absent ones)
    ok_, ot = np.concatenate([keys[1::4], q[-50:]]), np.concatenate([tids[1::4], qt[-50:]])
    nv = rng.integers(0, 1 << 63, ok_.size, dtype=np.uint64)
    if B == 1:
        nv &= np.uint64(0xFFFFFFFF)
    fw = g.overwrite(dev(ot, "u32"), dev(ok_, "u64"), dev(nv, "u32" if B == 1 else "u64"))
    fw = fw.cpu().numpy()
    for c0 in range(0, ok_.size, chunk):
        c1 = min(ok_.size, c0 + chunk)
        for t in range(nt):
            pos = np.nonzero(ot[c0:c1] == t)[0] + c0
            if pos.size:
                assert np.array_equal(fw[pos], orc[t].overwrite(ok_[pos], nv[pos])[0])
    # upserts through the group: stored keys, new keys (some twice), per table
    # and per chunk as the oracle's sub-batches
    nk, _ = inputs.keys_values(33, 400, value_bits=32 if B == 1 else 64)
    nt_ = rng.integers(0, nt, 400).astype(np.uint32)
    uk = np.concatenate([keys[2::7], nk, nk[:60]])
    ut = np.concatenate([tids[2::7], nt_, nt_[:60]])
    perm = rng.permutation(uk.size)
    uk, ut = uk[perm], ut[perm]
    uv = rng.integers(0, 1 << 63, uk.size, dtype=np.uint64)
    if B == 1:
        uv &= np.uint64(0xFFFFFFFF)
    base = g.insert_count
    ru = g.upsert(dev(ut, "u32"), dev(uk, "u64"), dev(uv, "u32" if B == 1 else "u64"))
    ru = {k: v.cpu().numpy().view(np.uint8 if k == "status" else np.uint32) for k, v in ru.items()}
    for c0 in range(0, uk.size, chunk):
        c1 = min(uk.size, c0 + chunk)
        for t in range(nt):
            pos = np.nonzero(ut[c0:c1] == t)[0] + c0
            if pos.size == 0:
                continue
            ro = orc[t].upsert(uk[pos], uv[pos], op_ids=base + pos)
            for f in ("status", "views", "kicks", "retries"):
                assert np.array_equal(ru[f][pos].astype(np.int64), ro[f].astype(np.int64)), \
                    (scheme, t, f, "upsert")
    assert (ru["status"] == oracle.ST_UPDATED).sum() >= (got["status"][2::7] == 1).sum()
    dk, dt = keys[::5], tids[::5]
    fd = g.delete(dev(dt, "u32"), dev(dk, "u64")).cpu().numpy()
    for c0 in range(0, dk.size, chunk):
        c1 = min(dk.size, c0 + chunk)
        for t in range(nt):
            pos = np.nonzero(dt[c0:c1] == t)[0] + c0
            if pos.size:
                assert np.array_equal(fd[pos], orc[t].delete(dk[pos])[0])
    for t in range(nt):
        img = g.export_table(t)
        assert_same_image(img, orc[t].export(), f"{scheme} table {t} after deletes")
        checks.check_invariants(img, int(bins[t]), B, d, 111, ghost=ghost,
                                rattle=scheme == "rattle")
    del torch


@pytest.mark.parametrize("scheme,B,d", [("random_walk", 4, 2), ("bfs", 2, 2), ("rattle", 1, 3)])
def test_group_stash_per_table(scheme, B, d):
    # Each table of a group has its own stash (Sec. 2): small tables driven
    # past their failure load give, table by table, what the oracle gives.
    rng = np.random.default_rng(9)
    nt = 12
    bins = np.maximum(inputs.log_uniform_int(6, nt, 4, 7), 8)
    chunk = 700
    kw = dict(max_chain=4, max_search=8, stash=4)
    g = make_group(bins, B, d, scheme, batch_ops=chunk, **kw)
    orc = [oracle.OracleTable(int(n), B, d, scheme, batch_ops=1 << 30, hash_seed=111,
                              rng_seed=222, **kw) for n in bins]
    per_table = [inputs.target_count(int(n), B, 1.05) for n in bins]
    keys, vals, tids = [], [], []
    start = 0
    for t, m in enumerate(per_table):
        k, v = inputs.keys_values(41, m, start=start, value_bits=32 if B == 1 else 64)
        start += m
        keys.append(k)
        vals.append(v)
        tids.append(np.full(m, t, np.uint32))
    keys, vals, tids = np.concatenate(keys), np.concatenate(vals), np.concatenate(tids)
    perm = rng.permutation(keys.size)
    keys, vals, tids = keys[perm], vals[perm], tids[perm]
    base = g.insert_count
    r = g.insert(dev(tids, "u32"), dev(keys, "u64"),
                 dev(vals & 0xFFFFFFFF, "u32") if B == 1 else dev(vals, "u64"))
    got = {k: v.cpu().numpy().view(np.uint8 if k == "status" else np.uint32) for k, v in r.items()}
    for c0 in range(0, keys.size, chunk):
        c1 = min(keys.size, c0 + chunk)
        for t in range(nt):
            pos = np.nonzero(tids[c0:c1] == t)[0] + c0
            if pos.size == 0:
                continue
            ro = orc[t].insert(keys[pos], vals[pos], op_ids=base + pos)
            for f in ("status", "views", "kicks", "retries"):
                assert np.array_equal(got[f][pos].astype(np.int64), ro[f].astype(np.int64)), \
                    (scheme, t, f)
    assert (got["status"] == oracle.ST_STASHED).sum() > 0
    for t in range(nt):
        assert_same_image(g.export_table(t), orc[t].export(), f"{scheme} table {t}")
    # every key held is found, stashed ones included
    held = np.isin(got["status"], (oracle.ST_OK, oracle.ST_STASHED))
    v, f = g.lookup(dev(tids[held], "u32"), dev(keys[held], "u64"))
    v = v.cpu().numpy()
    v = v.view(np.uint32).astype(np.uint64) if B == 1 else v.view(np.uint64)
    mask = np.uint64(0xFFFFFFFF) if B == 1 else np.uint64(0xFFFFFFFFFFFFFFFF)
    assert f.cpu().numpy().all() and np.array_equal(v, vals[held] & mask)
