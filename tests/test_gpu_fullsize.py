"""The workloads at their full sizes.

The single-table random-walk workload (2^16 bins x 4) is small enough for
element-by-element oracle parity.  The larger ones run in the launch
configuration the benchmark times and are checked through properties that
hold at any size, computed from the inputs alone:
  * every insert that reports success is found, with its value;
  * an insert that reports failure leaves its key absent;
  * never-inserted and deleted keys are absent;
  * the number of distinct stored keys equals successes minus deletes;
  * every stored key sits in one of its own bins, duplicates only as marked
    ghost twins, and rattle counters name the key's bin (independent torch
    re-implementation of the hash, `checks.check_image_torch`)."""
from __future__ import annotations

import numpy as np
import pytest

import checks
from gpu_util import assert_same_image, assert_same_ops, assert_same_stats, gpu_insert, \
    gpu_lookup, gpu_table, oracle_table
from paper_1605_05236_amd import inputs

pytestmark = pytest.mark.gpu


def _table(n, B, d, scheme, **kw):
    from paper_1605_05236_amd.table import CuckooTable
    return CuckooTable(n, B, d, scheme, **kw)


def _lookup_all(t, keys, vals, chunk=1 << 24):
    """All of `keys` found with `vals` (device tensors), in chunks."""
    import torch
    for c0 in range(0, keys.numel(), chunk):
        k = keys[c0:c0 + chunk]
        v, f = t.lookup(k)
        assert bool((f == 1).all()), "a stored key was not found"
        want = vals[c0:c0 + chunk]
        if t.B == 1:
            want = want & 0xFFFFFFFF
            v = v.to(torch.int64) & 0xFFFFFFFF
        assert bool((v == want).all()), "a lookup returned the wrong value"


def _absent(t, keys, chunk=1 << 24):
    for c0 in range(0, keys.numel(), chunk):
        _, f = t.lookup(keys[c0:c0 + chunk])
        assert not bool(f.any()), "an absent key was found"


def _values_for(vals, B):
    import torch
    return (vals & 0xFFFFFFFF).to(torch.int32) if B == 1 else vals


def test_random_walk_2e16x4_full_parity():
    """2^16 bins x 4 slots, two hash functions, random-walk kicking with chains
    capped at 500, filled to 95% in sub-batches of 2^12; then 2^16 lookups, half
    present and half absent.  Bit-exact against the oracle."""
    n, B, d = 1 << 16, 4, 2
    kw = dict(max_chain=500, batch_ops=1 << 12)
    m = inputs.target_count(n, B, 0.95)
    keys, vals = inputs.keys_values(1, m)
    print(f"random walk full parity: {m} inserts", flush=True)
    g = gpu_table(n, B, d, "random_walk", seed=1, **kw)
    o = oracle_table(n, B, d, "random_walk", seed=1, **kw)
    rg, ro = gpu_insert(g, keys, vals), o.insert(keys, vals)
    assert_same_ops(rg, ro, "fill")
    assert_same_image(g.export(), o.export(), "fill")
    assert_same_stats(g.stats(), o.stats(), "fill")
    assert (ro["status"] == 1).all()
    q, present = inputs.lookup_mix(301, keys, m, 1 << 16, 0.5, key_seed=1)
    vg, fg = gpu_lookup(g, q)
    vo, fo = o.lookup(q)
    assert np.array_equal(fg, fo) and np.array_equal(vg, vo)
    assert np.array_equal(fg.astype(bool), present)


@pytest.mark.parametrize("scheme", ["bfs", "sorted", "hybrid", "queue"])
def test_2e24x8_fill_properties(scheme):
    """2^24 bins x 8 slots (2 GiB), sub-batches of 2^20, one call to 95% as the
    benchmark makes it, then on to 98%, then 2^20 deletes."""
    import torch
    n, B = 1 << 24, 8
    t = _table(n, B, 2, scheme, max_search=500, batch_ops=1 << 20, hash_seed=102, rng_seed=202)
    m95 = inputs.target_count(n, B, 0.95)
    m98 = inputs.target_count(n, B, 0.98)
    keys, vals = inputs.keys_values_torch(2, m98)
    absent, _ = inputs.keys_values_torch(2, 1 << 22, start=m98)
    print(f"{scheme}: fill to 95% ({m95} keys)", flush=True)
    st = t.insert(keys[:m95], vals[:m95], diagnostics=False)["status"]
    assert bool((st == 1).all()), f"{int((st != 1).sum())} inserts failed below 95%"
    _lookup_all(t, keys[:m95], vals[:m95])
    _absent(t, absent)
    assert checks.check_image_torch(t.export(), n, B, 2, 102) == m95
    print(f"{scheme}: on to 98% ({m98 - m95} keys)", flush=True)
    st = t.insert(keys[m95:m98], vals[m95:m98], diagnostics=False)["status"]
    ok = torch.cat([torch.ones(m95, dtype=torch.bool, device="cuda"), st == 1])
    _lookup_all(t, keys[ok], vals[ok])
    _absent(t, keys[~ok])
    _absent(t, absent)
    stored = int(ok.sum())
    assert checks.check_image_torch(t.export(), n, B, 2, 102) == stored
    assert t.stats()["stored"] == stored
    g = torch.Generator(device="cuda").manual_seed(402)
    idx = torch.randperm(m95, generator=g, device="cuda")[: 1 << 20]
    f = t.delete(keys[idx])
    assert bool((f == 1).all()), "a stored key was not found by delete"
    _absent(t, keys[idx])
    keep = ok.clone()
    keep[idx] = False
    _lookup_all(t, keys[keep], vals[keep])
    assert checks.check_image_torch(t.export(), n, B, 2, 102) == stored - (1 << 20)


@pytest.mark.parametrize("d,scheme,loads", [(3, "rattle", (0.90, 0.95)),
                                           (3, "random_walk", (0.90, 0.95)),
                                           (4, "rattle", (0.97,)),
                                           (4, "random_walk", (0.97,))])
def test_dary_2e26_slots_properties(d, scheme, loads):
    """Single-slot bins, 2^26 slots of uint64 key + uint32 value, chains capped
    at 1000, sub-batches of 2^20.  Past the d-ary threshold (about 0.918 for
    d = 3) inserts may fail; a failed insert must leave its key absent."""
    import torch
    n = 1 << 26
    t = _table(n, 1, d, scheme, max_chain=1000, batch_ops=1 << 20, hash_seed=103,
               rng_seed=203)
    mt = inputs.target_count(n, 1, loads[-1])
    keys, vals = inputs.keys_values_torch(3, mt, value_bits=32)
    absent, _ = inputs.keys_values_torch(3, 1 << 22, start=mt)
    ok = torch.zeros(mt, dtype=torch.bool, device="cuda")
    done = 0
    for load in loads:
        m = inputs.target_count(n, 1, load)
        print(f"d={d} {scheme}: to {load} ({m} keys)", flush=True)
        st = t.insert(keys[done:m], _values_for(vals[done:m], 1), diagnostics=False)["status"]
        ok[done:m] = st == 1
        done = m
        _lookup_all(t, keys[:m][ok[:m]], vals[:m][ok[:m]])
        _absent(t, keys[:m][~ok[:m]])
        _absent(t, absent)
        stored = int(ok.sum())
        assert checks.check_image_torch(t.export(), n, 1, d, 103, rattle=scheme == "rattle") \
            == stored
        assert t.stats()["stored"] == stored


def test_steady_state_mixed_ghost_queue():
    """2^25 bins x 4 slots prefilled to 97% with queue-kicking and ghost
    insertions, then steps of 2^18 ops: 90% lookups drawn Zipf(0.99) over the
    stored keys, 5% inserts of fresh keys, 5% deletes of random stored keys
    (in each step: lookups, then deletes, then inserts)."""
    import torch
    n, B, steps, step_ops = 1 << 25, 4, 64, 1 << 18
    seed = 4
    t = _table(n, B, 2, "queue", ghost=True, batch_ops=step_ops, hash_seed=104, rng_seed=204)
    m = inputs.target_count(n, B, 0.97)
    print(f"steady state: prefill {m} keys", flush=True)
    rec = torch.arange(m, dtype=torch.int64, device="cuda")
    k, v = inputs.keys_at_torch(seed, rec)
    st = t.insert(k, v, diagnostics=False)["status"]
    stored = rec[st == 1]  # record ids currently stored
    del k, v, st
    zipf = inputs.ZipfTorch(stored.numel(), 0.99)
    gen = torch.Generator(device="cuda").manual_seed(504)
    n_look, n_ins = int(step_ops * 0.9), int(step_ops * 0.05)
    n_del = step_ops - n_look - n_ins
    fresh = m
    failed = 0
    for s in range(steps):
        r = zipf.sample(gen, n_look).clamp_(max=stored.numel() - 1)
        k, v = inputs.keys_at_torch(seed, stored[r])
        got, f = t.lookup(k)
        assert bool((f == 1).all()) and bool((got == v).all()), f"step {s}: lookups"
        pos = torch.unique(torch.randint(0, stored.numel(), (n_del,), generator=gen,
                                         device="cuda"))
        k, _ = inputs.keys_at_torch(seed, stored[pos])
        assert bool((t.delete(k) == 1).all()), f"step {s}: a stored key was not deleted"
        _absent(t, k)
        keep = torch.ones(stored.numel(), dtype=torch.bool, device="cuda")
        keep[pos] = False
        stored = stored[keep]
        new = torch.arange(fresh, fresh + n_ins, dtype=torch.int64, device="cuda")
        fresh += n_ins
        k, v = inputs.keys_at_torch(seed, new)
        st = t.insert(k, v, diagnostics=False)["status"]
        failed += int((st != 1).sum())
        _absent(t, k[st != 1])
        stored = torch.cat([stored, new[st == 1]])
    print(f"steady state: {steps} steps, {failed} failed inserts, stats {t.stats()}",
          flush=True)
    k, v = inputs.keys_at_torch(seed, stored)
    _lookup_all(t, k, v)
    assert checks.check_image_torch(t.export(), n, B, 2, 104, ghost=True) == stored.numel()
    assert t.stats()["stored"] == stored.numel()


def test_arena_growth_stays_bounded():
    """A d-ary random walk past its threshold overflows the first plan arena
    (long walks, many rounds).  The arena doubles only when a round runs out:
    it must end above its first size and below 2 m (max_chain + 1) moves, the
    most one round of m ops can need, doubled.  Results keep their
    properties: stored keys found with their values, failed keys absent."""
    import torch
    n, d, m, chain = 1 << 18, 3, 1 << 16, 1000
    t = _table(n, 1, d, "random_walk", max_chain=chain, batch_ops=m, hash_seed=106,
               rng_seed=206)
    arena0 = t.stats()["arena_moves"]
    total = inputs.target_count(n, 1, 0.93)
    keys, vals = inputs.keys_values_torch(7, total, value_bits=32)
    print(f"arena growth: {total} inserts, first arena {arena0} moves", flush=True)
    st = t.insert(keys, _values_for(vals, 1), diagnostics=False)["status"]
    s = t.stats()
    print(f"arena growth: arena {s['arena_moves']} moves, rounds {s['rounds']}, "
          f"failed {int((st != 1).sum())}", flush=True)
    assert arena0 < s["arena_moves"] <= 2 * m * (chain + 1)
    ok = st == 1
    _lookup_all(t, keys[ok], vals[ok])
    _absent(t, keys[~ok])
    assert checks.check_image_torch(t.export(), n, 1, d, 106) == int(ok.sum())


def test_2e24x8_upsert_properties():
    """The benchmark's table at 95% (queue-kicking), then one upsert call of
    2^21 ops: 2^20 stored keys with new values interleaved with 2^20 absent
    keys, the first 2^16 absent keys given twice more at the end.  A stored
    key reports UPDATED, an absent key OK the first time and UPDATED after;
    every key then holds the value of its last op, and nothing is stored twice."""
    import torch
    n, B = 1 << 24, 8
    t = _table(n, B, 2, "queue", batch_ops=1 << 20, hash_seed=102, rng_seed=202)
    m95 = inputs.target_count(n, B, 0.95)
    keys, vals = inputs.keys_values_torch(2, m95)
    st = t.insert(keys, vals, diagnostics=False)["status"]
    assert bool((st == 1).all())
    g = torch.Generator(device="cuda").manual_seed(403)
    idx = torch.randperm(m95, generator=g, device="cuda")[: 1 << 20]
    fresh, fresh_v = inputs.keys_values_torch(2, 1 << 20, start=m95)
    new_v = torch.randint(0, 1 << 62, (1 << 20,), generator=g, device="cuda", dtype=torch.int64)
    rep_v = torch.randint(0, 1 << 62, (1 << 16,), generator=g, device="cuda", dtype=torch.int64)
    ups = torch.stack([keys[idx], fresh], dim=1).reshape(-1)
    upv = torch.stack([new_v, fresh_v], dim=1).reshape(-1)
    ups = torch.cat([ups, fresh[: 1 << 16]])
    upv = torch.cat([upv, rep_v])
    print(f"upsert {ups.numel()} ops at 95%", flush=True)
    r = t.upsert(ups, upv, diagnostics=False)["status"]
    head = r[: 1 << 21].reshape(-1, 2)
    assert bool((head[:, 0] == 5).all()), "a stored key was not updated"
    assert bool((head[:, 1] == 1).all()), "an absent key was not inserted"
    assert bool((r[1 << 21:] == 5).all()), "a repeated new key was not updated"
    final_v = fresh_v.clone()
    final_v[: 1 << 16] = rep_v
    _lookup_all(t, keys[idx], new_v)
    _lookup_all(t, fresh, final_v)
    stored = m95 + (1 << 20)
    assert t.stats()["stored"] == stored
    assert checks.check_image_torch(t.export(), n, B, 2, 102) == stored


def test_2e24x8_stash_properties():
    """The benchmark's table filled to 98% by BFS with searches capped at 16
    bins, so chains fail in the last sub-batches, with a 64-entry stash: 64
    failures are stashed and found, the rest are absent, and the stash holds
    no key that also sits in a bin."""
    import torch
    n, B = 1 << 24, 8
    t = _table(n, B, 2, "bfs", max_search=16, batch_ops=1 << 20, hash_seed=102, rng_seed=202,
               stash=64)
    m = inputs.target_count(n, B, 0.98)
    keys, vals = inputs.keys_values_torch(2, m)
    print(f"fill to 98% with a stash ({m} keys)", flush=True)
    st = t.insert(keys, vals, diagnostics=False)["status"]
    n_ok, n_st, n_fail = (int((st == s).sum()) for s in (1, 6, 2))
    assert n_ok + n_st + n_fail == m and n_fail > 0, (n_ok, n_st, n_fail)
    assert n_st == 64
    held = (st == 1) | (st == 6)
    _lookup_all(t, keys[held], vals[held])
    _absent(t, keys[st == 2])
    assert t.stats()["stored"] == n_ok + n_st
    assert t.stats()["inserts_stashed"] == 64
    img = t.export()
    assert checks.check_image_torch(img, n, B, 2, 102) == n_ok
    sk = img["stash_keys"]
    stashed = torch.from_numpy(sk.view(np.int64)).cuda()
    assert bool((stashed != -1).all())
    want = torch.sort(keys[st == 6]).values
    assert bool((torch.sort(stashed).values == want).all())
