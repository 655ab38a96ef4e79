"""Pins of the oracle's transactional batches (Sec. 8).

* Transactional correctness (Sec. 8's definition): the table, and every
  answer the transactions got, equal those of running the committed
  transactions one at a time, in commit order, on a textbook dictionary.
* A transaction of one operation is that operation: serially, one-operation
  transactions give the same table and answers as the plain calls.
* Aborted transactions (max_rounds) leave no trace.
"""
from __future__ import annotations

import numpy as np
import pytest

import checks
import oracle
from paper_1605_05236_amd import inputs

LOOKUP, INSERT, DELETE, OVERWRITE = 0, 1, 2, 3


def workload(seed, n_txn, pool, max_ops=10, p_insert=0.35):
    """Transactions over a key pool: every key is inserted at most once (by
    one op), other ops pick any pool key (present or not); some transactions
    touch one key several times (insert, look up, overwrite, delete it)."""
    rng = np.random.default_rng(seed)
    keys_pool, vals_pool = inputs.keys_values(seed, pool)
    fresh = 0
    kinds, keys, vals, off = [], [], [], [0]
    for t in range(n_txn):
        for _ in range(int(rng.integers(1, max_ops + 1))):
            if fresh < pool and rng.random() < p_insert:
                k, v = keys_pool[fresh], vals_pool[fresh]
                fresh += 1
                kinds.append(INSERT)
                keys.append(k)
                vals.append(v)
                if rng.random() < 0.3:  # the transaction works on its own new key
                    for kd in rng.permutation([LOOKUP, OVERWRITE, LOOKUP, DELETE])[:3]:
                        kinds.append(int(kd))
                        keys.append(k)
                        vals.append(rng.integers(0, 1 << 63, dtype=np.uint64))
                continue
            kd = int(rng.choice([LOOKUP, LOOKUP, DELETE, OVERWRITE]))
            kinds.append(kd)
            keys.append(keys_pool[int(rng.integers(0, max(fresh, 1)))])
            vals.append(rng.integers(0, 1 << 63, dtype=np.uint64))
        off.append(len(keys))
    return (np.array(kinds, np.uint8), np.array(keys, np.uint64), np.array(vals, np.uint64),
            np.array(off, np.uint64))


def replay(kinds, keys, vals, off, res, batch, d=None, B=4):
    """Run the committed transactions one at a time in commit order (sub-batch,
    round, index) on a dict; check every answer; return the dict."""
    d = {} if d is None else d
    nt = off.size - 1
    order = sorted(range(nt), key=lambda t: (t // batch, int(res["round"][t]), t))
    mask = np.uint64(0xFFFFFFFF) if B == 1 else np.uint64(0xFFFFFFFFFFFFFFFF)
    for t in order:
        o0, o1 = int(off[t]), int(off[t + 1])
        if (res["status"][o0:o1] == oracle.ST_ABORTED).any():
            assert (res["status"][o0:o1] == oracle.ST_ABORTED).all()
            continue
        for j in range(o0, o1):
            k, st = int(keys[j]), int(res["status"][j])
            if kinds[j] == INSERT:
                assert k not in d
                if st == oracle.ST_OK:
                    d[k] = int(vals[j] & mask)
                else:
                    assert st == oracle.ST_FAIL
            elif kinds[j] == LOOKUP:
                assert st == (oracle.ST_OK if k in d else oracle.ST_NOT_FOUND), (t, j)
                if k in d:
                    assert int(res["value"][j]) == d[k], (t, j)
            elif kinds[j] == DELETE:
                assert st == (oracle.ST_OK if k in d else oracle.ST_NOT_FOUND), (t, j)
                d.pop(k, None)
            else:
                assert st == (oracle.ST_OK if k in d else oracle.ST_NOT_FOUND), (t, j)
                if k in d:
                    d[k] = int(vals[j] & mask)
    return d


def table_dict(t):
    img = t.export()
    occ = img["keys"] != oracle.EMPTY
    return dict(zip(img["keys"][occ].tolist(), img["vals"][occ].tolist()))


@pytest.mark.parametrize("scheme,B,d", [("random_walk", 4, 2), ("bfs", 4, 2), ("sorted", 8, 2),
                                        ("queue", 4, 2), ("hybrid", 2, 2), ("rattle", 1, 3),
                                        ("random_walk", 1, 4)])
@pytest.mark.parametrize("batch", [1, 7, 64])
def test_transactions_are_serializable(scheme, B, d, batch):
    n = 1 << 7 if B > 1 else 1 << 9
    pool = int(0.92 * n * B)
    kinds, keys, vals, off = workload(71, 300, pool)
    if B == 1:
        vals &= np.uint64(0xFFFFFFFF)
    t = oracle.OracleTable(n, B, d, scheme, batch_ops=batch, hash_seed=171, rng_seed=271,
                           max_chain=300, max_search=300)
    res = t.transactions(kinds, keys, vals, off)
    want = replay(kinds, keys, vals, off, res, batch, B=B)
    assert table_dict(t) == want
    held = checks.check_invariants(t.export(), n, B, d, 171, rattle=scheme == "rattle")
    assert held == set(want)
    assert t.stats()["stored"] == len(want)
    if batch == 64:
        assert res["retries"].sum() > 0  # transactions did conflict
        assert (res["status"][kinds == INSERT] == oracle.ST_OK).mean() > 0.9


def test_aborted_transactions_leave_no_trace():
    n, B = 1 << 6, 4
    kinds, keys, vals, off = workload(72, 200, int(0.9 * n * B))
    t = oracle.OracleTable(n, B, 2, "queue", batch_ops=100, max_rounds=1, hash_seed=172)
    res = t.transactions(kinds, keys, vals, off)
    aborted = sum((res["status"][int(off[i]):int(off[i + 1])] == oracle.ST_ABORTED).all()
                  for i in range(off.size - 1) if off[i + 1] > off[i])
    assert aborted > 0
    assert table_dict(t) == replay(kinds, keys, vals, off, res, 100)


def test_transactions_touching_too_many_bins_abort():
    # A plan that touches more distinct bins than the bound aborts whole (its
    # ops report ABORTED, nothing of it is applied); the rest stay serializable.
    n, B = 1 << 6, 4
    kinds, keys, vals, off = workload(75, 120, int(0.97 * n * B), max_ops=6, p_insert=0.8)
    t = oracle.OracleTable(n, B, 2, "random_walk", batch_ops=16, hash_seed=175, rng_seed=275)
    t.set_txn_bins(6)
    res = t.transactions(kinds, keys, vals, off)
    aborted = [i for i in range(off.size - 1)
               if (res["status"][int(off[i]):int(off[i + 1])] == oracle.ST_ABORTED).all()]
    assert 0 < len(aborted) < off.size - 1
    assert table_dict(t) == replay(kinds, keys, vals, off, res, 16)


@pytest.mark.parametrize("scheme", ["random_walk", "sorted", "queue"])
def test_one_op_transactions_are_the_plain_calls(scheme):
    # Serially, a transaction of one operation is that operation (Sec. 1):
    # inserts to 97% (kick-out chains included), then lookups, overwrites
    # and deletes of stored and absent keys.
    n, B = 1 << 9, 4
    m = inputs.target_count(n, B, 0.97)
    keys, vals = inputs.keys_values(73, m)
    kw = dict(batch_ops=1, hash_seed=173, rng_seed=273)
    a = oracle.OracleTable(n, B, 2, scheme, **kw)
    b = oracle.OracleTable(n, B, 2, scheme, **kw)
    b.set_txn_bins(1 << 20)  # no transaction is cut off by its bin count here
    ra = a.insert(keys, vals)
    rb = b.transactions(np.full(m, INSERT, np.uint8), keys, vals, np.arange(m + 1))
    assert np.array_equal(ra["status"], rb["status"])
    for f in ("keys", "vals", "meta"):
        assert np.array_equal(a.export()[f], b.export()[f]), f
    absent, _ = inputs.keys_values(74, 50)
    q = np.concatenate([keys[::5], absent])
    va, fa = a.lookup(q)
    r = b.transactions(np.full(q.size, LOOKUP, np.uint8), q, np.zeros(q.size, np.uint64),
                       np.arange(q.size + 1))
    assert np.array_equal(fa, r["status"]) and np.array_equal(va, r["value"])
    nv = np.arange(q.size, dtype=np.uint64) * np.uint64(7)
    fo, _ = a.overwrite(q, nv)
    r = b.transactions(np.full(q.size, OVERWRITE, np.uint8), q, nv, np.arange(q.size + 1))
    assert np.array_equal(fo, r["status"])
    fd, _ = a.delete(q[::2])
    r = b.transactions(np.full(q[::2].size, DELETE, np.uint8), q[::2],
                       np.zeros(q[::2].size, np.uint64), np.arange(q[::2].size + 1))
    assert np.array_equal(fd, r["status"])
    for f in ("keys", "vals", "meta"):
        assert np.array_equal(a.export()[f], b.export()[f]), f
