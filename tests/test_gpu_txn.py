"""GPU transactional batches (ck_transact, Sec. 8) against the oracle's,
bit-exact: per-op status and value, per-transaction commit round, the whole
image and the counters; and transactional correctness checked directly by a
serial dictionary replay in commit order."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_util import assert_same_image, assert_same_stats, gpu_insert, gpu_table, keys_for, \
    oracle_table, to_dev
from paper_1605_05236_amd import inputs
from test_oracle_txn import replay, table_dict, workload

pytestmark = pytest.mark.gpu


def run_both(g, o, kinds, keys, vals, off):
    import torch
    rg = g.transact(torch.from_numpy(kinds).cuda(), to_dev(keys), to_dev(vals),
                    torch.from_numpy(off.astype(np.int32)).cuda())
    ro = o.transactions(kinds, keys, vals, off)
    st = rg["status"].cpu().numpy()
    va = rg["value"].cpu().numpy().view(np.uint64)
    rd = rg["round"].cpu().numpy().astype(np.uint32)
    assert np.array_equal(st, ro["status"]), np.nonzero(st != ro["status"])[0][:8]
    assert np.array_equal(va, ro["value"])
    assert np.array_equal(rd, ro["round"])
    return ro


CASES = [("random_walk", 4, False), ("random_walk", 8, True), ("queue", 4, False),
         ("queue", 8, False), ("random_walk", 2, False)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(map(str, c)))
@pytest.mark.parametrize("batch", [1, 37, 1 << 12])
def test_transactions_parity(case, batch):
    scheme, B, lb = case
    n = 1 << 9
    pool = int(0.93 * n * B)
    print(f"transactions {case} batch={batch}", flush=True)
    kw = dict(load_balance=lb, batch_ops=batch, max_chain=200)
    g = gpu_table(n, B, 2, scheme, seed=81, **kw)
    o = oracle_table(n, B, 2, scheme, seed=81, **kw)
    # a prefill by plain inserts, then two calls of transactions
    pk, pv = keys_for(n, B, 0.5, seed=181)
    assert np.array_equal(gpu_insert(g, pk, pv)["status"], o.insert(pk, pv)["status"])
    d = dict(zip(pk.tolist(), pv.tolist()))
    for call in range(2):
        kinds, keys, vals, off = workload(82 + call, 400, pool)  # its own key pool
        ro = run_both(g, o, kinds, keys, vals, off)
        d = replay(kinds, keys, vals, off, ro, batch, d)
        assert_same_image(g.export(), o.export(), f"{case} call {call}")
        assert_same_stats(g.stats(), o.stats(), f"{case} call {call}")
    assert table_dict(o) == d
    if batch > 1:
        assert (o.stats()["rounds"] > 4)


def bench_like_workload(seed, n_txn, stored, ops=16):
    """Transactions shaped like the transaction benchmark's: `ops` ops each,
    inserts : deletes : overwrites : reads = 2:1:2:2, inserts of fresh keys,
    the other kinds on keys drawn uniformly from `stored` (present or, once
    deleted, absent)."""
    rng = np.random.default_rng(seed)
    m = n_txn * ops
    kinds = rng.choice(np.array([1, 1, 2, 3, 3, 0, 0], np.uint8), m)
    fresh, fvals = inputs.keys_values(seed + 1000, int((kinds == 1).sum()))
    keys = stored[rng.integers(0, stored.size, m)]
    keys[kinds == 1] = fresh
    vals = rng.integers(0, 1 << 63, m, dtype=np.uint64)
    vals[kinds == 1] = fvals
    off = np.arange(0, m + 1, ops, dtype=np.uint64)
    return kinds, keys, vals, off


def test_transactions_at_the_benchmark_call_shape():
    """2^14 transactions of 16 ops in one call (one sub-batch of the per-call
    cap), random kicking with load balancing on 8-slot bins prefilled to half
    load: the shape the transaction benchmark runs, on a smaller table (the
    oracle takes about 20 s)."""
    n, B = 1 << 19, 8
    kw = dict(load_balance=True, batch_ops=1 << 14, max_chain=500)
    g = gpu_table(n, B, 2, "random_walk", seed=87, **kw)
    o = oracle_table(n, B, 2, "random_walk", seed=87, **kw)
    pk, pv = keys_for(n, B, 0.5, seed=187)
    assert np.array_equal(gpu_insert(g, pk, pv)["status"], o.insert(pk, pv)["status"])
    kinds, keys, vals, off = bench_like_workload(88, 1 << 14, pk)
    print(f"transactions at call shape: {off.size - 1} transactions, {keys.size} ops", flush=True)
    ro = run_both(g, o, kinds, keys, vals, off)
    d = replay(kinds, keys, vals, off, ro, 1 << 14, dict(zip(pk.tolist(), pv.tolist())))
    assert_same_image(g.export(), o.export(), "call shape")
    assert_same_stats(g.stats(), o.stats(), "call shape")
    assert table_dict(o) == d
    assert (ro["round"] > 0).any()  # some transactions lost rounds to others


def test_transactions_abort_paths_parity():
    """A small bin bound and max_rounds: transactions abort for both causes."""
    n, B = 1 << 6, 4
    kinds, keys, vals, off = workload(85, 300, int(0.95 * n * B), max_ops=6, p_insert=0.8)
    g = gpu_table(n, B, 2, "random_walk", seed=85, batch_ops=64, max_rounds=2)
    o = oracle_table(n, B, 2, "random_walk", seed=85, batch_ops=64, max_rounds=2)
    ro = run_both(g, o, kinds, keys, vals, off)
    assert (ro["status"] == 3).any()
    assert_same_image(g.export(), o.export(), "aborts")
    assert_same_stats(g.stats(), o.stats(), "aborts")


def test_transactions_refused_where_unsupported():
    from paper_1605_05236_amd.table import CkError
    import torch
    kinds = torch.zeros(1, dtype=torch.uint8, device="cuda")
    keys = torch.zeros(1, dtype=torch.int64, device="cuda")
    off = torch.tensor([0, 1], dtype=torch.int32, device="cuda")
    for scheme, kw in [("bfs", {}), ("queue", {"ghost": True}), ("random_walk", {"stash": 4})]:
        t = gpu_table(1 << 8, 4, 2, scheme, seed=86, **kw)
        with pytest.raises(CkError):
            t.transact(kinds, keys, keys, off)
