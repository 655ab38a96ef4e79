"""GPU parity of k-at-a-time spawning (BFS and sorted search spawn the k
records at the front of their order together, Sec. 5 Prefetching) against the
oracle, bit-exact: per-op status, views, kicks and lost rounds, the image
(spawn counts included) and every counter."""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from gpu_util import (assert_same_image, assert_same_ops, assert_same_stats, gpu_insert,
                      gpu_lookup, gpu_table, gpu_upsert, keys_for, oracle_table)
from paper_1605_05236_amd import inputs

pytestmark = pytest.mark.gpu

CASES = [  # (scheme, B, ghost, k)
    ("bfs", 8, False, 2), ("bfs", 8, False, 4), ("sorted", 8, False, 2),
    ("sorted", 8, False, 4), ("sorted", 4, False, 8), ("bfs", 4, False, 3),
    ("sorted", 4, True, 4), ("bfs", 8, True, 4),
]


def ident(c):
    return "-".join(str(x) for x in c)


@pytest.mark.parametrize("case", CASES, ids=ident)
@pytest.mark.parametrize("batch", [1 << 8, 777])
def test_spawn_k_fill_parity(case, batch):
    scheme, B, ghost, k = case
    n = 1 << 12
    keys, vals = keys_for(n, B, 0.98, seed=61)
    kw = dict(ghost=ghost, max_search=300, batch_ops=batch, spawn_k=k)
    print(f"spawn_k fill parity {case} batch={batch}", flush=True)
    g = gpu_table(n, B, 2, scheme, seed=61, **kw)
    o = oracle_table(n, B, 2, scheme, seed=61, **kw)
    rg, ro = gpu_insert(g, keys, vals), o.insert(keys, vals)
    assert_same_ops(rg, ro, f"{case}")
    assert_same_image(g.export(), o.export(), f"{case}")
    assert_same_stats(g.stats(), o.stats(), f"{case}")
    ok = ro["status"] == 1
    v, f = gpu_lookup(g, keys[ok])
    assert f.all() and np.array_equal(v, vals[ok])


@pytest.mark.parametrize("case", [("sorted", 8, False, 4), ("bfs", 4, True, 8)], ids=ident)
def test_spawn_k_upsert_parity(case):
    scheme, B, ghost, k = case
    n = 1 << 11
    kw = dict(ghost=ghost, max_search=300, batch_ops=500, spawn_k=k)
    g = gpu_table(n, B, 2, scheme, seed=62, **kw)
    o = oracle_table(n, B, 2, scheme, seed=62, **kw)
    keys, _ = keys_for(n, B, 0.97, seed=62)
    rng = np.random.default_rng(62)
    seen = []
    for step in range(6):
        m = keys.size // 6
        new = keys[step * m:(step + 1) * m]
        old = np.array(seen, np.uint64)[rng.integers(0, len(seen), m // 4)] if seen else \
            np.zeros(0, np.uint64)
        batch = np.concatenate([new, old, new[:m // 10]])
        batch = batch[rng.permutation(batch.size)]
        vals = rng.integers(0, 1 << 63, batch.size, dtype=np.uint64)
        rg, ro = gpu_upsert(g, batch, vals), o.upsert(batch, vals)
        assert_same_ops(rg, ro, f"{case} step {step}")
        assert_same_image(g.export(), o.export(), f"{case} step {step}")
        seen.extend(new[np.isin(new, batch[ro["status"] == 1])].tolist())
    assert_same_stats(g.stats(), o.stats(), f"{case}")


N, BB = 1 << 18, 8
LOADS = (0.95, 0.98)
SHAPE = [("sorted", 4), ("sorted", 2), ("bfs", 4)]


@pytest.fixture(scope="module")
def shape_runs():
    cuts = [0] + [inputs.target_count(N, BB, x) for x in LOADS]
    keys, vals = inputs.keys_values(2, cuts[-1])

    def run(case):
        scheme, k = case
        o = oracle_table(N, BB, 2, scheme, seed=2, max_search=500, batch_ops=1 << 20,
                         spawn_k=k)
        return [(o.insert(keys[a:b], vals[a:b]), o.export(), o.stats())
                for a, b in zip(cuts[:-1], cuts[1:])]

    print(f"oracle: {N} x {BB}, {cuts[-1]} inserts, {SHAPE}", flush=True)
    with ThreadPoolExecutor(len(SHAPE)) as ex:
        runs = dict(zip(SHAPE, ex.map(run, SHAPE)))
    return keys, vals, cuts, runs


@pytest.mark.parametrize("case", SHAPE, ids=ident)
def test_spawn_k_benchmark_shape_parity(shape_runs, case):
    """The benchmark's launch configuration (bins of 8 slots, sub-batches of
    2^20, searches capped at 500 views) on a 2^18 x 8 table, to 95% then 98%."""
    keys, vals, cuts, runs = shape_runs
    scheme, k = case
    g = gpu_table(N, BB, 2, scheme, seed=2, max_search=500, batch_ops=1 << 20, spawn_k=k)
    top = 0
    for (a, b), load, (ro, img, st) in zip(zip(cuts[:-1], cuts[1:]), LOADS, runs[case]):
        what = f"{case} to {load}"
        rg = gpu_insert(g, keys[a:b], vals[a:b])
        assert_same_ops(rg, ro, what)
        assert_same_image(g.export(), img, what)
        assert_same_stats(g.stats(), st, what)
        top = max(top, int(ro["views"].max()))
    assert top > 130, top
