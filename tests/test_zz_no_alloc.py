"""The no-allocation delete (ck_delete_noalloc) against ck_delete: the same
found flags, table image and counters on twin tables, over two calls in a
row (the second smaller), with tables of different geometries sharing the
library's one fixed scratch array in turn; sizes past its limit are refused
before any device work."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_util import assert_same_image, assert_same_stats, gpu_insert, gpu_table, keys_for, \
    to_dev

pytestmark = pytest.mark.gpu

CASES = [  # (scheme, B, d, ghost, stash, batch_ops)
    ("queue", 4, 2, True, 0, 300),
    ("sorted", 8, 2, False, 0, 1 << 12),
    ("random_walk", 4, 2, False, 16, 1 << 16),
    ("rattle", 1, 3, False, 0, 1 << 20),
]


def _twins(scheme, B, d, ghost, stash, batch, seed):
    n = 1 << 11 if B > 1 else 1 << 13
    kw = dict(ghost=ghost, stash=stash, batch_ops=batch, max_chain=8 if stash else 1000,
              max_search=500)
    a = gpu_table(n, B, d, scheme, seed=seed, **kw)
    b = gpu_table(n, B, d, scheme, seed=seed, **kw)
    keys, vals = keys_for(n, B, 1.1 if stash else (0.9 if B == 1 else 0.97), seed=seed + 40)
    ra, rb = gpu_insert(a, keys, vals), gpu_insert(b, keys, vals)
    assert np.array_equal(ra["status"], rb["status"])
    if stash:
        assert (ra["status"] == 6).sum() == stash, "the stash did not fill"
    return a, b, keys, ra["status"]


def _delete_both(a, b, q, what):
    fa = a.delete(to_dev(q)).cpu().numpy()
    fb = b.delete_noalloc(to_dev(q)).cpu().numpy()
    assert np.array_equal(fa, fb), f"{what}: found flags differ"
    assert_same_image(a.export(), b.export(), what)
    sa, sb = a.stats(), b.stats()
    assert_same_stats(sb, sa, what)
    return fa


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(map(str, c)))
def test_noalloc_delete_matches_delete(case):
    scheme, B, d, ghost, stash, batch = case
    print(f"no-alloc delete {case}", flush=True)
    a, b, keys, st = _twins(scheme, B, d, ghost, stash, batch, seed=31)
    held = keys[(st == 1) | (st == 6)]
    rng = np.random.default_rng(31)
    absent = keys_for(64, 4, 1.0, seed=99)[0]
    # call 1: stored keys (some twice), absent keys and the reserved key
    pick = held[rng.permutation(held.size)[: held.size // 2]]
    q1 = np.concatenate([pick, pick[:50], absent, np.array([0xFFFFFFFFFFFFFFFF], np.uint64)])
    q1 = q1[rng.permutation(q1.size)]
    f1 = _delete_both(a, b, q1, f"{case} call 1")
    assert (f1 == 1).sum() == pick.size
    # call 2, smaller: the rest of the stored keys in part, and keys already gone
    rest = np.setdiff1d(held, pick)
    q2 = np.concatenate([rest[: rest.size // 3], pick[:20]])
    f2 = _delete_both(a, b, q2, f"{case} call 2")
    assert (f2 == 1).sum() == rest.size // 3
    assert q2.size < q1.size


def test_noalloc_shared_scratch_across_tables():
    """Two tables of different geometries take turns on the one array: each
    call starts from cleared round counters, whatever the last call left."""
    a1, b1, k1, s1 = _twins("queue", 8, 2, False, 0, 1 << 12, seed=33)
    a2, b2, k2, s2 = _twins("bfs", 2, 2, True, 0, 500, seed=34)
    for step in range(3):
        q1 = k1[(s1 == 1)][step::7][:600]
        q2 = k2[(s2 == 1)][step::5][:900 - 200 * step]
        _delete_both(a1, b1, q1, f"table 1 step {step}")
        _delete_both(a2, b2, q2, f"table 2 step {step}")


def test_noalloc_refuses_oversize_sub_batch():
    from paper_1605_05236_amd import table
    t = gpu_table(1 << 12, 4, 2, "queue", seed=35, batch_ops=1 << 20)
    keys, vals = keys_for(1 << 12, 4, 0.5, seed=35)
    gpu_insert(t, keys, vals)
    before = t.export()
    big = np.concatenate([keys, keys_for(1 << 14, 4, 1.0, seed=36)[0]])
    q = np.resize(big, 65537)  # repeats keys: only a key's first delete finds it
    with pytest.raises(table.CkError):
        t.delete_noalloc(to_dev(q))
    assert_same_image(t.export(), before, "refused call")
    # exactly the limit is accepted
    f = t.delete_noalloc(to_dev(q[:65536])).cpu().numpy()
    assert (f == 1).sum() == np.unique(q[:65536][np.isin(q[:65536], keys)]).size
